// gfx950 matrix-core wrappers used by the LLOID kernels.
//
// Lane layout of the 16x16 MFMA family (wave64), for C = A x B with
// A [16][K], B [K][16], C [16][16]:
//   A: lane l supplies row  l % 16, the K-group l / 16
//   B: lane l supplies column l % 16, the K-group l / 16
//   C: lane l holds rows 4 (l / 16) + v, v = 0..3, of column l % 16
// 16x16x4 f32: one K element per lane and group (K = 4);
// 16x16x32 bf16/f16: eight consecutive K elements per lane and group (K = 32).
// A and B must use the same K assignment; the sum over K does not depend
// on which lane holds which K element.
#pragma once
#include <hip/hip_runtime.h>

namespace lloid {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma_16x16x4_f32(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_16x16x32_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_16x16x32_f16(halfx8 a, halfx8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) { return mfma_16x16x32_bf16(a, b, c); }
__device__ __forceinline__ floatx4 mfma16(halfx8 a, halfx8 b, floatx4 c) { return mfma_16x16x32_f16(a, b, c); }

}  // namespace lloid
