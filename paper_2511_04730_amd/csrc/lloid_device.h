// Small device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lloid_internal.h"

namespace lloid {

// a mod m in [0, m) for negative a too
__device__ __forceinline__ int64_t posmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

// trigger candidate: max |z|^2, first index on ties
struct PeakCand {
    float p2;
    int idx;
    float re, im;
};

__device__ __forceinline__ bool better(float p2, int idx, float bp2, int bidx) {
    return p2 > bp2 || (p2 == bp2 && idx < bidx);
}

// Raw buffer resource over [base, base + bytes) (gfx9 descriptor word 3);
// loads through it take a 32-bit per-lane offset plus a scalar offset, and
// return zero outside the range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename V>
__device__ __forceinline__ V buffer_load16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// A load through a pointer known to address global memory (pointers read
// from work tables are generic; flat loads also count against the LDS
// counter, so their waits cover both).
template <typename V>
__device__ __forceinline__ V ld_global(const void *p) {
    return *(const __attribute__((address_space(1))) V *)(p);
}

// Element (pos, l) of one plane of a basis-output ring and element (r, l) of
// a mixing matrix in fragment order (layouts in MixSlice); G = 16 / element size.
template <int G>
__device__ __forceinline__ int64_t ring_index(int64_t pos, int l, int capY) {
    return ((int64_t)(l / G) * 2 * capY + pos) * G + l % G;
}
template <int G>
__device__ __forceinline__ int64_t frag_index(int r, int l, int Lpad) {
    return ((int64_t)(r >> 4) * (Lpad / G) + l / G) * (16 * G) + (r & 15) * G + l % G;
}

// Work item of this work group when `group` consecutive items are to share
// one XCD (and its L2): the dispatcher deals work groups to the XCDs in turn,
// so group b runs on XCD b mod kXcds.  group <= 0 keeps the launch order.
// The grid is xcd_grid(n, group) long; items >= n exit at once.
__device__ __forceinline__ int xcd_item(int group) {
    const int b = blockIdx.x;
    if (group <= 0) return b;
    const int x = b % kXcds, k = b / kXcds;
    return ((k / group) * kXcds + x) * group + k % group;
}

}  // namespace lloid
