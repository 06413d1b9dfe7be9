// Small device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace lloid
