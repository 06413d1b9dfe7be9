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
