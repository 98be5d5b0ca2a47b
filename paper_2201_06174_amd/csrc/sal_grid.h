// sal_grid.h -- launch geometry for grids of any size (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sal {

// A dispatch counts the work-items of each grid dimension in 32 bits, so a launch of
// `nblocks` workgroups of `block` threads spreads over y when x alone would pass 2^31
// work-items.  x stays a multiple of 8, so a workgroup's linear id y * gridDim.x + x has the
// same residue modulo 8 (its XCD in the round-robin over the 8 XCDs) as in a 1D launch.
// Workgroups with a linear id >= nblocks are padding.
inline dim3 wide_grid(int64_t nblocks, int block) {
    const int64_t xmax = (((int64_t)1 << 31) / block) / 8 * 8;
    if (nblocks <= xmax) return dim3((unsigned)(nblocks > 0 ? nblocks : 1));
    return dim3((unsigned)xmax, (unsigned)((nblocks + xmax - 1) / xmax));
}

// The y extent a wide_grid launch may take (HIP's limit for the second grid dimension).
constexpr int64_t kMaxGridY = 65535;

inline bool wide_grid_fits(int64_t nblocks, int block) {
    const int64_t xmax = (((int64_t)1 << 31) / block) / 8 * 8;
    return (nblocks + xmax - 1) / xmax <= kMaxGridY;
}

__device__ __forceinline__ int64_t block_id() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }

// Workgroups are dealt to the 8 XCDs round-robin.  xcd_block(nblocks) renumbers a launch of
// xcd_grid(nblocks) workgroups so that each XCD takes a contiguous eighth of the range
// [0, nblocks) (its neighbour reads then stay in that XCD's L2); a result >= nblocks is
// padding and does nothing.
inline int64_t xcd_grid(int64_t nblocks) { return 8 * ((nblocks + 7) / 8); }

__device__ __forceinline__ int64_t xcd_block(int64_t nblocks) {
    const int64_t b = block_id(), per = (nblocks + 7) / 8;
    return b < 8 * per ? (b % 8) * per + b / 8 : nblocks;
}

}  // namespace sal
