// sal_stage.h -- staging of a tile plus its window halo from HBM into LDS (shared by the
// feature and adjoint kernels; not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sal {

// Half-sample reflection, then a clamp that keeps the (never used) positions of
// centres beyond the grid inside the volume.
__device__ __forceinline__ int64_t reflect_clamp_s(int64_t p, int64_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p < 0 ? 0 : (p >= N ? N - 1 : p);
}

// Copy the region [RT][RI][RX] starting at voxel (t0, i0, x0) into Vt with row pitch RXp.
// Waves take (t, il) rows, lanes the xl samples of a row (two rows per wave when a row
// fits in 32 lanes), so each lane's xl index and its reflection are fixed.
template <int NT>
__device__ __forceinline__ void stage_tile(const float* __restrict__ V, int64_t T, int64_t IL, int64_t XL,
                                           int64_t t0, int64_t i0, int64_t x0, int RT, int RI, int RX, int RXp,
                                           float* __restrict__ Vt) {
    constexpr int NWAVES = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool two = RX <= 32;
    const int sub = two ? (lane >> 5) : 0;
    const int rx = two ? (lane & 31) : lane;
    const int step = two ? 2 * NWAVES : NWAVES;
    const int nrows = RT * RI;
    const bool act = rx < RX;
    const int64_t gx = reflect_clamp_s(x0 + rx, XL);
    for (int r = (two ? 2 * wave : wave) + sub; r < nrows + sub; r += step) {
        if (r < nrows && act) {
            const int rt = r / RI, ri = r - rt * RI;
            const int64_t gt = reflect_clamp_s(t0 + rt, T), gi = reflect_clamp_s(i0 + ri, IL);
            Vt[r * RXp + rx] = V[(gt * IL + gi) * XL + gx];
        }
    }
}

}  // namespace sal
