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
// A lane owns one (il, xl) column of the region, so its reflected in-plane offset is
// computed once; the lanes split into as many groups as there are whole columns sets in
// the workgroup, and group g walks the t planes g, g + G, ...  The loads of up to
// kStageBatch planes are issued before any of them is stored; every address is reflected
// and clamped into the volume, so the loads are unconditional and only the stores are
// masked.
constexpr int kStageBatch = 16;

template <int NT>
__device__ __forceinline__ void stage_tile(const float* __restrict__ V, int64_t T, int64_t IL, int64_t XL,
                                           int64_t t0, int64_t i0, int64_t x0, int RT, int RI, int RX, int RXp,
                                           float* __restrict__ Vt) {
    const int PQ = RI * RX;
    const int G = PQ >= NT ? 1 : NT / PQ;
    const int g = (int)threadIdx.x / PQ;
    if (g >= G) return;
    const int64_t PS = IL * XL;
    const int plane = RI * RXp;
    for (int q = (int)threadIdx.x - g * PQ; q < PQ; q += NT) {
        const int ri = q / RX, rx = q - ri * RX;
        const int64_t off = reflect_clamp_s(i0 + ri, IL) * XL + reflect_clamp_s(x0 + rx, XL);
        const float* src = V + off;
        float* dst = Vt + ri * RXp + rx;
        for (int rt0 = g; rt0 < RT; rt0 += G * kStageBatch) {
            float v[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; u++) {
                const int rt = min(rt0 + u * G, RT - 1);
                v[u] = src[reflect_clamp_s(t0 + rt, T) * PS];
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; u++) {
                const int rt = rt0 + u * G;
                if (rt < RT) dst[rt * plane] = v[u];
            }
        }
    }
}

}  // namespace sal
