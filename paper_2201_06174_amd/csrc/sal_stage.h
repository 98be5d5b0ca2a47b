// sal_stage.h -- staging of a tile plus its window halo from HBM into LDS (shared by the
// feature and adjoint kernels; not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace sal {

// Half-sample reflection, then a clamp that keeps the (never used) positions of
// centres beyond the grid inside the volume.
__device__ __forceinline__ int64_t reflect_clamp_s(int64_t p, int64_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p < 0 ? 0 : (p >= N ? N - 1 : p);
}
// The same in 32 bits: for a wave-uniform plane index it stays on the scalar unit, which
// has no 64-bit signed compare.
__device__ __forceinline__ int32_t reflect_clamp_s32(int32_t p, int32_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p < 0 ? 0 : (p >= N ? N - 1 : p);
}

// Hand every sample of the region [RT][RI][RX] starting at voxel (t0, i0, x0) to
// store(rt, ri, rx, value).
// A lane owns one (il, xl) column of the region, so its reflected in-plane offset is
// computed once.  Whole waves form groups that each cover every column (64 lanes per wave,
// the last wave of a group partly idle); group g walks the t planes g, g + G, ..., so a
// plane index, its reflection and its base address are the same across the wave and stay
// in scalar registers.  The loads of up to kStageBatch planes are issued before any of them
// is stored; every address is reflected and clamped into the volume, so the loads are
// unconditional and only the stores are masked.
constexpr int kStageBatch = 16;

// MAXU bounds the t planes one group loads per batch (at most kStageBatch); a kernel whose
// region extents are fixed at compile time passes stage_batch(...) so the unrolled batch has
// only the steps a group can own.
template <int NT, int MAXU = kStageBatch, typename Store>
__device__ __forceinline__ void stage_tile_with(const float* __restrict__ V, int64_t T, int64_t IL, int64_t XL,
                                                int64_t t0, int64_t i0, int64_t x0, int RT, int RI, int RX,
                                                Store store) {
    constexpr int NWV = NT / 64;
    const int PQ = RI * RX;
    const int WPG = (PQ + 63) / 64;                // waves per column set
    const int G = WPG <= NWV ? NWV / WPG : 1;       // groups of waves
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = wave / WPG;
    if (g >= G) return;
    const int64_t PS = IL * XL;
    // a volume below 2^31 samples takes 32-bit plane offsets (scalar) on a 32-bit lane offset
    const bool small = T * PS < (int64_t(1) << 31);
    // waves of a group (or, with fewer waves than a column set, all waves in turn) take
    // consecutive 64-column slices
    const int wstep = G == 1 ? NWV : WPG;
    for (int q = (wave - g * WPG) * 64 + lane, q0 = (wave - g * WPG) * 64; q0 < PQ; q += wstep * 64, q0 += wstep * 64) {
        const bool act = q < PQ;
        const int qc = act ? q : PQ - 1;
        const int ri = qc / RX, rx = qc - ri * RX;
        const int64_t off = reflect_clamp_s(i0 + ri, IL) * XL + reflect_clamp_s(x0 + rx, XL);
        const uint32_t off32 = (uint32_t)off;
        // SMALL: 32-bit plane offsets, reflected on the scalar unit
        auto planes = [&](auto is_small) {
            constexpr bool SMALL = decltype(is_small)::value;
            for (int rt0 = g; rt0 < RT; rt0 += G * MAXU) {
                float v[MAXU];
#pragma unroll
                for (int u = 0; u < MAXU; u++) {
                    // a group of a small region owns far fewer planes than a batch: steps past
                    // every group's last plane are not issued (a test uniform over the workgroup,
                    // fixed at compile time for fixed extents); a group's last step may still
                    // read the last plane again
                    if (u * G >= RT) break;
                    const int rt = min(rt0 + u * G, RT - 1);
                    const float* pb =
                        SMALL ? V + (uint32_t)reflect_clamp_s32((int32_t)t0 + rt, (int32_t)T) * (uint32_t)PS
                              : V + reflect_clamp_s(t0 + rt, T) * PS;
                    // a plane below 2^30 samples takes a 32-bit lane offset on a scalar base
                    v[u] = SMALL || PS < (int64_t(1) << 30) ? pb[off32] : pb[off];
                }
#pragma unroll
                for (int u = 0; u < MAXU; u++) {
                    const int rt = rt0 + u * G;
                    if (rt < RT && act) store(rt, ri, rx, v[u]);
                }
            }
        };
        if (small) planes(std::true_type{});
        else planes(std::false_type{});
    }
}

// Split form of stage_tile for a region whose columns fit the waves in one pass
// (RI * RX <= NT) and whose planes fit NPL per lane (stage_planes() <= NPL):
// stage_issue starts the loads of a region into registers, stage_commit stores them, so
// their latency is covered by the work in between (the next tile's region is fetched while
// the current tile finishes).  The lane's position is recomputed by stage_commit, so only
// the loaded values stay live in between.
struct StageLane {
    int g, G, ri, rx;
    bool act;
};

template <int NT>
__device__ __forceinline__ StageLane stage_lane(int RI, int RX) {
    constexpr int NWV = NT / 64;
    const int PQ = RI * RX;
    const int WPG = (PQ + 63) / 64;
    StageLane L;
    L.G = NWV / WPG;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    L.g = wave / WPG;
    const int q = (wave - L.g * WPG) * 64 + (int)(threadIdx.x & 63);
    L.act = L.g < L.G && q < PQ;
    const int qc = q < PQ ? q : PQ - 1;
    L.ri = qc / RX;
    L.rx = qc - L.ri * RX;
    return L;
}

// t planes per lane of the split form (0 if the columns do not fit the waves in one pass)
template <int NT>
__host__ __device__ constexpr int stage_planes(int RT, int RI, int RX) {
    return (RI * RX + 63) / 64 > NT / 64 ? 0 : (RT + NT / 64 / ((RI * RX + 63) / 64) - 1) / (NT / 64 / ((RI * RX + 63) / 64));
}

// Batch bound of stage_tile for a region of at most RT x RI x RX samples: the planes a group
// owns, or a full batch where the columns take several passes.
template <int NT>
__host__ __device__ constexpr int stage_batch(int RT, int RI, int RX) {
    return stage_planes<NT>(RT, RI, RX) > 0 && stage_planes<NT>(RT, RI, RX) < kStageBatch ? stage_planes<NT>(RT, RI, RX)
                                                                                           : kStageBatch;
}

template <int NT, int NPL>
__device__ __forceinline__ void stage_issue(float (&v)[NPL], const float* __restrict__ V, int64_t T, int64_t IL,
                                            int64_t XL, int64_t t0, int64_t i0, int64_t x0, int RT, int RI, int RX) {
    const StageLane L = stage_lane<NT>(RI, RX);
    if (L.g >= L.G) return;  // wave-uniform: idle waves issue nothing
    const int64_t PS = IL * XL;
    const int64_t off = reflect_clamp_s(i0 + L.ri, IL) * XL + reflect_clamp_s(x0 + L.rx, XL);
    // a volume below 2^31 samples takes 32-bit offsets (the plane's on the scalar unit)
    if (T * PS < (int64_t(1) << 31)) {
#pragma unroll
        for (int u = 0; u < NPL; u++) {
            const int rt = min(L.g + u * L.G, RT - 1);
            const float* pb = V + (uint32_t)reflect_clamp_s32((int32_t)t0 + rt, (int32_t)T) * (uint32_t)PS;
            v[u] = pb[(uint32_t)off];
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < NPL; u++) {
        const int rt = min(L.g + u * L.G, RT - 1);
        v[u] = V[reflect_clamp_s(t0 + rt, T) * PS + off];
    }
}

template <int NT, int NPL>
__device__ __forceinline__ void stage_commit(const float (&v)[NPL], int RT, int RI, int RX, int RXp,
                                             float* __restrict__ Vt) {
    const StageLane L = stage_lane<NT>(RI, RX);
    if (L.g >= L.G) return;
#pragma unroll
    for (int u = 0; u < NPL; u++) {
        const int rt = L.g + u * L.G;
        if (rt < RT && L.act) Vt[(rt * RI + L.ri) * RXp + L.rx] = v[u];
    }
}

// fp32 rows of pitch RXp: Vt[(rt * RI + ri) * RXp + rx]
template <int NT, int MAXU = kStageBatch>
__device__ __forceinline__ void stage_tile(const float* __restrict__ V, int64_t T, int64_t IL, int64_t XL,
                                           int64_t t0, int64_t i0, int64_t x0, int RT, int RI, int RX, int RXp,
                                           float* __restrict__ Vt) {
    stage_tile_with<NT, MAXU>(V, T, IL, XL, t0, i0, x0, RT, RI, RX,
                        [&](int rt, int ri, int rx, float v) { Vt[(rt * RI + ri) * RXp + rx] = v; });
}

}  // namespace sal
