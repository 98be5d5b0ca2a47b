// sal_adapt.hip -- sequential LMS / NLMS / RLS adaptation of the fusion weights (Sec. 2, fusion
// paragraph and Fig. 6): the weights W of Eq. 4 updated sample by sample towards the desired
// map D over the masked grid points of each weight group, in memory order, `passes` sweeps.
//
// Samples must be taken one after the other, so the recursion itself runs on one wavefront
// per weight group; what can run wide runs wide: the masked points of each group are first
// compacted into an index list in memory order (a count and a write kernel over many blocks,
// each block's offset the sum of the counts before it, in a fixed order), and the wave loads
// 64 samples at a time with one lane per sample before walking them in order.  Every lane
// runs the same FP64 update on values broadcast from the sample's lane, so the result is
// independent of timing and bitwise reproducible.
#include <hip/hip_runtime.h>

#include "sal_aux.h"
#include "sal_grid.h"

namespace sal {

constexpr int kSeqBlocks = 256;  // compaction blocks per weight group

// Range [lo, hi) of group positions (memory order inside the group) handled by block b.
__device__ __forceinline__ void seq_chunk(int64_t count, int b, int64_t* lo, int64_t* hi) {
    const int64_t per = (count + kSeqBlocks - 1) / kSeqBlocks;
    *lo = (int64_t)b * per < count ? (int64_t)b * per : count;
    *hi = *lo + per < count ? *lo + per : count;
}

__device__ __forceinline__ int64_t group_point(int64_t e, int64_t slab, int64_t plane, int64_t first) {
    return (e / slab) * plane + first + e % slab;
}

// Masked points per (group, block).
__global__ __launch_bounds__(256) void k_seq_count(const uint8_t* __restrict__ mask, int64_t Tg, int64_t ILg,
                                                   int64_t XLg, int64_t sections, int* __restrict__ counts) {
    __shared__ int red[256];
    const int64_t k = blockIdx.y;
    const int64_t il0 = sections > 0 ? k * sections : 0;
    const int64_t nk = sections > 0 ? (ILg - il0 < sections ? ILg - il0 : sections) : ILg;
    const int64_t slab = nk * XLg, plane = ILg * XLg, first = il0 * XLg, count = Tg * slab;
    int64_t lo, hi;
    seq_chunk(count, blockIdx.x, &lo, &hi);
    int c = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x)
        c += !mask || mask[group_point(e, slab, plane, first)] != 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[k * kSeqBlocks + blockIdx.x] = red[0];
}

// The masked points of each group in memory order: idx[base_k + rank] = grid point, base_k =
// the group's first position in the whole grid (Tg * XLg * k * sections).
__global__ __launch_bounds__(256) void k_seq_compact(const uint8_t* __restrict__ mask, int64_t Tg, int64_t ILg,
                                                     int64_t XLg, int64_t sections, const int* __restrict__ counts,
                                                     int* __restrict__ idx) {
    __shared__ int scan[256];
    __shared__ int64_t base;
    const int64_t k = blockIdx.y;
    const int64_t il0 = sections > 0 ? k * sections : 0;
    const int64_t nk = sections > 0 ? (ILg - il0 < sections ? ILg - il0 : sections) : ILg;
    const int64_t slab = nk * XLg, plane = ILg * XLg, first = il0 * XLg, count = Tg * slab;
    if (threadIdx.x == 0) {
        int64_t o = Tg * XLg * il0;
        for (int b = 0; b < (int)blockIdx.x; b++) o += counts[k * kSeqBlocks + b];
        base = o;
    }
    __syncthreads();
    int64_t lo, hi;
    seq_chunk(count, blockIdx.x, &lo, &hi);
    int64_t out = base;
    for (int64_t e0 = lo; e0 < hi; e0 += blockDim.x) {
        const int64_t e = e0 + threadIdx.x;
        const int64_t j = e < hi ? group_point(e, slab, plane, first) : 0;
        const int in = e < hi && (!mask || mask[j] != 0);
        // inclusive scan of the flags (Hillis-Steele in LDS; integer, so order-free)
        scan[threadIdx.x] = in;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int v = (int)threadIdx.x >= d ? scan[threadIdx.x - d] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        if (in) idx[out + scan[threadIdx.x] - 1] = (int)j;
        out += scan[255];
        __syncthreads();
    }
}

// One wavefront per weight group: the recursion over the group's compacted samples.
// W: [K][4] (weights, then 0); err2: [K][cap] squared a priori errors in update order (or
// nullptr); count: [K] samples per pass (or nullptr).
__global__ __launch_bounds__(64) void k_seq_adapt(const float* __restrict__ Sm, const float* __restrict__ D,
                                                  int64_t Tg, int64_t ILg, int64_t XLg, int64_t sections,
                                                  const int* __restrict__ counts, const int* __restrict__ idx, int rule,
                                                  double mu, double eps, double lambda, double delta, double w00,
                                                  double w01, double w02, int passes, double* __restrict__ W,
                                                  float* __restrict__ err2, int64_t cap, int64_t* __restrict__ count) {
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t G = Tg * ILg * XLg;
    const int64_t il0 = sections > 0 ? k * sections : 0;
    // samples of the group: lane-strided sums of the block counts, then a fixed tree
    int64_t m = 0;
    for (int b = lane; b < kSeqBlocks; b += 64) m += counts[k * kSeqBlocks + b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o);
    const int* list = idx + Tg * XLg * il0;
    double w0 = w00, w1 = w01, w2 = w02;
    const double p0 = 1.0 / delta;
    double P00 = p0, P01 = 0.0, P02 = 0.0, P11 = p0, P12 = 0.0, P22 = p0;  // symmetric
    int64_t it = 0;
    for (int pass = 0; pass < passes; pass++) {
        for (int64_t c0 = 0; c0 < m; c0 += 64) {
            // lane l holds sample c0 + l
            double ul0 = 0.0, ul1 = 0.0, ul2 = 0.0, dl = 0.0;
            if (c0 + lane < m) {
                const int64_t j = list[c0 + lane];
                ul0 = Sm[j];
                ul1 = Sm[G + j];
                ul2 = Sm[2 * G + j];
                dl = D[j];
            }
            const int nc = m - c0 < 64 ? (int)(m - c0) : 64;
            for (int i = 0; i < nc; i++) {
                const double u0 = __shfl(ul0, i), u1 = __shfl(ul1, i), u2 = __shfl(ul2, i), d = __shfl(dl, i);
                const double e = d - (w0 * u0 + w1 * u1 + w2 * u2);
                if (err2 && lane == 0 && it < cap) err2[k * cap + it] = (float)(e * e);
                if (rule == SAL_FUSE_LMS) {
                    const double g = mu * e;
                    w0 += g * u0;
                    w1 += g * u1;
                    w2 += g * u2;
                } else if (rule == SAL_FUSE_NLMS) {
                    const double g = mu * e / (eps + (u0 * u0 + u1 * u1 + u2 * u2));
                    w0 += g * u0;
                    w1 += g * u1;
                    w2 += g * u2;
                } else {
                    const double q0 = P00 * u0 + P01 * u1 + P02 * u2;
                    const double q1 = P01 * u0 + P11 * u1 + P12 * u2;
                    const double q2 = P02 * u0 + P12 * u1 + P22 * u2;
                    const double den = lambda + (u0 * q0 + u1 * q1 + u2 * q2);
                    const double k0 = q0 / den, k1 = q1 / den, k2 = q2 / den;
                    w0 += k0 * e;
                    w1 += k1 * e;
                    w2 += k2 * e;
                    P00 = (P00 - k0 * q0) / lambda;
                    P01 = (P01 - k0 * q1) / lambda;
                    P02 = (P02 - k0 * q2) / lambda;
                    P11 = (P11 - k1 * q1) / lambda;
                    P12 = (P12 - k1 * q2) / lambda;
                    P22 = (P22 - k2 * q2) / lambda;
                }
                it++;
            }
        }
    }
    if (lane == 0) {
        W[4 * k] = w0;
        W[4 * k + 1] = w1;
        W[4 * k + 2] = w2;
        W[4 * k + 3] = 0.0;
        if (count) count[k] = m;
    }
}

size_t seq_workspace_bytes(int64_t G, int64_t K) {
    return ((size_t)G * sizeof(int) + 255) / 256 * 256 + (size_t)K * kSeqBlocks * sizeof(int);
}

sal_status launch_seq_adapt(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion& f,
                            const float* D, const uint8_t* mask, double* W, float* err2, int64_t cap, int64_t* count,
                            void* ws, hipStream_t stream) {
    const int64_t G = Tg * ILg * XLg;
    const int64_t K = fuse_groups(f.sections, ILg);
    const int64_t sections = K > 1 ? f.sections : 0;
    if (G >= (int64_t(1) << 31)) return fail(SAL_ERR_UNSUPPORTED, "sequential adaptation needs fewer than 2^31 grid points");
    if (K > 65535) return fail(SAL_ERR_SHAPE, "too many weight groups for one launch");
    int* idx = (int*)ws;
    int* counts = (int*)((char*)ws + ((size_t)G * sizeof(int) + 255) / 256 * 256);
    hipLaunchKernelGGL(k_seq_count, dim3(kSeqBlocks, (unsigned)K), dim3(256), 0, stream, mask, Tg, ILg, XLg, sections,
                       counts);
    sal_status st = check_hip(hipGetLastError(), "launch k_seq_count");
    if (st) return st;
    hipLaunchKernelGGL(k_seq_compact, dim3(kSeqBlocks, (unsigned)K), dim3(256), 0, stream, mask, Tg, ILg, XLg,
                       sections, counts, idx);
    if ((st = check_hip(hipGetLastError(), "launch k_seq_compact"))) return st;
    hipLaunchKernelGGL(k_seq_adapt, dim3((unsigned)K), dim3(64), 0, stream, Sm, D, Tg, ILg, XLg, sections, counts, idx,
                       f.mode, f.mu, f.eps, f.lambda, f.delta, f.w_fixed[0], f.w_fixed[1], f.w_fixed[2], f.passes, W,
                       err2, cap, count);
    return check_hip(hipGetLastError(), "launch k_seq_adapt");
}

}  // namespace sal
