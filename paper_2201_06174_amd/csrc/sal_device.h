// sal_device.h -- device helpers shared by the single-volume and batched kernels of the
// center-surround and fusion steps (not part of the ABI).
#pragma once

#include <type_traits>

#include "sal_aux.h"
#include "sal_grid.h"

namespace sal {

// S_m at grid point j of one volume (Sec. 2, Eq. 3): (1/Q) sum over in-grid neighbours.
// A point at least the stencil reach away from every border has all q neighbours in the
// grid and skips the bounds tests (same terms, same order).  PLANES: per-plane stencils,
// each plane summing over its own members with its own weights and its own count Q_m.
template <typename I, bool PLANES>
__device__ __forceinline__ void dcs_point_t(const float* __restrict__ E, float* __restrict__ S, I Tg, I ILg, I XLg,
                                            const DcsStencil& st, I j) {
    const I G = Tg * ILg * XLg;
    const I gx = j % XLg, gi = (j / XLg) % ILg, gt = j / (XLg * ILg);
    const bool inner = gt >= st.reach[0] && gt + st.reach[0] < Tg && gi >= st.reach[1] && gi + st.reach[1] < ILg &&
                       gx >= st.reach[2] && gx + st.reach[2] < XLg;
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    const float e0 = E[j], e1 = E[G + j], e2 = E[2 * G + j];
    int Q = 0, Q1 = 0, Q2 = 0;
    auto term = [&](float ec, float en, float w) { return st.literal ? fabsf(ec - w * en) : w * fabsf(ec - en); };
    for (int k = 0; k < st.q; k++) {
        const I nt = gt + st.o[k][0], ni = gi + st.o[k][1], nx = gx + st.o[k][2];
        if (!inner && (nt < 0 || nt >= Tg || ni < 0 || ni >= ILg || nx < 0 || nx >= XLg)) continue;
        const I jn = (nt * ILg + ni) * XLg + nx;
        if constexpr (PLANES) {
            const unsigned mb = st.member[k];
            if (mb & 1u) { acc0 += term(e0, E[jn], st.wp[k][0]); Q++; }
            if (mb & 2u) { acc1 += term(e1, E[G + jn], st.wp[k][1]); Q1++; }
            if (mb & 4u) { acc2 += term(e2, E[2 * G + jn], st.wp[k][2]); Q2++; }
        } else {
            const float w = st.w[k];
            acc0 += term(e0, E[jn], w);
            acc1 += term(e1, E[G + jn], w);
            acc2 += term(e2, E[2 * G + jn], w);
            Q++;
        }
    }
    if constexpr (!PLANES) Q1 = Q2 = Q;
    S[j] = Q ? acc0 / (float)Q : 0.f;
    S[G + j] = Q1 ? acc1 / (float)Q1 : 0.f;
    S[2 * G + j] = Q2 ? acc2 / (float)Q2 : 0.f;
}

// 32-bit index arithmetic whenever the grid's three planes fit it
__device__ __forceinline__ void dcs_point(const float* __restrict__ E, float* __restrict__ S, int64_t Tg,
                                          int64_t ILg, int64_t XLg, const DcsStencil& st, int64_t j) {
    const bool i32 = 3 * Tg * ILg * XLg < (int64_t(1) << 31);
    if (st.planes) {
        if (i32) dcs_point_t<int32_t, true>(E, S, (int32_t)Tg, (int32_t)ILg, (int32_t)XLg, st, (int32_t)j);
        else dcs_point_t<int64_t, true>(E, S, Tg, ILg, XLg, st, j);
    } else {
        if (i32) dcs_point_t<int32_t, false>(E, S, (int32_t)Tg, (int32_t)ILg, (int32_t)XLg, st, (int32_t)j);
        else dcs_point_t<int64_t, false>(E, S, Tg, ILg, XLg, st, j);
    }
}

// The grid points of one weight group (inline planes [k N, k N + N) of the grid), numbered
// e = 0 .. count-1 in memory order: point e is j = (e / slab) * plane + first + e % slab.
// Without sections the group is the whole grid and j = e.
struct GroupMap {
    int64_t count;  // points in the group
    int64_t slab;   // points per t plane inside the group (its inline planes x XLg)
    int64_t plane;  // ILg * XLg
    int64_t first;  // k N XLg
};

__device__ __forceinline__ GroupMap group_map(int64_t Tg, int64_t ILg, int64_t XLg, int64_t sections, int64_t k) {
    GroupMap g;
    const int64_t il0 = sections > 0 ? k * sections : 0;
    const int64_t nk = sections > 0 ? (ILg - il0 < sections ? ILg - il0 : sections) : ILg;
    g.slab = nk * XLg;
    g.plane = ILg * XLg;
    g.first = il0 * XLg;
    g.count = Tg * g.slab;
    return g;
}

// One block's FP64 partial sums of u u^T, u D, D^2 and the count over the masked points
// e = first, first + stride, ... of a weight group (fixed order: deterministic).  256 threads.
// G is the size of a whole plane of Sm; SECT maps group positions to grid points.
template <bool SECT>
__device__ __forceinline__ void fuse_stats_group(const float* __restrict__ Sm, const float* __restrict__ D,
                                                 const uint8_t* __restrict__ mask, int64_t G, const GroupMap gm,
                                                 int64_t first, int64_t stride, double* __restrict__ out,
                                                 double* red) {
    double st[kStats];
    for (int k = 0; k < kStats; k++) st[k] = 0.0;
    auto add = [&](float f0, float f1, float f2, float fd) {
        const double u0 = f0, u1 = f1, u2 = f2, d = fd;
        st[0] += u0 * u0; st[1] += u0 * u1; st[2] += u0 * u2;
        st[3] += u1 * u1; st[4] += u1 * u2; st[5] += u2 * u2;
        st[6] += u0 * d; st[7] += u1 * d; st[8] += u2 * d;
        st[9] += d * d; st[10] += 1.0;
    };
    auto J = [&](int64_t e) -> int64_t { return SECT ? (e / gm.slab) * gm.plane + gm.first + e % gm.slab : e; };
    const int64_t cnt = SECT ? gm.count : G;
    // Four of a thread's points at a time: their loads are issued together, the sums still
    // taken point by point in increasing e (the same order, so the same result, as one at a time).
    auto sweep = [&](auto masked) {
        constexpr bool MASKED = decltype(masked)::value;
        int64_t e = first + threadIdx.x;
        for (; e + 3 * stride < cnt; e += 4 * stride) {
            bool in[4];
            float v[4][4];
            int64_t jp[4];
#pragma unroll
            for (int p = 0; p < 4; p++) jp[p] = J(e + p * stride);
#pragma unroll
            for (int p = 0; p < 4; p++) in[p] = MASKED ? mask[jp[p]] != 0 : true;
#pragma unroll
            for (int p = 0; p < 4; p++) {
                if (in[p]) {
                    v[p][0] = Sm[jp[p]];
                    v[p][1] = Sm[G + jp[p]];
                    v[p][2] = Sm[2 * G + jp[p]];
                    v[p][3] = D[jp[p]];
                }
            }
#pragma unroll
            for (int p = 0; p < 4; p++)
                if (in[p]) add(v[p][0], v[p][1], v[p][2], v[p][3]);
        }
        for (; e < cnt; e += stride) {
            const int64_t j = J(e);
            if (!MASKED || mask[j]) add(Sm[j], Sm[G + j], Sm[2 * G + j], D[j]);
        }
    };
    if (mask)
        sweep(std::true_type{});
    else
        sweep(std::false_type{});
    for (int k = 0; k < kStats; k++) {
        red[threadIdx.x] = st[k];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

// The whole grid as one group.
__device__ __forceinline__ void fuse_stats_block(const float* __restrict__ Sm, const float* __restrict__ D,
                                                 const uint8_t* __restrict__ mask, int64_t G, int64_t first,
                                                 int64_t stride, double* __restrict__ out, double* red) {
    fuse_stats_group<false>(Sm, D, mask, G, GroupMap{}, first, stride, out, red);
}

// 3x3 Cholesky solve; 1 if A is not numerically positive definite.
__device__ __forceinline__ int chol3(const double A[9], const double b[3], double x[3]) {
    double dmax = 0.0;
    for (int i = 0; i < 3; i++) {
        if (!isfinite(A[4 * i])) return 1;
        dmax = A[4 * i] > dmax ? A[4 * i] : dmax;
    }
    if (!(dmax > 0.0)) return 1;
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < 3; j++) {
        double d = A[3 * j + j];
        for (int k = 0; k < j; k++) d -= L[3 * j + k] * L[3 * j + k];
        if (!(d > 1e-12 * dmax) || !isfinite(d)) return 1;
        L[3 * j + j] = sqrt(d);
        for (int i = j + 1; i < 3; i++) {
            double v = A[3 * i + j];
            for (int k = 0; k < j; k++) v -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = v / L[3 * j + j];
        }
    }
    double y[3];
    for (int i = 0; i < 3; i++) {
        double v = b[i];
        for (int k = 0; k < i; k++) v -= L[3 * i + k] * y[k];
        y[i] = v / L[3 * i + i];
    }
    for (int i = 2; i >= 0; i--) {
        double v = y[i];
        for (int k = i + 1; k < 3; k++) v -= L[3 * k + i] * x[k];
        x[i] = v / L[3 * i + i];
    }
    return 0;
}

// Column sums of an FP64 table part[nparts][ncols] (ncols <= 16) by a block of 64 threads in a
// fixed order (deterministic): thread t adds rows t, t + 64, ... in turn, then the 64 partial
// sums of a column are combined by a pairwise tree.  red: 16 x 64 doubles of shared memory.
__device__ __forceinline__ void sum_columns64(const double* __restrict__ part, int nparts, int ncols, double* red,
                                              double* out) {
    const int t = threadIdx.x;
    for (int k = 0; k < ncols; k++) {
        double s = 0.0;
#pragma unroll 4
        for (int b = t; b < nparts; b += 64) s += part[(int64_t)b * ncols + k];
        red[k * 64 + t] = s;
    }
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < ncols; k++) red[k * 64 + t] += red[k * 64 + t + w];
        __syncthreads();
    }
    if (t < ncols) out[t] = red[t * 64];
    __syncthreads();
}

// Weights of one volume from its reduced statistics (block of 64 threads): sums the
// partials (sum_columns64), then solves; writes W[0..2] and the status word W[3].
__device__ __forceinline__ void solve_weights(const double* __restrict__ part, int nparts, int mode, double w0,
                                              double w1, double w2, double delta, double* __restrict__ W,
                                              double* __restrict__ stats_out, double* st) {
    if (mode == SAL_FUSE_ADAPT_LS) {
        __shared__ double red[16 * 64];
        sum_columns64(part, nparts, kStats, red, st);
        if (stats_out && threadIdx.x < kStats) stats_out[threadIdx.x] = st[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (mode == SAL_FUSE_EQUAL) {
        W[0] = W[1] = W[2] = 1.0 / 3.0;
        W[3] = 0.0;
        return;
    }
    if (mode == SAL_FUSE_FIXED) {
        W[0] = w0; W[1] = w1; W[2] = w2;
        W[3] = 0.0;
        return;
    }
    const double A[9] = {st[0] + delta, st[1], st[2], st[1], st[3] + delta, st[4], st[2], st[4], st[5] + delta};
    const double b[3] = {st[6], st[7], st[8]};
    double x[3];
    if (chol3(A, b, x)) {
        W[0] = W[1] = W[2] = 1.0 / 3.0;
        W[3] = 1.0;
    } else {
        W[0] = x[0]; W[1] = x[1]; W[2] = x[2];
        W[3] = 0.0;
    }
}

__device__ __forceinline__ int64_t cell_of(int64_t v, int s, int64_t Ng) {
    const int64_t g = (v + (s - 1) / 2) / s;
    return g < Ng - 1 ? g : Ng - 1;
}

// One (t, il) row of S(v) = sum_m W_m S_m(g(v)) (Eq. 4), threads striding along xl; with
// sections > 0 the row takes the weights of its grid cell's group (W: [K][4]).
__device__ __forceinline__ void combine_row(const float* __restrict__ Sm, const double* __restrict__ W, int64_t Tg,
                                            int64_t ILg, int64_t XLg, int64_t IL, int64_t XL, int s, int64_t row,
                                            float* __restrict__ S, int64_t sections = 0) {
    const int64_t t = row / IL, i = row % IL;
    const int64_t G = Tg * ILg * XLg;
    const int64_t gi = cell_of(i, s, ILg);
    const int64_t base = (cell_of(t, s, Tg) * ILg + gi) * XLg;
    const double* Wr = W + 4 * (sections > 0 ? gi / sections : 0);
    const double W0 = Wr[0], W1 = Wr[1], W2 = Wr[2];
    const int sh = (s - 1) / 2;
    for (int x = threadIdx.x; x < XL; x += blockDim.x) {
        int gx = (x + sh) / s;
        gx = gx < XLg - 1 ? gx : (int)XLg - 1;
        const int64_t j = base + gx;
        S[row * XL + x] = (float)(W0 * (double)Sm[j] + W1 * (double)Sm[G + j] + W2 * (double)Sm[2 * G + j]);
    }
}

}  // namespace sal
