// sal_aux.hip -- the bandwidth-bound steps: full local spectra (checks), directional
// center-surround (Sec. 2 step 4, Eq. 3) and fusion (Sec. 2 step 5, Eq. 4), with
// their adjoints.
#include "sal_device.h"

namespace sal {

// Half-sample reflection, then a clamp that keeps any (invalid) far-off index in bounds.
__device__ __forceinline__ int64_t reflect_index(int64_t p, int64_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p < 0 ? 0 : (p >= N ? N - 1 : p);
}

// ---------------------------------------------------------------- local spectra (Eq. 2)
// One workgroup per centre: gather the tapered cube into LDS, then three complex
// DFT passes (xl, il, t), each output a direct n-term sum.
__global__ __launch_bounds__(256) void k_local_spectra(const float* __restrict__ V, int64_t T, int64_t IL, int64_t XL,
                                                       int n, int window, const int32_t* __restrict__ centers,
                                                       int64_t cnt, float* __restrict__ F) {
    extern __shared__ float sh[];
    const int n3 = n * n * n;
    float* xr = sh;
    float* xi = sh + n3;
    float* yr = sh + 2 * n3;
    float* yi = sh + 3 * n3;
    float* tw = sh + 4 * n3;  // [n][n][2] cos/sin(2 pi k a / n)
    float* h = tw + 2 * n * n;
    const int64_t c = block_id();
    if (c >= cnt) return;
    const int64_t ct = centers[3 * c], ci = centers[3 * c + 1], cx = centers[3 * c + 2];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int k = e / n, a = e % n;
        const int r = (k * a) % n;
        float sn, cs;
        sincospif(2.0f * (float)r / (float)n, &sn, &cs);
        tw[2 * e] = cs;
        tw[2 * e + 1] = sn;
    }
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const float v = sinpif((float)a / (float)n);
        h[a] = window == SAL_WINDOW_HANN ? v * v : 1.0f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n3; e += blockDim.x) {
        const int at = e / (n * n), ai = (e / n) % n, ax = e % n;
        const int64_t pt = reflect_index(ct - n / 2 + at, T), pi = reflect_index(ci - n / 2 + ai, IL),
                      px = reflect_index(cx - n / 2 + ax, XL);
        xr[e] = h[at] * h[ai] * h[ax] * V[(pt * IL + pi) * XL + px];
        xi[e] = 0.f;
    }
    __syncthreads();
    float *inr = xr, *ini = xi, *outr = yr, *outi = yi;
    for (int axis = 2; axis >= 0; axis--) {
        const int stride = axis == 0 ? n * n : (axis == 1 ? n : 1);
        for (int e = threadIdx.x; e < n3; e += blockDim.x) {
            const int k = (e / stride) % n;
            const int base = e - k * stride;
            float sr = 0.f, si = 0.f;
            for (int a = 0; a < n; a++) {
                const float cr = tw[2 * (k * n + a)], cs = -tw[2 * (k * n + a) + 1];
                const float vr = inr[base + a * stride], vi = ini[base + a * stride];
                sr = fmaf(vr, cr, fmaf(-vi, cs, sr));
                si = fmaf(vr, cs, fmaf(vi, cr, si));
            }
            outr[e] = sr;
            outi[e] = si;
        }
        __syncthreads();
        float* t;
        t = inr; inr = outr; outr = t;
        t = ini; ini = outi; outi = t;
    }
    for (int e = threadIdx.x; e < n3; e += blockDim.x) {
        F[(c * n3 + e) * 2] = inr[e];
        F[(c * n3 + e) * 2 + 1] = ini[e];
    }
}

sal_status launch_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int window,
                                const int32_t* centers, int64_t cnt, float* F, hipStream_t stream) {
    if (cnt == 0) return SAL_OK;
    const size_t lds = sizeof(float) * (4 * (size_t)n * n * n + 2 * n * n + n);
    static std::atomic<uint64_t> attr{0};
    sal_status st = lds_limit_once((const void*)k_local_spectra, 160 * 1024, attr, "hipFuncSetAttribute(local_spectra)");
    if (st) return st;
    if (!wide_grid_fits(cnt, 256)) return fail(SAL_ERR_SHAPE, "too many centres for one launch");
    hipLaunchKernelGGL(k_local_spectra, wide_grid(cnt, 256), dim3(256), lds, stream, V, T, IL, XL, n, window, centers,
                       cnt, F);
    return check_hip(hipGetLastError(), "launch k_local_spectra");
}

// ---------------------------------------------------------------- center-surround (Eq. 3)

__global__ __launch_bounds__(256) void k_dcs(const float* __restrict__ E, float* __restrict__ S, int64_t Tg,
                                             int64_t ILg, int64_t XLg, DcsStencil st) {
    const int64_t G = Tg * ILg * XLg;
    const int64_t j = xcd_block((G + 255) / 256) * 256 + threadIdx.x;
    if (j >= G) return;
    dcs_point(E, S, Tg, ILg, XLg, st, j);
}

sal_status launch_dcs(const float* E, float* S, int64_t Tg, int64_t ILg, int64_t XLg, const DcsStencil& st,
                      hipStream_t stream) {
    const int64_t G = Tg * ILg * XLg;
    if (G == 0) return SAL_OK;
    const int64_t blocks = xcd_grid((G + 255) / 256);
    if (!wide_grid_fits(blocks, 256)) return fail(SAL_ERR_SHAPE, "grid too large for one launch");
    hipLaunchKernelGGL(k_dcs, wide_grid(blocks, 256), dim3(256), 0, stream, E, S, Tg, ILg, XLg, st);
    return check_hip(hipGetLastError(), "launch k_dcs");
}

// Adjoint of Eq. 3 as a gather: each grid point collects its own terms and the terms in
// which it is the neighbour of g - o, with sgn(0) = 0.  R = gS_m / Q carries the division by
// each point's neighbour count.  For a symmetric stencil the neighbour term of the mirrored
// offset reads the same point g + o as the own term of o, so every neighbour is read once;
// a point at least the stencil reach away from every border skips the bounds tests.
template <typename I, bool SYM, bool PLANES>
__device__ __forceinline__ void dcs_adjoint_point(const float* __restrict__ E, const float* __restrict__ R,
                                                  float* __restrict__ gE, I Tg, I ILg, I XLg, const DcsStencil& st,
                                                  I j) {
    const I G = Tg * ILg * XLg;
    const I gx = j % XLg, gi = (j / XLg) % ILg, gt = j / (XLg * ILg);
    auto inside = [&](I a, I b, I c) { return a >= 0 && a < Tg && b >= 0 && b < ILg && c >= 0 && c < XLg; };
    auto sgn = [](float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); };
    const bool inner = gt >= st.reach[0] && gt + st.reach[0] < Tg && gi >= st.reach[1] && gi + st.reach[1] < ILg &&
                       gx >= st.reach[2] && gx + st.reach[2] < XLg;
    // own[m] = sum_k (literal ? 1 : w_k) sgn(e0 - (literal ? w_k : 1) e_k); nbr[m] = the
    // neighbour terms without their sign flip
    float e0[3], own[3] = {0.f, 0.f, 0.f}, nbr[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 3; m++) e0[m] = E[m * G + j];
    for (int k = 0; k < st.q; k++) {
        const I nt = gt + st.o[k][0], ni = gi + st.o[k][1], nx = gx + st.o[k][2];
        if (!inner && !inside(nt, ni, nx)) continue;
        const I jn = (nt * ILg + ni) * XLg + nx;
#pragma unroll
        for (int m = 0; m < 3; m++) {
            // with per-plane stencils an offset outside plane m's stencil adds nothing there
            // (a mirrored pair shares its planes)
            if (PLANES && !((st.member[k] >> m) & 1u)) continue;
            const float wk = PLANES ? st.wp[k][m] : st.w[k];
            const float e1 = E[m * G + jn];
            own[m] += st.literal ? sgn(e0[m] - wk * e1) : wk * sgn(e0[m] - e1);
            if (SYM) {
                // g = (g + o_k) - o_mirror: the mirrored offset's neighbour term
                const float wm = PLANES ? st.wp[st.mirror[k]][m] : st.w[st.mirror[k]];
                nbr[m] += R[m * G + jn] * wm * sgn(st.literal ? e1 - wm * e0[m] : e1 - e0[m]);
            }
        }
    }
    if (!SYM) {
        for (int k = 0; k < st.q; k++) {
            const I pt = gt - st.o[k][0], pi = gi - st.o[k][1], px = gx - st.o[k][2];
            if (!inner && !inside(pt, pi, px)) continue;
            const I jp = (pt * ILg + pi) * XLg + px;
#pragma unroll
            for (int m = 0; m < 3; m++) {
                if (PLANES && !((st.member[k] >> m) & 1u)) continue;
                const float wk = PLANES ? st.wp[k][m] : st.w[k];
                const float ep = E[m * G + jp];
                nbr[m] += R[m * G + jp] * wk * sgn(st.literal ? ep - wk * e0[m] : ep - e0[m]);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 3; m++) gE[m * G + j] = R[m * G + j] * own[m] - nbr[m];
}

template <bool SYM, bool PLANES>
__global__ __launch_bounds__(256) void k_dcs_adjoint(const float* __restrict__ E, const float* __restrict__ R,
                                                     float* __restrict__ gE, int64_t Tg, int64_t ILg, int64_t XLg,
                                                     DcsStencil st) {
    const int64_t G = Tg * ILg * XLg;
    const int64_t j = xcd_block((G + 255) / 256) * 256 + threadIdx.x;
    if (j >= G) return;
    if (3 * G < (int64_t(1) << 31))
        dcs_adjoint_point<int32_t, SYM, PLANES>(E, R, gE, (int32_t)Tg, (int32_t)ILg, (int32_t)XLg, st, (int32_t)j);
    else
        dcs_adjoint_point<int64_t, SYM, PLANES>(E, R, gE, Tg, ILg, XLg, st, j);
}

sal_status launch_dcs_adjoint(const float* E, const float* R, float* gE, int64_t Tg, int64_t ILg, int64_t XLg,
                              const DcsStencil& st, hipStream_t stream) {
    const int64_t G = Tg * ILg * XLg;
    if (G == 0) return SAL_OK;
    const int64_t blocks = xcd_grid((G + 255) / 256);
    if (!wide_grid_fits(blocks, 256)) return fail(SAL_ERR_SHAPE, "grid too large for one launch");
    const dim3 grid = wide_grid(blocks, 256);
    if (st.symmetric && st.planes)
        hipLaunchKernelGGL((k_dcs_adjoint<true, true>), grid, dim3(256), 0, stream, E, R, gE, Tg, ILg, XLg, st);
    else if (st.symmetric)
        hipLaunchKernelGGL((k_dcs_adjoint<true, false>), grid, dim3(256), 0, stream, E, R, gE, Tg, ILg, XLg, st);
    else if (st.planes)
        hipLaunchKernelGGL((k_dcs_adjoint<false, true>), grid, dim3(256), 0, stream, E, R, gE, Tg, ILg, XLg, st);
    else
        hipLaunchKernelGGL((k_dcs_adjoint<false, false>), grid, dim3(256), 0, stream, E, R, gE, Tg, ILg, XLg, st);
    return check_hip(hipGetLastError(), "launch k_dcs_adjoint");
}

// ---------------------------------------------------------------- fusion (Eq. 4)

// Per-block FP64 partial sums over the masked grid points of
// u u^T (6), u D (3), D^2, count, in a fixed order (deterministic).  Block (b, k) covers part
// b of weight group k (part: [K][kFuseParts][kStats]); one group is the whole grid in memory
// order.
__global__ __launch_bounds__(256) void k_fuse_stats(const float* __restrict__ Sm, const float* __restrict__ D,
                                                    const uint8_t* __restrict__ mask, int64_t Tg, int64_t ILg,
                                                    int64_t XLg, int64_t sections, double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t G = Tg * ILg * XLg;
    const int64_t k = blockIdx.y;
    double* out = part + (k * kFuseParts + blockIdx.x) * kStats;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x, stride = (int64_t)gridDim.x * blockDim.x;
    if (sections > 0)
        fuse_stats_group<true>(Sm, D, mask, G, group_map(Tg, ILg, XLg, sections, k), first, stride, out, red);
    else
        fuse_stats_block(Sm, D, mask, G, first, stride, out, red);
}

// One block per weight group: fixed-order reduction of the group's partials and the 3x3
// solve.  Writes W[4k .. 4k+2] and the status word W[4k+3]; also the reduced statistics of
// group k to stats_out[16k ..].
__global__ __launch_bounds__(64) void k_fuse_solve(const double* __restrict__ part, int nparts, int mode,
                                                   double w0, double w1, double w2, double delta,
                                                   double* __restrict__ W, double* __restrict__ stats_out) {
    __shared__ double st[kStats];
    const int64_t k = blockIdx.x;
    solve_weights(part + k * nparts * kStats, nparts, mode, w0, w1, w2, delta, W + 4 * k,
                  stats_out ? stats_out + 16 * k : nullptr, st);
}

// S(v) = sum_m W_m S_m(g(v)) (same arithmetic as combine_row): kCombineRows (t, il) rows per
// block, each thread writing four consecutive xl samples with one 16-byte store (XL % 4 == 0
// and a 16-byte aligned S), the stride fixed at compile time (SS > 0) so the nearest-centre
// division is a constant one.  The block's rows are resolved once (one division, then a step
// along il), and an element finds its row by comparisons, so the loop has no 64-bit division.
constexpr int kCombineRows = 4;

// SECT: each row takes the weights of its grid cell's group (W: [K][4], `sections` inline
// planes per group).
template <int SS, bool SECT>
__global__ __launch_bounds__(256) void k_combine4(const float* __restrict__ Sm, const double* __restrict__ W,
                                                  int64_t Tg, int64_t ILg, int64_t XLg, int64_t T, int64_t IL,
                                                  int64_t XL, int s_rt, int64_t sections, float* __restrict__ S) {
    const int s = SS > 0 ? SS : s_rt;
    const int64_t G = Tg * ILg * XLg;
    double W0 = W[0], W1 = W[1], W2 = W[2];
    const int sh = (s - 1) / 2;
    const int64_t q = XL / 4;
    const int64_t row0 = block_id() * kCombineRows;
    const int64_t nrow = T * IL - row0 < kCombineRows ? T * IL - row0 : kCombineRows;
    int64_t base[kCombineRows], orow[kCombineRows], wrow[kCombineRows];
    {
        int64_t t = row0 / IL, i = row0 - t * IL;
#pragma unroll
        for (int r = 0; r < kCombineRows; r++) {
            const int64_t gi = cell_of(i, s, ILg);
            base[r] = (cell_of(t, s, Tg) * ILg + gi) * XLg;
            orow[r] = (row0 + r) * XL;
            wrow[r] = SECT ? 4 * (gi / sections) : 0;
            if (++i == IL) {
                i = 0;
                t++;
            }
        }
    }
    for (int64_t e = threadIdx.x; e < nrow * q; e += blockDim.x) {
        int r = 0;
#pragma unroll
        for (int k = 1; k < kCombineRows; k++) r += e >= k * q;
        int64_t b = base[0], ob = orow[0], wo = wrow[0];
#pragma unroll
        for (int k = 1; k < kCombineRows; k++)
            if (r == k) {
                b = base[k];
                ob = orow[k];
                wo = wrow[k];
            }
        if constexpr (SECT) {
            W0 = W[wo];
            W1 = W[wo + 1];
            W2 = W[wo + 2];
        }
        const int x0 = (int)(e - r * q) * 4;
        auto value = [&](int gx) {
            const int64_t j = b + gx;
            return (float)(W0 * (double)Sm[j] + W1 * (double)Sm[G + j] + W2 * (double)Sm[2 * G + j]);
        };
        float4 o;
        if constexpr (SS == 2) {
            // x0 = 4u: samples x0, x0 + 1 take centre 2u, the next two 2u + 1 (< XLg as XL % 4 == 0)
            const float a0 = value(x0 / 2), a1 = value(x0 / 2 + 1);
            o = make_float4(a0, a0, a1, a1);
        } else {
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int gx = (x0 + k + sh) / s;
                v[k] = value(gx < XLg - 1 ? gx : (int)XLg - 1);
            }
            o = make_float4(v[0], v[1], v[2], v[3]);
        }
        *(float4*)&S[ob + x0] = o;
    }
}

// S(v) = sum_m W_m S_m(g(v)); one block per (t, il) row (any XL).
__global__ __launch_bounds__(256) void k_combine(const float* __restrict__ Sm, const double* __restrict__ W,
                                                 int64_t Tg, int64_t ILg, int64_t XLg, int64_t T, int64_t IL,
                                                 int64_t XL, int s, int64_t sections, float* __restrict__ S) {
    const int64_t row = block_id();  // one block per (t, il) row
    if (row >= T * IL) return;
    combine_row(Sm, W, Tg, ILg, XLg, IL, XL, s, row, S, sections);
}

// Forward workspace over K groups: partials [K][kFuseParts][kStats], then [K][16] reduced
// statistics.
size_t fuse_workspace_bytes(int64_t K) { return sizeof(double) * (size_t)K * (kFuseParts * kStats + 16); }

template <int SS>
static void launch_combine4(bool sect, dim3 grid, hipStream_t stream, const float* Sm, const double* W, int64_t Tg,
                            int64_t ILg, int64_t XLg, int64_t T, int64_t IL, int64_t XL, int s, int64_t sections,
                            float* S) {
    if (sect)
        hipLaunchKernelGGL((k_combine4<SS, true>), grid, dim3(256), 0, stream, Sm, W, Tg, ILg, XLg, T, IL, XL, s,
                           sections, S);
    else
        hipLaunchKernelGGL((k_combine4<SS, false>), grid, dim3(256), 0, stream, Sm, W, Tg, ILg, XLg, T, IL, XL, s,
                           sections, S);
}

sal_status launch_fuse(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion& f, const float* D,
                       const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int s, double* W, float* S, double* ws,
                       hipStream_t stream) {
    const int64_t K = fuse_groups(f.sections, ILg);
    const int64_t sections = K > 1 ? f.sections : 0;  // one group covers the grid: the plain path
    if (K > 65535) return fail(SAL_ERR_SHAPE, "too many weight groups for one launch");
    if (f.mode == SAL_FUSE_ADAPT_LS) {
        hipLaunchKernelGGL(k_fuse_stats, dim3(kFuseParts, (unsigned)K), dim3(256), 0, stream, Sm, D, mask, Tg, ILg,
                           XLg, sections, ws);
        sal_status st = check_hip(hipGetLastError(), "launch k_fuse_stats");
        if (st) return st;
    }
    hipLaunchKernelGGL(k_fuse_solve, dim3((unsigned)K), dim3(64), 0, stream, ws, kFuseParts, f.mode, f.w_fixed[0],
                       f.w_fixed[1], f.w_fixed[2], f.delta, W,
                       f.mode == SAL_FUSE_ADAPT_LS ? ws + K * kFuseParts * kStats : nullptr);
    sal_status st = check_hip(hipGetLastError(), "launch k_fuse_solve");
    if (st) return st;
    return launch_combine(Sm, Tg, ILg, XLg, sections, T, IL, XL, s, W, S, stream);
}

sal_status launch_combine(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, int64_t sections, int64_t T,
                          int64_t IL, int64_t XL, int s, const double* W, float* S, hipStream_t stream) {
    if (T * IL * XL == 0) return SAL_OK;
    if (!wide_grid_fits(T * IL, 256)) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    if (XL % 4 == 0 && reinterpret_cast<uintptr_t>(S) % 16 == 0) {
        const dim3 grid = wide_grid((T * IL + kCombineRows - 1) / kCombineRows, 256);
        const bool sect = sections > 0;
        if (s == 1)
            launch_combine4<1>(sect, grid, stream, Sm, W, Tg, ILg, XLg, T, IL, XL, s, sections, S);
        else if (s == 2)
            launch_combine4<2>(sect, grid, stream, Sm, W, Tg, ILg, XLg, T, IL, XL, s, sections, S);
        else
            launch_combine4<0>(sect, grid, stream, Sm, W, Tg, ILg, XLg, T, IL, XL, s, sections, S);
    } else {
        hipLaunchKernelGGL(k_combine, wide_grid(T * IL, 256), dim3(256), 0, stream, Sm, W, Tg, ILg, XLg, T, IL, XL,
                           s, sections, S);
    }
    return check_hip(hipGetLastError(), "launch k_combine");
}

// ---------------------------------------------------------------- fusion adjoint

// Cell sum c(g) = sum of gS over the voxels whose nearest centre is g.  I = int32_t when
// the volume fits it.
template <typename I>
__device__ __forceinline__ float cell_sum(const float* __restrict__ gS, I T, I IL, I XL, int s, I Tg, I ILg, I XLg,
                                          I gt, I gi, I gx) {
    const I N3[3] = {T, IL, XL}, Ng[3] = {Tg, ILg, XLg}, g3[3] = {gt, gi, gx};
    I lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = g3[a] * s - (s - 1) / 2;
        if (lo[a] < 0) lo[a] = 0;
        hi[a] = (g3[a] == Ng[a] - 1) ? N3[a] - 1 : g3[a] * s + s - 1 - (s - 1) / 2;
        if (hi[a] > N3[a] - 1) hi[a] = N3[a] - 1;
    }
    double acc = 0.0;
    for (I t = lo[0]; t <= hi[0]; t++)
        for (I i = lo[1]; i <= hi[1]; i++)
            for (I x = lo[2]; x <= hi[2]; x++) acc += (double)gS[(t * IL + i) * XL + x];
    return (float)acc;
}

template <typename I>
__global__ __launch_bounds__(256) void k_cell_sum(const float* __restrict__ gS, int64_t T, int64_t IL, int64_t XL,
                                                  int s, int64_t Tg_, int64_t ILg_, int64_t XLg_,
                                                  float* __restrict__ cell) {
    const I Tg = (I)Tg_, ILg = (I)ILg_, XLg = (I)XLg_;
    const int64_t j64 = block_id() * blockDim.x + threadIdx.x;
    if (j64 >= (int64_t)Tg_ * ILg_ * XLg_) return;
    const I j = (I)j64;
    cell[j] = cell_sum<I>(gS, (I)T, (I)IL, (I)XL, s, Tg, ILg, XLg, j / (XLg * ILg), (j / XLg) % ILg, j % XLg);
}

// Per-block FP64 partials of gW_m = sum_g S_m(g) c(g) over weight group blockIdx.y (part:
// [K][kFuseParts][3]); the lambda terms need the solved gW first.
__global__ __launch_bounds__(256) void k_gw_partials(const float* __restrict__ Sm, const float* __restrict__ cell,
                                                     int64_t Tg, int64_t ILg, int64_t XLg, int64_t sections,
                                                     double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t G = Tg * ILg * XLg;
    const int64_t k = blockIdx.y;
    const GroupMap gm = group_map(Tg, ILg, XLg, sections, k);
    const int64_t cnt = sections > 0 ? gm.count : G;
    double a[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += stride) {
        const int64_t j = sections > 0 ? (e / gm.slab) * gm.plane + gm.first + e % gm.slab : e;
        const double c = cell[j];
        a[0] += (double)Sm[j] * c;
        a[1] += (double)Sm[G + j] * c;
        a[2] += (double)Sm[2 * G + j] * c;
    }
    double* out = part + (k * gridDim.x + blockIdx.x) * 3;
    for (int m = 0; m < 3; m++) {
        red[threadIdx.x] = a[m];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[m] = red[0];
        __syncthreads();
    }
}

// One block per weight group k: lambda_k = (G_k + delta I)^-1 gW_k from the group's reduced
// statistics of the forward (stats: [K][16], lambda written at stats[16k + 11 ..]).
__global__ __launch_bounds__(64) void k_gw_solve(const double* __restrict__ part, int nparts,
                                                 double* __restrict__ stats, double delta) {
    __shared__ double gw[3];
    __shared__ double red[16 * 64];
    const int64_t k = blockIdx.x;
    sum_columns64(part + k * nparts * 3, nparts, 3, red, gw);
    if (threadIdx.x != 0) return;
    double* st = stats + 16 * k;
    const double A[9] = {st[0] + delta, st[1], st[2], st[1], st[3] + delta, st[4], st[2], st[4], st[5] + delta};
    double x[3] = {0.0, 0.0, 0.0};
    if (chol3(A, gw, x)) x[0] = x[1] = x[2] = 0.0;
    st[11] = x[0]; st[12] = x[1]; st[13] = x[2];
}

// gS_m(g) = W_m c(g) (+ on the mask, ADAPT_LS: lambda_m (D - W.u) - W_m (lambda.u)), stored
// divided by the neighbour count Q_m(g), with W and lambda of g's weight group (W: [K][4],
// lambda at lam[16k ..]).  Without a cell-sum buffer (cell == nullptr) c(g) is summed here
// from gS.  I = int32_t when the grid's three planes fit it.
template <typename I>
__global__ __launch_bounds__(256) void k_gsm(const float* __restrict__ Sm, const float* __restrict__ cell,
                                             const double* __restrict__ W, const double* __restrict__ lam,
                                             const float* __restrict__ D, const uint8_t* __restrict__ mask,
                                             int64_t Tg_, int64_t ILg_, int64_t XLg_, DcsStencil ds, int adapt,
                                             int64_t sections, const float* __restrict__ gS, int64_t T, int64_t IL,
                                             int64_t XL, int s, float* __restrict__ R) {
    const I Tg = (I)Tg_, ILg = (I)ILg_, XLg = (I)XLg_;
    const I G = Tg * ILg * XLg;
    const int64_t j64 = block_id() * blockDim.x + threadIdx.x;
    if (j64 >= (int64_t)G) return;
    const I j = (I)j64;
    // neighbours of g inside the grid (all q of them away from the borders), per plane with
    // per-plane stencils
    const I gx = j % XLg, gi = (j / XLg) % ILg, gt = j / (XLg * ILg);
    int Q[3];
    if (!ds.planes) {
        Q[0] = ds.q;
        if (!(gt >= ds.reach[0] && gt + ds.reach[0] < Tg && gi >= ds.reach[1] && gi + ds.reach[1] < ILg &&
              gx >= ds.reach[2] && gx + ds.reach[2] < XLg)) {
            Q[0] = 0;
            for (int k = 0; k < ds.q; k++) {
                const I a = gt + ds.o[k][0], b = gi + ds.o[k][1], c = gx + ds.o[k][2];
                Q[0] += a >= 0 && a < Tg && b >= 0 && b < ILg && c >= 0 && c < XLg;
            }
        }
        Q[1] = Q[2] = Q[0];
    } else {
        Q[0] = Q[1] = Q[2] = 0;
        for (int k = 0; k < ds.q; k++) {
            const I a = gt + ds.o[k][0], b = gi + ds.o[k][1], c = gx + ds.o[k][2];
            if (!(a >= 0 && a < Tg && b >= 0 && b < ILg && c >= 0 && c < XLg)) continue;
            const unsigned mb = ds.member[k];
            Q[0] += mb & 1u;
            Q[1] += (mb >> 1) & 1u;
            Q[2] += (mb >> 2) & 1u;
        }
    }
    const int64_t grp = sections > 0 ? (int64_t)gi / sections : 0;
    const double* Wg = W + 4 * grp;
    const double c = cell ? cell[j] : cell_sum<I>(gS, (I)T, (I)IL, (I)XL, s, Tg, ILg, XLg, gt, gi, gx);
    double g[3] = {Wg[0] * c, Wg[1] * c, Wg[2] * c};
    if (adapt && Wg[3] == 0.0 && (!mask || mask[j])) {
        const double* lg = lam + 16 * grp;
        const double u0 = Sm[j], u1 = Sm[G + j], u2 = Sm[2 * G + j];
        const double r = (double)D[j] - (Wg[0] * u0 + Wg[1] * u1 + Wg[2] * u2);
        const double lu = lg[0] * u0 + lg[1] * u1 + lg[2] * u2;
        for (int m = 0; m < 3; m++) g[m] += lg[m] * r - Wg[m] * lu;
    }
#pragma unroll
    for (int m = 0; m < 3; m++) R[m * G + j] = Q[m] ? (float)g[m] / (float)Q[m] : 0.f;
}

// Adjoint workspace over K groups (doubles): forward partials [K][P][kStats] | statistics
// [K][16] (kStats values, lambda at +11) | gW partials [K][P][3] | the solve's weights [K][4].
size_t fuse_adjoint_workspace_bytes(int64_t K) {
    return sizeof(double) * (size_t)K * (kFuseParts * kStats + 16 + 3 * kFuseParts + 4);
}

sal_status launch_fuse_adjoint(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion& f,
                               const float* D, const uint8_t* mask, const double* W, const float* gS, int64_t T,
                               int64_t IL, int64_t XL, int s, const DcsStencil& ds, float* cell, double* ws, float* R,
                               hipStream_t stream) {
    const int64_t G = Tg * ILg * XLg;
    if (G == 0) return SAL_OK;
    const int64_t K = fuse_groups(f.sections, ILg);
    const int64_t sections = K > 1 ? f.sections : 0;
    if (K > 65535) return fail(SAL_ERR_SHAPE, "too many weight groups for one launch");
    const int64_t nb = (G + 255) / 256;
    if (!wide_grid_fits(nb, 256)) return fail(SAL_ERR_SHAPE, "grid too large for one launch");
    const dim3 blocks = wide_grid(nb, 256);
    // 32-bit index arithmetic when the volume and the grid's three planes fit it
    const bool i32 = T * IL * XL < (int64_t(1) << 31) && 3 * G < (int64_t(1) << 31);
    const int adapt = f.mode == SAL_FUSE_ADAPT_LS;
    sal_status st = SAL_OK;
    // the adapted weights need every c(g) before gS_m; otherwise k_gsm sums its own cell
    if (adapt) {
        if (i32)
            hipLaunchKernelGGL(k_cell_sum<int32_t>, blocks, dim3(256), 0, stream, gS, T, IL, XL, s, Tg, ILg,
                               XLg, cell);
        else
            hipLaunchKernelGGL(k_cell_sum<int64_t>, blocks, dim3(256), 0, stream, gS, T, IL, XL, s, Tg, ILg,
                               XLg, cell);
        if ((st = check_hip(hipGetLastError(), "launch k_cell_sum"))) return st;
    }
    const float* cellp = adapt ? cell : nullptr;
    double* part = ws;
    double* stats = ws + K * kFuseParts * kStats;  // [K][16]: statistics, then lambda at +11
    double* gwp = stats + 16 * K;
    double* wtmp = gwp + 3 * K * kFuseParts;
    if (adapt) {
        // statistics of the forward, recomputed here so the adjoint does not depend on workspace state
        hipLaunchKernelGGL(k_fuse_stats, dim3(kFuseParts, (unsigned)K), dim3(256), 0, stream, Sm, D, mask, Tg, ILg,
                           XLg, sections, part);
        if ((st = check_hip(hipGetLastError(), "launch k_fuse_stats"))) return st;
        hipLaunchKernelGGL(k_fuse_solve, dim3((unsigned)K), dim3(64), 0, stream, part, kFuseParts,
                           (int)SAL_FUSE_ADAPT_LS, 0.0, 0.0, 0.0, f.delta, wtmp, stats);
        if ((st = check_hip(hipGetLastError(), "launch k_fuse_solve"))) return st;
        hipLaunchKernelGGL(k_gw_partials, dim3(kFuseParts, (unsigned)K), dim3(256), 0, stream, Sm, cell, Tg, ILg,
                           XLg, sections, gwp);
        if ((st = check_hip(hipGetLastError(), "launch k_gw_partials"))) return st;
        hipLaunchKernelGGL(k_gw_solve, dim3((unsigned)K), dim3(64), 0, stream, gwp, kFuseParts, stats, f.delta);
        if ((st = check_hip(hipGetLastError(), "launch k_gw_solve"))) return st;
    }
    const double* lam = stats + 11;
    if (i32)
        hipLaunchKernelGGL(k_gsm<int32_t>, blocks, dim3(256), 0, stream, Sm, cellp, W, lam, D, mask, Tg, ILg,
                           XLg, ds, adapt, sections, gS, T, IL, XL, s, R);
    else
        hipLaunchKernelGGL(k_gsm<int64_t>, blocks, dim3(256), 0, stream, Sm, cellp, W, lam, D, mask, Tg, ILg,
                           XLg, ds, adapt, sections, gS, T, IL, XL, s, R);
    return check_hip(hipGetLastError(), "launch k_gsm");
}

}  // namespace sal
