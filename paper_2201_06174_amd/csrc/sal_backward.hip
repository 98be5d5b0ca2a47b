// sal_backward.hip -- hand-written adjoint of the saliency path.
//
// For the loss L = sum_v gS(v) S(v):
//   1. fusion adjoint (Eq. 4): gS_m(g) = W_m c(g), c(g) the cell sum of gS, plus,
//      for adapted weights, the terms through W = (G + delta I)^-1 p;
//   2. center-surround adjoint (Eq. 3), a gather with sgn(0) = 0;
//   3. spectral adjoint (Eq. 1-2 and the feature step): per window, recompute
//      F (the same three passes as the forward), form
//      Y(k) = c(k) F(k)/|F(k)| with c(k) = sum_m gE_m mult(kx) alpha_m(k) / n^3,
//      and run the transposed passes: inverse DFT along t with the taper and an
//      overlap-add over the window centres, the same along il, and along xl the
//      real part accumulated in registers over every kx.  Local spectra are
//      never stored.
// Each workgroup writes the unfolded contribution of its tile region to a
// workspace; a gather kernel then sums, for every voxel, the regions that cover
// it directly or through the border reflection, in a fixed order (no atomics,
// bitwise reproducible).
#include <algorithm>

#include "sal_aux.h"
#include "sal_device.h"
#include "sal_passb.h"
#include "sal_stage.h"

namespace sal {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4b(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void lds_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
// Keeps the compiler from moving LDS accesses across this point.  The LDS itself executes a
// wave's accesses in issue order, so a read issued after another lane's write of the same
// wave sees that write without waiting for it first.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// LDS floats of an adjoint tile of CT t-centres (with or without the separate inverse buffer)
constexpr size_t adj_base_floats(int N, int S, int CT) {
    const size_t RT = (size_t)(CT - 1) * S + N, RI = (size_t)3 * S + N, RXp = (size_t)(3 * S + N) | 1;
    return ((RT * RI * RXp + 3) & ~(size_t)3) + 2 * RT * RI * 4 + 2 * (size_t)N * RT * 16 +
           (size_t)(N / 2 + 1) * N * 2 + (size_t)CT * 16 * 3;
}
constexpr size_t adj_band_floats(int N, int CT) { return N == 8 ? (size_t)CT / 2 * 4 * 64 + 8 * 64 : 0; }

// t-centres per adjoint tile: 8, or the deepest of 4, 2, 1 whose tile fits the LDS (wide
// strides of n = 12 and 16)
constexpr int adj_ct(int N, int S) {
    for (int CT = 8; CT > 1; CT /= 2)
        if ((adj_base_floats(N, S, CT) + adj_band_floats(N, CT)) * sizeof(float) <= 160 * 1024) return CT;
    return 1;
}

struct AdjParams {
    const float* V;
    int64_t T, IL, XL;
    int64_t Tg, ILg, XLg;
    int64_t tilesT, tilesI, tilesX, ntiles;
    const float* gE;
    const float* passA;
    const float* mat;
    const float* inv;
    const float4* wts;
    float* part;  // [tilesT][tilesI][RT][RI][tilesX][RX]: each region row next to its xl neighbours'
};

template <int N, int S>
struct AdjGeom {
    static constexpr int CT = adj_ct(N, S);
    static constexpr int KH = N / 2 + 1;
    static constexpr int NK = N / 4;
    static constexpr int RT = (CT - 1) * S + N;
    static constexpr int RI = 3 * S + N;
    static constexpr int RX = 3 * S + N;
    static constexpr int RXp = RX | 1;
    static constexpr int ROWS = (RT * RI + 511) / 512;
    static constexpr size_t base_floats = adj_base_floats(N, S, CT);
    // SEP: the inverse pass C accumulates into a buffer of its own, so each t-centre's
    // forward contraction, Y and inverse contraction run back to back (few live registers)
    static constexpr bool SEP = (base_floats + 2 * (size_t)N * RT * 16) * sizeof(float) <= 160 * 1024;
    static constexpr size_t lds_floats = base_floats + (SEP ? 2 * (size_t)N * RT * 16 : 0) + adj_band_floats(N, CT);
    // PAIR (n = 8): the 8 packed rows of an n = 8 transform fill half of a 16-row matrix
    // operand, so pass C takes two t-centres per contraction: rows 8..15 hold the second
    // centre's (banded, K = n + s samples; block-diagonal for the inverse)
    static constexpr bool PAIR = N == 8 && SEP && CT % 2 == 0;
    // BANDB (n = 8, RI <= 16): the transposed pass B is one banded contraction per four t
    // rows, with the il rows of a whole tile as the 16 matrix rows
    static constexpr bool BANDB = PAIR && RI <= 16;
    // BANDC (n = 8, RT <= 16): the inverse t-DFT of all t-centres of a ki slot accumulates in
    // one 16-row register tile (banded operand over K = (centre, packed row), 16 per-lane
    // values per centre pair kept in LDS), stored once
    static constexpr bool BANDC = PAIR && RT <= 16;
    // the banded paired operand spans K = 12 samples: both centres of a pair fit for s <= 4
    // (the stride of an n = 8 window is at most 3)
    static_assert(!PAIR || N + S <= 12, "paired contraction too short for this stride");
    static_assert(lds_floats * sizeof(float) <= 160 * 1024, "adjoint tile exceeds the LDS");
};

// With a separate inverse buffer two tiles share a CU (4 waves per SIMD, at most 128
// registers each), three for n = 8 at s <= 2 (6 waves, at most 85 registers; its LDS tile
// is 45 KB); otherwise, or where a thread's synthesis accumulators (ROWS x RX registers)
// are many, one tile takes the CU.
template <int N, int S>
constexpr int adj_waves_per_simd() {
    using Gm = AdjGeom<N, S>;
    return Gm::SEP && Gm::ROWS * Gm::RX <= 40 ? (N <= 8 && S <= 2 ? 6 : 4) : 2;
}

// Y = c F/|F| (EN: Y = 2 c F) of the two bins of a packed row pair, as packed inverse-DFT
// inputs.  (Ca, Sb) and (Cai, Sbi) are the pair's cos and sin rows from the real and imaginary
// channels, giving the bins +q and -q; the special pair sp (cos 0, cos n/2) holds the bins 0 and
// n/2 directly.  c = sum_m gE_m w_m with the window's upstream gradient ge and the bins' weights
// wa, wb.  The cos row of the output takes Y(+q) + Y(-q), the sin row i (Y(+q) - Y(-q)).
// The special pair's selections are products with f = 0 where they can be (fma(f, x, y) is y + x
// for f = 1, y for f = 0), and |F|^2 is floored at the smallest normal float instead of tested:
// a zero spectrum still gives Y = 0, as c F times any finite scale.
template <bool EN>
__device__ __forceinline__ void pack_y(bool sp, float Ca, float Sb, float Cai, float Sbi, float4 wa, float4 wb,
                                       const float* ge, float* y) {
    const float f = sp ? 0.f : 1.f;
    const float re1 = fmaf(f, Sbi, Ca), im1 = fmaf(-f, Sb, Cai);
    const float re2 = sp ? Sb : Ca - Sbi, im2 = sp ? Sbi : Cai + Sb;
    const float c1 = fmaf(ge[0], wa.x, fmaf(ge[1], wa.y, ge[2] * wa.z));
    const float c2 = fmaf(ge[0], wb.x, fmaf(ge[1], wb.y, ge[2] * wb.z));
    const float q1 = fmaf(re1, re1, im1 * im1), q2 = fmaf(re2, re2, im2 * im2);
    const float s1 = EN ? 2.f * c1 : c1 * __builtin_amdgcn_rsqf(fmaxf(q1, 1.17549435e-38f));
    const float s2 = EN ? 2.f * c2 : c2 * __builtin_amdgcn_rsqf(fmaxf(q2, 1.17549435e-38f));
    const float y1r = s1 * re1, y1i = s1 * im1, y2r = s2 * re2, y2i = s2 * im2;
    y[0] = fmaf(f, y2r, y1r);           // real chain, cos row
    y[1] = sp ? y2r : y2i - y1i;        // real chain, sin row
    y[2] = fmaf(f, y2i, y1i);           // imaginary chain, cos row
    y[3] = sp ? y2i : y1r - y2r;        // imaginary chain, sin row
}

// EN: the adjoint of the energy feature, Y = 2 c(k) F(k) with c(k) from the squared projection
// weights (p.wts), instead of c(k) F(k) / |F(k)|.
template <int N, int S, bool EN = false>
__global__ __launch_bounds__(512, (adj_waves_per_simd<N, S>())) void k_spectral_adjoint(AdjParams p) {
    using Gm = AdjGeom<N, S>;
    constexpr int CT = Gm::CT, KH = Gm::KH, NK = Gm::NK, RT = Gm::RT, RI = Gm::RI, RX = Gm::RX, RXp = Gm::RXp,
                  ROWS = Gm::ROWS;
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over waves stay scalar
    const int col = lane & 15;
    const int grp = lane >> 4;

    const int64_t tile = xcd_block(p.ntiles);
    if (tile >= p.ntiles) return;
    const int64_t tx = tile % p.tilesX;
    const int64_t ti = (tile / p.tilesX) % p.tilesI;
    const int64_t tt = tile / (p.tilesX * p.tilesI);

    float* Vt = lds;                          // [RT][RI][RXp]
    float* Ab = Vt + (((size_t)RT * RI * RXp + 3) & ~(size_t)3);  // [2][RT][RI][4]  forward A, then adjoint A'
    float* Gb = Ab + (size_t)2 * RT * RI * 4; // [2][N][RT][16]  forward G, then adjoint G'
    float* tab = Gb + (size_t)2 * N * RT * 16;  // [KH][N][2] h cos, -h sin
    float* gel = tab + (size_t)KH * N * 2;        // [CT][16][3] upstream gradient of the tile's features
    float* Gi = Gm::SEP ? gel + CT * 16 * 3 : Gb;  // [2][N][RT][16] inverse pass C output
    float* atab = Gi + (Gm::SEP ? 2 * N * RT * 16 : 0);  // [CT/2][4][64] banded inverse t operand (n = 8)
    float* btab = atab + (N == 8 ? CT / 2 * 4 * 64 : 0);  // [8][64] banded inverse il operand (n = 8)
    constexpr int abStride = RT * RI * 4;
    constexpr int gbStride = N * RT * 16;

    const int64_t t0 = tt * CT * S - N / 2, i0 = ti * 4 * S - N / 2, x0 = tx * 4 * S - N / 2;
    stage_tile<512, stage_batch<512>(RT, RI, RX)>(p.V, p.T, p.IL, p.XL, t0, i0, x0, RT, RI, RX, RXp, Vt);
    for (int e = tid; e < KH * N * 2; e += 512) tab[e] = p.passA[e];
    if constexpr (Gm::BANDB) {
        // banded transposed pass B: lane l at step k has row il = l & 15 and K slot
        // (il-centre l >> 4, packed row k): the adjoint coefficient of sample il - centre*S.
        // Every lane of a step takes the same packed row, so the inputs are formed alike.
        for (int e = tid; e < 8 * 64; e += 512) {
            const int l = e & 63, k = e >> 6, a = (l & 15) - (l >> 4) * S;
            btab[e] = a >= 0 && a < N ? p.inv[a * 16 + k] : 0.f;
        }
    }
    if constexpr (Gm::BANDC) {
        // lane l at step (pair pp, j): row t = l & 15, K slot l >> 4 = (centre 2 pp + (l >> 5),
        // packed row 4 ((l >> 4) & 1) + j)
        for (int e = tid; e < CT / 2 * 4 * 64; e += 512) {
            const int l = e & 63, j = (e >> 6) & 3, pp = e >> 8;
            const int a = (l & 15) - (2 * pp + (l >> 5)) * S;
            atab[e] = a >= 0 && a < N ? p.inv[a * 16 + 4 * ((l >> 4) & 1) + j] : 0.f;
        }
    }

    float amat[NK], ainvB[NK], ainvC[4];
#pragma unroll
    for (int ks = 0; ks < NK; ks++) {
        amat[ks] = p.mat[col * N + 4 * ks + grp];
        ainvB[ks] = p.inv[col * 16 + 4 * ks + grp];
    }
#pragma unroll
    for (int j = 0; j < 4; j++) ainvC[j] = p.inv[col * 16 + 4 * grp + j];
    // paired operands: forward row col of centre col >> 3 at K slot 4 ks + grp (its sample
    // k - (col >> 3) S), inverse block-diagonal in (output centre, packed-row centre)
    float amatP[3], ainvP[4];
#pragma unroll
    for (int ks = 0; ks < 3; ks++) {
        const int a = 4 * ks + grp - (col >> 3) * S;
        amatP[ks] = a >= 0 && a < N ? p.mat[(col & 7) * N + a] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) ainvP[j] = (col >> 3) == (grp >> 1) ? p.inv[(col & 7) * 16 + ((4 * grp + j) & 7)] : 0.f;

    // upstream gradient of the tile's features (zero outside the grid)
    const int64_t G = p.Tg * p.ILg * p.XLg;
    for (int e = tid; e < CT * 16 * 3; e += 512) {
        const int m = e % 3, w = (e / 3) % 16, tc = e / 48;
        const int64_t gt = tt * CT + tc, gi = ti * 4 + (w >> 2), gx = tx * 4 + (w & 3);
        const bool ok = gt < p.Tg && gi < p.ILg && gx < p.XLg;
        gel[e] = ok ? p.gE[m * G + (gt * p.ILg + gi) * p.XLg + gx] : 0.f;
    }

    float acc[ROWS][RX];
#pragma unroll
    for (int r = 0; r < ROWS; r++)
#pragma unroll
        for (int x = 0; x < RX; x++) acc[r][x] = 0.f;

    __syncthreads();

    for (int kx = 0; kx < KH; kx++) {
        const float* tk = tab + kx * N * 2;
        // ---- forward pass A (as in the feature kernel)
        for (int r = tid; r < RT * RI; r += 512) {
            const float* row = Vt + r * RXp;
            float o[8];
#pragma unroll
            for (int xc = 0; xc < 4; xc++) {
                float ar = 0.f, ai = 0.f;
#pragma unroll
                for (int a = 0; a < N; a++) {
                    const float v = row[xc * S + a];
                    ar = fmaf(tk[2 * a], v, ar);
                    ai = fmaf(tk[2 * a + 1], v, ai);
                }
                o[xc] = ar;
                o[4 + xc] = ai;
            }
            *(float4*)&Ab[r * 4] = make_float4(o[0], o[1], o[2], o[3]);
            *(float4*)&Ab[abStride + r * 4] = make_float4(o[4], o[5], o[6], o[7]);
        }
        __syncthreads();
        // ---- forward pass B
        if constexpr (Gm::PAIR) {
            // two il-centres per contraction with the banded operand pass C uses along t;
            // raised issue priority while a wave issues a run of products (in every pass B and
            // the banded inverse t- and il-DFTs): about 1.5 % off the adjoint in A/B runs
            pass_b_pair8<true>(Ab, abStride, Gb, gbStride, RT, RI, S, amatP, wave, 8, col, grp);
        } else {
            const int ilc = col >> 2, xc = col & 3;
            for (int rt = wave; rt < RT; rt += 8) {
                f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    const int idx = (rt * RI + ilc * S + 4 * ks + grp) * 4 + xc;
                    dr = mfma4b(amat[ks], Ab[idx], dr);
                    di = mfma4b(amat[ks], Ab[abStride + idx], di);
                }
                __builtin_amdgcn_s_setprio(0);
#pragma unroll
                for (int pr = 0; pr < 2; pr++) {
                    const int ra = 4 * grp + 2 * pr;
                    if (ra >= N) continue;
                    const float Ca = dr[2 * pr], Sb = dr[2 * pr + 1], Cai = di[2 * pr], Sbi = di[2 * pr + 1];
                    int u1, u2;
                    float g1r, g1i, g2r, g2i;
                    if (ra == 0) {
                        u1 = 0; u2 = N / 2;
                        g1r = Ca; g1i = Cai; g2r = Sb; g2i = Sbi;
                    } else {
                        const int q = ra >> 1;
                        u1 = q; u2 = N - q;
                        g1r = Ca + Sbi; g1i = Cai - Sb;
                        g2r = Ca - Sbi; g2i = Cai + Sb;
                    }
                    Gb[(u1 * RT + rt) * 16 + col] = g1r;
                    Gb[gbStride + (u1 * RT + rt) * 16 + col] = g1i;
                    Gb[(u2 * RT + rt) * 16 + col] = g2r;
                    Gb[gbStride + (u2 * RT + rt) * 16 + col] = g2i;
                }
            }
        }
        __syncthreads();
        // ---- pass C, Y = c F/|F|, and the transposed pass C with overlap-add over the t-centres.
        // One wave owns each ki slot u, so its rows of the inverse buffer are written by it alone.
        // On the planes kx = 0 and kx = n/2 (their own Hermitian mirrors, Y(-k) = conj Y(k)) only
        // the real part of the synthesis is kept, to which the bins k and -k contribute equally:
        // the ki slots (0, n/2) are visited with twice their weight, their mirrors not at all
        // (zero rows), and the self-mirrored slots 0 and n/2 as they are.
        const bool mirror = kx == 0 || 2 * kx == N;
        for (int u = wave; u < N; u += 8) {
            if (mirror && 2 * u > N) {
                for (int e = lane; e < RT * 16; e += 64) {
                    Gi[u * RT * 16 + e] = 0.f;
                    Gi[gbStride + u * RT * 16 + e] = 0.f;
                }
                continue;
            }
            const float fold = mirror && u > 0 && 2 * u < N ? 2.f : 1.f;
            auto scaled = [&](float4 w) { return make_float4(fold * w.x, fold * w.y, fold * w.z, fold * w.w); };
            const float4* wrow = p.wts + ((size_t)(kx * N + u) * 16 + 4 * grp);
            const float4 w0 = scaled(wrow[0]), w1 = scaled(wrow[1]), w2 = scaled(wrow[2]), w3 = scaled(wrow[3]);
            // forward contraction of t-centre tc and Y = c F/|F| as packed inverse-DFT inputs
            auto fwd_y = [&](int tc, float (&y)[8]) {
                f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
                const float* gr = Gb + (u * RT + tc * S + grp) * 16 + col;
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    dr = mfma4b(amat[ks], gr[ks * 64], dr);
                    di = mfma4b(amat[ks], gr[gbStride + ks * 64], di);
                }
                const float* ge = gel + (tc * 16 + col) * 3;
#pragma unroll
                for (int pr = 0; pr < 2; pr++) {
                    const bool sp = (grp == 0) && (pr == 0);
                    pack_y<EN>(sp, dr[2 * pr], dr[2 * pr + 1], di[2 * pr], di[2 * pr + 1], pr ? w2 : w0, pr ? w3 : w1, ge,
                           &y[4 * pr]);
                }
            };
            // inverse contraction of t-centre tc, overlap-added into rows tc*S + a of slot u;
            // the rows of slot u belong to this wave alone, whose LDS accesses run in order
            auto inv_add = [&](int tc, const float (&y)[8]) {
                f4 zr = {0.f, 0.f, 0.f, 0.f}, zi = {0.f, 0.f, 0.f, 0.f};
                // K-permuted contraction: step j takes packed row 4*grp + j from this lane's registers
                zr = mfma4b(ainvC[0], y[0], zr);
                zi = mfma4b(ainvC[0], y[2], zi);
                zr = mfma4b(ainvC[1], y[1], zr);
                zi = mfma4b(ainvC[1], y[3], zi);
                zr = mfma4b(ainvC[2], y[4], zr);
                zi = mfma4b(ainvC[2], y[6], zi);
                zr = mfma4b(ainvC[3], y[5], zr);
                zi = mfma4b(ainvC[3], y[7], zi);
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int a = 4 * grp + j;
                    if (a < N) {
                        float* dst = Gi + (u * RT + tc * S + a) * 16 + col;
                        dst[0] += zr[j];
                        dst[gbStride] += zi[j];
                    }
                }
                lds_order();
            };
            if constexpr (Gm::PAIR) {
                if constexpr (!Gm::BANDC)
                    for (int e = lane; e < RT * 16; e += 64) {
                        Gi[u * RT * 16 + e] = 0.f;
                        Gi[gbStride + u * RT * 16 + e] = 0.f;
                    }
                f4 Zr = {0.f, 0.f, 0.f, 0.f}, Zi = {0.f, 0.f, 0.f, 0.f};  // banded: rows t of slot u
                // a lane's rows belong to centre tc0 + (grp >> 1), packed rows 4 (grp & 1) + j
                const float4* wp = p.wts + ((size_t)(kx * N + u) * 16 + 4 * (grp & 1));
                const float4 v0 = scaled(wp[0]), v1 = scaled(wp[1]), v2 = scaled(wp[2]), v3 = scaled(wp[3]);
#pragma unroll 1
                for (int tc0 = 0; tc0 < CT; tc0 += 2) {
                    f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
                    // samples tc0*S + k, k < 12 (past the last row only zero coefficients meet
                    // the finite LDS that follows)
                    const float* gr = Gb + (u * RT + tc0 * S + grp) * 16 + col;
#pragma unroll
                    for (int ks = 0; ks < 3; ks++) {
                        dr = mfma4b(amatP[ks], gr[ks * 64], dr);
                        di = mfma4b(amatP[ks], gr[gbStride + ks * 64], di);
                    }
                    const float* ge = gel + ((tc0 + (grp >> 1)) * 16 + col) * 3;
                    float y[8];
#pragma unroll
                    for (int pr = 0; pr < 2; pr++) {
                        const bool sp = ((grp & 1) == 0) && (pr == 0);
                        pack_y<EN>(sp, dr[2 * pr], dr[2 * pr + 1], di[2 * pr], di[2 * pr + 1], pr ? v2 : v0, pr ? v3 : v1, ge,
                               &y[4 * pr]);
                    }
                    if constexpr (Gm::BANDC) {
                        const float* at = atab + (tc0 >> 1) * 256 + lane;
                        __builtin_amdgcn_s_setprio(1);
                        Zr = mfma4b(at[0], y[0], Zr);
                        Zi = mfma4b(at[0], y[2], Zi);
                        Zr = mfma4b(at[64], y[1], Zr);
                        Zi = mfma4b(at[64], y[3], Zi);
                        Zr = mfma4b(at[128], y[4], Zr);
                        Zi = mfma4b(at[128], y[6], Zi);
                        Zr = mfma4b(at[192], y[5], Zr);
                        Zi = mfma4b(at[192], y[7], Zi);
                        __builtin_amdgcn_s_setprio(0);
                        continue;
                    }
                    f4 zr = {0.f, 0.f, 0.f, 0.f}, zi = {0.f, 0.f, 0.f, 0.f};
                    zr = mfma4b(ainvP[0], y[0], zr);
                    zi = mfma4b(ainvP[0], y[2], zi);
                    zr = mfma4b(ainvP[1], y[1], zr);
                    zi = mfma4b(ainvP[1], y[3], zi);
                    zr = mfma4b(ainvP[2], y[4], zr);
                    zi = mfma4b(ainvP[2], y[6], zi);
                    zr = mfma4b(ainvP[3], y[5], zr);
                    zi = mfma4b(ainvP[3], y[7], zi);
                    // output rows 4 grp + j: sample (4 grp + j) & 7 of centre tc0 + (grp >> 1); the
                    // two centres' rows overlap, so they are added one centre after the other
#pragma unroll
                    for (int blk = 0; blk < 2; blk++) {
                        if ((grp >> 1) == blk) {
#pragma unroll
                            for (int j = 0; j < 4; j++) {
                                float* dst = Gi + (u * RT + (tc0 + blk) * S + 4 * (grp & 1) + j) * 16 + col;
                                dst[0] += zr[j];
                                dst[gbStride] += zi[j];
                            }
                        }
                        lds_order();
                    }
                }
                if constexpr (Gm::BANDC) {
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int t = 4 * grp + j;
                        if (t < RT) {
                            Gi[(u * RT + t) * 16 + col] = Zr[j];
                            Gi[gbStride + (u * RT + t) * 16 + col] = Zi[j];
                        }
                    }
                }
            } else if constexpr (Gm::SEP) {
                for (int e = lane; e < RT * 16; e += 64) {
                    Gi[u * RT * 16 + e] = 0.f;
                    Gi[gbStride + u * RT * 16 + e] = 0.f;
                }
#pragma unroll 1
                for (int tc = 0; tc < CT; tc++) {
                    float y[8];
                    fwd_y(tc, y);
                    inv_add(tc, y);
                }
            } else {
                // the inverse overwrites the rows the forward reads: every t-centre's Y first
                float y[CT][8];
#pragma unroll
                for (int tc = 0; tc < CT; tc++) fwd_y(tc, y[tc]);
                lds_fence();
                for (int e = lane; e < RT * 16; e += 64) {
                    Gi[u * RT * 16 + e] = 0.f;
                    Gi[gbStride + u * RT * 16 + e] = 0.f;
                }
#pragma unroll
                for (int tc = 0; tc < CT; tc++) inv_add(tc, y[tc]);
            }
        }
        if constexpr (!Gm::BANDB)
            for (int e = tid; e < 2 * abStride; e += 512) Ab[e] = 0.f;
        __syncthreads();
        if constexpr (Gm::BANDB) {
            // ---- transposed pass B as one banded contraction per (4 t rows, channel): output
            // rows il, columns (t row, xc), K = (il-centre, packed row); the overlap-add over the
            // il-centres happens inside the contraction and every output is stored once.  Step k
            // takes packed row k (0: ki 0, 1: ki n/2, 2q: cos q, 2q+1: sin q) of il-centre grp,
            // formed from this channel's plane P and the other one, Q: the cos row of the real
            // channel is G(+q) + G(-q), its sin row i (G(+q) - G(-q)).
            const int rtp = col >> 2, xc = col & 3;
            for (int item = wave; item < 2 * ((RT + 3) / 4); item += 8) {
                const int ch = item & 1, rt = 4 * (item >> 1) + rtp;
                // a t row past the tile reads the last one; its outputs are dropped
                const int at = (rt < RT ? rt : RT - 1) * 16 + grp * 4 + xc;
                const float* P = Gi + ch * gbStride + at;
                const float* Q = Gi + (1 - ch) * gbStride + at;
                float gp[N], gq[N];
#pragma unroll
                for (int u = 0; u < N; u++) {
                    gp[u] = P[u * RT * 16];
                    gq[u] = 2 * u % N ? Q[u * RT * 16] : 0.f;
                }
                float x[8];
                x[0] = gp[0];
                x[1] = gp[N / 2];
#pragma unroll
                for (int q = 1; q < N / 2; q++) {
                    x[2 * q] = gp[q] + gp[N - q];
                    const float d = gq[q] - gq[N - q];
                    x[2 * q + 1] = ch ? d : -d;
                }
                f4 z = {0.f, 0.f, 0.f, 0.f};
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int k = 0; k < 8; k++) z = mfma4b(btab[k * 64 + lane], x[k], z);
                __builtin_amdgcn_s_setprio(0);
                if (rt < RT) {
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int il = 4 * grp + j;
                        if (il < RI) Ab[ch * abStride + (rt * RI + il) * 4 + xc] = z[j];
                    }
                }
            }
        } else {
            // ---- transposed pass B (ki -> il samples) with overlap-add over the il-centres
            const int ilc = col >> 2, xc = col & 3;
            for (int rt = wave; rt < RT; rt += 8) {
                f4 zr = {0.f, 0.f, 0.f, 0.f}, zi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    const int r = 4 * ks + grp;
                    float xr, xi;
                    if (r == 0 || r == 1) {
                        const int u = r == 0 ? 0 : N / 2;
                        xr = Gi[(u * RT + rt) * 16 + col];
                        xi = Gi[gbStride + (u * RT + rt) * 16 + col];
                    } else {
                        const int q = r >> 1;
                        const float pr_ = Gi[(q * RT + rt) * 16 + col], pi_ = Gi[gbStride + (q * RT + rt) * 16 + col];
                        const float mr_ = Gi[((N - q) * RT + rt) * 16 + col],
                                    mi_ = Gi[gbStride + ((N - q) * RT + rt) * 16 + col];
                        if (r & 1) {  // sin row: i (G(+q) - G(-q))
                            xr = mi_ - pi_;
                            xi = pr_ - mr_;
                        } else {
                            xr = pr_ + mr_;
                            xi = pi_ + mi_;
                        }
                    }
                    zr = mfma4b(ainvB[ks], xr, zr);
                    zi = mfma4b(ainvB[ks], xi, zi);
                }
                // rows b = 4 grp + j of column (ilc, xc) add into il row ilc*S + b, one ilc at a
                // time; the rows of rt belong to this wave alone, whose LDS accesses run in order
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    if (ilc == k) {
#pragma unroll
                        for (int j = 0; j < 4; j++) {
                            const int b = 4 * grp + j;
                            if (b < N) {
                                float* dst = Ab + (rt * RI + k * S + b) * 4 + xc;
                                dst[0] += zr[j];
                                dst[abStride] += zi[j];
                            }
                        }
                    }
                    lds_order();
                }
            }
        }
        __syncthreads();
        // ---- transposed pass A: real part of the kx term into the register accumulators
#pragma unroll
        for (int rr = 0; rr < ROWS; rr++) {
            const int r = tid + 512 * rr;
            if (r < RT * RI) {
#pragma unroll
                for (int xc = 0; xc < 4; xc++) {
                    const float ar = Ab[r * 4 + xc], ai = Ab[abStride + r * 4 + xc];
#pragma unroll
                    for (int a = 0; a < N; a++) acc[rr][xc * S + a] = fmaf(ar, tk[2 * a], fmaf(ai, tk[2 * a + 1], acc[rr][xc * S + a]));
                }
            }
        }
        __syncthreads();
    }

    // stage the tile's contributions through LDS for coalesced workspace writes
#pragma unroll
    for (int rr = 0; rr < ROWS; rr++) {
        const int r = tid + 512 * rr;
        if (r < RT * RI) {
#pragma unroll
            for (int x = 0; x < RX; x++) Vt[r * RXp + x] = acc[rr][x];
        }
    }
    __syncthreads();
    // region row r = (rt, ri) of this tile goes next to the same row of its xl neighbours
    float* out = p.part + ((tt * p.tilesI + ti) * (int64_t)(RT * RI) * p.tilesX + tx) * RX;
    for (int e = tid; e < RT * RI * RX; e += 512) {
        const int rx = e % RX, r = e / RX;
        out[(int64_t)r * p.tilesX * RX + rx] = Vt[r * RXp + rx];
    }
}

// gV(p) = sum over tiles and reflections of the tile contributions at virtual positions
// q with reflect(q) = p, in a fixed order.
struct GatherParams {
    const float* part;
    float* gV;
    int64_t N3[3];
    int64_t tiles[3];
    int C[3];   // centres per tile along each axis
    int R[3];   // region extent along each axis
    int n, s;
};

// Per axis, a voxel p is reached at up to three virtual positions (itself and its two
// half-sample reflections); each lies in the regions of a contiguous range of tiles.
// The ranges are found on the fly (no per-thread arrays, which would live in scratch) and
// visited axis by axis in a fixed order: virtual position, then tile.
template <typename I>
struct GatherAxis {
    I q[3];    // virtual positions relative to the start of tile 0's region
    I lo[3], hi[3];
    int nq;
};

template <typename I>
__device__ __forceinline__ GatherAxis<I> gather_axis(I pa, I Na, int half, int R, I step, I ntiles) {
    GatherAxis<I> g;
    g.nq = 0;
    g.q[0] = g.q[1] = g.q[2] = 0;
    g.q[g.nq++] = pa + half;
    if (-1 - pa >= -half) g.q[g.nq++] = -1 - pa + half;
    if (Na - 1 - pa < half) g.q[g.nq++] = (Na - 1 - pa) + Na + half;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const I lo = g.q[k] - R + 1;
        g.lo[k] = lo <= 0 ? 0 : (lo + step - 1) / step;
        const I hi = g.q[k] / step;
        g.hi[k] = hi > ntiles - 1 ? ntiles - 1 : hi;
    }
    return g;
}

// One workgroup per (t, il) row of the volume: the t and il ranges of covering tiles are the
// same for the whole row (scalar work), each lane then walks the xl tiles of its voxels.
// The sum runs over virtual position, then tile, axis by axis, a fixed order.
template <typename I>
__global__ __launch_bounds__(256) void k_gather(GatherParams p) {
    const int64_t nrows = p.N3[0] * p.N3[1];
    const int64_t r = xcd_block(nrows);
    if (r >= nrows) return;
    const I N1 = (I)p.N3[1], N2 = (I)p.N3[2];
    const int half = p.n / 2;
    const GatherAxis<I> a0 = gather_axis<I>((I)(r / N1), (I)p.N3[0], half, p.R[0], (I)p.C[0] * p.s, (I)p.tiles[0]);
    const GatherAxis<I> a1 = gather_axis<I>((I)(r % N1), N1, half, p.R[1], (I)p.C[1] * p.s, (I)p.tiles[1]);
    const I step0 = (I)p.C[0] * p.s, step1 = (I)p.C[1] * p.s, step2 = (I)p.C[2] * p.s;
    // workspace [tilesT][tilesI][R0][R1][tilesX][R2]
    const I T1 = (I)p.tiles[1], T2 = (I)p.tiles[2];
    // element k of a 3-array by selects (a dynamic index would put the array in scratch)
    auto sel = [](const I* x, int k) { return k == 0 ? x[0] : (k == 1 ? x[1] : x[2]); };
    for (I x = (I)threadIdx.x; x < N2; x += (I)blockDim.x) {
        const GatherAxis<I> a2 = gather_axis<I>(x, N2, half, p.R[2], step2, T2);
        float acc = 0.f;
        for (int k0 = 0; k0 < a0.nq; k0++) {
            const I q0 = sel(a0.q, k0), hi0 = sel(a0.hi, k0);
            for (I t0 = sel(a0.lo, k0); t0 <= hi0; t0++) {
                const I o0 = q0 - t0 * step0;
                for (int k1 = 0; k1 < a1.nq; k1++) {
                    const I q1 = sel(a1.q, k1), hi1 = sel(a1.hi, k1);
                    for (I t1 = sel(a1.lo, k1); t1 <= hi1; t1++) {
                        const I row = ((t0 * T1 + t1) * p.R[0] + o0) * p.R[1] + (q1 - t1 * step1);
                        const float* pr = p.part + row * T2 * p.R[2];
                        for (int k2 = 0; k2 < a2.nq; k2++) {
                            const I q2 = sel(a2.q, k2), hi2 = sel(a2.hi, k2);
                            for (I t2 = sel(a2.lo, k2); t2 <= hi2; t2++) acc += pr[t2 * p.R[2] + (q2 - t2 * step2)];
                        }
                    }
                }
            }
        }
        p.gV[r * N2 + x] = acc;
    }
}

struct AdjLayout {
    int CT, RT, RI, RX;
    int64_t tilesT, tilesI, tilesX, ntiles;
    size_t lds;
    size_t part_bytes;
};

template <int N, int S>
static AdjLayout adj_layout(int64_t T, int64_t IL, int64_t XL) {
    using Gm = AdjGeom<N, S>;
    AdjLayout L;
    L.CT = Gm::CT; L.RT = Gm::RT; L.RI = Gm::RI; L.RX = Gm::RX;
    L.tilesT = ceil_div(ceil_div(T, S), Gm::CT);
    L.tilesI = ceil_div(ceil_div(IL, S), 4);
    L.tilesX = ceil_div(ceil_div(XL, S), 4);
    L.ntiles = L.tilesT * L.tilesI * L.tilesX;
    L.lds = Gm::lds_floats * sizeof(float);
    L.part_bytes = (size_t)L.ntiles * Gm::RT * Gm::RI * Gm::RX * sizeof(float);
    return L;
}

static sal_status adj_layout_dispatch(int n, int s, int64_t T, int64_t IL, int64_t XL, AdjLayout* L) {
#define SAL_ADJ_CASE(NN, SS) \
    if (n == NN && s == SS) { *L = adj_layout<NN, SS>(T, IL, XL); return SAL_OK; }
    SAL_ADJ_CASE(4, 1)
    SAL_ADJ_CASE(8, 1) SAL_ADJ_CASE(8, 2) SAL_ADJ_CASE(8, 3)
    SAL_ADJ_CASE(12, 1) SAL_ADJ_CASE(12, 2) SAL_ADJ_CASE(12, 3) SAL_ADJ_CASE(12, 4) SAL_ADJ_CASE(12, 5)
    SAL_ADJ_CASE(16, 1) SAL_ADJ_CASE(16, 2) SAL_ADJ_CASE(16, 3) SAL_ADJ_CASE(16, 4) SAL_ADJ_CASE(16, 5)
    SAL_ADJ_CASE(16, 6) SAL_ADJ_CASE(16, 7)
#undef SAL_ADJ_CASE
    return fail(SAL_ERR_UNSUPPORTED, "adjoint built for n in {4, 8, 12, 16} and 1 <= s < n/2");
}

template <int N, int S, bool EN>
static sal_status launch_adj(const AdjParams& p, const AdjLayout& L, hipStream_t stream) {
    static std::atomic<uint64_t> attr{0};
    sal_status st = lds_limit_once((const void*)k_spectral_adjoint<N, S, EN>, 160 * 1024, attr,
                                   "hipFuncSetAttribute(adjoint)");
    if (st) return st;
    const int64_t grid = xcd_grid(L.ntiles);
    if (!wide_grid_fits(grid, 512)) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    hipLaunchKernelGGL((k_spectral_adjoint<N, S, EN>), wide_grid(grid, 512), dim3(512), L.lds, stream, p);
    return check_hip(hipGetLastError(), "launch k_spectral_adjoint");
}

template <int N, int S>
static sal_status launch_adj_feature(bool energy, const AdjParams& p, const AdjLayout& L, hipStream_t stream) {
    return energy ? launch_adj<N, S, true>(p, L, stream) : launch_adj<N, S, false>(p, L, stream);
}

static sal_status launch_adj_dispatch(int n, int s, bool energy, const AdjParams& p, const AdjLayout& L,
                                      hipStream_t stream) {
#define SAL_ADJ_CASE(NN, SS) \
    if (n == NN && s == SS) return launch_adj_feature<NN, SS>(energy, p, L, stream);
    SAL_ADJ_CASE(4, 1)
    SAL_ADJ_CASE(8, 1) SAL_ADJ_CASE(8, 2) SAL_ADJ_CASE(8, 3)
    SAL_ADJ_CASE(12, 1) SAL_ADJ_CASE(12, 2) SAL_ADJ_CASE(12, 3) SAL_ADJ_CASE(12, 4) SAL_ADJ_CASE(12, 5)
    SAL_ADJ_CASE(16, 1) SAL_ADJ_CASE(16, 2) SAL_ADJ_CASE(16, 3) SAL_ADJ_CASE(16, 4) SAL_ADJ_CASE(16, 5)
    SAL_ADJ_CASE(16, 6) SAL_ADJ_CASE(16, 7)
#undef SAL_ADJ_CASE
    return fail(SAL_ERR_UNSUPPORTED, "adjoint not built for this window/stride");
}

// Workspace layout of sal_backward (each part 256-byte aligned):
//   cell [G] f32 | gS_m / Q [3G] f32 | gE [3G] f32 | fusion-adjoint doubles | tile partials
struct BwdWs {
    size_t cell, gsm, ge, fus, part, total;
};

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

static BwdWs bwd_ws(int64_t G, const AdjLayout& L, int64_t K) {
    BwdWs w;
    w.cell = 0;
    w.gsm = w.cell + al256(sizeof(float) * G);
    w.ge = w.gsm + al256(sizeof(float) * 3 * G);
    w.fus = w.ge + al256(sizeof(float) * 3 * G);
    w.part = w.fus + al256(fuse_adjoint_workspace_bytes(K));
    w.total = w.part + al256(L.part_bytes);
    return w;
}

}  // namespace sal

using namespace sal;

extern "C" {

size_t sal_backward_workspace_size(int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                                   const sal_fusion* fusion) {
    if (check_spec(spec, T, IL, XL) != SAL_OK) return 0;
    AdjLayout L;
    if (adj_layout_dispatch(spec->n, spec->s, T, IL, XL, &L) != SAL_OK) return 0;
    const int64_t ILg = ceil_div(IL, spec->s);
    const int64_t G = ceil_div(T, spec->s) * ILg * ceil_div(XL, spec->s);
    const int64_t K = fusion && fusion->sections > 0 ? fuse_groups(fusion->sections, ILg) : 1;
    return bwd_ws(G, L, K).total;
}

static sal_status sal_backward_body(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                        const sal_stencil* stencil, const sal_fusion* fusion, const float* E, const float* Sm,
                        const double* W, const float* D, const uint8_t* mask, const float* gS, float* gV_out,
                        void* ws, size_t ws_bytes, sal_stream stream_) {
    hipStream_t stream = (hipStream_t)stream_;
    sal_status st = check_spec(spec, T, IL, XL);
    if (st) return st;
    if (spec->precision != SAL_PREC_FP32) return fail(SAL_ERR_UNSUPPORTED, "the adjoint runs in fp32 only");
    if (!V || !E || !Sm || !W || !gS || !gV_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (!fusion) return fail(SAL_ERR_ARG, "fusion is NULL");
    if (fuse_sequential(fusion->mode))
        return fail(SAL_ERR_UNSUPPORTED, "the adjoint of the LMS / NLMS / RLS recursions is not built (fix their "
                                         "weights with SAL_FUSE_FIXED to differentiate the rest of the path)");
    if (fusion->mode != SAL_FUSE_EQUAL && fusion->mode != SAL_FUSE_FIXED && fusion->mode != SAL_FUSE_ADAPT_LS)
        return fail(SAL_ERR_ARG, "unknown fusion mode");
    if (fusion->mode == SAL_FUSE_ADAPT_LS && (!D || !(fusion->delta >= 0.0)))
        return fail(SAL_ERR_ARG, "ADAPT_LS needs D and delta >= 0");
    if (fusion->sections < 0) return fail(SAL_ERR_ARG, "sections must be >= 0");
    DcsStencil ds;
    if ((st = make_stencil(stencil, spec->s, &ds))) return st;
    AdjLayout L;
    if ((st = adj_layout_dispatch(spec->n, spec->s, T, IL, XL, &L))) return st;
    const int s = spec->s;
    const int64_t Tg = ceil_div(T, s), ILg = ceil_div(IL, s), XLg = ceil_div(XL, s), G = Tg * ILg * XLg;
    const BwdWs lay = bwd_ws(G, L, fuse_groups(fusion->sections, ILg));
    if (!ws || ws_bytes < lay.total) return fail(SAL_ERR_NOMEM, "workspace smaller than sal_backward_workspace_size()");
    char* base = (char*)ws;
    float* cell = (float*)(base + lay.cell);
    float* gSq = (float*)(base + lay.gsm);  // gS_m / Q
    float* gE = (float*)(base + lay.ge);
    double* fws = (double*)(base + lay.fus);
    float* part = (float*)(base + lay.part);
    const Tables* tb = nullptr;
    if ((st = get_tables(stream, spec->n, spec->window, &tb))) return st;

    if ((st = launch_fuse_adjoint(Sm, Tg, ILg, XLg, *fusion, D, mask, W, gS, T, IL, XL, s, ds, cell, fws, gSq,
                                  stream)))
        return st;
    if ((st = launch_dcs_adjoint(E, gSq, gE, Tg, ILg, XLg, ds, stream))) return st;

    AdjParams p;
    p.V = V;
    p.T = T; p.IL = IL; p.XL = XL;
    p.Tg = Tg; p.ILg = ILg; p.XLg = XLg;
    p.tilesT = L.tilesT; p.tilesI = L.tilesI; p.tilesX = L.tilesX; p.ntiles = L.ntiles;
    p.gE = gE;
    p.passA = tb->passA;
    p.mat = tb->mat;
    p.inv = tb->inv;
    const bool energy = spec->feature == SAL_FEATURE_ENERGY;
    p.wts = (const float4*)(energy ? tb->wts_e : tb->wts);
    p.part = part;
    if ((st = launch_adj_dispatch(spec->n, s, energy, p, L, stream))) return st;

    GatherParams gp;
    gp.part = part;
    gp.gV = gV_out;
    gp.N3[0] = T; gp.N3[1] = IL; gp.N3[2] = XL;
    gp.tiles[0] = L.tilesT; gp.tiles[1] = L.tilesI; gp.tiles[2] = L.tilesX;
    gp.C[0] = L.CT; gp.C[1] = 4; gp.C[2] = 4;
    gp.R[0] = L.RT; gp.R[1] = L.RI; gp.R[2] = L.RX;
    gp.n = spec->n;
    gp.s = s;
    const int64_t NV = T * IL * XL;
    const int64_t parts = L.tilesT * L.tilesI * L.tilesX * (int64_t)L.RT * L.RI * L.RX;
    const int64_t lim = int64_t(1) << 30;
    const int64_t nb = xcd_grid(T * IL);  // one workgroup per (t, il) row
    if (!wide_grid_fits(nb, 256)) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    const dim3 grid = wide_grid(nb, 256);
    const dim3 block((unsigned)std::min<int64_t>(256, (XL + 63) / 64 * 64));
    if (parts < 2 * lim && NV < 2 * lim && T < lim && IL < lim && XL < lim)
        hipLaunchKernelGGL(k_gather<int32_t>, grid, block, 0, stream, gp);
    else
        hipLaunchKernelGGL(k_gather<int64_t>, grid, block, 0, stream, gp);
    return check_hip(hipGetLastError(), "launch k_gather");
}

sal_status sal_backward(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                        const sal_stencil* stencil, const sal_fusion* fusion, const float* E, const float* Sm,
                        const double* W, const float* D, const uint8_t* mask, const float* gS, float* gV_out,
                        void* ws, size_t ws_bytes, sal_stream stream_) {
    CallScope cs("sal_backward");
    return cs.done(sal_backward_body(V, T, IL, XL, spec, stencil, fusion, E, Sm, W, D, mask, gS, gV_out, ws, ws_bytes, stream_));
}

}  // extern "C"
