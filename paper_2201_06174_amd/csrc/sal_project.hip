// sal_project.hip -- fused local-spectrum / projection / feature kernel (Sec. 2 steps 1-3).
//
// One workgroup owns a tile of CT x 4 x 4 window centres (t, il, xl).  The
// volume tile plus its window halo is staged once in LDS (reflected at the
// borders), then the windowed 3D DFT of every centre is formed separably,
// streaming over the xl frequency kx in [0, n/2] (the input is real, so the
// other half of the spectrum is its conjugate mirror):
//
//   pass A (VALU)  A(t, il, xc; kx)  = sum_a h(a) V(t, il, xc*s+a) e^{-2 pi i kx a/n}
//   pass B (MFMA)  G(t, ic, xc; ki, kx) = sum_b h(b) A(t, ic*s+b, xc; kx) e^{-2 pi i ki b/n}
//   pass C (MFMA)  F(tc, ic, xc; kt, ki, kx) = sum_a h(a) G(tc*s+a, ic, xc; ki, kx) e^{-2 pi i kt a/n}
//
// Passes B and C are real 16 x n x 16 contractions on the matrix cores: the
// A operand is the tapered cos/sin matrix with packed rows (cos 0, cos n/2,
// cos 1, sin 1, ...), the B operand a sliding (Hankel) view of LDS rows.
// The complex combinations of the cos/sin outputs happen in registers, and
// pass C ends in the projection epilogue (Eq. 1 and the third step): |F| of
// each bin times its per-plane weight mult(kx) alpha_m(k) / n^3, accumulated
// per window and reduced across lane groups at the end.  Nothing but E
// leaves the chip.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sal_aux.h"
#include "sal_grid.h"
#include "sal_passb.h"
#include "sal_stage.h"

namespace sal {

typedef float f4 __attribute__((ext_vector_type(4)));

struct ProjParams {
    const float* V;
    int64_t T, IL, XL;
    int64_t Tg, ILg, XLg;
    int s;
    int CT, RT, RI, RX, RXp;
    int64_t tilesT, tilesI, tilesX, ntiles;
    const float* passA;
    const float* mat;
    const float4* wts;
    float* E;
};

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kNT = 1024;  // threads per workgroup: 16 waves, 4 per SIMD

// Persistent form with a prefetched region (n >= 12 at a compile-time stride whose full-depth
// region takes at most 16 t planes per lane; shallower tiles take fewer): a workgroup walks
// several tiles, and during the last kx step of a tile, when no pass reads the staged region
// any more, the next tile's region is loaded into registers and stored over it, so the
// staging latency is hidden.
template <int N, int S, int CTW>
constexpr int fp32_prefetch_planes() {
    return N >= 12 && S > 0 && CTW == 1 ? stage_planes<kNT>(7 * S + N, 3 * S + N, 3 * S + N) : 0;
}
template <int N, int S, int CTW>
constexpr bool fp32_prefetch() {
    return fp32_prefetch_planes<N, S, CTW>() > 0 && fp32_prefetch_planes<N, S, CTW>() <= 16;
}

// One tile of CT x 4 x 4 centres.  S > 0 fixes the stride at compile time (rows of
// pass A then live in registers); S == 0 reads it from the parameters.  With `staged` the
// region is already in LDS; with `has_next` the region of tile `next` (of the volume pn, of
// the same window class and tile depth) is fetched into LDS during the last kx step
// (fp32_prefetch instances).
// EN: the energy feature, |F|^2 against the squared projection weights (p.wts then holds
// mult(kx) alpha_m^2 / n^3), instead of |F|.
template <int N, int S, int CTW, bool EN = false>
__device__ __forceinline__ void project_tile_fp32(const ProjParams& p, const int64_t tile, float* lds,
                                                  bool staged = false, bool has_next = false, int64_t next = 0,
                                                  const ProjParams* pn = nullptr) {
    constexpr int KH = N / 2 + 1;
    constexpr int NK = N / 4;
    constexpr int NW = kNT / 64;           // waves per workgroup (8 or 16)
    constexpr int UH = N * 8 / NW;        // ki slots per wave
    static_assert(NW == 16, "the ki slots are split between two halves of 8 waves");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over waves stay scalar
    const int col = lane & 15;
    const int grp = lane >> 4;

    const int64_t tx = tile % p.tilesX;
    const int64_t ti = (tile / p.tilesX) % p.tilesI;
    const int64_t tt = tile / (p.tilesX * p.tilesI);

    const int s = S > 0 ? S : p.s;
    const int RT = p.RT, CT = p.CT;
    const int RI = S > 0 ? 3 * S + N : p.RI, RX = RI, RXp = S > 0 ? ((3 * S + N) | 1) : p.RXp;
    float* Vt = lds;                                               // [RT][RI][RXp]
    float* Ab = Vt + (((size_t)RT * RI * RXp + 3) & ~(size_t)3);  // [2][RT][RI][4], 16-byte aligned
    float* Gb = Ab + (size_t)2 * RT * RI * 4;                      // [2][N][RT][16]
    float4* Wl = (float4*)(Gb + (size_t)2 * N * RT * 16);          // [N][16] bin weights of the current kx
    const int abStride = RT * RI * 4;
    const int gbStride = N * RT * 16;

    // stage the tile and its halo, reflected at the volume borders
    if (!staged) {
        const int64_t t0 = tt * CT * s - N / 2, i0 = ti * 4 * s - N / 2, x0 = tx * 4 * s - N / 2;
        // with a compile-time stride the deepest region is (8 CTW - 1) s + n planes
        constexpr int MAXU = S > 0 ? stage_batch<kNT>((8 * CTW - 1) * S + N, 3 * S + N, 3 * S + N) : kStageBatch;
        stage_tile<kNT, MAXU>(p.V, p.T, p.IL, p.XL, t0, i0, x0, RT, RI, RX, RXp, Vt);
    }

    // A operand of both MFMA passes: packed taper*DFT rows
    float amat[NK];
#pragma unroll
    for (int ks = 0; ks < NK; ks++) amat[ks] = p.mat[col * N + 4 * ks + grp];
    // PAIR (n = 8): the 8 packed rows fill half of the 16-row operand, so pass C stacks two
    // t-centres: row col of centre col >> 3 at K slot 4 ks + grp (its sample k - (col >> 3) s);
    // 12 samples in 3 K steps instead of 2 x 2
    constexpr bool PAIR = N == 8 && CTW == 1;
    float amatP[3];
#pragma unroll
    for (int ks = 0; ks < 3; ks++) {
        const int a = 4 * ks + grp - (col >> 3) * s;
        amatP[ks] = PAIR && a >= 0 && a < N ? p.mat[(col & 7) * N + a] : 0.f;
    }

    // pass C work of this wave: t-centres wave%8 (+8c), ki slots of one half
    const int wtc = wave & 7;
    float acc[CTW][3];
#pragma unroll
    for (int c = 0; c < CTW; c++) acc[c][0] = acc[c][1] = acc[c][2] = 0.f;

    __syncthreads();

    // PLANE: 0 when kx may be a mirror plane (tested at run time), 1 for a plane known not to be one,
    // 2 for a mirror plane (kx = 0 or n/2)
    auto kstep = [&](const int kx, auto plane) {
        constexpr int PLANE = decltype(plane)::value;
        // ---- pass A: real DFT along xl at bin kx for every staged (t, il) row
        {
            float cA[N], sA[N];
#pragma unroll
            for (int a = 0; a < N; a++) {
                cA[a] = p.passA[(kx * N + a) * 2];
                sA[a] = p.passA[(kx * N + a) * 2 + 1];
            }
            for (int r = tid; r < RT * RI; r += kNT) {
                const float* row = Vt + r * RXp;
                float o[8];
                if constexpr (S > 0) {
                    constexpr int RXc = 3 * S + N;
                    float v[RXc];
#pragma unroll
                    for (int k = 0; k < RXc; k++) v[k] = row[k];
#pragma unroll
                    for (int xc = 0; xc < 4; xc++) {
                        float ar = 0.f, ai = 0.f;
#pragma unroll
                        for (int a = 0; a < N; a++) {
                            ar = fmaf(cA[a], v[xc * S + a], ar);
                            ai = fmaf(sA[a], v[xc * S + a], ai);
                        }
                        o[xc] = ar;
                        o[4 + xc] = ai;
                    }
                } else {
#pragma unroll
                    for (int xc = 0; xc < 4; xc++) {
                        float ar = 0.f, ai = 0.f;
#pragma unroll
                        for (int a = 0; a < N; a++) {
                            const float v = row[xc * s + a];
                            ar = fmaf(cA[a], v, ar);
                            ai = fmaf(sA[a], v, ai);
                        }
                        o[xc] = ar;
                        o[4 + xc] = ai;
                    }
                }
                *(float4*)&Ab[r * 4] = make_float4(o[0], o[1], o[2], o[3]);
                *(float4*)&Ab[abStride + r * 4] = make_float4(o[4], o[5], o[6], o[7]);
            }
        }
        __syncthreads();
        // bin weights of this kx (their previous readers all passed the barrier above).  The
        // planes kx = 0 and kx = n/2 are their own Hermitian mirrors (|F(-k)| = |F(k)|): only
        // the ki slots [0, n/2] are visited there, and a slot whose mirror is skipped counts twice.
        const bool mirror = PLANE == 2 || (PLANE == 0 && (kx == 0 || 2 * kx == N));
        // at n = 8 pass B keeps waves 0..7 busy, so waves from 8 on copy the weights: the latency
        // of their global loads overlaps the products instead of delaying them
        for (int e = PAIR ? tid - kNT / 2 : tid; e < N * 16; e += kNT) {
            if (e < 0) break;
            const int u = e >> 4;
            const float f = mirror && u >= 1 && u < N / 2 ? 2.f : 1.f;
            const float4 w = p.wts[(size_t)kx * N * 16 + e];
            Wl[e] = make_float4(f * w.x, f * w.y, f * w.z, f * w.w);
        }
        // ---- pass B: complex DFT along il on the matrix cores, combined into signed ki slots
        if constexpr (PAIR) {
            pass_b_pair8<false>(Ab, abStride, Gb, gbStride, RT, RI, s, amatP, wave, kNT / 64, col, grp);
        } else {
            const int ilc = col >> 2, xc = col & 3;
            for (int rt = wave; rt < RT; rt += kNT / 64) {
                f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
                float xr[NK], xi[NK];
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    const int idx = (rt * RI + ilc * s + 4 * ks + grp) * 4 + xc;
                    xr[ks] = Ab[idx];
                    xi[ks] = Ab[abStride + idx];
                }
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    dr = mfma4(amat[ks], xr[ks], dr);
                    di = mfma4(amat[ks], xi[ks], di);
                }
#pragma unroll
                for (int pr = 0; pr < 2; pr++) {
                    const int ra = 4 * grp + 2 * pr;
                    if (ra >= N) continue;
                    const float Ca = dr[2 * pr], Sb = dr[2 * pr + 1], Cai = di[2 * pr], Sbi = di[2 * pr + 1];
                    int u1, u2;
                    float g1r, g1i, g2r, g2i;
                    if (ra == 0) {  // cos 0 and cos n/2 rows: no sine partner
                        u1 = 0; u2 = N / 2;
                        g1r = Ca; g1i = Cai; g2r = Sb; g2i = Sbi;
                    } else {
                        const int q = ra >> 1;
                        u1 = q; u2 = N - q;
                        g1r = Ca + Sbi; g1i = Cai - Sb;   // +q
                        g2r = Ca - Sbi; g2i = Cai + Sb;   // -q
                    }
                    Gb[(u1 * RT + rt) * 16 + col] = g1r;
                    Gb[gbStride + (u1 * RT + rt) * 16 + col] = g1i;
                    Gb[(u2 * RT + rt) * 16 + col] = g2r;
                    Gb[gbStride + (u2 * RT + rt) * 16 + col] = g2i;
                }
            }
        }
        __syncthreads();
        // ---- pass C along t on the matrix cores, then |F| * weights into the window sums.
        // The contraction of slot u+1 is issued before the epilogue of slot u, so the
        // matrix cores and the VALU work on different slots at the same time.  The two
        // wave halves split the ki slots to visit, [0, n) or [0, n/2] on a mirror plane.
        if constexpr (PAIR) {
            // wave: centre pair wave & 3 (lanes grp >> 1 pick the centre), ki slots
            // [2q, 2q + 2) of quarter q = wave >> 2, cut to [0, n/2] on a mirror plane
            const int tc0 = 2 * (wave & 3), ua = 2 * (wave >> 2);
            const int nu = mirror ? N / 2 + 1 : N;
            const int cnt = nu - ua >= 2 ? 2 : (nu - ua > 0 ? nu - ua : 0);
            // samples tc0*s + k, k < 12; past the tile's last row only zero coefficients meet
            // the finite LDS that follows
            const float* gbase = Gb + (tc0 * s + grp) * 16 + col;
            auto contractP = [&](int u, f4& dr, f4& di) {
                const float* gr = gbase + u * RT * 16;
                float br[3], bi[3];
#pragma unroll
                for (int ks = 0; ks < 3; ks++) {
                    br[ks] = gr[ks * 64];
                    bi[ks] = gr[gbStride + ks * 64];
                }
                dr = f4{0.f, 0.f, 0.f, 0.f};
                di = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 3; ks++) {
                    dr = mfma4(amatP[ks], br[ks], dr);
                    di = mfma4(amatP[ks], bi[ks], di);
                }
            };
            auto epilogue = [&](int u, const f4& dr, const f4& di) {
                const float4* wrow = Wl + u * 16 + 4 * (grp & 1);
                const float4 w0 = wrow[0], w1 = wrow[1], w2 = wrow[2], w3 = wrow[3];
#pragma unroll
                for (int pr = 0; pr < 2; pr++) {
                    const bool sp = ((grp & 1) == 0) && (pr == 0);
                    const float Ca = dr[2 * pr], Sb = dr[2 * pr + 1], Cai = di[2 * pr], Sbi = di[2 * pr + 1];
                    const float re1 = sp ? Ca : Ca + Sbi, im1 = sp ? Cai : Cai - Sb;
                    const float re2 = sp ? Sb : Ca - Sbi, im2 = sp ? Sbi : Cai + Sb;
                    const float q1 = fmaf(re1, re1, im1 * im1), q2 = fmaf(re2, re2, im2 * im2);
                    const float m1 = EN ? q1 : __builtin_amdgcn_sqrtf(q1);
                    const float m2 = EN ? q2 : __builtin_amdgcn_sqrtf(q2);
                    const float4 wa = pr ? w2 : w0, wb = pr ? w3 : w1;
                    acc[0][0] = fmaf(wa.x, m1, fmaf(wb.x, m2, acc[0][0]));
                    acc[0][1] = fmaf(wa.y, m1, fmaf(wb.y, m2, acc[0][1]));
                    acc[0][2] = fmaf(wa.z, m1, fmaf(wb.z, m2, acc[0][2]));
                }
            };
            if (cnt == 2) {
                f4 d0r, d0i, d1r, d1i;
                contractP(ua, d0r, d0i);
                contractP(ua + 1, d1r, d1i);
                epilogue(ua, d0r, d0i);
                epilogue(ua + 1, d1r, d1i);
            } else if (cnt == 1) {
                f4 d0r, d0i;
                contractP(ua, d0r, d0i);
                epilogue(ua, d0r, d0i);
            }
            return;
        }
        const int ua = (wave >> 3) ? (mirror ? (N / 2 + 2) / 2 : UH) : 0;
#pragma unroll
        for (int c = 0; c < CTW; c++) {
            const int tc = wtc + 8 * c;
            if (tc >= CT) break;
            const float* gbase = Gb + (tc * s + grp) * 16 + col;
            auto contract = [&](int u, f4& dr, f4& di) {
                const float* gr = gbase + u * RT * 16;
                // the wave loading and issuing a slot's products goes first, so the matrix cores
                // start the next contraction while the other waves finish their epilogues (3.4 %
                // faster at n = 16; the paired n = 8 form and pass B are not helped)
                __builtin_amdgcn_s_setprio(1);
                float br[NK], bi[NK];
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    br[ks] = gr[ks * 64];
                    bi[ks] = gr[gbStride + ks * 64];
                }
                dr = f4{0.f, 0.f, 0.f, 0.f};
                di = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    dr = mfma4(amat[ks], br[ks], dr);
                    di = mfma4(amat[ks], bi[ks], di);
                }
                __builtin_amdgcn_s_setprio(0);
            };
            auto run = [&](auto count) {
                constexpr int CNT = decltype(count)::value;
                f4 dr, di;
                contract(ua, dr, di);
#pragma unroll
                for (int uu = 0; uu < CNT; uu++) {
                    const int u = ua + uu;
                    const float4* wrow = Wl + u * 16 + 4 * grp;
                    const float4 w0 = wrow[0], w1 = wrow[1], w2 = wrow[2], w3 = wrow[3];
                    f4 nr, ni;
                    const bool more = uu + 1 < CNT;
                    if (more) contract(u + 1, nr, ni);
#pragma unroll
                    for (int pr = 0; pr < 2; pr++) {
                        const bool sp = (grp == 0) && (pr == 0);
                        const float Ca = dr[2 * pr], Sb = dr[2 * pr + 1], Cai = di[2 * pr], Sbi = di[2 * pr + 1];
                        // the special pair (cos 0, cos n/2) only drops a term in re1, im1: fma(f, x, y)
                        // is y + x for f = 1 and y for f = 0
                        const float f = sp ? 0.f : 1.f;
                        const float re1 = fmaf(f, Sbi, Ca), im1 = fmaf(-f, Sb, Cai);
                        const float re2 = sp ? Sb : Ca - Sbi, im2 = sp ? Sbi : Cai + Sb;
                        const float q1 = fmaf(re1, re1, im1 * im1), q2 = fmaf(re2, re2, im2 * im2);
                        const float m1 = EN ? q1 : __builtin_amdgcn_sqrtf(q1);
                        const float m2 = EN ? q2 : __builtin_amdgcn_sqrtf(q2);
                        const float4 wa = pr ? w2 : w0, wb = pr ? w3 : w1;
                        acc[c][0] = fmaf(wa.x, m1, fmaf(wb.x, m2, acc[c][0]));
                        acc[c][1] = fmaf(wa.y, m1, fmaf(wb.y, m2, acc[c][1]));
                        acc[c][2] = fmaf(wa.z, m1, fmaf(wb.z, m2, acc[c][2]));
                    }
                    if (more) {
                        dr = nr;
                        di = ni;
                    }
                }
            };
            // slot counts are compile-time per case so each loop stays fully unrolled
            if (PLANE == 1 || !mirror) run(std::integral_constant<int, UH>{});
            else if (wave >> 3) run(std::integral_constant<int, (N / 2 + 1) / 2>{});
            else run(std::integral_constant<int, (N / 2 + 2) / 2>{});
        }
        // the next pass A writes only Ab, whose readers (pass B) all passed the barrier above
    };
    if constexpr (fp32_prefetch<N, S, CTW>()) {
        kstep(0, std::integral_constant<int, 2>{});
        for (int kx = 1; kx + 1 < KH; kx++) kstep(kx, std::integral_constant<int, 1>{});
        // the last kx step reads the region in pass A only; its loads for the next tile are in
        // flight meanwhile and land after the step (every wave passed the barrier behind pass A)
        constexpr int NPL = fp32_prefetch_planes<N, S, CTW>();
        float pf[NPL];
        if (has_next) {
            const ProjParams& q = pn ? *pn : p;
            const int64_t nx = next % q.tilesX, ni = (next / q.tilesX) % q.tilesI, nt = next / (q.tilesX * q.tilesI);
            stage_issue<kNT, NPL>(pf, q.V, q.T, q.IL, q.XL, nt * CT * s - N / 2, ni * 4 * s - N / 2,
                                  nx * 4 * s - N / 2, RT, RI, RX);
        }
        kstep(KH - 1, std::integral_constant<int, 2>{});
        if (has_next) stage_commit<kNT, NPL>(pf, RT, RI, RX, RXp, Vt);
    } else {
        // the mirror planes kx = 0 and n/2 peeled off, so every step's slot counts are fixed
        kstep(0, std::integral_constant<int, 2>{});
        for (int kx = 1; kx + 1 < KH; kx++) kstep(kx, std::integral_constant<int, 1>{});
        kstep(KH - 1, std::integral_constant<int, 2>{});
    }

    const int64_t G = p.Tg * p.ILg * p.XLg;
    if constexpr (PAIR) {
        // lane groups 0|1 and 2|3 hold the two centres of a pair; the four ki quarters
        // (waves w, w + 4, w + 8, w + 12) are summed through LDS in a fixed order
        __syncthreads();
        float* red = Gb;  // [3 quarters][4 pairs][2 centres][16][3]
        const int tp = wave & 3, q = wave >> 2, blk = grp >> 1;
        float v[3];
#pragma unroll
        for (int m = 0; m < 3; m++) v[m] = acc[0][m] + __shfl_xor(acc[0][m], 16);
        if (q > 0 && (grp & 1) == 0) {
#pragma unroll
            for (int m = 0; m < 3; m++) red[((((q - 1) * 4 + tp) * 2 + blk) * 16 + col) * 3 + m] = v[m];
        }
        __syncthreads();
        if (q == 0 && (grp & 1) == 0) {
            const int tc = 2 * tp + blk;
            const int64_t gt = tt * CT + tc, gi = ti * 4 + (col >> 2), gx = tx * 4 + (col & 3);
            if (tc < CT && gt < p.Tg && gi < p.ILg && gx < p.XLg) {
                const int64_t j = (gt * p.ILg + gi) * p.XLg + gx;
#pragma unroll
                for (int m = 0; m < 3; m++) {
                    float x = v[m];
#pragma unroll
                    for (int qq = 0; qq < 3; qq++) x += red[(((qq * 4 + tp) * 2 + blk) * 16 + col) * 3 + m];
                    p.E[m * G + j] = x;
                }
            }
        }
        return;
    }
    // reduce the lane groups holding partial sums of the same window, then the two
    // halves of the ki slots (waves w and w + 8) through LDS
    __syncthreads();  // every wave is done with Gb; reuse it for the partial sums
    float* red = Gb;  // [CTW][8][16][3]
    float v[CTW][3];
#pragma unroll
    for (int c = 0; c < CTW; c++)
#pragma unroll
        for (int m = 0; m < 3; m++) {
            float x = acc[c][m];
            x += __shfl_xor(x, 16);
            x += __shfl_xor(x, 32);
            v[c][m] = x;
        }
    if (NW > 8 && wave >= 8 && grp == 0) {
#pragma unroll
        for (int c = 0; c < CTW; c++)
#pragma unroll
            for (int m = 0; m < 3; m++) red[((c * 8 + wtc) * 16 + col) * 3 + m] = v[c][m];
    }
    __syncthreads();
    if (wave < 8 && grp == 0) {
#pragma unroll
        for (int c = 0; c < CTW; c++) {
            const int tc = wtc + 8 * c;
            const int64_t gt = tt * CT + tc, gi = ti * 4 + (col >> 2), gx = tx * 4 + (col & 3);
            if (tc < CT && gt < p.Tg && gi < p.ILg && gx < p.XLg) {
                const int64_t j = (gt * p.ILg + gi) * p.XLg + gx;
#pragma unroll
                for (int m = 0; m < 3; m++) p.E[m * G + j] = v[c][m] + (NW > 8 ? red[((c * 8 + wtc) * 16 + col) * 3 + m] : 0.f);
            }
        }
    }
}

// One tile per workgroup; consecutive workgroups land on different XCDs, so
// each XCD gets a contiguous run of tiles (neighbouring halos share its L2).
// An n = 8 tile is small enough (about 30 KB of LDS) for two workgroups per CU when each
// wave stays within 64 registers; the second workgroup covers the first one's barriers and
// staging.
template <int N>
constexpr int fp32_waves_per_simd() { return N == 8 ? 8 : 4; }

template <int N, int S, int CTW, bool EN = false>
__global__ __launch_bounds__(kNT, (fp32_waves_per_simd<N>())) void k_project_fp32(ProjParams p) {
    extern __shared__ float lds[];
    if constexpr (fp32_prefetch<N, S, CTW>()) {
        // persistent: workgroup b of XCD b % 8 walks that XCD's contiguous share of the tiles
        // with a static stride
        const int64_t per = (p.ntiles + 7) / 8, stride = gridDim.x / 8;
        const int64_t lo = (int64_t)(blockIdx.x % 8) * per, hi = lo + per < p.ntiles ? lo + per : p.ntiles;
        for (int64_t g = lo + blockIdx.x / 8; g < hi; g += stride)
            project_tile_fp32<N, S, CTW, EN>(p, g, lds, g != lo + blockIdx.x / 8, g + stride < hi, g + stride);
        return;
    }
    const int64_t tile = xcd_block(p.ntiles);
    if (tile >= p.ntiles) return;
    project_tile_fp32<N, S, CTW, EN>(p, tile, lds);
}

// Persistent form over the concatenated tiles of many volumes of one window
// class: workgroup b of XCD b % 8 walks that XCD's contiguous share of the
// global tile range with a static stride (every tile is independent, so the
// result does not depend on which workgroup computes it).
template <int N, int S, int CTW>
__global__ __launch_bounds__(kNT, (fp32_waves_per_simd<N>())) void k_project_fp32_batch(const ProjParams* __restrict__ items,
                                                            const int64_t* __restrict__ prefix, int nitems,
                                                            int64_t total) {
    extern __shared__ float lds[];
    const int64_t per = (total + 7) / 8;
    const int64_t xcd = blockIdx.x % 8, local = blockIdx.x / 8, stride = gridDim.x / 8;
    const int64_t lo = xcd * per, hi = lo + per < total ? lo + per : total;
    auto item_of = [&](int64_t g) {  // last item with prefix[item] <= g
        int a = 0, b = nitems - 1;
        while (a < b) {
            const int m = (a + b + 1) / 2;
            if (prefix[m] <= g) a = m; else b = m - 1;
        }
        return a;
    };
    if constexpr (fp32_prefetch<N, S, CTW>()) {
        // each next region (possibly of the next member) is fetched during the current tile
        int64_t g = lo + local;
        if (g >= hi) return;
        int a = item_of(g);
        for (bool staged = false; g < hi; g += stride, staged = true) {
            const bool more = g + stride < hi;
            const int an = more ? item_of(g + stride) : a;
            project_tile_fp32<N, S, CTW>(items[a], g - prefix[a], lds, staged, more, g + stride - prefix[an],
                                         &items[an]);
            a = an;
        }
        return;
    }
    for (int64_t g = lo + local; g < hi; g += stride) {
        const int a = item_of(g);
        __syncthreads();
        project_tile_fp32<N, S, CTW>(items[a], g - prefix[a], lds);
    }
}

// n = 8 (two workgroups per CU within 64 registers): the batch takes one tile per workgroup
// like the single-volume kernel, since the persistent loop's extra live state does not fit
// that register budget.
template <int N>
constexpr bool fp32_batch_one_tile() { return fp32_waves_per_simd<N>() > 4; }

template <int N, int S, int CTW>
__global__ __launch_bounds__(kNT, (fp32_waves_per_simd<N>())) void k_project_fp32_batch1(const ProjParams* __restrict__ items,
                                                             const int64_t* __restrict__ prefix, int nitems,
                                                             int64_t total) {
    extern __shared__ float lds[];
    const int64_t g = xcd_block(total);
    if (g >= total) return;
    int a = 0, b = nitems - 1;  // last item with prefix[item] <= g
    while (a < b) {
        const int m = (a + b + 1) / 2;
        if (prefix[m] <= g) a = m; else b = m - 1;
    }
    project_tile_fp32<N, S, CTW>(items[a], g - prefix[a], lds);
}

static size_t proj_lds_bytes(int n, int s, int CT, int* RT, int* RI, int* RX, int* RXp) {
    *RT = (CT - 1) * s + n;
    *RI = 3 * s + n;
    *RX = 3 * s + n;
    *RXp = *RX | 1;  // odd row pitch: conflict-free row reads in pass A
    const size_t gb = std::max<size_t>(2 * (size_t)n * (*RT) * 16, 8 * 16 * 3 * 4);  // also holds the final sums
    return sizeof(float) * ((((size_t)(*RT) * (*RI) * (*RXp) + 3) & ~(size_t)3) + 2 * (size_t)(*RT) * (*RI) * 4 + gb +
                            (size_t)n * 16 * 4);
}

static constexpr size_t kLdsMax = 160 * 1024;

static int fp32_ctw(int n) { return n == 4 ? 2 : 1; }

// Tile depths (t-centres per tile) that fit the LDS, deepest first.
void project_fp32_ct_candidates(int n, int s, std::vector<int>* out) {
    out->clear();
    const int mx = 8 * fp32_ctw(n);
    int RT, RI, RX, RXp;
    for (int CT = mx; CT >= 1; CT--) {
        if (proj_lds_bytes(n, s, CT, &RT, &RI, &RX, &RXp) > kLdsMax) continue;
        if (out->empty() || CT == mx / 2 || CT == (3 * mx) / 4 || CT == mx / 4) out->push_back(CT);
    }
}

sal_status project_fp32_params(int n, int s, int CT, const float* V, int64_t T, int64_t IL, int64_t XL,
                               const Tables* tb, float* E, void* out, int64_t* ntiles, size_t* lds) {
    ProjParams p;
    p.V = V;
    p.T = T; p.IL = IL; p.XL = XL;
    p.Tg = ceil_div(T, s); p.ILg = ceil_div(IL, s); p.XLg = ceil_div(XL, s);
    p.s = s;
    if (CT <= 0) {
        std::vector<int> c;
        project_fp32_ct_candidates(n, s, &c);
        if (c.empty()) return fail(SAL_ERR_UNSUPPORTED, "stride too large for the LDS tile");
        CT = c[0];
    }
    if (CT > 8 * fp32_ctw(n)) return fail(SAL_ERR_ARG, "tile depth too large");
    *lds = proj_lds_bytes(n, s, CT, &p.RT, &p.RI, &p.RX, &p.RXp);
    if (*lds > kLdsMax) return fail(SAL_ERR_UNSUPPORTED, "tile does not fit the LDS");
    p.CT = CT;
    p.tilesT = ceil_div(p.Tg, CT);
    p.tilesI = ceil_div(p.ILg, 4);
    p.tilesX = ceil_div(p.XLg, 4);
    p.ntiles = p.tilesT * p.tilesI * p.tilesX;
    p.passA = tb->passA;
    p.mat = tb->mat;
    p.wts = (const float4*)tb->wts;
    p.E = E;
    *ntiles = p.ntiles;
    if (out) memcpy(out, &p, sizeof(p));
    return SAL_OK;
}

size_t project_fp32_param_bytes() { return sizeof(ProjParams); }

template <typename K>
static sal_status set_lds_attr(K kernel, const char* what) {
    return check_hip(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax),
                     what);
}

// (n, s) -> the compiled kernel: strides 1..3 have their own instances, larger ones
// take the run-time-stride form.
#define SAL_FP32_DISPATCH(CALL)                                            \
    switch (n) {                                                           \
        case 4: return CALL(4, 1, 2);                                      \
        case 8:                                                            \
            if (s == 1) return CALL(8, 1, 1);                              \
            if (s == 2) return CALL(8, 2, 1);                              \
            if (s == 3) return CALL(8, 3, 1);                              \
            return CALL(8, 0, 1);                                          \
        case 12:                                                           \
            if (s == 1) return CALL(12, 1, 1);                             \
            if (s == 2) return CALL(12, 2, 1);                             \
            if (s == 3) return CALL(12, 3, 1);                             \
            return CALL(12, 0, 1);                                         \
        case 16:                                                           \
            if (s == 1) return CALL(16, 1, 1);                             \
            if (s == 2) return CALL(16, 2, 1);                             \
            if (s == 3) return CALL(16, 3, 1);                             \
            return CALL(16, 0, 1);                                         \
        default: return fail(SAL_ERR_UNSUPPORTED, "window side not built"); \
    }

template <int N, int S, int CTW, bool EN>
static sal_status launch_project(const ProjParams& p, size_t lds, hipStream_t stream) {
    static std::atomic<uint64_t> attr{0};
    sal_status st = lds_limit_once((const void*)k_project_fp32<N, S, CTW, EN>, (int)kLdsMax, attr,
                                   "hipFuncSetAttribute(project)");
    if (st) return st;
    int64_t grid = xcd_grid(p.ntiles);
    if constexpr (fp32_prefetch<N, S, CTW>()) {
        // as many workgroups as are resident at once, a multiple of 8 (one share per XCD)
        int dev = 0, cus = 0, per_cu = 0;
        if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice"))) return st;
        if ((st = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                            "hipDeviceGetAttribute")))
            return st;
        if ((st = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_project_fp32<N, S, CTW, EN>, kNT,
                                                                         lds),
                            "hipOccupancyMaxActiveBlocksPerMultiprocessor")))
            return st;
        grid = std::min<int64_t>(grid, std::max<int64_t>(8, (int64_t)cus * std::max(per_cu, 1) / 8 * 8));
    }
    if (!wide_grid_fits(grid, kNT)) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    hipLaunchKernelGGL((k_project_fp32<N, S, CTW, EN>), wide_grid(grid, kNT), dim3(kNT), lds, stream, p);
    return check_hip(hipGetLastError(), "launch k_project_fp32");
}

sal_status launch_project_fp32(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int feature,
                               const Tables* tb, float* E, hipStream_t stream) {
    ProjParams p;
    int64_t nt = 0;
    size_t lds = 0;
    sal_status st = project_fp32_params(n, s, 0, V, T, IL, XL, tb, E, &p, &nt, &lds);
    if (st) return st;
    if (nt == 0) return SAL_OK;
    if (feature == SAL_FEATURE_ENERGY) {
        p.wts = (const float4*)tb->wts_e;
#define CALL(NN, SS, CC) launch_project<NN, SS, CC, true>(p, lds, stream)
        SAL_FP32_DISPATCH(CALL)
#undef CALL
    }
#define CALL(NN, SS, CC) launch_project<NN, SS, CC, false>(p, lds, stream)
    SAL_FP32_DISPATCH(CALL)
#undef CALL
}

template <int N, int S, int CTW>
static sal_status launch_batch(const void* items, const int64_t* prefix, int nitems, int64_t total, size_t lds,
                               int grid, hipStream_t stream) {
    // the LDS attribute was set by project_fp32_batch_occupancy(), outside any stream capture
    if constexpr (fp32_batch_one_tile<N>()) {
        (void)grid;
        const int64_t g1 = xcd_grid(total);
        if (!wide_grid_fits(g1, kNT)) return fail(SAL_ERR_SHAPE, "batch too large for one launch");
        hipLaunchKernelGGL((k_project_fp32_batch1<N, S, CTW>), wide_grid(g1, kNT), dim3(kNT), lds, stream,
                           (const ProjParams*)items, prefix, nitems, total);
    } else {
        hipLaunchKernelGGL((k_project_fp32_batch<N, S, CTW>), dim3((unsigned)grid), dim3(kNT), lds, stream,
                           (const ProjParams*)items, prefix, nitems, total);
    }
    return check_hip(hipGetLastError(), "launch k_project_fp32_batch");
}

template <int N, int S, int CTW>
static sal_status batch_occupancy(size_t lds, int* per_cu) {
    if constexpr (fp32_batch_one_tile<N>()) {
        sal_status st = set_lds_attr(k_project_fp32_batch1<N, S, CTW>, "hipFuncSetAttribute(project batch)");
        if (st) return st;
        return check_hip(
            hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_project_fp32_batch1<N, S, CTW>, kNT, lds),
            "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    } else {
        sal_status st = set_lds_attr(k_project_fp32_batch<N, S, CTW>, "hipFuncSetAttribute(project batch)");
        if (st) return st;
        return check_hip(
            hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_project_fp32_batch<N, S, CTW>, kNT, lds),
            "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    }
}

// Workgroups of a batched launch: one per tile for the one-tile form, else `resident`.
int64_t project_fp32_batch_grid(int n, int64_t total, int64_t resident) {
    return n == 8 ? 8 * ((total + 7) / 8) : resident;
}

sal_status project_fp32_batch(int n, int s, const void* items, const int64_t* prefix, int nitems, int64_t total,
                              size_t lds, int grid, hipStream_t stream) {
#define CALL(NN, SS, CC) launch_batch<NN, SS, CC>(items, prefix, nitems, total, lds, grid, stream)
    SAL_FP32_DISPATCH(CALL)
#undef CALL
}

sal_status project_fp32_batch_occupancy(int n, int s, size_t lds, int* per_cu) {
#define CALL(NN, SS, CC) batch_occupancy<NN, SS, CC>(lds, per_cu)
    SAL_FP32_DISPATCH(CALL)
#undef CALL
}

}  // namespace sal
