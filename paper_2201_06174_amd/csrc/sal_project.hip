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
#include "sal_internal.h"

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

__device__ __forceinline__ int64_t reflect_clamp(int64_t p, int64_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p < 0 ? 0 : (p >= N ? N - 1 : p);
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int N, int CTW>
__global__ __launch_bounds__(512) void k_project_fp32(ProjParams p) {
    constexpr int KH = N / 2 + 1;
    constexpr int NK = N / 4;
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 15;
    const int grp = lane >> 4;

    // consecutive workgroups land on different XCDs: give each XCD a contiguous run of tiles
    const int64_t per = (p.ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= p.ntiles) return;
    const int64_t tx = tile % p.tilesX;
    const int64_t ti = (tile / p.tilesX) % p.tilesI;
    const int64_t tt = tile / (p.tilesX * p.tilesI);

    const int s = p.s, RT = p.RT, RI = p.RI, RX = p.RX, RXp = p.RXp, CT = p.CT;
    float* Vt = lds;                                  // [RT][RI][RXp]
    float* Ab = Vt + (size_t)RT * RI * RXp;           // [2][RT][RI][4]
    float* Gb = Ab + (size_t)2 * RT * RI * 4;         // [2][N][RT][16]
    const int abStride = RT * RI * 4;
    const int gbStride = N * RT * 16;

    // stage the tile and its halo, reflected at the volume borders
    const int64_t t0 = tt * CT * s - N / 2, i0 = ti * 4 * s - N / 2, x0 = tx * 4 * s - N / 2;
    const int nreg = RT * RI * RX;
    for (int e = tid; e < nreg; e += 512) {
        const int rx = e % RX;
        const int r = e / RX;
        const int ri = r % RI, rt = r / RI;
        const int64_t gt = reflect_clamp(t0 + rt, p.T), gi = reflect_clamp(i0 + ri, p.IL),
                      gx = reflect_clamp(x0 + rx, p.XL);
        Vt[(rt * RI + ri) * RXp + rx] = p.V[(gt * p.IL + gi) * p.XL + gx];
    }

    // A operand of both MFMA passes: packed taper*DFT rows
    float amat[NK];
#pragma unroll
    for (int ks = 0; ks < NK; ks++) amat[ks] = p.mat[col * N + 4 * ks + grp];

    float acc[CTW][3];
#pragma unroll
    for (int c = 0; c < CTW; c++) acc[c][0] = acc[c][1] = acc[c][2] = 0.f;

    __syncthreads();

    for (int kx = 0; kx < KH; kx++) {
        // ---- pass A: real DFT along xl at bin kx for every staged (t, il) row
        {
            float cA[N], sA[N];
#pragma unroll
            for (int a = 0; a < N; a++) {
                cA[a] = p.passA[(kx * N + a) * 2];
                sA[a] = p.passA[(kx * N + a) * 2 + 1];
            }
            for (int r = tid; r < RT * RI; r += 512) {
                const float* row = Vt + r * RXp;
                float o[8];
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
                *(float4*)&Ab[r * 4] = make_float4(o[0], o[1], o[2], o[3]);
                *(float4*)&Ab[abStride + r * 4] = make_float4(o[4], o[5], o[6], o[7]);
            }
        }
        __syncthreads();
        // ---- pass B: complex DFT along il on the matrix cores, combined into signed ki slots
        {
            const int ilc = col >> 2, xc = col & 3;
            for (int rt = wave; rt < RT; rt += 8) {
                f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    const int idx = (rt * RI + ilc * s + 4 * ks + grp) * 4 + xc;
                    dr = mfma4(amat[ks], Ab[idx], dr);
                    di = mfma4(amat[ks], Ab[abStride + idx], di);
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
        // ---- pass C along t on the matrix cores, then |F| * weights into the window sums
        for (int u = 0; u < N; u++) {
            const float4* wrow = p.wts + ((size_t)(kx * N + u) * 16 + 4 * grp);
            const float4 w0 = wrow[0], w1 = wrow[1], w2 = wrow[2], w3 = wrow[3];
#pragma unroll
            for (int c = 0; c < CTW; c++) {
                const int tc = wave + 8 * c;
                if (tc >= CT) continue;
                f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
                const float* gr = Gb + (u * RT + tc * s + grp) * 16 + col;
#pragma unroll
                for (int ks = 0; ks < NK; ks++) {
                    dr = mfma4(amat[ks], gr[ks * 64], dr);
                    di = mfma4(amat[ks], gr[gbStride + ks * 64], di);
                }
#pragma unroll
                for (int pr = 0; pr < 2; pr++) {
                    const bool sp = (grp == 0) && (pr == 0);
                    const float Ca = dr[2 * pr], Sb = dr[2 * pr + 1], Cai = di[2 * pr], Sbi = di[2 * pr + 1];
                    const float re1 = sp ? Ca : Ca + Sbi, im1 = sp ? Cai : Cai - Sb;
                    const float re2 = sp ? Sb : Ca - Sbi, im2 = sp ? Sbi : Cai + Sb;
                    const float m1 = __builtin_amdgcn_sqrtf(fmaf(re1, re1, im1 * im1));
                    const float m2 = __builtin_amdgcn_sqrtf(fmaf(re2, re2, im2 * im2));
                    const float4 wa = pr ? w2 : w0, wb = pr ? w3 : w1;
                    acc[c][0] = fmaf(wa.x, m1, fmaf(wb.x, m2, acc[c][0]));
                    acc[c][1] = fmaf(wa.y, m1, fmaf(wb.y, m2, acc[c][1]));
                    acc[c][2] = fmaf(wa.z, m1, fmaf(wb.z, m2, acc[c][2]));
                }
            }
        }
        // the next pass A writes only Ab, whose readers (pass B) all passed the barrier above
    }

    // reduce the four lane groups that hold partial sums of the same window
    const int64_t G = p.Tg * p.ILg * p.XLg;
#pragma unroll
    for (int c = 0; c < CTW; c++) {
        const int tc = wave + 8 * c;
        float v[3];
#pragma unroll
        for (int m = 0; m < 3; m++) {
            float x = acc[c][m];
            x += __shfl_xor(x, 16);
            x += __shfl_xor(x, 32);
            v[m] = x;
        }
        const int64_t gt = tt * CT + tc, gi = ti * 4 + (col >> 2), gx = tx * 4 + (col & 3);
        if (grp == 0 && tc < CT && gt < p.Tg && gi < p.ILg && gx < p.XLg) {
            const int64_t j = (gt * p.ILg + gi) * p.XLg + gx;
#pragma unroll
            for (int m = 0; m < 3; m++) p.E[m * G + j] = v[m];
        }
    }
}

static size_t proj_lds_bytes(int n, int s, int CT, int* RT, int* RI, int* RX, int* RXp) {
    *RT = (CT - 1) * s + n;
    *RI = 3 * s + n;
    *RX = 3 * s + n;
    *RXp = *RX | 1;  // odd row pitch: conflict-free row reads in pass A
    return sizeof(float) * ((size_t)(*RT) * (*RI) * (*RXp) + 2 * (size_t)(*RT) * (*RI) * 4 + 2 * (size_t)n * (*RT) * 16);
}

static constexpr size_t kLdsMax = 160 * 1024;

template <int N, int CTW>
static sal_status launch_project(const float* V, int64_t T, int64_t IL, int64_t XL, int s, const Tables* tb,
                                 float* E, hipStream_t stream) {
    ProjParams p;
    p.V = V;
    p.T = T; p.IL = IL; p.XL = XL;
    p.Tg = ceil_div(T, s); p.ILg = ceil_div(IL, s); p.XLg = ceil_div(XL, s);
    p.s = s;
    int CT = 8 * CTW;
    size_t lds = 0;
    for (; CT >= 1; CT--) {
        lds = proj_lds_bytes(N, s, CT, &p.RT, &p.RI, &p.RX, &p.RXp);
        if (lds <= kLdsMax) break;
    }
    if (CT < 1) return fail(SAL_ERR_UNSUPPORTED, "stride too large for the LDS tile");
    p.CT = CT;
    p.tilesT = ceil_div(p.Tg, CT);
    p.tilesI = ceil_div(p.ILg, 4);
    p.tilesX = ceil_div(p.XLg, 4);
    p.ntiles = p.tilesT * p.tilesI * p.tilesX;
    p.passA = tb->passA;
    p.mat = tb->mat;
    p.wts = (const float4*)tb->wts;
    p.E = E;
    if (p.ntiles == 0) return SAL_OK;
    static bool attr_set = false;
    if (!attr_set) {
        sal_status st = check_hip(hipFuncSetAttribute((const void*)k_project_fp32<N, CTW>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax),
                                  "hipFuncSetAttribute(project)");
        if (st) return st;
        attr_set = true;
    }
    const int64_t grid = 8 * ((p.ntiles + 7) / 8);
    if (grid > INT32_MAX) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    hipLaunchKernelGGL((k_project_fp32<N, CTW>), dim3((unsigned)grid), dim3(512), lds, stream, p);
    return check_hip(hipGetLastError(), "launch k_project_fp32");
}

sal_status launch_project_fp32(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, const Tables* tb,
                               float* E, hipStream_t stream) {
    switch (n) {
        case 4: return launch_project<4, 4>(V, T, IL, XL, s, tb, E, stream);
        case 8: return launch_project<8, 2>(V, T, IL, XL, s, tb, E, stream);
        case 12: return launch_project<12, 1>(V, T, IL, XL, s, tb, E, stream);
        case 16: return launch_project<16, 1>(V, T, IL, XL, s, tb, E, stream);
        default: return fail(SAL_ERR_UNSUPPORTED, "window side not built");
    }
}

}  // namespace sal
