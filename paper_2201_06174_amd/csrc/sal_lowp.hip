// sal_lowp.hip -- the feature kernel with reduced-precision DFT contractions.
//
// Same tiling and streaming over kx as the fp32 kernel, but passes B and C are
// complex contractions on the 16x16x32 bf16/fp16 matrix cores: the K dimension
// holds [real part samples | imaginary part samples] of the window (n <= 16
// each, zero padded), the rows are the 16 DFT bins in natural order, and one
// instruction pair (real and imaginary output tiles) covers a whole 1D DFT of
// 16 windows.  Operands are rounded to bfloat16 twice (hi = bf16(x),
// lo = bf16(x - hi)) and the three products hi*hi + hi*lo + lo*hi are
// accumulated in fp32 (SPLIT_BF16), or rounded once to fp16 (FP16).  Pass A,
// the magnitudes and the projection sums stay in fp32.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sal_aux.h"
#include "sal_stage.h"

namespace sal {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

struct LowpParams {
    const float* V;
    int64_t T, IL, XL;
    int64_t Tg, ILg, XLg;
    int s;
    int CT, RT, RTp, RI, RX, RXp;
    int64_t tilesT, tilesI, tilesX, ntiles;
    const float* passA;
    const uint16_t* cpx_a;  // hi (bf16) or fp16 operand table [2][16][32]
    const uint16_t* cpx_b;  // lo (bf16) table, unused for fp16
    const float4* wts;      // natural-order weights
    float* E;
};

__device__ __forceinline__ int64_t reflect_clamp_l(int64_t p, int64_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p < 0 ? 0 : (p >= N ? N - 1 : p);
}

template <int PREC>
struct Lp;

template <>
struct Lp<SAL_PREC_SPLIT_BF16> {
    typedef bf8 vec;
    static constexpr bool split = true;
    __device__ static __forceinline__ uint16_t hi(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
    __device__ static __forceinline__ uint16_t lo(float x, uint16_t h) {
        const float hf = (float)__builtin_bit_cast(__bf16, h);
        return __builtin_bit_cast(uint16_t, (__bf16)(x - hf));
    }
    __device__ static __forceinline__ vec from_bits(const uint16_t (&b)[8]) {
        vec v;
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = __builtin_bit_cast(__bf16, b[i]);
        return v;
    }
    __device__ static __forceinline__ f4 mma(vec a, vec b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Lp<SAL_PREC_FP16> {
    typedef h8 vec;
    static constexpr bool split = false;
    __device__ static __forceinline__ uint16_t hi(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
    __device__ static __forceinline__ uint16_t lo(float, uint16_t) { return 0; }
    __device__ static __forceinline__ vec from_bits(const uint16_t (&b)[8]) {
        vec v;
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = __builtin_bit_cast(_Float16, b[i]);
        return v;
    }
    __device__ static __forceinline__ f4 mma(vec a, vec b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// D += A * B in the chosen precision (three products for the split form).
template <int PREC>
__device__ __forceinline__ f4 contract(typename Lp<PREC>::vec ah, typename Lp<PREC>::vec al,
                                       typename Lp<PREC>::vec bh, typename Lp<PREC>::vec bl, f4 d) {
    d = Lp<PREC>::mma(ah, bh, d);
    if constexpr (Lp<PREC>::split) {
        d = Lp<PREC>::mma(ah, bl, d);
        d = Lp<PREC>::mma(al, bh, d);
    }
    return d;
}

constexpr int kNTL = 1024;  // threads per workgroup: 16 waves, 4 per SIMD

// Eight consecutive 16-bit samples starting at element t0 of an LDS row whose base is
// 4-byte aligned, read as aligned dwords; an odd start (ODD, known per wave) reads one
// more dword and realigns in registers.  The empty asm statements keep the dword loads
// from being fused into one wide, misaligned access.
template <bool ODD>
__device__ __forceinline__ void load8_u16(const uint16_t* row, int t0, uint32_t (&w)[4]) {
    const uint32_t* p = (const uint32_t*)(row + (t0 & ~1));
    uint32_t a[ODD ? 5 : 4];
#pragma unroll
    for (int i = 0; i < (ODD ? 5 : 4); i++) {
        a[i] = p[i];
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if constexpr (ODD) w[i] = __builtin_amdgcn_alignbyte(a[i + 1], a[i], 2);
        else w[i] = a[i];
    }
}

template <int PREC>
__device__ __forceinline__ typename Lp<PREC>::vec vec_from_words(const uint32_t (&w)[4]) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    u4 v = {w[0], w[1], w[2], w[3]};
    return __builtin_bit_cast(typename Lp<PREC>::vec, v);
}

template <int N, int S, int PREC, int CTW>
__device__ __forceinline__ void project_tile_lowp(const LowpParams& p, const int64_t tile, float* lds) {
    using L = Lp<PREC>;
    typedef typename L::vec vec;
    constexpr int KH = N / 2 + 1;
    constexpr int NW = kNTL / 64;
    constexpr int UH = N * 8 / NW;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 15;
    const int grp = lane >> 4;

    const int64_t tx = tile % p.tilesX;
    const int64_t ti = (tile / p.tilesX) % p.tilesI;
    const int64_t tt = tile / (p.tilesX * p.tilesI);

    const int s = S > 0 ? S : p.s;
    const int RT = p.RT, RTp = p.RTp, CT = p.CT;
    const int RI = S > 0 ? 3 * S + N : p.RI, RX = RI, RXp = S > 0 ? ((3 * S + N) | 1) : p.RXp;
    float* Vt = lds;                                               // [RT][RI][RXp]
    float* Ab = Vt + (((size_t)RT * RI * RXp + 3) & ~(size_t)3);  // [2][RT][RI][4], 16-byte aligned
    uint16_t* Gh = (uint16_t*)(Ab + (size_t)2 * RT * RI * 4);     // [2][N][16][RTp]
    uint16_t* Gl = Gh + (size_t)2 * N * 16 * RTp;                 // same, lo parts (split only)
    float4* Wl = (float4*)(Gl + (L::split ? (size_t)2 * N * 16 * RTp : 0));  // [N][16] weights of this kx
    const int abStride = RT * RI * 4;
    const int gRow = RTp;  // one (ri, u, col) sample row; RTp is even, rows stay 4-byte aligned
    const int gStrideRi = N * 16 * RTp;

    const int64_t t0 = tt * CT * s - N / 2, i0 = ti * 4 * s - N / 2, x0 = tx * 4 * s - N / 2;
    stage_tile<kNTL>(p.V, p.T, p.IL, p.XL, t0, i0, x0, RT, RI, RX, RXp, Vt);
    // the samples past the last staged row only meet zero coefficients; keep them finite
    for (int e = tid; e < 2 * N * 16 * (RTp - RT); e += kNTL) {
        const int pad = RTp - RT;
        const int r = e / pad, k = RT + e % pad;
        Gh[r * RTp + k] = 0;
        if constexpr (L::split) Gl[r * RTp + k] = 0;
    }

    // A operands: lane supplies row = col, K slots 8*grp .. 8*grp+7
    vec are_h, are_l, aim_h, aim_l;
    {
        uint16_t b[8];
#pragma unroll
        for (int i = 0; i < 8; i++) b[i] = p.cpx_a[(0 * 16 + col) * 32 + 8 * grp + i];
        are_h = L::from_bits(b);
#pragma unroll
        for (int i = 0; i < 8; i++) b[i] = p.cpx_a[(1 * 16 + col) * 32 + 8 * grp + i];
        aim_h = L::from_bits(b);
        if constexpr (L::split) {
#pragma unroll
            for (int i = 0; i < 8; i++) b[i] = p.cpx_b[(0 * 16 + col) * 32 + 8 * grp + i];
            are_l = L::from_bits(b);
#pragma unroll
            for (int i = 0; i < 8; i++) b[i] = p.cpx_b[(1 * 16 + col) * 32 + 8 * grp + i];
            aim_l = L::from_bits(b);
        } else {
            are_l = are_h;
            aim_l = aim_h;
        }
    }

    const int wtc = wave & 7;
    const int u0 = (wave >> 3) * UH;
    float acc[CTW][3];
#pragma unroll
    for (int c = 0; c < CTW; c++) acc[c][0] = acc[c][1] = acc[c][2] = 0.f;

    const int half = grp >> 1;       // 0: real part samples, 1: imaginary part samples
    const int b0 = 8 * (grp & 1);    // first sample of this lane's K slots

    __syncthreads();

    for (int kx = 0; kx < KH; kx++) {
        // ---- pass A (fp32)
        {
            float cA[N], sA[N];
#pragma unroll
            for (int a = 0; a < N; a++) {
                cA[a] = p.passA[(kx * N + a) * 2];
                sA[a] = p.passA[(kx * N + a) * 2 + 1];
            }
            for (int r = tid; r < RT * RI; r += kNTL) {
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
        for (int e = tid; e < N * 16; e += kNTL) Wl[e] = p.wts[(size_t)kx * N * 16 + e];
        // ---- pass B: complex DFT along il, one contraction per output tile
        {
            const int ilc = col >> 2, xc = col & 3;
            for (int rt = wave; rt < RT; rt += kNTL / 64) {
                uint16_t bh[8], bl[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const int b = b0 + i;
                    const float x = b < N ? Ab[half * abStride + (rt * RI + ilc * s + b) * 4 + xc] : 0.f;
                    bh[i] = L::hi(x);
                    bl[i] = L::lo(x, bh[i]);
                }
                const vec vh = L::from_bits(bh), vl = L::from_bits(bl);
                f4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
                dre = contract<PREC>(are_h, are_l, vh, vl, dre);
                dim = contract<PREC>(aim_h, aim_l, vh, vl, dim);
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int u = 4 * grp + j;
                    if (u < N) {
                        const uint16_t rh = L::hi(dre[j]), ih = L::hi(dim[j]);
                        Gh[(u * 16 + col) * gRow + rt] = rh;
                        Gh[gStrideRi + (u * 16 + col) * gRow + rt] = ih;
                        if constexpr (L::split) {
                            Gl[(u * 16 + col) * gRow + rt] = L::lo(dre[j], rh);
                            Gl[gStrideRi + (u * 16 + col) * gRow + rt] = L::lo(dim[j], ih);
                        }
                    }
                }
            }
        }
        __syncthreads();
        // ---- pass C along t and the projection epilogue; slot u+1 is contracted before
        // the epilogue of slot u so the matrix cores and the VALU overlap
#pragma unroll
        for (int c = 0; c < CTW; c++) {
            const int tc = wtc + 8 * c;
            if (tc >= CT) break;
            const int ts = tc * s + b0;
            const uint16_t* ghb = Gh + half * gStrideRi + col * gRow;
            const uint16_t* glb = Gl + half * gStrideRi + col * gRow;
            auto run = [&](auto odd) {
                constexpr bool ODD = decltype(odd)::value;
                auto contract_c = [&](int u, f4& dre, f4& dim) {
                    uint32_t wh[4], wl[4];
                    load8_u16<ODD>(ghb + u * 16 * gRow, ts, wh);
                    if constexpr (L::split) load8_u16<ODD>(glb + u * 16 * gRow, ts, wl);
                    const vec vh = vec_from_words<PREC>(wh);
                    const vec vl = L::split ? vec_from_words<PREC>(wl) : vh;
                    dre = contract<PREC>(are_h, are_l, vh, vl, f4{0.f, 0.f, 0.f, 0.f});
                    dim = contract<PREC>(aim_h, aim_l, vh, vl, f4{0.f, 0.f, 0.f, 0.f});
                };
                f4 dre, dim;
                contract_c(u0, dre, dim);
#pragma unroll
                for (int uu = 0; uu < UH; uu++) {
                    const int u = u0 + uu;
                    const float4* wrow = Wl + u * 16 + 4 * grp;
                    const float4 w0 = wrow[0], w1 = wrow[1], w2 = wrow[2], w3 = wrow[3];
                    f4 nre, nim;
                    if (uu + 1 < UH) contract_c(u + 1, nre, nim);
                    float m[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) m[j] = __builtin_amdgcn_sqrtf(fmaf(dre[j], dre[j], dim[j] * dim[j]));
                    acc[c][0] = fmaf(w0.x, m[0], fmaf(w1.x, m[1], fmaf(w2.x, m[2], fmaf(w3.x, m[3], acc[c][0]))));
                    acc[c][1] = fmaf(w0.y, m[0], fmaf(w1.y, m[1], fmaf(w2.y, m[2], fmaf(w3.y, m[3], acc[c][1]))));
                    acc[c][2] = fmaf(w0.z, m[0], fmaf(w1.z, m[1], fmaf(w2.z, m[2], fmaf(w3.z, m[3], acc[c][2]))));
                    if (uu + 1 < UH) {
                        dre = nre;
                        dim = nim;
                    }
                }
            };
            // the window start's parity is the same for the whole wave
            if ((S > 0 && (S & 1) == 0) || (ts & 1) == 0) run(std::false_type{});
            else run(std::true_type{});
        }
    }

    // reduce the lane groups, then the two halves of the ki slots through LDS
    __syncthreads();
    float* red = (float*)Gh;  // [CTW][8][16][3]
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
    const int64_t G = p.Tg * p.ILg * p.XLg;
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

template <int N, int S, int PREC, int CTW>
__global__ __launch_bounds__(kNTL) void k_project_lowp(LowpParams p) {
    extern __shared__ float lds[];
    const int64_t per = (p.ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= p.ntiles) return;
    project_tile_lowp<N, S, PREC, CTW>(p, tile, lds);
}

template <int N, int S, int PREC, int CTW>
__global__ __launch_bounds__(kNTL) void k_project_lowp_batch(const LowpParams* __restrict__ items,
                                                             const int64_t* __restrict__ prefix, int nitems,
                                                             int64_t total) {
    extern __shared__ float lds[];
    const int64_t per = (total + 7) / 8;
    const int64_t xcd = blockIdx.x % 8, local = blockIdx.x / 8, stride = gridDim.x / 8;
    const int64_t lo = xcd * per, hi = lo + per < total ? lo + per : total;
    for (int64_t g = lo + local; g < hi; g += stride) {
        int a = 0, b = nitems - 1;
        while (a < b) {
            const int m = (a + b + 1) / 2;
            if (prefix[m] <= g) a = m; else b = m - 1;
        }
        __syncthreads();
        project_tile_lowp<N, S, PREC, CTW>(items[a], g - prefix[a], lds);
    }
}

static size_t lowp_lds_bytes(int n, int s, int CT, bool split, LowpParams* p) {
    p->RT = (CT - 1) * s + n;
    // row pitch in 16-bit samples: even (dword-aligned rows), one sample of slack for realigned
    // odd starts, and an odd-times-4-plus-3 dword pitch so the 16 columns of a wave's reads
    // and writes fall into distinct LDS banks
    int R = ((CT - 1) * s + 18) / 2;
    while ((R & 3) != 3) R++;
    p->RTp = 2 * R;
    p->RI = 3 * s + n;
    p->RX = 3 * s + n;
    p->RXp = p->RX | 1;
    const size_t f32 = (((size_t)p->RT * p->RI * p->RXp + 3) & ~(size_t)3) + 2 * (size_t)p->RT * p->RI * 4;
    const size_t u16 = std::max<size_t>((size_t)2 * n * 16 * p->RTp * (split ? 2 : 1), 8 * 16 * 3 * 2 * 2);
    return sizeof(float) * f32 + 2 * u16 + sizeof(float) * 4 * 16 * n;
}

static constexpr size_t kLdsMaxL = 160 * 1024;

static int lowp_ctw(int n) { return n == 4 ? 2 : 1; }

void project_lowp_ct_candidates(int n, int s, int precision, std::vector<int>* out) {
    out->clear();
    const int mx = 8 * lowp_ctw(n);
    LowpParams p;
    for (int CT = mx; CT >= 1; CT--) {
        if (lowp_lds_bytes(n, s, CT, precision == SAL_PREC_SPLIT_BF16, &p) > kLdsMaxL) continue;
        if (out->empty() || CT == mx / 2 || CT == (3 * mx) / 4 || CT == mx / 4) out->push_back(CT);
    }
}

sal_status project_lowp_params(int n, int s, int precision, int CT, const float* V, int64_t T, int64_t IL,
                               int64_t XL, const Tables* tb, float* E, void* out, int64_t* ntiles, size_t* lds) {
    LowpParams p;
    p.V = V;
    p.T = T; p.IL = IL; p.XL = XL;
    p.Tg = ceil_div(T, s); p.ILg = ceil_div(IL, s); p.XLg = ceil_div(XL, s);
    p.s = s;
    const bool split = precision == SAL_PREC_SPLIT_BF16;
    if (CT <= 0) {
        std::vector<int> c;
        project_lowp_ct_candidates(n, s, precision, &c);
        if (c.empty()) return fail(SAL_ERR_UNSUPPORTED, "stride too large for the LDS tile");
        CT = c[0];
    }
    if (CT > 8 * lowp_ctw(n)) return fail(SAL_ERR_ARG, "tile depth too large");
    *lds = lowp_lds_bytes(n, s, CT, split, &p);
    if (*lds > kLdsMaxL) return fail(SAL_ERR_UNSUPPORTED, "tile does not fit the LDS");
    p.CT = CT;
    p.tilesT = ceil_div(p.Tg, CT);
    p.tilesI = ceil_div(p.ILg, 4);
    p.tilesX = ceil_div(p.XLg, 4);
    p.ntiles = p.tilesT * p.tilesI * p.tilesX;
    p.passA = tb->passA;
    p.cpx_a = split ? tb->cpx_hi : tb->cpx_h16;
    p.cpx_b = tb->cpx_lo;
    p.wts = (const float4*)tb->wts_nat;
    p.E = E;
    *ntiles = p.ntiles;
    if (out) memcpy(out, &p, sizeof(p));
    return SAL_OK;
}

size_t project_lowp_param_bytes() { return sizeof(LowpParams); }

template <typename K>
static sal_status set_lds_attr_l(K kernel, const char* what) {
    return check_hip(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)kLdsMaxL), what);
}

template <int N, int S, int PREC, int CTW>
static sal_status launch_lowp(const LowpParams& p, size_t lds, hipStream_t stream) {
    static bool attr = false;
    if (!attr) {
        sal_status st = set_lds_attr_l(k_project_lowp<N, S, PREC, CTW>, "hipFuncSetAttribute(project lowp)");
        if (st) return st;
        attr = true;
    }
    const int64_t grid = 8 * ((p.ntiles + 7) / 8);
    if (grid > INT32_MAX) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    hipLaunchKernelGGL((k_project_lowp<N, S, PREC, CTW>), dim3((unsigned)grid), dim3(kNTL), lds, stream, p);
    return check_hip(hipGetLastError(), "launch k_project_lowp");
}

template <int N, int S, int PREC, int CTW>
static sal_status launch_lowp_batch(const void* items, const int64_t* prefix, int nitems, int64_t total, size_t lds,
                                   int grid, hipStream_t stream) {
    // the LDS attribute was set by project_lowp_batch_occupancy(), outside any stream capture
    hipLaunchKernelGGL((k_project_lowp_batch<N, S, PREC, CTW>), dim3((unsigned)grid), dim3(kNTL), lds, stream,
                       (const LowpParams*)items, prefix, nitems, total);
    return check_hip(hipGetLastError(), "launch k_project_lowp_batch");
}

template <int N, int S, int PREC, int CTW>
static sal_status lowp_occupancy(size_t lds, int* per_cu) {
    sal_status st = set_lds_attr_l(k_project_lowp_batch<N, S, PREC, CTW>, "hipFuncSetAttribute(project lowp batch)");
    if (st) return st;
    return check_hip(
        hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_project_lowp_batch<N, S, PREC, CTW>, kNTL, lds),
        "hipOccupancyMaxActiveBlocksPerMultiprocessor");
}

#define SAL_LP_S(NN, CC, PP)                       \
    if (s == 1) return CALL(NN, 1, PP, CC);        \
    if (s == 2 && NN > 4) return CALL(NN, 2, PP, CC); \
    if (s == 3 && NN > 6) return CALL(NN, 3, PP, CC); \
    return CALL(NN, 0, PP, CC);
#define SAL_LP_P(NN, CC)                                                     \
    if (precision == SAL_PREC_SPLIT_BF16) { SAL_LP_S(NN, CC, SAL_PREC_SPLIT_BF16) } \
    SAL_LP_S(NN, CC, SAL_PREC_FP16)
#define SAL_LP_DISPATCH                                                   \
    switch (n) {                                                          \
        case 4: SAL_LP_P(4, 2)                                            \
        case 8: SAL_LP_P(8, 1)                                            \
        case 12: SAL_LP_P(12, 1)                                          \
        case 16: SAL_LP_P(16, 1)                                          \
        default: return fail(SAL_ERR_UNSUPPORTED, "window side not built"); \
    }

sal_status launch_project_lowp(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int precision,
                               const Tables* tb, float* E, hipStream_t stream) {
    LowpParams p;
    int64_t nt = 0;
    size_t lds = 0;
    sal_status st = project_lowp_params(n, s, precision, 0, V, T, IL, XL, tb, E, &p, &nt, &lds);
    if (st) return st;
    if (nt == 0) return SAL_OK;
#define CALL(NN, SS, PP, CC) launch_lowp<NN, SS, PP, CC>(p, lds, stream)
    SAL_LP_DISPATCH
#undef CALL
}

sal_status project_lowp_batch(int n, int s, int precision, const void* items, const int64_t* prefix, int nitems,
                              int64_t total, size_t lds, int grid, hipStream_t stream) {
#define CALL(NN, SS, PP, CC) launch_lowp_batch<NN, SS, PP, CC>(items, prefix, nitems, total, lds, grid, stream)
    SAL_LP_DISPATCH
#undef CALL
}

sal_status project_lowp_batch_occupancy(int n, int s, int precision, size_t lds, int* per_cu) {
#define CALL(NN, SS, PP, CC) lowp_occupancy<NN, SS, PP, CC>(lds, per_cu)
    SAL_LP_DISPATCH
#undef CALL
}

}  // namespace sal
