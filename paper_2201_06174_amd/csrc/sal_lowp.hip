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
#include "sal_aux.h"

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

template <int N, int PREC, int CTW>
__global__ __launch_bounds__(512) void k_project_lowp(LowpParams p) {
    using L = Lp<PREC>;
    typedef typename L::vec vec;
    constexpr int KH = N / 2 + 1;
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 15;
    const int grp = lane >> 4;

    const int64_t per = (p.ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= p.ntiles) return;
    const int64_t tx = tile % p.tilesX;
    const int64_t ti = (tile / p.tilesX) % p.tilesI;
    const int64_t tt = tile / (p.tilesX * p.tilesI);

    const int s = p.s, RT = p.RT, RTp = p.RTp, RI = p.RI, RX = p.RX, RXp = p.RXp, CT = p.CT;
    float* Vt = lds;                                         // [RT][RI][RXp]
    float* Ab = Vt + (size_t)RT * RI * RXp;                  // [2][RT][RI][4]
    uint16_t* Gh = (uint16_t*)(Ab + (size_t)2 * RT * RI * 4);  // [2][N][16][RTp]
    uint16_t* Gl = Gh + (size_t)2 * N * 16 * RTp;            // same, lo parts (split only)
    const int abStride = RT * RI * 4;
    const int gRow = RTp;                                    // one (ri, u, col) sample row
    const int gStrideRi = N * 16 * RTp;

    const int64_t t0 = tt * CT * s - N / 2, i0 = ti * 4 * s - N / 2, x0 = tx * 4 * s - N / 2;
    for (int e = tid; e < RT * RI * RX; e += 512) {
        const int rx = e % RX;
        const int r = e / RX;
        const int ri = r % RI, rt = r / RI;
        const int64_t gt = reflect_clamp_l(t0 + rt, p.T), gi = reflect_clamp_l(i0 + ri, p.IL),
                      gx = reflect_clamp_l(x0 + rx, p.XL);
        Vt[(rt * RI + ri) * RXp + rx] = p.V[(gt * p.IL + gi) * p.XL + gx];
    }
    // the samples past the last staged row only meet zero coefficients; keep them finite
    for (int e = tid; e < 2 * N * 16 * (RTp - RT); e += 512) {
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
        // ---- pass B: complex DFT along il, one contraction per output tile
        {
            const int ilc = col >> 2, xc = col & 3;
            for (int rt = wave; rt < RT; rt += 8) {
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
        // ---- pass C along t and the projection epilogue
        for (int u = 0; u < N; u++) {
            const float4* wrow = p.wts + ((size_t)(kx * N + u) * 16 + 4 * grp);
            const float4 w0 = wrow[0], w1 = wrow[1], w2 = wrow[2], w3 = wrow[3];
            const uint16_t* gh = Gh + half * gStrideRi + (u * 16 + col) * gRow + b0;
            const uint16_t* gl = Gl + half * gStrideRi + (u * 16 + col) * gRow + b0;
#pragma unroll
            for (int c = 0; c < CTW; c++) {
                const int tc = wave + 8 * c;
                if (tc >= CT) continue;
                uint16_t bh[8], bl[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    bh[i] = gh[tc * s + i];
                    bl[i] = L::split ? gl[tc * s + i] : 0;
                }
                const vec vh = L::from_bits(bh), vl = L::from_bits(bl);
                f4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
                dre = contract<PREC>(are_h, are_l, vh, vl, dre);
                dim = contract<PREC>(aim_h, aim_l, vh, vl, dim);
                float m[4];
#pragma unroll
                for (int j = 0; j < 4; j++) m[j] = __builtin_amdgcn_sqrtf(fmaf(dre[j], dre[j], dim[j] * dim[j]));
                acc[c][0] = fmaf(w0.x, m[0], fmaf(w1.x, m[1], fmaf(w2.x, m[2], fmaf(w3.x, m[3], acc[c][0]))));
                acc[c][1] = fmaf(w0.y, m[0], fmaf(w1.y, m[1], fmaf(w2.y, m[2], fmaf(w3.y, m[3], acc[c][1]))));
                acc[c][2] = fmaf(w0.z, m[0], fmaf(w1.z, m[1], fmaf(w2.z, m[2], fmaf(w3.z, m[3], acc[c][2]))));
            }
        }
    }

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

static size_t lowp_lds_bytes(int n, int s, int CT, bool split, LowpParams* p) {
    p->RT = (CT - 1) * s + n;
    p->RTp = (CT - 1) * s + 16;
    p->RI = 3 * s + n;
    p->RX = 3 * s + n;
    p->RXp = p->RX | 1;
    const size_t f32 = (size_t)p->RT * p->RI * p->RXp + 2 * (size_t)p->RT * p->RI * 4;
    const size_t u16 = (size_t)2 * n * 16 * p->RTp * (split ? 2 : 1);
    return sizeof(float) * f32 + 2 * u16;
}

template <int N, int PREC, int CTW>
static sal_status launch_lowp(const float* V, int64_t T, int64_t IL, int64_t XL, int s, const Tables* tb, float* E,
                              hipStream_t stream) {
    LowpParams p;
    p.V = V;
    p.T = T; p.IL = IL; p.XL = XL;
    p.Tg = ceil_div(T, s); p.ILg = ceil_div(IL, s); p.XLg = ceil_div(XL, s);
    p.s = s;
    const bool split = PREC == SAL_PREC_SPLIT_BF16;
    int CT = 8 * CTW;
    size_t lds = 0;
    for (; CT >= 1; CT--) {
        lds = lowp_lds_bytes(N, s, CT, split, &p);
        if (lds <= 160 * 1024) break;
    }
    if (CT < 1) return fail(SAL_ERR_UNSUPPORTED, "stride too large for the LDS tile");
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
    if (p.ntiles == 0) return SAL_OK;
    static bool attr = false;
    if (!attr) {
        sal_status st = check_hip(hipFuncSetAttribute((const void*)k_project_lowp<N, PREC, CTW>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024),
                                  "hipFuncSetAttribute(project lowp)");
        if (st) return st;
        attr = true;
    }
    const int64_t grid = 8 * ((p.ntiles + 7) / 8);
    if (grid > INT32_MAX) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    hipLaunchKernelGGL((k_project_lowp<N, PREC, CTW>), dim3((unsigned)grid), dim3(512), lds, stream, p);
    return check_hip(hipGetLastError(), "launch k_project_lowp");
}

sal_status launch_project_lowp(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int precision,
                               const Tables* tb, float* E, hipStream_t stream) {
#define SAL_LP(NN, CTW)                                                                                    \
    if (n == NN) {                                                                                         \
        if (precision == SAL_PREC_SPLIT_BF16)                                                              \
            return launch_lowp<NN, SAL_PREC_SPLIT_BF16, CTW>(V, T, IL, XL, s, tb, E, stream);              \
        return launch_lowp<NN, SAL_PREC_FP16, CTW>(V, T, IL, XL, s, tb, E, stream);                       \
    }
    SAL_LP(4, 4)
    SAL_LP(8, 2)
    SAL_LP(12, 1)
    SAL_LP(16, 1)
#undef SAL_LP
    return fail(SAL_ERR_UNSUPPORTED, "window side not built");
}

}  // namespace sal
