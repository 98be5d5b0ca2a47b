// sal_lowp.hip -- the feature kernel with reduced-precision DFT contractions.
//
// Same tiling and streaming over kx as the fp32 kernel, but passes B and C are
// complex contractions on the 16x16x32 bf16/fp16 matrix cores: the K dimension
// holds [real part samples | imaginary part samples] of the window (n <= 16
// each, zero padded), the rows are the 16 DFT bins in natural order, and one
// instruction pair (real and imaginary output tiles) covers a whole 1D DFT of
// 16 windows.  Operands are rounded to bfloat16 twice (hi = bf16(x),
// lo = bf16(x - hi)) and the three products hi*hi + hi*lo + lo*hi are
// accumulated in fp32 (SPLIT_BF16), or rounded once to fp16 (FP16).  Pass A
// and the magnitudes stay in fp32; so do the projection sums of the split form,
// while FP16 takes them on the bf16 matrix cores (magnitudes rounded once,
// weights split into hi + lo, fp32 accumulation).
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sal_aux.h"
#include "sal_grid.h"
#include "sal_stage.h"

namespace sal {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

struct LowpParams {
    const float* V;
    int64_t T, IL, XL;
    int64_t Tg, ILg, XLg;
    int s;
    int CT, RT, RTp, RI, RX, RXp, IQ2;
    int64_t tilesT, tilesI, tilesX, ntiles;
    const float* passA;
    const uint16_t* cpx_a;  // hi (bf16) or fp16 operand table [2][16][32]
    const uint16_t* cpx_b;  // lo (bf16) table, unused for fp16
    const float4* wts;      // natural-order weights, Hermitian mirror folded in (wts_nat_h)
    const uint32_t* wproj;  // FP16 projection operand [KH][N][64 lanes][2 words] (Tables::wproj)
    const uint16_t* pa_ops; // pass-A operands of this stride (fixed tiles)
    float* E;
};

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
    // a in the low half, b in the high half, each rounded to nearest even
    __device__ static __forceinline__ uint32_t pack_hi(float a, float b) {
        const bf2 v = {(__bf16)a, (__bf16)b};
        return __builtin_bit_cast(uint32_t, v);
    }
    // the rounded residuals x - hi (exact in fp32) of the pair packed by pack_hi.  The low
    // element's hi is h << 16, written as a byte alignment so that it stays one instruction
    // (a plain shift is turned back into a second rounding of a plus a shift)
    __device__ static __forceinline__ uint32_t pack_lo(float a, float b, uint32_t h) {
        return pack_hi(a - __uint_as_float(__builtin_amdgcn_alignbyte(h, 0u, 2)), b - __uint_as_float(h & 0xffff0000u));
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
    __device__ static __forceinline__ uint32_t pack_hi(float a, float b) {
        const h2 v = {(_Float16)a, (_Float16)b};
        return __builtin_bit_cast(uint32_t, v);
    }
    __device__ static __forceinline__ uint32_t pack_lo(float, float, uint32_t) { return 0; }
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

// Eight consecutive il samples of one (plane, rt, xc) from an Ab row laid out as
// [il/2][xc][il&1] (dword k*4 + xc holds il = 2k, 2k+1).  `rowx` points at dword xc of
// il/2 = 0.  An even stride keeps every lane's start even; otherwise each lane realigns
// by its own start parity.
template <int S>
__device__ __forceinline__ void load8_ab(const uint32_t* rowx, int il0, uint32_t (&w)[4]) {
    const uint32_t* q = rowx + (il0 >> 1) * 4;
    if constexpr (S > 0 && (S & 1) == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) w[k] = q[4 * k];
    } else {
        uint32_t a[5];
#pragma unroll
        for (int k = 0; k < 5; k++) a[k] = q[4 * k];
        const uint32_t sh = (il0 & 1) * 2;
#pragma unroll
        for (int k = 0; k < 4; k++) w[k] = __builtin_amdgcn_alignbyte(a[k + 1], a[k], sh);
    }
}

// Row pitch of the pass-B output rows in 16-bit samples for a tile of CT t-centres: even
// (dword-aligned rows), room for the furthest realigned read, and an odd-times-4-plus-3
// dword pitch so the 16 columns of a wave's reads and writes fall into distinct LDS banks.
__host__ __device__ constexpr int lowp_rtp(int CT, int s) {
    int R = ((CT - 1) * s + 18) / 2;
    while ((R & 3) != 3) R++;
    return 2 * R;
}

// Offset between the real and imaginary planes of a pass output, in 16-bit samples: the
// plane size rounded up to 16 modulo 32 dwords.  The two planes then start in opposite
// halves of the 32 LDS banks, so the lane groups of a wave that read both planes at the same
// position (rows of 16 consecutive banks, or of an odd dword pitch) never share a bank.
__host__ __device__ constexpr int plane_pitch16(int n16) {
    return 2 * (n16 / 2 + (16 - (n16 / 2) % 32 + 32) % 32);
}

// Two magnitudes rounded to bf16 (nearest even), a in the low half.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
    const bf2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// Sum over the 16 lanes of a DPP row (the bins kt of one lane group): rotations by 8, 4, 2
// and 1 within the row leave the total in every lane, without a trip through LDS.
__device__ __forceinline__ float row_sum16(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xf, 0xf, false));
    return x;
}

// dword columns per Ab row plane: cover the furthest read of pass B, which starts at
// il = 3s + 8 (last window column, upper K half) and spans 4 dwords for an even stride,
// 5 for an odd one
__host__ __device__ constexpr int ab_iq2(int s) { return (3 * s + 8) / 2 + ((s & 1) ? 5 : 4); }

// Extents of the fixed-tile LDS layout, where the staged volume is held as 16-bit planes
// for pass A on the matrix cores: rows r = rt * RIE + il of XP samples (RIE = RI rounded up
// to even so that rows r, r + 1 with r even are il pairs of one rt; XP = RX rounded up to 8
// for 16-byte operand reads), MT tiles of 16 rows, plus the rows that the 32-sample operand
// reads of the last tile run past.
struct FixGeom {
    int RT, RTe, RI, RIE, RX, XP, MROWS, MT, VROWS, VP;
};
__host__ __device__ constexpr FixGeom fix_geom(int n, int s, int CT) {
    FixGeom g{};
    g.RT = (CT - 1) * s + n;
    g.RTe = (g.RT + 1) & ~1;
    g.RI = 3 * s + n;
    g.RIE = (g.RI + 1) & ~1;
    g.RX = 3 * s + n;
    g.XP = (g.RX + 7) & ~7;
    g.MROWS = g.RTe * g.RIE;
    g.MT = (g.MROWS + 15) / 16;
    g.VROWS = g.MT * 16 + (32 - g.XP + g.XP - 1) / g.XP;
    g.VP = g.VROWS * g.XP;
    return g;
}

// FIX: the tile has its full depth 8*CTW and a compile-time stride, so every LDS extent
// and pitch is a compile-time constant (addresses fold into instruction offsets), and the
// volume is staged once per tile as 16-bit operands: pass A then also runs on the matrix
// cores, and the bin weights are read from the (cached) global table.
// Persistent form with a prefetched region (fixed tile, n >= 12, at most 16 t planes per
// lane): during the last kx step of a tile, when pass A no longer reads the staged planes,
// the next tile's region is loaded into registers and its rounded samples are stored after
// the step.  FP16 only: the split form already uses all 128 registers, and neither the
// registers' spills nor loading the fp32 region straight into LDS (whose wait then lands
// on the first weight load of pass C) cost less than the staging they hide (measured).
template <int N, int S, int PREC, int CTW, bool FIX>
constexpr int lowp_prefetch_planes() {
    return FIX && N >= 12 && S > 0 && CTW == 1 ? stage_planes<kNTL>(7 * S + N, 3 * S + N, 3 * S + N) : 0;
}
template <int N, int S, int PREC, int CTW, bool FIX>
constexpr bool lowp_prefetch() {
    return PREC == SAL_PREC_FP16 && lowp_prefetch_planes<N, S, PREC, CTW, FIX>() > 0 &&
           lowp_prefetch_planes<N, S, PREC, CTW, FIX>() <= 16;
}

// One tile.  With `staged` the region (and the constant pads) are already in LDS; with
// `has_next` the region of tile `next` of pn (same window class) is fetched during the last
// kx step (lowp_prefetch instances).
template <int N, int S, int PREC, int CTW, bool FIX>
__device__ __forceinline__ void project_tile_lowp(const LowpParams& p, const int64_t tile, float* lds,
                                                  bool staged = false, bool has_next = false, int64_t next = 0,
                                                  const LowpParams* pn = nullptr) {
    using L = Lp<PREC>;
    typedef typename L::vec vec;
    constexpr int KH = N / 2 + 1;
    constexpr int NW = kNTL / 64;
    constexpr int UH = N * 8 / NW;
    static_assert(NW == 16, "the ki slots are split between two halves of 8 waves");
    constexpr int NPL = L::split ? 4 : 2;  // Ab planes: (hi, lo) x (real, imaginary)
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over waves stay scalar
    const int col = lane & 15;
    const int grp = lane >> 4;

    const int64_t tx = tile % p.tilesX;
    const int64_t ti = (tile / p.tilesX) % p.tilesI;
    const int64_t tt = tile / (p.tilesX * p.tilesI);

    const int s = S > 0 ? S : p.s;
    static_assert(!FIX || S > 0, "a fixed tile needs a compile-time stride");
    constexpr int CTF = 8 * CTW;
    constexpr FixGeom FG = fix_geom(N, S > 0 ? S : 1, CTF);
    const int CT = FIX ? CTF : p.CT;
    const int RT = FIX ? FG.RT : p.RT;
    const int RTe = (RT + 1) & ~1;
    const int RTp = FIX ? lowp_rtp(CTF, S > 0 ? S : 1) : p.RTp;
    const int RI = S > 0 ? 3 * S + N : p.RI, RX = RI, RXp = S > 0 ? ((3 * S + N) | 1) : p.RXp;
    const int IQ2 = S > 0 ? ab_iq2(S) : p.IQ2;
    // fixed tile: Vb [hi, lo][VROWS][XP] 16-bit; otherwise Vt [RT][RI][RXp] fp32
    float* Vt = lds;
    uint16_t* Vb = (uint16_t*)lds;
    constexpr int NVP = L::split ? 2 : 1;
    const size_t vbytes = FIX ? (size_t)NVP * FG.VP * 2 : (((size_t)RT * RI * RXp + 3) & ~(size_t)3) * 4;
    uint16_t* Ab = (uint16_t*)((char*)lds + vbytes);                      // [NPL][RTe][IQ2][4][2]
    const int abPlane = plane_pitch16(RTe * IQ2 * 8);
    const int gStrideRi = N * 16 * RTp;         // one plane [N][16][RTp]
    const int gPlane = plane_pitch16(gStrideRi);  // real plane to imaginary plane
    uint16_t* Gh = Ab + (size_t)NPL * abPlane;                          // [re, im][N][16][RTp]
    uint16_t* Gl = Gh + (size_t)gPlane + gStrideRi;                      // same, lo parts (split only)
    float4* Wl = (float4*)(Gl + (L::split ? (size_t)gPlane + gStrideRi : 0));  // [N][16] weights of this kx
    const int gRow = RTp;  // one (ri, u, col) sample row; RTp is even, rows stay 4-byte aligned

    // zero the pads the operand reads cover (disjoint from the staged samples): columns
    // [RX, XP) of every row, the odd il row of each rt, and the rows from rt = RT on
    auto zero_vb_pads = [&]() {
        if constexpr (FIX) {
            constexpr int XPAD = FG.XP - FG.RX;
            if constexpr (XPAD > 0)
                for (int e = tid; e < FG.VROWS * XPAD; e += kNTL) {
                    const int at = (e / XPAD) * FG.XP + FG.RX + e % XPAD;
                    Vb[at] = 0;
                    if constexpr (L::split) Vb[FG.VP + at] = 0;
                }
            if constexpr (FG.RIE > FG.RI)
                for (int e = tid; e < FG.RT * FG.RX; e += kNTL) {
                    const int at = ((e / FG.RX) * FG.RIE + FG.RI) * FG.XP + e % FG.RX;
                    Vb[at] = 0;
                    if constexpr (L::split) Vb[FG.VP + at] = 0;
                }
            for (int e = tid; e < (FG.VROWS - FG.RT * FG.RIE) * FG.RX; e += kNTL) {
                const int at = (FG.RT * FG.RIE + e / FG.RX) * FG.XP + e % FG.RX;
                Vb[at] = 0;
                if constexpr (L::split) Vb[FG.VP + at] = 0;
            }
        }
    };
    const int64_t t0 = tt * CT * s - N / 2, i0 = ti * 4 * s - N / 2, x0 = tx * 4 * s - N / 2;
    if (staged) {
        // region and pads are in place (the pads are never overwritten)
    } else if constexpr (FIX) {
        stage_tile_with<kNTL, stage_batch<kNTL>(FG.RT, FG.RI, FG.RX)>(p.V, p.T, p.IL, p.XL, t0, i0, x0, RT, RI, RX, [&](int rt, int ri, int rx, float v) {
            const int at = (rt * FG.RIE + ri) * FG.XP + rx;
            const uint16_t h = L::hi(v);
            Vb[at] = h;
            if constexpr (L::split) Vb[FG.VP + at] = L::lo(v, h);
        });
        zero_vb_pads();
        // Ab columns il/2 in [RIE/2, IQ2) are read by pass B but never written by pass A
        constexpr int CPAD = ab_iq2(S > 0 ? S : 1) - FG.RIE / 2;
        if constexpr (CPAD > 0)
            for (int e = tid; e < NPL * FG.RTe * CPAD * 4; e += kNTL) {
                const int pl = e / (FG.RTe * CPAD * 4), r = e % (FG.RTe * CPAD * 4);
                const int rt = r / (CPAD * 4), k = r % (CPAD * 4);
                ((uint32_t*)(Ab + (size_t)pl * abPlane))[(rt * IQ2 + FG.RIE / 2) * 4 + k] = 0u;
            }
    } else {
        stage_tile<kNTL>(p.V, p.T, p.IL, p.XL, t0, i0, x0, RT, RI, RX, RXp, Vt);
    }

    // The K slots of passes B and C are (channel, sample): K = 16 * half + b0 + i, half = the
    // real or imaginary plane of the data, b0 + i the sample.  Lane group grp takes half =
    // grp & 1 and b0 = 8 (grp >> 1), so the 32 lanes that the LDS serves together read the two
    // planes at the same sample offset (no bank shared, see plane_pitch16).
    const int half = grp & 1;
    const int b0 = 8 * (grp >> 1);
    const int kslot = 16 * half + b0;
    // DFT operands: lane supplies bin = col, K slots kslot .. kslot + 7
    vec are_h, are_l, aim_h, aim_l;
    {
        uint16_t b[8];
#pragma unroll
        for (int i = 0; i < 8; i++) b[i] = p.cpx_a[(0 * 16 + col) * 32 + kslot + i];
        are_h = L::from_bits(b);
#pragma unroll
        for (int i = 0; i < 8; i++) b[i] = p.cpx_a[(1 * 16 + col) * 32 + kslot + i];
        aim_h = L::from_bits(b);
        if constexpr (L::split) {
#pragma unroll
            for (int i = 0; i < 8; i++) b[i] = p.cpx_b[(0 * 16 + col) * 32 + kslot + i];
            are_l = L::from_bits(b);
#pragma unroll
            for (int i = 0; i < 8; i++) b[i] = p.cpx_b[(1 * 16 + col) * 32 + kslot + i];
            aim_l = L::from_bits(b);
        } else {
            are_l = are_h;
            aim_l = aim_h;
        }
    }
    // pass-A operands of a bin kx (fixed tile): lane supplies column col (cos|sin x window
    // column), K slots = staged samples 8*grp .. 8*grp+7
    auto pass_a_ops = [&](int kx, vec& bh, vec& bl) {
        const uint16_t* o = p.pa_ops + ((size_t)(kx * 3 + (L::split ? 0 : 2)) * 16 + col) * 32 + 8 * grp;
        bh = __builtin_bit_cast(vec, *(const uint4*)o);
        bl = L::split ? __builtin_bit_cast(vec, *(const uint4*)(o + 16 * 32)) : bh;
    };
    vec pbh, pbl;
    if constexpr (FIX) pass_a_ops(0, pbh, pbl);

    const int wtc = wave & 7;
    // split form: acc[c][j][m], window 4*grp + j of t slot wtc + 8c, plane m, summed over this
    // lane's bins.  FP16: pacc[c], row m' = 4 grp + j of window col of t slot wtc + 8c (j = 0..2:
    // plane m = j from the weights' hi parts in lane group 0, from their lo parts in group 1).
    float acc[CTW][4][3];
    f4 pacc[CTW];
#pragma unroll
    for (int c = 0; c < CTW; c++) {
        pacc[c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; j++) acc[c][j][0] = acc[c][j][1] = acc[c][j][2] = 0.f;
    }

    __syncthreads();
    // the samples past the last staged row only meet zero coefficients; keep them finite.
    // Written after the barrier: the previous tile of a persistent workgroup reduced its sums
    // in these rows, and pass C reads them only after two more barriers.
    for (int e = tid; e < 2 * N * 16 * (RTp - RT); e += kNTL) {
        const int pad = RTp - RT;
        const int r = e / pad, k = RT + e % pad;
        const int at = (r >= N * 16 ? gPlane - gStrideRi : 0) + r * RTp + k;
        Gh[at] = 0;
        if constexpr (L::split) Gl[at] = 0;
    }

    // PLANE: 0 when kx may be a mirror plane (tested at run time), 1 for a plane known not to be one,
    // 2 for a mirror plane (kx = 0 or n/2)
    auto kstep = [&](const int kx, auto plane) {
        constexpr int PLANE = decltype(plane)::value;
        if constexpr (FIX) {
            // ---- pass A on the matrix cores: 16 staged rows x 32 samples times the 32 x 16
            // operand of this kx (columns cos|sin x window column); the il pairs of the result
            // are rounded once and stored packed for pass B
            for (int mt = wave; mt < FG.MT; mt += NW) {
                const uint16_t* ra = Vb + (size_t)(mt * 16 + col) * FG.XP + 8 * grp;
                const vec ah = __builtin_bit_cast(vec, *(const uint4*)ra);
                const vec al = L::split ? __builtin_bit_cast(vec, *(const uint4*)(ra + FG.VP)) : ah;
                const f4 d = contract<PREC>(ah, al, pbh, pbl, f4{0.f, 0.f, 0.f, 0.f});
                if (col < 8) {
                    const int h = col >> 2, xc = col & 3;
                    if constexpr (2 * ab_iq2(S > 0 ? S : 1) == FG.RIE) {
                        // the Ab rows hold exactly the il pairs of a staged row set (pitch RIE / 2
                        // pairs), so row pair r / 2 of the staged planes lands at dword r / 2 * 4 + xc:
                        // a running address instead of a division per row
                        uint32_t* dst = (uint32_t*)(Ab + (size_t)h * abPlane) + (mt * 8 + 2 * grp) * 4 + xc;
                        const bool full = (mt + 1) * 16 <= FG.MROWS;  // only the last tile is partial
#pragma unroll
                        for (int pr = 0; pr < 2; pr++) {
                            if (full || mt * 16 + 4 * grp + 2 * pr < FG.MROWS) {
                                const uint32_t hw = L::pack_hi(d[2 * pr], d[2 * pr + 1]);
                                dst[4 * pr] = hw;
                                if constexpr (L::split) dst[abPlane + 4 * pr] = L::pack_lo(d[2 * pr], d[2 * pr + 1], hw);
                            }
                        }
                        continue;
                    }
#pragma unroll
                    for (int pr = 0; pr < 2; pr++) {
                        const int r = mt * 16 + 4 * grp + 2 * pr;
                        if (r < FG.MROWS) {
                            const int rt = r / FG.RIE, il2 = (r - rt * FG.RIE) >> 1;
                            const int at = (rt * IQ2 + il2) * 4 + xc;
                            const uint32_t hw = L::pack_hi(d[2 * pr], d[2 * pr + 1]);
                            ((uint32_t*)(Ab + (size_t)h * abPlane))[at] = hw;
                            if constexpr (L::split)
                                ((uint32_t*)(Ab + (size_t)(2 + h) * abPlane))[at] = L::pack_lo(d[2 * pr], d[2 * pr + 1], hw);
                        }
                    }
                }
            }
            if (kx + 1 < KH) pass_a_ops(kx + 1, pbh, pbl);
        } else {
            // ---- pass A (fp32 sums): one thread per (rt, il pair, cos|sin); the two rows'
            // results are rounded once and stored as packed pairs for pass B
            for (int e = tid; e < RTe * IQ2 * 2; e += kNTL) {
                const int h = e & 1;
                const int q = e >> 1;
                const int rt = q / IQ2, il2 = q - rt * IQ2;
                float cf[N];
#pragma unroll
                for (int a = 0; a < N; a++) cf[a] = p.passA[(kx * N + a) * 2 + h];
                float o[2][4];
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    const int il = 2 * il2 + r;
#pragma unroll
                    for (int xc = 0; xc < 4; xc++) o[r][xc] = 0.f;
                    if (rt < RT && il < RI) {
                        const float* row = Vt + (rt * RI + il) * RXp;
                        if constexpr (S > 0) {
                            constexpr int RXc = 3 * S + N;
                            float v[RXc];
#pragma unroll
                            for (int k = 0; k < RXc; k++) v[k] = row[k];
#pragma unroll
                            for (int xc = 0; xc < 4; xc++) {
                                float acc_a = 0.f;
#pragma unroll
                                for (int a = 0; a < N; a++) acc_a = fmaf(cf[a], v[xc * S + a], acc_a);
                                o[r][xc] = acc_a;
                            }
                        } else {
#pragma unroll
                            for (int xc = 0; xc < 4; xc++) {
                                float acc_a = 0.f;
#pragma unroll
                                for (int a = 0; a < N; a++) acc_a = fmaf(cf[a], row[xc * s + a], acc_a);
                                o[r][xc] = acc_a;
                            }
                        }
                    }
                }
                uint4 wh, wl;
                wh.x = L::pack_hi(o[0][0], o[1][0]);
                wh.y = L::pack_hi(o[0][1], o[1][1]);
                wh.z = L::pack_hi(o[0][2], o[1][2]);
                wh.w = L::pack_hi(o[0][3], o[1][3]);
                const size_t at = (size_t)(rt * IQ2 + il2) * 8;
                *(uint4*)(Ab + (size_t)h * abPlane + at) = wh;
                if constexpr (L::split) {
                    wl.x = L::pack_lo(o[0][0], o[1][0], wh.x);
                    wl.y = L::pack_lo(o[0][1], o[1][1], wh.y);
                    wl.z = L::pack_lo(o[0][2], o[1][2], wh.z);
                    wl.w = L::pack_lo(o[0][3], o[1][3], wh.w);
                    *(uint4*)(Ab + (size_t)(2 + h) * abPlane + at) = wl;
                }
            }
        }
        __syncthreads();
        // bin weights of this kx.  The planes kx = 0 and kx = n/2 are their own Hermitian
        // mirrors (|F(-k)| = |F(k)|): only the ki slots [0, n/2] are visited there, with the
        // skipped mirrors folded into the table's weights.
        const bool mirror = PLANE == 2 || (PLANE == 0 && (kx == 0 || 2 * kx == N));
        const float4* wk = p.wts + (size_t)kx * N * 16;
        if constexpr (!FIX && L::split)
            for (int e = tid; e < N * 16; e += kNTL) Wl[e] = wk[e];
        // ---- pass B: complex DFT along il for a pair of rows per wave; the outputs of the
        // two rows are rounded and written as packed pairs along t
        {
            const int il0 = (col >> 2) * s + b0, xc = col & 3;
            const uint32_t* abh = (const uint32_t*)(Ab + (size_t)half * abPlane) + xc;
            const uint32_t* abl = (const uint32_t*)(Ab + (size_t)(2 + half) * abPlane) + xc;
            for (int pi = wave; pi < RTe / 2; pi += NW) {
                f4 dre[2], dim[2];
#pragma unroll
                for (int r = 0; r < 2; r++) {
                    const int rowoff = (2 * pi + r) * IQ2 * 4;
                    uint32_t wh[4], wl[4];
                    load8_ab<S>(abh + rowoff, il0, wh);
                    if constexpr (L::split) load8_ab<S>(abl + rowoff, il0, wl);
                    const vec vh = vec_from_words<PREC>(wh);
                    const vec vl = L::split ? vec_from_words<PREC>(wl) : vh;
                    dre[r] = contract<PREC>(are_h, are_l, vh, vl, f4{0.f, 0.f, 0.f, 0.f});
                    dim[r] = contract<PREC>(aim_h, aim_l, vh, vl, f4{0.f, 0.f, 0.f, 0.f});
                }
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int u = 4 * grp + j;
                    if (u < N) {
                        uint32_t* gre = (uint32_t*)(Gh + (u * 16 + col) * gRow) + pi;
                        uint32_t* gim = (uint32_t*)(Gh + gPlane + (u * 16 + col) * gRow) + pi;
                        const uint32_t rh = L::pack_hi(dre[0][j], dre[1][j]);
                        const uint32_t ih = L::pack_hi(dim[0][j], dim[1][j]);
                        *gre = rh;
                        *gim = ih;
                        if constexpr (L::split) {
                            uint32_t* lre = (uint32_t*)(Gl + (u * 16 + col) * gRow) + pi;
                            uint32_t* lim = (uint32_t*)(Gl + gPlane + (u * 16 + col) * gRow) + pi;
                            *lre = L::pack_lo(dre[0][j], dre[1][j], rh);
                            *lim = L::pack_lo(dim[0][j], dim[1][j], ih);
                        }
                    }
                }
            }
        }
        __syncthreads();
        // ---- pass C along t and the projection.  Split form: the product is taken transposed
        // (windows x bins), so a lane holds one bin kt = col of four windows and needs one weight
        // triple per ki, summed in fp32.  FP16: the product puts the bins in the rows and the 16
        // windows of the t-centre in the columns, so a lane holds bins 4 grp .. 4 grp + 3 of window
        // col; the magnitudes of two ki slots, rounded to bf16, form the B operand of one bf16
        // product against the weights (rows m: their hi parts, rows 4 + m: their lo parts),
        // accumulated in fp32 over all slots and kx.  Slot u+1 is contracted before the epilogue
        // of slot u so the matrix cores and the VALU overlap.  The two wave halves split the ki
        // slots to visit, [0, n) or [0, n/2] on a mirror plane.
        const int ua = (wave >> 3) ? (mirror ? (N / 2 + 2) / 2 : UH) : 0;
        const uint32_t* wpk = p.wproj + ((size_t)kx * N * 64 + lane) * 2;  // FP16: this lane's words of slot 0
#pragma unroll
        for (int c = 0; c < CTW; c++) {
            const int tc = wtc + 8 * c;
            if (tc >= CT) break;
            const int ts = tc * s + b0;
            const uint16_t* ghb = Gh + half * gPlane + col * gRow;
            const uint16_t* glb = Gl + half * gPlane + col * gRow;
            auto run = [&](auto odd, auto count) {
                constexpr bool ODD = decltype(odd)::value;
                constexpr int CNT = decltype(count)::value;
                auto contract_c = [&](int u, f4& dre, f4& dim) {
                    uint32_t wh[4], wl[4];
                    load8_u16<ODD>(ghb + u * 16 * gRow, ts, wh);
                    if constexpr (L::split) load8_u16<ODD>(glb + u * 16 * gRow, ts, wl);
                    const vec vh = vec_from_words<PREC>(wh);
                    const vec vl = L::split ? vec_from_words<PREC>(wl) : vh;
                    // split form: the wave issuing its six products goes first, so the matrix
                    // cores are fed while the other waves run their epilogues (about 1 % faster;
                    // the single-product FP16 form is not helped)
                    if constexpr (L::split) __builtin_amdgcn_s_setprio(1);
                    dre = contract<PREC>(vh, vl, are_h, are_l, f4{0.f, 0.f, 0.f, 0.f});
                    dim = contract<PREC>(vh, vl, aim_h, aim_l, f4{0.f, 0.f, 0.f, 0.f});
                    if constexpr (L::split) __builtin_amdgcn_s_setprio(0);
                };
                // weights of bin (kt = col, ki = u): from LDS, or on the fixed tile straight
                // from the global table, fetched one slot ahead
                auto weight = [&](int u) { return FIX ? wk[u * 16 + col] : Wl[u * 16 + col]; };
                f4 dre, dim;
                float4 w = weight(ua);
                contract_c(ua, dre, dim);
#pragma unroll
                for (int uu = 0; uu < CNT; uu++) {
                    const int u = ua + uu;
                    f4 nre, nim;
                    float4 wn;
                    if (uu + 1 < CNT) {
                        wn = weight(u + 1);
                        contract_c(u + 1, nre, nim);
                    }
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const float m = __builtin_amdgcn_sqrtf(fmaf(dre[j], dre[j], dim[j] * dim[j]));
                        acc[c][j][0] = fmaf(w.x, m, acc[c][j][0]);
                        acc[c][j][1] = fmaf(w.y, m, acc[c][j][1]);
                        acc[c][j][2] = fmaf(w.z, m, acc[c][j][2]);
                    }
                    if (uu + 1 < CNT) {
                        dre = nre;
                        dim = nim;
                        w = wn;
                    }
                }
            };
            auto run16 = [&](auto odd, auto count) {
                constexpr bool ODD = decltype(odd)::value;
                constexpr int CNT = decltype(count)::value;
                auto contract_c = [&](int u, f4& dre, f4& dim) {
                    uint32_t wh[4];
                    load8_u16<ODD>(ghb + u * 16 * gRow, ts, wh);
                    const vec vh = vec_from_words<PREC>(wh);
                    dre = contract<PREC>(are_h, are_l, vh, vh, f4{0.f, 0.f, 0.f, 0.f});
                    dim = contract<PREC>(aim_h, aim_l, vh, vh, f4{0.f, 0.f, 0.f, 0.f});
                };
                auto weight = [&](int u) { return *(const uint2*)(wpk + (size_t)u * 128); };
                f4 dre, dim;
                // wp[q]: weights of the slot at position q of the current pair
                uint2 wp[2] = {weight(ua), make_uint2(0u, 0u)};
                uint32_t mag[4];
                contract_c(ua, dre, dim);
#pragma unroll
                for (int uu = 0; uu < CNT; uu++) {
                    const int u = ua + uu;
                    f4 nre, nim;
                    uint2 wn;
                    if (uu + 1 < CNT) {
                        wn = weight(u + 1);
                        contract_c(u + 1, nre, nim);
                    }
                    float m[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) m[j] = __builtin_amdgcn_sqrtf(fmaf(dre[j], dre[j], dim[j] * dim[j]));
                    const int q = 2 * (uu & 1);
                    mag[q] = bf16_pair(m[0], m[1]);
                    mag[q + 1] = bf16_pair(m[2], m[3]);
                    if ((uu & 1) || uu + 1 == CNT) {
                        // a lone last slot pairs with zero weights and magnitudes
                        if (!(uu & 1)) {
                            mag[2] = mag[3] = 0u;
                            wp[1] = make_uint2(0u, 0u);
                        }
                        typedef uint32_t u4w __attribute__((ext_vector_type(4)));
                        pacc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf8, u4w{wp[0].x, wp[0].y, wp[1].x, wp[1].y}),
                            __builtin_bit_cast(bf8, u4w{mag[0], mag[1], mag[2], mag[3]}), pacc[c], 0, 0, 0);
                    }
                    if (uu + 1 < CNT) {
                        dre = nre;
                        dim = nim;
                        wp[(uu + 1) & 1] = wn;
                    }
                }
            };
            // slot counts are compile-time per case so each loop stays fully unrolled
            auto run_form = [&](auto odd, auto count) {
                if constexpr (L::split) run(odd, count);
                else run16(odd, count);
            };
            auto run_slots = [&](auto odd) {
                if (PLANE == 1 || !mirror) run_form(odd, std::integral_constant<int, UH>{});
                else if (wave >> 3) run_form(odd, std::integral_constant<int, (N / 2 + 1) / 2>{});
                else run_form(odd, std::integral_constant<int, (N / 2 + 2) / 2>{});
            };
            // the window start's parity is the same for the whole wave
            if ((S > 0 && (S & 1) == 0) || (ts & 1) == 0) run_slots(std::false_type{});
            else run_slots(std::true_type{});
        }
    };
    if constexpr (lowp_prefetch<N, S, PREC, CTW, FIX>()) {
        kstep(0, std::integral_constant<int, 2>{});
        for (int kx = 1; kx + 1 < KH; kx++) kstep(kx, std::integral_constant<int, 1>{});
        // the last kx step reads the staged planes in pass A only; the next region's loads
        // are in flight meanwhile and are stored after the step
        constexpr int NPF = lowp_prefetch_planes<N, S, PREC, CTW, FIX>();
        float pf[NPF];
        if (has_next) {
            const LowpParams& q = pn ? *pn : p;
            const int64_t nx = next % q.tilesX, ni = (next / q.tilesX) % q.tilesI, nt = next / (q.tilesX * q.tilesI);
            stage_issue<kNTL, NPF>(pf, q.V, q.T, q.IL, q.XL, nt * CT * s - N / 2, ni * 4 * s - N / 2,
                                   nx * 4 * s - N / 2, RT, RI, RX);
        }
        kstep(KH - 1, std::integral_constant<int, 2>{});
        if (has_next) {
            const StageLane sl = stage_lane<kNTL>(RI, RX);
            if (sl.g < sl.G) {
#pragma unroll
                for (int u = 0; u < NPF; u++) {
                    const int rt = sl.g + u * sl.G;
                    if (rt < RT && sl.act) {
                        const int at = (rt * FG.RIE + sl.ri) * FG.XP + sl.rx;
                        const uint16_t h = L::hi(pf[u]);
                        Vb[at] = h;
                        if constexpr (L::split) Vb[FG.VP + at] = L::lo(pf[u], h);
                    }
                }
            }
        }
    } else {
        kstep(0, std::integral_constant<int, 2>{});
        for (int kx = 1; kx + 1 < KH; kx++) kstep(kx, std::integral_constant<int, 1>{});
        kstep(KH - 1, std::integral_constant<int, 2>{});
    }

    const int64_t G = p.Tg * p.ILg * p.XLg;
    float* red = (float*)Gh;  // [CTW][8][16][3]
    if constexpr (!L::split) {
        // plane m of window col: row m (lane group 0) plus row 4 + m (lane group 1), then the two
        // halves of the ki slots through LDS
        __syncthreads();
        float e[CTW][3];
#pragma unroll
        for (int c = 0; c < CTW; c++)
#pragma unroll
            for (int m = 0; m < 3; m++) e[c][m] = pacc[c][m] + __shfl_down(pacc[c][m], 16);
        if (NW > 8 && wave >= 8 && lane < 16) {
#pragma unroll
            for (int c = 0; c < CTW; c++)
#pragma unroll
                for (int m = 0; m < 3; m++) red[((c * 8 + wtc) * 16 + col) * 3 + m] = e[c][m];
        }
        __syncthreads();
        if (wave < 8 && lane < 16) {
#pragma unroll
            for (int c = 0; c < CTW; c++) {
                const int tc = wtc + 8 * c;
                const int64_t gt = tt * CT + tc, gi = ti * 4 + (col >> 2), gx = tx * 4 + (col & 3);
                if (tc < CT && gt < p.Tg && gi < p.ILg && gx < p.XLg) {
                    const int64_t at = (gt * p.ILg + gi) * p.XLg + gx;
#pragma unroll
                    for (int m = 0; m < 3; m++)
                        p.E[m * G + at] = e[c][m] + (NW > 8 ? red[((c * 8 + wtc) * 16 + col) * 3 + m] : 0.f);
                }
            }
        }
        return;
    }
    // reduce over the 16 bins of a lane group, then over the two halves of the ki slots
    // through LDS
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CTW; c++)
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int m = 0; m < 3; m++) {
                acc[c][j][m] = row_sum16(acc[c][j][m]);
            }
    if (NW > 8 && wave >= 8 && col == 0) {
#pragma unroll
        for (int c = 0; c < CTW; c++)
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
                for (int m = 0; m < 3; m++) red[((c * 8 + wtc) * 16 + 4 * grp + j) * 3 + m] = acc[c][j][m];
    }
    __syncthreads();
    if (wave < 8 && col == 0) {
#pragma unroll
        for (int c = 0; c < CTW; c++) {
            const int tc = wtc + 8 * c;
            const int64_t gt = tt * CT + tc, gi = ti * 4 + grp;
            if (tc < CT && gt < p.Tg && gi < p.ILg) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int64_t gx = tx * 4 + j;
                    if (gx < p.XLg) {
                        const int64_t at = (gt * p.ILg + gi) * p.XLg + gx;
#pragma unroll
                        for (int m = 0; m < 3; m++)
                            p.E[m * G + at] =
                                acc[c][j][m] + (NW > 8 ? red[((c * 8 + wtc) * 16 + 4 * grp + j) * 3 + m] : 0.f);
                    }
                }
            }
        }
    }
}

template <int N, int S, int PREC, int CTW, bool FIX>
__global__ __launch_bounds__(kNTL) void k_project_lowp(LowpParams p) {
    extern __shared__ float lds[];
    if constexpr (lowp_prefetch<N, S, PREC, CTW, FIX>()) {
        // persistent: workgroup b of XCD b % 8 walks that XCD's contiguous share of the tiles
        const int64_t per = (p.ntiles + 7) / 8, stride = gridDim.x / 8;
        const int64_t lo = (int64_t)(blockIdx.x % 8) * per, hi = lo + per < p.ntiles ? lo + per : p.ntiles;
        for (int64_t g = lo + blockIdx.x / 8; g < hi; g += stride)
            project_tile_lowp<N, S, PREC, CTW, FIX>(p, g, lds, g != lo + blockIdx.x / 8, g + stride < hi,
                                                    g + stride);
        return;
    }
    const int64_t tile = xcd_block(p.ntiles);
    if (tile >= p.ntiles) return;
    project_tile_lowp<N, S, PREC, CTW, FIX>(p, tile, lds);
}

template <int N, int S, int PREC, int CTW, bool FIX>
__global__ __launch_bounds__(kNTL) void k_project_lowp_batch(const LowpParams* __restrict__ items,
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
    if constexpr (lowp_prefetch<N, S, PREC, CTW, FIX>()) {
        // each next region (possibly of the next member) is fetched during the current tile
        int64_t g = lo + local;
        if (g >= hi) return;
        int a = item_of(g);
        for (bool staged = false; g < hi; g += stride, staged = true) {
            const bool more = g + stride < hi;
            const int an = more ? item_of(g + stride) : a;
            project_tile_lowp<N, S, PREC, CTW, FIX>(items[a], g - prefix[a], lds, staged, more,
                                                    g + stride - prefix[an], &items[an]);
            a = an;
        }
        return;
    }
    for (int64_t g = lo + local; g < hi; g += stride) {
        const int a = item_of(g);
        __syncthreads();
        project_tile_lowp<N, S, PREC, CTW, FIX>(items[a], g - prefix[a], lds);
    }
}

static int lowp_ctw(int n) { return n == 4 ? 2 : 1; }

// Whether a launch takes the fixed-tile kernel: a stride built at compile time for this n
// (the dispatch below) and the full tile depth.
static bool lowp_fixed(int n, int s, int CT) {
    const bool compiled = s == 1 || (s == 2 && n > 4) || (s == 3 && n > 6);
    return compiled && CT == 8 * lowp_ctw(n);
}

static size_t lowp_lds_bytes(int n, int s, int CT, bool split, LowpParams* p) {
    p->RT = (CT - 1) * s + n;
    p->RTp = lowp_rtp(CT, s);
    p->RI = 3 * s + n;
    p->RX = 3 * s + n;
    p->RXp = p->RX | 1;
    p->IQ2 = ab_iq2(s);
    const size_t RTe = (size_t)((p->RT + 1) & ~1);
    const size_t ab = (split ? 4 : 2) * (size_t)plane_pitch16((int)RTe * p->IQ2 * 8);
    const size_t plane = (size_t)n * 16 * p->RTp;
    const size_t g = std::max<size_t>((plane + plane_pitch16((int)plane)) * (split ? 2 : 1), 8 * 16 * 3 * 2 * 2);
    if (lowp_fixed(n, s, CT)) {
        // 16-bit staged planes, no weight staging
        const FixGeom fg = fix_geom(n, s, CT);
        return 2 * ((split ? 2 : 1) * (size_t)fg.VP + ab + g);
    }
    const size_t f32 = ((size_t)p->RT * p->RI * p->RXp + 3) & ~(size_t)3;
    return sizeof(float) * f32 + 2 * (ab + g) + sizeof(float) * 4 * 16 * n;
}

static constexpr size_t kLdsMaxL = 160 * 1024;

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
    p.wts = (const float4*)tb->wts_nat_h;
    p.wproj = tb->wproj;
    p.pa_ops = nullptr;
    if (lowp_fixed(n, s, CT)) {
        sal_status st = get_pass_a_ops(nullptr, n, s, tb->window, &p.pa_ops);  // the tables are uploaded by now
        if (st) return st;
    }
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

template <int N, int S, int PREC, int CTW, bool FIX>
static sal_status launch_lowp_k(const LowpParams& p, size_t lds, hipStream_t stream) {
    static std::atomic<uint64_t> attr{0};
    sal_status st = lds_limit_once((const void*)k_project_lowp<N, S, PREC, CTW, FIX>, (int)kLdsMaxL, attr,
                                   "hipFuncSetAttribute(project lowp)");
    if (st) return st;
    int64_t grid = xcd_grid(p.ntiles);
    if constexpr (lowp_prefetch<N, S, PREC, CTW, FIX>()) {
        // as many workgroups as are resident at once, a multiple of 8 (one share per XCD)
        int dev = 0, cus = 0, per_cu = 0;
        if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice"))) return st;
        if ((st = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                            "hipDeviceGetAttribute")))
            return st;
        if ((st = check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &per_cu, k_project_lowp<N, S, PREC, CTW, FIX>, kNTL, lds),
                            "hipOccupancyMaxActiveBlocksPerMultiprocessor")))
            return st;
        grid = std::min<int64_t>(grid, std::max<int64_t>(8, (int64_t)cus * std::max(per_cu, 1) / 8 * 8));
    }
    if (!wide_grid_fits(grid, kNTL)) return fail(SAL_ERR_SHAPE, "volume too large for one launch");
    hipLaunchKernelGGL((k_project_lowp<N, S, PREC, CTW, FIX>), wide_grid(grid, kNTL), dim3(kNTL), lds, stream, p);
    return check_hip(hipGetLastError(), "launch k_project_lowp");
}

// the full-depth tile of a compile-time stride takes the kernel with fixed extents
template <int N, int S, int PREC, int CTW>
static constexpr bool fixed_tile(int CT) { return S > 0 && CT == 8 * CTW; }

template <int N, int S, int PREC, int CTW>
static sal_status launch_lowp(const LowpParams& p, size_t lds, hipStream_t stream) {
    if constexpr (S > 0)
        if (fixed_tile<N, S, PREC, CTW>(p.CT)) return launch_lowp_k<N, S, PREC, CTW, true>(p, lds, stream);
    return launch_lowp_k<N, S, PREC, CTW, false>(p, lds, stream);
}

template <int N, int S, int PREC, int CTW>
static sal_status launch_lowp_batch(int CT, const void* items, const int64_t* prefix, int nitems, int64_t total,
                                   size_t lds, int grid, hipStream_t stream) {
    // the LDS attribute was set by project_lowp_batch_occupancy(), outside any stream capture
    if constexpr (S > 0)
        if (fixed_tile<N, S, PREC, CTW>(CT)) {
            hipLaunchKernelGGL((k_project_lowp_batch<N, S, PREC, CTW, true>), dim3((unsigned)grid), dim3(kNTL), lds,
                               stream, (const LowpParams*)items, prefix, nitems, total);
            return check_hip(hipGetLastError(), "launch k_project_lowp_batch");
        }
    hipLaunchKernelGGL((k_project_lowp_batch<N, S, PREC, CTW, false>), dim3((unsigned)grid), dim3(kNTL), lds, stream,
                       (const LowpParams*)items, prefix, nitems, total);
    return check_hip(hipGetLastError(), "launch k_project_lowp_batch");
}

template <int N, int S, int PREC, int CTW, bool FIX>
static sal_status lowp_occupancy_k(size_t lds, int* per_cu) {
    sal_status st =
        set_lds_attr_l(k_project_lowp_batch<N, S, PREC, CTW, FIX>, "hipFuncSetAttribute(project lowp batch)");
    if (st) return st;
    return check_hip(
        hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_project_lowp_batch<N, S, PREC, CTW, FIX>, kNTL, lds),
        "hipOccupancyMaxActiveBlocksPerMultiprocessor");
}

template <int N, int S, int PREC, int CTW>
static sal_status lowp_occupancy(int CT, size_t lds, int* per_cu) {
    if constexpr (S > 0)
        if (fixed_tile<N, S, PREC, CTW>(CT)) return lowp_occupancy_k<N, S, PREC, CTW, true>(lds, per_cu);
    return lowp_occupancy_k<N, S, PREC, CTW, false>(lds, per_cu);
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

sal_status project_lowp_batch(int n, int s, int precision, int CT, const void* items, const int64_t* prefix,
                              int nitems, int64_t total, size_t lds, int grid, hipStream_t stream) {
#define CALL(NN, SS, PP, CC) launch_lowp_batch<NN, SS, PP, CC>(CT, items, prefix, nitems, total, lds, grid, stream)
    SAL_LP_DISPATCH
#undef CALL
}

sal_status project_lowp_batch_occupancy(int n, int s, int precision, int CT, size_t lds, int* per_cu) {
#define CALL(NN, SS, PP, CC) lowp_occupancy<NN, SS, PP, CC>(CT, lds, per_cu)
    SAL_LP_DISPATCH
#undef CALL
}

}  // namespace sal
