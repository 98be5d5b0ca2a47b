// sal_passb.h -- the il-DFT (pass B) of an n = 8 window with two il-centres per matrix
// product (shared by the feature and adjoint kernels; not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace sal {

// Pass B of an n = 8 window on the 16x16x4 fp32 matrix cores, from the pass-A output Ab
// ([2][RT][RI][4]: real and imaginary planes abStride apart, xl centre innermost) into Gb
// ([2][8][RT][16]: signed ki slots in natural order, planes gbStride apart, window column
// il-centre * 4 + xc innermost).
//
// The 8 packed DFT rows (cos 0, cos n/2, cos 1, sin 1, ..., sin 3) fill half of the 16-row
// A operand, so rows 8..15 hold the next il-centre: amatP is the banded operand of a centre
// pair (row r of centre r >> 3 at K slot k takes sample k - (r >> 3) s; 12 samples cover
// both centres for s <= 4), the columns are (t row parity, centre pair, xc), and one product
// covers two t rows.  The t-row pairs are dealt to the waves `wave` of `nwaves`; every lane
// stores its four rows (no divergent epilogue).  PRIO raises the issue priority while a wave
// issues its products.
template <bool PRIO>
__device__ __forceinline__ void pass_b_pair8(const float* __restrict__ Ab, int abStride, float* __restrict__ Gb,
                                             int gbStride, int RT, int RI, int s, const float (&amatP)[3],
                                             int wave, int nwaves, int col, int grp) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    constexpr int N = 8;
    const int pp = (col >> 2) & 1, xc = col & 3;
    // this lane's sample of step ks is 2 pp s + 4 ks + grp; in the last step the samples past
    // the row (they meet zero coefficients) read its last one
    const int ib = (2 * pp * s + grp) * 4 + xc;
    const int i2 = min(2 * pp * s + 8 + grp, RI - 1) * 4 + xc;
    const int cw = (2 * pp + (grp >> 1)) * 4 + xc;  // window column of this lane's output rows
    for (int it = wave; it < (RT + 1) / 2; it += nwaves) {
        const int rt = 2 * it + (col >> 3);
        const float* ar = Ab + (rt < RT ? rt : RT - 1) * RI * 4;  // a row past the tile is dropped
        float br[3], bi[3];
#pragma unroll
        for (int ks = 0; ks < 3; ks++) {
            const int io = ks < 2 ? ib + 16 * ks : i2;
            br[ks] = ar[io];
            bi[ks] = ar[abStride + io];
        }
        f4v dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < 3; ks++) {
            dr = __builtin_amdgcn_mfma_f32_16x16x4f32(amatP[ks], br[ks], dr, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x4f32(amatP[ks], bi[ks], di, 0, 0, 0);
        }
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        // a lane's rows are packed rows 4 (grp & 1) + j of centre 2 pp + (grp >> 1): the pairs
        // 2q, 2q + 1 are (cos q, sin q), or (cos 0, cos n/2) for q = 0
        if (rt < RT) {
#pragma unroll
            for (int pr = 0; pr < 2; pr++) {
                const int q = 2 * (grp & 1) + pr;
                const bool sp = q == 0;
                const float Ca = dr[2 * pr], Sb = dr[2 * pr + 1], Cai = di[2 * pr], Sbi = di[2 * pr + 1];
                const int u1 = sp ? 0 : q, u2 = sp ? N / 2 : N - q;
                Gb[(u1 * RT + rt) * 16 + cw] = sp ? Ca : Ca + Sbi;               // +q
                Gb[gbStride + (u1 * RT + rt) * 16 + cw] = sp ? Cai : Cai - Sb;
                Gb[(u2 * RT + rt) * 16 + cw] = sp ? Sb : Ca - Sbi;               // -q
                Gb[gbStride + (u2 * RT + rt) * 16 + cw] = sp ? Sbi : Cai + Sb;
            }
        }
    }
}

}  // namespace sal
