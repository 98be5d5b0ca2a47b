// sal_aux.h -- launchers of the bandwidth-bound kernels (not part of the ABI).
#pragma once

#include <vector>

#include "sal_internal.h"

namespace sal {

constexpr int kStats = 11;       // G00 G01 G02 G11 G12 G22 p0 p1 p2 sum(D^2) count
constexpr int kFuseParts = 256;  // fixed number of partial-sum blocks (deterministic reduction)

// Stencil in grid units, passed by value as a kernel argument.  With per-plane stencils
// (planes = 1) the offsets are the union of the three planes' stencils: offset k belongs to
// plane m's stencil when bit m of member[k] is set, with weight wp[k][m] there.
struct DcsStencil {
    int q;
    int literal;
    int reach[3];  // largest |offset| per axis, in grid units
    int symmetric; // every offset has its negation in the stencil: mirror[] pairs them one to one
                   // (with per-plane stencils, a pair also shares its planes)
    int planes;    // 0: every offset on all three planes with weight w[k]; 1: member / wp
    int o[SAL_MAX_STENCIL][3];
    float w[SAL_MAX_STENCIL];
    int mirror[SAL_MAX_STENCIL];  // o[mirror[k]] == -o[k] (symmetric stencils only)
    float wp[SAL_MAX_STENCIL][3];
    unsigned char member[SAL_MAX_STENCIL];
};

// Weight groups of the fusion (re-adaptation every `sections` inline sections of the grid):
// group k holds the inline planes [k N, k N + N) of the grid; N = 0 is one group.
inline int64_t fuse_groups(int64_t sections, int64_t ILg) {
    return sections > 0 ? (ILg + sections - 1) / sections : 1;
}

// Resolves a stencil (validation, Gaussian default weights) into grid units.
sal_status make_stencil(const sal_stencil* st, int s, DcsStencil* out);

sal_status launch_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int window,
                                const int32_t* centers, int64_t cnt, float* F, hipStream_t stream);
sal_status launch_dcs(const float* E, float* S, int64_t Tg, int64_t ILg, int64_t XLg, const DcsStencil& st,
                      hipStream_t stream);
// gE from E and R = gS_m / Q (the output of launch_fuse_adjoint).
sal_status launch_dcs_adjoint(const float* E, const float* R, float* gE, int64_t Tg, int64_t ILg, int64_t XLg,
                              const DcsStencil& st, hipStream_t stream);
// Workspace bytes of the fusion over K weight groups (ADAPT_LS partial sums and statistics).
size_t fuse_workspace_bytes(int64_t K);
// W: K x 4 doubles (sal_fuse's W_out).
sal_status launch_fuse(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion& f, const float* D,
                       const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int s, double* W, float* S, double* ws,
                       hipStream_t stream);
size_t fuse_adjoint_workspace_bytes(int64_t K);
// The sequential rules (LMS, NLMS, RLS).
inline bool fuse_sequential(int mode) {
    return mode == SAL_FUSE_LMS || mode == SAL_FUSE_NLMS || mode == SAL_FUSE_RLS;
}
// Workspace of the sequential rules: the index list of the masked points and the block counts.
size_t seq_workspace_bytes(int64_t G, int64_t K);
// W: K x 4 doubles; err2: K x cap floats or nullptr; count: K int64 or nullptr.
sal_status launch_seq_adapt(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion& f,
                            const float* D, const uint8_t* mask, double* W, float* err2, int64_t cap, int64_t* count,
                            void* ws, hipStream_t stream);
// S(v) = sum_m W_m S_m(g(v)) with the weights of each row's group (W: K x 4).
sal_status launch_combine(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, int64_t sections, int64_t T,
                          int64_t IL, int64_t XL, int s, const double* W, float* S, hipStream_t stream);
// Writes R_m(g) = gS_m(g) / Q(g), the fusion adjoint divided by the number Q(g) of stencil
// neighbours of g inside the grid (0 where Q(g) = 0): the per-point factor of every term of
// the center-surround adjoint.
sal_status launch_fuse_adjoint(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion& f,
                               const float* D, const uint8_t* mask, const double* W, const float* gS, int64_t T,
                               int64_t IL, int64_t XL, int s, const DcsStencil& ds, float* cell, double* ws, float* R,
                               hipStream_t stream);
sal_status launch_project_lowp(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int precision,
                               const Tables* tb, float* E, hipStream_t stream);
sal_status launch_project_fp32(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int feature,
                               const Tables* tb, float* E, hipStream_t stream);

// Batched (persistent) feature launches over many volumes of one window class.  The
// per-volume kernel parameters are opaque blocks of *_param_bytes() bytes.
void project_fp32_ct_candidates(int n, int s, std::vector<int>* out);
void project_lowp_ct_candidates(int n, int s, int precision, std::vector<int>* out);
size_t project_fp32_param_bytes();
size_t project_lowp_param_bytes();
sal_status project_fp32_params(int n, int s, int CT, const float* V, int64_t T, int64_t IL, int64_t XL,
                               const Tables* tb, float* E, void* out, int64_t* ntiles, size_t* lds);
sal_status project_lowp_params(int n, int s, int precision, int CT, const float* V, int64_t T, int64_t IL,
                               int64_t XL, const Tables* tb, float* E, void* out, int64_t* ntiles, size_t* lds);
sal_status project_fp32_batch(int n, int s, const void* items, const int64_t* prefix, int nitems, int64_t total,
                              size_t lds, int grid, hipStream_t stream);
sal_status project_lowp_batch(int n, int s, int precision, int CT, const void* items, const int64_t* prefix,
                              int nitems, int64_t total, size_t lds, int grid, hipStream_t stream);
sal_status project_fp32_batch_occupancy(int n, int s, size_t lds, int* per_cu);
int64_t project_fp32_batch_grid(int n, int64_t total, int64_t resident);
sal_status project_lowp_batch_occupancy(int n, int s, int precision, int CT, size_t lds, int* per_cu);

}  // namespace sal
