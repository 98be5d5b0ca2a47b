/*
 * sal.h -- C ABI of libsal, the MI355X (gfx950) implementation of the seismic
 * saliency hot path of Shafiq, Long, Di, AlRegib, "A novel attention model
 * for salient structure detection in seismic volumes" (ACI 2021,
 * arXiv 2201.06174), Section 2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Volume V: float32 [T][IL][XL], XL fastest (time, inline, crossline; the
 *   paper's T x X x Y volume, Sec. 2 first paragraph).
 * Grid: window centres at g*s on each axis, Tg = ceil(T/s) etc.  Feature and
 *   saliency maps are planar float32 [3][Tg][ILg][XLg] with plane order
 *   (t, x = crossline = XL axis, y = inline = IL axis), the order of Eq. 1/4.
 * Window: side n (even), samples c-n/2 .. c+n/2-1 around the centre c, taper
 *   periodic Hann sin^2(pi a/n) or flat; indices outside the volume are
 *   reflected half-sample symmetrically (-1 -> 0, N -> N-1), so every axis
 *   must hold at least n/2 voxels.
 * Memory: every pointer named in a call is caller-owned; device pointers must
 *   be device memory of the current HIP device, host pointers are read during
 *   the call only.  No call keeps a pointer past its return (plans excepted,
 *   see sal_plan_create).
 * Execution: all device work is enqueued on the given stream, and no call but
 *   sal_plan_create allocates device memory.  The constant tables the kernels read live in
 *   static device memory and are uploaded once per device: by sal_init(), or
 *   else by the first call on that device that needs them, which then blocks
 *   the host until the upload is done.  After sal_init() on a device no call
 *   synchronises the host with it (sal_plan_create and sal_plan_status
 *   excepted, as documented there), so every call can be captured in a HIP
 *   graph; a first call inside a capture before sal_init() returns
 *   SAL_ERR_STATE without enqueueing anything.  Results are bitwise identical
 *   run to run.
 * Errors: every call validates its arguments on the host before launching
 *   anything and returns a sal_status; sal_last_error() then gives a message
 *   (thread-local).  NaN/Inf inputs propagate without a check.
 */
#ifndef SAL_H
#define SAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* sal_stream; /* a hipStream_t; NULL is the null stream */

typedef enum {
    SAL_OK = 0,
    SAL_ERR_ARG = 1,         /* bad pointer, size, or option value */
    SAL_ERR_SHAPE = 2,       /* inconsistent shapes (e.g. an axis shorter than n/2), or more work
                                than one launch holds (about 2^47 work-items: far beyond HBM) */
    SAL_ERR_UNSUPPORTED = 3, /* valid for the method, not built into this library (e.g. n = 10) */
    SAL_ERR_NOMEM = 4,       /* workspace too small or allocation failed */
    SAL_ERR_DEVICE = 5,      /* a HIP runtime call failed */
    SAL_ERR_STATE = 6        /* the call needs sal_init() on this device first (a first call inside a
                                stream capture) */
} sal_status;

typedef enum { SAL_WINDOW_HANN = 0, SAL_WINDOW_RECT = 1 } sal_window;

/* Arithmetic of the windowed-DFT contractions.  FP32: fp32 matrix-core
 * products; SPLIT_BF16: each operand split into hi + lo bfloat16 parts, three
 * bf16 products (hi*hi + hi*lo + lo*hi) accumulated in fp32; FP16: one fp16
 * product accumulated in fp32.  Every other step runs in fp32 (fp64 for the
 * fusion statistics). */
typedef enum { SAL_PREC_FP32 = 0, SAL_PREC_SPLIT_BF16 = 1, SAL_PREC_FP16 = 2 } sal_precision;

/* Feature of the third step of Sec. 2, the mean over the n^3 cube of the
 * projected spectrum F_m = alpha_m F (Eq. 1): of its magnitude |F_m|
 * (MAGNITUDE, the default), or of its energy |F_m|^2 = alpha_m^2 |F|^2
 * (ENERGY; FP32 only, not batched). */
typedef enum { SAL_FEATURE_MAGNITUDE = 0, SAL_FEATURE_ENERGY = 1 } sal_feature;

/* Window and sampling (Sec. 2 step 1: local cube of side n, sliding window
 * with more than 50 % overlap).  n in {4, 8, 12, 16}; 1 <= s < n/2. */
typedef struct {
    int32_t n;         /* cube side (even) */
    int32_t s;         /* stride between window centres, voxels */
    int32_t window;    /* sal_window */
    int32_t precision; /* sal_precision */
    int32_t feature;   /* sal_feature */
} sal_spec;

/* Directional center-surround stencil (Sec. 2 step 4, Eq. 3 and Fig. 4).
 * offsets: host int32 [q][3] (dt, dil, dxl) in voxels, each a multiple of s,
 * not all zero; 1 <= q <= SAL_MAX_STENCIL.  weights: host float [q], or NULL
 * for Gaussian weights exp(-|o|^2 / 2d^2) (d = the stencil's Chebyshev reach)
 * scaled to mean 1.  literal = 0 puts the weight outside the modulus,
 * w |E(c) - E(c+o)|; literal = 1 keeps Eq. 3 as printed, |E(c) - w E(c+o)|.
 * per_plane: NULL, or a host array of three stencils, one per projection
 * plane (t, x, y), for the step's "different directional filters" per
 * spectral projection; each is resolved on its own (its own Gaussian default
 * and neighbour count Q), their union may hold at most SAL_MAX_STENCIL
 * distinct offsets, and q, offsets and weights of the outer stencil are then
 * ignored (its literal flag applies to all three; their per_plane must be
 * NULL). */
#define SAL_MAX_STENCIL 64
typedef struct sal_stencil {
    int32_t q;
    const int32_t* offsets;
    const float* weights;
    int32_t literal;
    const struct sal_stencil* per_plane;
} sal_stencil;

/*
 * sal_line_template -- a graded directional line template (Sec. 2 step 4,
 * Fig. 4: comparisons along t, x or t-x with weights that fall off away from
 * the centre).  Offsets j * dir for j = +-1 .. +-length (dir: host int32 [3],
 * in voxels, a multiple of the stride, not zero), weights
 * exp(-j^2 / (2 sigma^2)) scaled to mean 1 over the 2 * length offsets.
 *   offsets_out  host int32 [2 * length][3], ordered j = -length .. -1, 1 .. length
 *   weights_out  host float [2 * length]
 * 1 <= length <= SAL_MAX_STENCIL / 2, sigma > 0.  Host only.
 */
sal_status sal_line_template(const int32_t* dir, int32_t length, double sigma, int32_t* offsets_out,
                             float* weights_out);

typedef enum {
    SAL_FUSE_EQUAL = 0,
    SAL_FUSE_FIXED = 1,
    SAL_FUSE_ADAPT_LS = 2,
    SAL_FUSE_LMS = 3,
    SAL_FUSE_NLMS = 4,
    SAL_FUSE_RLS = 5
} sal_fusion_mode;

/* Fusion of the three directional maps (Sec. 2 step 5, Eq. 4).  EQUAL: 1/3
 * each; FIXED: w_fixed (the "empirical" template); ADAPT_LS: the
 * least-squares weights W = (G + delta I)^-1 p, G = sum u u^T, p = sum u D
 * over the masked grid points, u = (S_t, S_x, S_y) -- the fixed point the
 * paper's LMS/NLMS/RLS adaptation converges to.  A Gram matrix that is not
 * numerically positive definite falls back to EQUAL and raises the status
 * word (see sal_fuse).
 * LMS, NLMS, RLS: the sequential recursions themselves (Sec. 2: the weights
 * are adapted with LMS, NLMS or RLS; Fig. 6), starting from W0 = w_fixed and
 * sweeping the masked grid points in memory order `passes` times; at each
 * sample u = (S_t, S_x, S_y) with a priori error e = D - W.u:
 *   LMS  W += mu e u;   NLMS W += mu e u / (eps + u.u);
 *   RLS  P0 = I / delta, k = P u / (lambda + u.P u), W += k e,
 *        P = (P - k (P u)^T) / lambda.
 * RLS with lambda = 1 and W0 = 0 ends at the ADAPT_LS weights with the same
 * delta.  Their status word is 0.  sal_adapt_weights also returns the
 * learning curve.  The adjoint (sal_backward), the batched plans and
 * sal_fuse_noalloc do not take these modes (SAL_ERR_UNSUPPORTED).
 * sections: 0 fits one W for the whole volume; N > 0 re-adapts every N
 * inline sections (Sec. 2, last paragraph): the grid's inline planes are cut
 * into K = ceil(ILg / N) groups [kN, kN + N), each with its own W fitted on
 * its own masked points, and every voxel takes the W of its grid cell's
 * group.  sal_fuse_groups() gives K. */
typedef struct {
    int32_t mode;
    double w_fixed[3];  /* FIXED: the weights; LMS / NLMS / RLS: the starting weights */
    double delta;       /* >= 0; ADAPT_LS: the ridge term; RLS: P0 = I / delta (> 0) */
    int64_t sections;   /* >= 0 */
    double mu;          /* LMS / NLMS step (> 0) */
    double eps;         /* NLMS regulariser (>= 0) */
    double lambda;      /* RLS forgetting factor, in (0, 1] */
    int32_t passes;     /* LMS / NLMS / RLS sweeps over the masked points (>= 1) */
} sal_fusion;

/* Number of weight groups K of a fusion over a grid with ILg inline planes
 * (1 without sections); 0 for a NULL fusion or negative sizes. */
int64_t sal_fuse_groups(const sal_fusion* fusion, int64_t ILg);

/* Uploads the constant tables of the current device and resolves its static
 * scratch (idempotent, blocking).  Call it once per device before capturing
 * any call in a HIP graph. */
sal_status sal_init(void);

/* Human-readable message of the last failed call on this thread. */
const char* sal_last_error(void);

/* Library version string. */
const char* sal_version(void);

/* Grid extent along an axis of N voxels: ceil(N / s). */
int64_t sal_grid_extent(int64_t N, int32_t s);

/*
 * sal_local_spectra -- Sec. 2 step 1, Eq. 2.
 * The full, unnormalised local 3D DFT F(k) = sum_a H(a) V(c - n/2 + a)
 * e^{-2 pi i k.a/n} at cnt arbitrary voxel centres.
 *   V        device float [T][IL][XL]
 *   centers  device int32 [cnt][3] voxel coordinates (t, il, xl), each inside the volume
 *   F_out    device float [cnt][n][n][n][2]: bins (kt, ki, kx) unshifted, interleaved re/im
 * spec->precision is ignored (fp32).  Intended for checks; cnt may be 0.
 */
sal_status sal_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                             const int32_t* centers, int64_t cnt, float* F_out, sal_stream stream);

/*
 * sal_project -- Sec. 2 steps 1-3, Eq. 1-2.
 * Features E_m(g) = n^-3 sum_{k != 0} alpha_m(k) |F_g(k)| (or, with the
 * energy feature, n^-3 sum_{k != 0} alpha_m(k)^2 |F_g(k)|^2) with
 * alpha_t = sqrt(ki^2 + kx^2)/|k|, alpha_x = sqrt(kt^2 + ki^2)/|k|,
 * alpha_y = sqrt(kt^2 + kx^2)/|k| (signed bin frequencies; the DC bin, the
 * centre of the spectral cube, is not computed).
 *   V      device float [T][IL][XL]
 *   E_out  device float [3][Tg][ILg][XLg]
 */
sal_status sal_project(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec, float* E_out,
                       sal_stream stream);

/*
 * sal_center_surround -- Sec. 2 step 4, Eq. 3.
 * S_m(g) = (1/Q_g) sum over in-grid neighbours g + o/s of w_o |E_m(g) - E_m(g + o/s)|
 * (or the literal form), Q_g = the number of in-grid neighbours (S = 0 if none).
 *   E       device float [3][Tg][ILg][XLg]
 *   Sm_out  device float [3][Tg][ILg][XLg] (must not alias E)
 */
sal_status sal_center_surround(const float* E, int64_t Tg, int64_t ILg, int64_t XLg, int32_t s,
                               const sal_stencil* stencil, float* Sm_out, sal_stream stream);

/*
 * sal_fuse -- Sec. 2 step 5, Eq. 4.
 * Weights W (per fusion->mode) and the full-resolution map
 * S(v) = sum_m W_m S_m(g(v)), g(v) the nearest grid centre (ties to the lower).
 *   Sm      device float [3][Tg][ILg][XLg]
 *   D       device float [Tg][ILg][XLg] desired map (ADAPT_LS only, else ignored)
 *   mask    device uint8 [Tg][ILg][XLg] points used for the fit, or NULL for all
 *   W_out   device double [K][4], K = sal_fuse_groups(): per group W_t, W_x, W_y,
 *           then the status word (0, or 1 if ADAPT_LS fell back to equal weights)
 *   S_out   device float [T][IL][XL]
 *   ws      device workspace of at least sal_fuse_workspace_size() bytes (ADAPT_LS,
 *           LMS, NLMS, RLS)
 */
size_t sal_fuse_workspace_size(int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion);
sal_status sal_fuse(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion, const float* D,
                    const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s, double* W_out, float* S_out,
                    void* ws, size_t ws_bytes, sal_stream stream);

/*
 * sal_adapt_weights -- the sequential LMS / NLMS / RLS weights of Eq. 4 and
 * their learning curve (Sec. 2, fusion paragraph; Fig. 6), without the combine.
 *   fusion     mode SAL_FUSE_LMS, SAL_FUSE_NLMS or SAL_FUSE_RLS (see sal_fusion)
 *   Sm, D, mask as in sal_fuse
 *   W_out      device double [K][4] (the status words are 0)
 *   err2_out   device float [K][cap]: the squared a priori errors e^2 of the first
 *              cap updates of each group, in update order (NULL: not written)
 *   count_out  device int64 [K]: the samples of one pass of each group (NULL: not written)
 *   ws         device workspace of at least sal_fuse_workspace_size() bytes
 * Needs fewer than 2^31 grid points.  sal_fuse with the same fusion gives the
 * same W bit for bit.
 */
sal_status sal_adapt_weights(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion,
                             const float* D, const uint8_t* mask, double* W_out, float* err2_out, int64_t cap,
                             int64_t* count_out, void* ws, size_t ws_bytes, sal_stream stream);

/*
 * sal_fuse_noalloc -- for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * sal_fuse with its workspace in a static device array of
 * sal_fuse_noalloc_max_bytes() bytes, which the library holds on each device
 * it runs on until the process ends.  Arguments and results are those of
 * sal_fuse (bit for bit) without ws / ws_bytes.  ADAPT_LS takes at most 64
 * weight groups (sal_fuse_groups()); more returns SAL_ERR_NOMEM (use sal_fuse
 * with a workspace).  Every call on a device shares that device's array, so
 * calls that overlap on one device (two streams or threads) race: serialise
 * them.  Call sal_init() on the device before capturing a call in a graph
 * (otherwise the first call resolves the array and, inside a capture, returns
 * SAL_ERR_STATE).  Never allocates or frees device memory.
 */
size_t sal_fuse_noalloc_max_bytes(void);
sal_status sal_fuse_noalloc(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion,
                            const float* D, const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s,
                            double* W_out, float* S_out, sal_stream stream);

/*
 * sal_backward -- adjoint of the whole path (sal_project, sal_center_surround,
 * sal_fuse) for the scalar loss L = sum_v gS(v) S(v): gV = dL/dV.  Local
 * spectra are recomputed from V, never stored.  With ADAPT_LS the weights'
 * dependence on the maps is differentiated (D is held fixed); where a |.| or
 * |F| has a kink the subgradient 0 is used.
 *   V, E, Sm     the forward's inputs and outputs (device)
 *   W            device double [K][4] from sal_fuse
 *   D, mask      as given to sal_fuse
 *   gS           device float [T][IL][XL]
 *   gV_out       device float [T][IL][XL]
 *   ws           device workspace of at least sal_backward_workspace_size() bytes
 * spec->precision must be FP32 (the adjoint runs in fp32).
 */
size_t sal_backward_workspace_size(int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                                   const sal_fusion* fusion);
sal_status sal_backward(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                        const sal_stencil* stencil, const sal_fusion* fusion, const float* E, const float* Sm,
                        const double* W, const float* D, const uint8_t* mask, const float* gS, float* gV_out,
                        void* ws, size_t ws_bytes, sal_stream stream);

/*
 * Batched form: the whole forward path (sal_project, sal_center_surround,
 * sal_fuse) for many volumes of uneven sizes and window classes, replayed as
 * one captured HIP graph of persistent kernels (Sec. 2 applied to every
 * member).  Each member's outputs equal those of the single-volume calls
 * bit for bit.
 */
typedef struct {
    const float* V;       /* device float [T][IL][XL] */
    int64_t T, IL, XL;
    sal_spec spec;        /* n, s, window, precision of this member */
    sal_stencil stencil;  /* host arrays, copied by sal_plan_create */
    sal_fusion fusion;    /* sections must be 0 */
    const float* D;       /* device [Tg][ILg][XLg], ADAPT_LS only */
    const uint8_t* mask;  /* device [Tg][ILg][XLg] or NULL */
    float* E_out;         /* device [3][Tg][ILg][XLg] */
    float* Sm_out;        /* device [3][Tg][ILg][XLg] */
    double* W_out;        /* device [4] (as in sal_fuse) */
    float* S_out;         /* device [T][IL][XL] */
} sal_batch_item;

#define SAL_PLAN_AUTOTUNE 1u /* time the candidate tile depths of every window class at creation */
#define SAL_PLAN_NO_GRAPH 2u /* enqueue the kernels directly at each launch instead of replaying a graph */

typedef struct sal_plan_s sal_plan;

/*
 * sal_plan_create -- validates every member, groups them into window classes
 * (n, s, window, precision), picks a tile depth per class (the deepest that
 * fits, or, with SAL_PLAN_AUTOTUNE, the fastest of the candidates, timed on
 * the members themselves and remembered for the process), uploads the
 * descriptor tables and captures the launch sequence in a HIP graph.  The
 * plan keeps the member pointers: the buffers must stay allocated and at the
 * same addresses until sal_plan_destroy.  Creation synchronises the device.
 *   items  host array [count]; count >= 1
 *   out    receives the plan
 */
sal_status sal_plan_create(const sal_batch_item* items, int64_t count, uint32_t flags, sal_plan** out);

/* Enqueues one run of the whole batch on the stream (graph replay). */
sal_status sal_plan_launch(sal_plan* plan, sal_stream stream);

/* Reads the plan's device status word, written by the last launch enqueued on
 * `stream`: the number of members whose ADAPT_LS fit fell back to equal weights
 * and the lowest such member index (-1 if none).  Waits for `stream`. */
sal_status sal_plan_status(const sal_plan* plan, sal_stream stream, int64_t* fallback_count,
                           int64_t* first_fallback);

/* Human-readable description of the classes, tile depths and timings (owned by the plan). */
const char* sal_plan_describe(const sal_plan* plan);

/* Frees the plan's device tables and graph (the member buffers are the caller's). */
sal_status sal_plan_destroy(sal_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* SAL_H */
