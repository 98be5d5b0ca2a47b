/*
 * sal_oracle.c -- plain FP64 CPU oracle of the seismic saliency hot path.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product library (libsal) never
 * links, loads or calls it, and the two share no code, header or table.
 *
 * Method: Shafiq, Long, Di, AlRegib, "A novel attention model for salient
 * structure detection in seismic volumes" (ACI 2021, arXiv 2201.06174),
 * Section 2 "Proposed algorithm".  Every routine below is the definition
 * written out, in FP64, with no FFT, no blocking and no reuse between windows:
 *
 *   step 1 (Sec. 2, Eq. 2): local 3D DFT of the cube of side n around each
 *          grid centre, as three direct 1D DFT passes (the Kronecker product
 *          D_t (x) D_il (x) D_xl applied axis by axis);
 *   step 2 (Sec. 2, Eq. 1): projection F_m = F * P_m / |k|, DC bin excluded;
 *   step 3 (Sec. 2, third step): feature E_m = mean over the n^3 cube of |F_m|;
 *   step 4 (Sec. 2, Eq. 3): directional center-surround S_m, with one
 *          stencil for all planes or a stencil per plane, and graded line
 *          templates along a direction (Fig. 4);
 *   step 5 (Sec. 2, Eq. 4): S = W_t S_t + W_x S_x + W_y S_y with equal, fixed
 *          or least-squares-adapted weights (the fixed point of the LMS/NLMS
 *          and the exact result of RLS with unit forgetting factor), or the
 *          weights of the sequential LMS, NLMS and RLS recursions themselves,
 *          fitted once or again every N inline sections (last paragraph of
 *          Sec. 2).
 *
 * Readings taken where the paper is silent (each is listed in the design doc):
 *   - volume V is float32 [T][IL][XL] (XL fastest); feature/saliency planes
 *     are ordered (t, x = crossline = XL axis, y = inline = IL axis); P_m
 *     omits the frequency of axis m;
 *   - grid centres are g*s on every axis, Ng = ceil(N/s);
 *   - the window of an even side n spans c-n/2 .. c+n/2-1 and is tapered by
 *     the separable periodic Hann h(a) = sin^2(pi a/n) (or a flat window);
 *   - indices outside the volume are reflected half-sample symmetrically
 *     (-1 -> 0, N -> N-1), which needs N >= n/2;
 *   - DFT e^{-2 pi i k.a/n}, unnormalised, phase origin at the window start;
 *     bin u has signed frequency u (u <= n/2) or u-n;
 *   - E_m divides by n^3 and gives the DC bin weight 0;
 *   - DCS: S_m(g) = (1/Q_g) sum_{o valid} w_o |E_m(g) - E_m(g+o/s)|
 *     (weight outside the modulus; the literal form |E(g) - w E(g+o)| is a
 *     flag), Q_g = number of in-volume neighbours, default weights Gaussian
 *     with sigma = the stencil's Chebyshev reach, scaled to mean 1;
 *   - adapted weights: W = (G + delta I)^{-1} p with G = sum u u^T and
 *     p = sum u D over the mask, u = (S_t, S_x, S_y); a Gram matrix that is
 *     not positive definite falls back to equal weights; with re-adaptation
 *     every N sections, one such fit per group of N grid inline planes;
 *   - a line template holds the offsets j * dir, j = +-1 .. +-L, with
 *     weights exp(-j^2 / 2 sigma^2) scaled to mean 1;
 *   - S at full resolution takes the nearest grid centre, ties to the lower.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EARG 1
#define ORC_ENOMEM 4

static const double ORC_PI = 3.14159265358979323846264338327950288;

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/* Half-sample symmetric reflection of an index into [0, N). */
static int64_t reflect_index(int64_t p, int64_t N) {
    if (p < 0) p = -1 - p;
    if (p >= N) p = 2 * N - 1 - p;
    return p;
}

/* Signed frequency of DFT bin u of an n-point transform. */
static int signed_freq(int u, int n) { return (u <= n / 2) ? u : u - n; }

static int check_spec(int64_t T, int64_t IL, int64_t XL, int n, int s, int window) {
    if (n < 2 || (n & 1) || n > 64) return ORC_EARG;
    if (s < 1) return ORC_EARG;
    if (window != 0 && window != 1) return ORC_EARG;
    if (T < n / 2 || IL < n / 2 || XL < n / 2) return ORC_EARG;
    return ORC_OK;
}

/* Window taper: 0 = periodic Hann sin^2(pi a/n), 1 = flat. */
int orc_window(int n, int window, double* h) {
    if (n < 2 || (window != 0 && window != 1)) return ORC_EARG;
    for (int a = 0; a < n; a++) {
        double v = sin(ORC_PI * (double)a / (double)n);
        h[a] = window == 0 ? v * v : 1.0;
    }
    return ORC_OK;
}

/* cos/sin of 2 pi k a / n with the product reduced mod n first. */
static void twiddle_tables(int n, double* c, double* sn) {
    for (int k = 0; k < n; k++)
        for (int a = 0; a < n; a++) {
            int r = (k * a) % n;
            c[k * n + a] = cos(2.0 * ORC_PI * (double)r / (double)n);
            sn[k * n + a] = sin(2.0 * ORC_PI * (double)r / (double)n);
        }
}

/* Projection weights of Eq. 1 for every bin of the n^3 spectrum:
 * alpha_t = sqrt(ki^2+kx^2)/|k|, alpha_x = sqrt(kt^2+ki^2)/|k|,
 * alpha_y = sqrt(kt^2+kx^2)/|k|, and 0 at the DC bin. */
static void alpha_tables(int n, double* at, double* ax, double* ay) {
    for (int ut = 0; ut < n; ut++)
        for (int ui = 0; ui < n; ui++)
            for (int ux = 0; ux < n; ux++) {
                int64_t idx = ((int64_t)ut * n + ui) * n + ux;
                double ft = signed_freq(ut, n), fi = signed_freq(ui, n), fx = signed_freq(ux, n);
                double k2 = ft * ft + fi * fi + fx * fx;
                if (k2 == 0.0) {
                    at[idx] = ax[idx] = ay[idx] = 0.0;
                    continue;
                }
                double kn = sqrt(k2);
                at[idx] = sqrt(fi * fi + fx * fx) / kn;
                ax[idx] = sqrt(ft * ft + fi * fi) / kn;
                ay[idx] = sqrt(ft * ft + fx * fx) / kn;
            }
}

typedef struct {
    int n;
    double* h;   /* [n] */
    double* c;   /* [n][n] cos(2 pi k a/n) */
    double* sn;  /* [n][n] sin(2 pi k a/n) */
    double* at;  /* [n^3] projection weights */
    double* ax;
    double* ay;
} orc_tables;

static int tables_init(orc_tables* tb, int n, int window) {
    int64_t n3 = (int64_t)n * n * n;
    tb->n = n;
    tb->h = (double*)malloc(sizeof(double) * n);
    tb->c = (double*)malloc(sizeof(double) * n * n);
    tb->sn = (double*)malloc(sizeof(double) * n * n);
    tb->at = (double*)malloc(sizeof(double) * n3);
    tb->ax = (double*)malloc(sizeof(double) * n3);
    tb->ay = (double*)malloc(sizeof(double) * n3);
    if (!tb->h || !tb->c || !tb->sn || !tb->at || !tb->ax || !tb->ay) return ORC_ENOMEM;
    orc_window(n, window, tb->h);
    twiddle_tables(n, tb->c, tb->sn);
    alpha_tables(n, tb->at, tb->ax, tb->ay);
    return ORC_OK;
}

static void tables_free(orc_tables* tb) {
    free(tb->h); free(tb->c); free(tb->sn); free(tb->at); free(tb->ax); free(tb->ay);
}

/* Scratch for one window: three complex n^3 buffers. */
typedef struct {
    double *xr, *xi, *yr, *yi;
} orc_work;

static int work_init(orc_work* w, int n) {
    int64_t n3 = (int64_t)n * n * n;
    w->xr = (double*)malloc(sizeof(double) * n3);
    w->xi = (double*)malloc(sizeof(double) * n3);
    w->yr = (double*)malloc(sizeof(double) * n3);
    w->yi = (double*)malloc(sizeof(double) * n3);
    return (w->xr && w->xi && w->yr && w->yi) ? ORC_OK : ORC_ENOMEM;
}

static void work_free(orc_work* w) { free(w->xr); free(w->xi); free(w->yr); free(w->yi); }

/* One direct 1D DFT pass along axis `ax` (0 = t, 1 = il, 2 = xl) of the
 * complex cube (ir, ii) into (or, oi), with sign -1 (forward) or +1
 * (inverse, unnormalised).  out[.., k, ..] = sum_a in[.., a, ..] e^{sign 2 pi i k a/n}. */
static void dft_pass(const orc_tables* tb, int axis, int sign, const double* ir, const double* ii,
                     double* outr, double* outi) {
    int n = tb->n;
    int64_t stride = axis == 0 ? (int64_t)n * n : (axis == 1 ? n : 1);
    for (int p = 0; p < n; p++)
        for (int q = 0; q < n; q++) {
            /* base offset of the line: the two other axes take values p, q */
            int64_t base;
            if (axis == 0) base = (int64_t)p * n + q;
            else if (axis == 1) base = (int64_t)p * n * n + q;
            else base = ((int64_t)p * n + q) * n;
            for (int k = 0; k < n; k++) {
                double sr = 0.0, si = 0.0;
                for (int a = 0; a < n; a++) {
                    double cr = tb->c[k * n + a], cs = sign * tb->sn[k * n + a];
                    double vr = ir[base + a * stride], vi = ii[base + a * stride];
                    /* (vr + i vi)(cr + i cs) */
                    sr += vr * cr - vi * cs;
                    si += vr * cs + vi * cr;
                }
                outr[base + k * stride] = sr;
                outi[base + k * stride] = si;
            }
        }
}

/* Gather the tapered cube around voxel centre (ct, ci, cx) and take its
 * 3D DFT (Sec. 2 step 1, Eq. 2).  Result in (w->xr, w->xi), layout [kt][ki][kx]. */
static void window_spectrum(const float* V, int64_t T, int64_t IL, int64_t XL, const orc_tables* tb,
                            int64_t ct, int64_t ci, int64_t cx, orc_work* w) {
    int n = tb->n, half = n / 2;
    for (int at = 0; at < n; at++) {
        int64_t pt = reflect_index(ct - half + at, T);
        for (int ai = 0; ai < n; ai++) {
            int64_t pi = reflect_index(ci - half + ai, IL);
            for (int axx = 0; axx < n; axx++) {
                int64_t px = reflect_index(cx - half + axx, XL);
                int64_t idx = ((int64_t)at * n + ai) * n + axx;
                w->xr[idx] = tb->h[at] * tb->h[ai] * tb->h[axx] * (double)V[(pt * IL + pi) * XL + px];
                w->xi[idx] = 0.0;
            }
        }
    }
    dft_pass(tb, 2, -1, w->xr, w->xi, w->yr, w->yi);
    dft_pass(tb, 1, -1, w->yr, w->yi, w->xr, w->xi);
    dft_pass(tb, 0, -1, w->xr, w->xi, w->yr, w->yi);
    int64_t n3 = (int64_t)n * n * n;
    memcpy(w->xr, w->yr, sizeof(double) * n3);
    memcpy(w->xi, w->yi, sizeof(double) * n3);
}

/* Features of one window (Sec. 2 steps 2-3, Eq. 1), the mean over the n^3 cube of the
 * projected spectrum F_m = alpha_m F:
 *   feature 0 (magnitude): E_m = n^-3 sum_k |F_m(k)| = n^-3 sum_k alpha_m(k) |F(k)|;
 *   feature 1 (energy):    E_m = n^-3 sum_k |F_m(k)|^2 = n^-3 sum_k alpha_m(k)^2 |F(k)|^2. */
static void window_features(const orc_tables* tb, const orc_work* w, int feature, double* E3) {
    int n = tb->n;
    int64_t n3 = (int64_t)n * n * n;
    double et = 0.0, ex = 0.0, ey = 0.0;
    for (int64_t k = 0; k < n3; k++) {
        double p = w->xr[k] * w->xr[k] + w->xi[k] * w->xi[k];
        if (feature == 1) {
            et += tb->at[k] * tb->at[k] * p;
            ex += tb->ax[k] * tb->ax[k] * p;
            ey += tb->ay[k] * tb->ay[k] * p;
        } else {
            double mag = sqrt(p);
            et += tb->at[k] * mag;
            ex += tb->ax[k] * mag;
            ey += tb->ay[k] * mag;
        }
    }
    E3[0] = et / (double)n3;
    E3[1] = ex / (double)n3;
    E3[2] = ey / (double)n3;
}

/* Full local spectra at arbitrary voxel centres: F[cnt][n][n][n][2]. */
int orc_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int window,
                      const int64_t* centers, int64_t cnt, double* F) {
    int rc = check_spec(T, IL, XL, n, 1, window);
    if (rc) return rc;
    orc_tables tb;
    if (tables_init(&tb, n, window)) { tables_free(&tb); return ORC_ENOMEM; }
    orc_work w;
    if (work_init(&w, n)) { work_free(&w); tables_free(&tb); return ORC_ENOMEM; }
    int64_t n3 = (int64_t)n * n * n;
    for (int64_t j = 0; j < cnt; j++) {
        int64_t ct = centers[3 * j], ci = centers[3 * j + 1], cx = centers[3 * j + 2];
        if (ct < 0 || ct >= T || ci < 0 || ci >= IL || cx < 0 || cx >= XL) { rc = ORC_EARG; break; }
        window_spectrum(V, T, IL, XL, &tb, ct, ci, cx, &w);
        for (int64_t k = 0; k < n3; k++) {
            F[(j * n3 + k) * 2] = w.xr[k];
            F[(j * n3 + k) * 2 + 1] = w.xi[k];
        }
    }
    work_free(&w);
    tables_free(&tb);
    return rc;
}

/* E at a list of grid points g[cnt][3]; output E[cnt][3]. */
int orc_features_at_ex(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int feature,
                       const int64_t* g, int64_t cnt, double* E, int nthreads) {
    int rc = check_spec(T, IL, XL, n, s, window);
    if (rc) return rc;
    if (feature != 0 && feature != 1) return ORC_EARG;
    int64_t Tg = ceil_div(T, s), ILg = ceil_div(IL, s), XLg = ceil_div(XL, s);
    for (int64_t j = 0; j < cnt; j++)
        if (g[3 * j] < 0 || g[3 * j] >= Tg || g[3 * j + 1] < 0 || g[3 * j + 1] >= ILg || g[3 * j + 2] < 0 ||
            g[3 * j + 2] >= XLg)
            return ORC_EARG;
    orc_tables tb;
    if (tables_init(&tb, n, window)) { tables_free(&tb); return ORC_ENOMEM; }
    int fail = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        int ok = work_init(&w, n) == ORC_OK;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < cnt; j++) {
            if (!ok) continue;
            window_spectrum(V, T, IL, XL, &tb, g[3 * j] * s, g[3 * j + 1] * s, g[3 * j + 2] * s, &w);
            window_features(&tb, &w, feature, E + 3 * j);
        }
        work_free(&w);
    }
    tables_free(&tb);
    return fail ? ORC_ENOMEM : ORC_OK;
}

int orc_features_at(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window,
                    const int64_t* g, int64_t cnt, double* E, int nthreads) {
    return orc_features_at_ex(V, T, IL, XL, n, s, window, 0, g, cnt, E, nthreads);
}

/* E on the whole grid, planar layout E[3][Tg][ILg][XLg]. */
int orc_features_ex(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int feature,
                    double* E, int nthreads) {
    int rc = check_spec(T, IL, XL, n, s, window);
    if (rc) return rc;
    if (feature != 0 && feature != 1) return ORC_EARG;
    int64_t Tg = ceil_div(T, s), ILg = ceil_div(IL, s), XLg = ceil_div(XL, s);
    int64_t G = Tg * ILg * XLg;
    orc_tables tb;
    if (tables_init(&tb, n, window)) { tables_free(&tb); return ORC_ENOMEM; }
    int fail = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w;
        int ok = work_init(&w, n) == ORC_OK;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < G; j++) {
            if (!ok) continue;
            int64_t gt = j / (ILg * XLg), gi = (j / XLg) % ILg, gx = j % XLg;
            double e3[3];
            window_spectrum(V, T, IL, XL, &tb, gt * s, gi * s, gx * s, &w);
            window_features(&tb, &w, feature, e3);
            E[j] = e3[0];
            E[G + j] = e3[1];
            E[2 * G + j] = e3[2];
        }
        work_free(&w);
    }
    tables_free(&tb);
    return fail ? ORC_ENOMEM : ORC_OK;
}

int orc_features(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, double* E,
                 int nthreads) {
    return orc_features_ex(V, T, IL, XL, n, s, window, 0, E, nthreads);
}

/* Default DCS weights: Gaussian exp(-|o|^2 / (2 d^2)) with d the stencil's
 * Chebyshev reach, scaled to mean 1 over the stencil (Sec. 2, Eq. 3 text). */
int orc_default_weights(int q, const int32_t* off, double* w) {
    if (q <= 0) return ORC_EARG;
    int d = 0;
    for (int j = 0; j < q; j++)
        for (int a = 0; a < 3; a++) {
            int v = abs(off[3 * j + a]);
            if (v > d) d = v;
        }
    if (d == 0) return ORC_EARG;
    double sum = 0.0;
    for (int j = 0; j < q; j++) {
        double r2 = 0.0;
        for (int a = 0; a < 3; a++) r2 += (double)off[3 * j + a] * off[3 * j + a];
        w[j] = exp(-r2 / (2.0 * (double)d * d));
        sum += w[j];
    }
    for (int j = 0; j < q; j++) w[j] *= (double)q / sum;
    return ORC_OK;
}

static int check_stencil(int s, int q, const int32_t* off) {
    if (q <= 0 || s < 1) return ORC_EARG;
    for (int j = 0; j < 3 * q; j++)
        if (off[j] % s != 0) return ORC_EARG;
    return ORC_OK;
}

/* Directional center-surround at one grid point of one plane (Sec. 2, Eq. 3). */
static double dcs_point(const double* Em, int64_t Tg, int64_t ILg, int64_t XLg, int s, int q,
                        const int32_t* off, const double* w, int literal, int64_t gt, int64_t gi, int64_t gx) {
    double e0 = Em[(gt * ILg + gi) * XLg + gx];
    double acc = 0.0;
    int Q = 0;
    for (int j = 0; j < q; j++) {
        int64_t nt = gt + off[3 * j] / s, ni = gi + off[3 * j + 1] / s, nx = gx + off[3 * j + 2] / s;
        if (nt < 0 || nt >= Tg || ni < 0 || ni >= ILg || nx < 0 || nx >= XLg) continue;
        double e1 = Em[(nt * ILg + ni) * XLg + nx];
        acc += literal ? fabs(e0 - w[j] * e1) : w[j] * fabs(e0 - e1);
        Q++;
    }
    return Q ? acc / (double)Q : 0.0;
}

/* S_m on the whole grid from E (both planar [3][Tg][ILg][XLg]). */
int orc_dcs(const double* E, int64_t Tg, int64_t ILg, int64_t XLg, int s, int q, const int32_t* off,
            const double* w, int literal, double* S) {
    if (check_stencil(s, q, off)) return ORC_EARG;
    int64_t G = Tg * ILg * XLg;
    for (int m = 0; m < 3; m++)
        for (int64_t j = 0; j < G; j++) {
            int64_t gt = j / (ILg * XLg), gi = (j / XLg) % ILg, gx = j % XLg;
            S[m * G + j] = dcs_point(E + m * G, Tg, ILg, XLg, s, q, off, w, literal, gt, gi, gx);
        }
    return ORC_OK;
}

/* Graded directional line template (Sec. 2 step 4 and Fig. 4: comparisons
 * along a direction with weights that are largest next to the centre and fall
 * off with distance).  Reading: offsets j * dir for j = -L .. -1, 1 .. L in
 * that order, weights exp(-j^2 / (2 sigma^2)) scaled to mean 1 over the 2L
 * offsets.  off: [2L][3], w: [2L]. */
int orc_line_template(const int32_t* dir, int L, double sigma, int32_t* off, double* w) {
    if (L < 1 || !(sigma > 0.0) || (dir[0] == 0 && dir[1] == 0 && dir[2] == 0)) return ORC_EARG;
    int k = 0;
    double sum = 0.0;
    for (int j = -L; j <= L; j++) {
        if (j == 0) continue;
        for (int a = 0; a < 3; a++) off[3 * k + a] = j * dir[a];
        w[k] = exp(-(double)j * j / (2.0 * sigma * sigma));
        sum += w[k];
        k++;
    }
    for (int e = 0; e < k; e++) w[e] *= (double)k / sum;
    return ORC_OK;
}

/* S_m with a stencil of its own for every plane (Sec. 2 step 4: different
 * directional filters per spectral projection).  Plane m uses the q3[m]
 * offsets and weights that follow those of the planes before it in off_all
 * ([sum q3][3]) and w_all ([sum q3]). */
int orc_dcs_planes(const double* E, int64_t Tg, int64_t ILg, int64_t XLg, int s, const int* q3,
                   const int32_t* off_all, const double* w_all, int literal, double* S) {
    int64_t G = Tg * ILg * XLg;
    int base = 0;
    for (int m = 0; m < 3; m++) {
        const int32_t* off = off_all + 3 * base;
        const double* w = w_all + base;
        if (check_stencil(s, q3[m], off)) return ORC_EARG;
        for (int64_t j = 0; j < G; j++) {
            int64_t gt = j / (ILg * XLg), gi = (j / XLg) % ILg, gx = j % XLg;
            S[m * G + j] = dcs_point(E + m * G, Tg, ILg, XLg, s, q3[m], off, w, literal, gt, gi, gx);
        }
        base += q3[m];
    }
    return ORC_OK;
}

/* S_m (and E) at a list of grid points, computing E at each point and at its
 * in-volume stencil neighbours directly from V.  Sm, E: [cnt][3]. */
int orc_saliency_at(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int q,
                    const int32_t* off, const double* w, int literal, const int64_t* g, int64_t cnt, double* Sm,
                    double* E, int nthreads) {
    int rc = check_spec(T, IL, XL, n, s, window);
    if (rc) return rc;
    if (check_stencil(s, q, off)) return ORC_EARG;
    int64_t Tg = ceil_div(T, s), ILg = ceil_div(IL, s), XLg = ceil_div(XL, s);
    for (int64_t j = 0; j < cnt; j++)
        if (g[3 * j] < 0 || g[3 * j] >= Tg || g[3 * j + 1] < 0 || g[3 * j + 1] >= ILg || g[3 * j + 2] < 0 ||
            g[3 * j + 2] >= XLg)
            return ORC_EARG;
    orc_tables tb;
    if (tables_init(&tb, n, window)) { tables_free(&tb); return ORC_ENOMEM; }
    int fail = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work w_;
        int ok = work_init(&w_, n) == ORC_OK;
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < cnt; j++) {
            if (!ok) continue;
            int64_t gt = g[3 * j], gi = g[3 * j + 1], gx = g[3 * j + 2];
            double e0[3], e1[3], acc[3] = {0, 0, 0};
            int Q = 0;
            window_spectrum(V, T, IL, XL, &tb, gt * s, gi * s, gx * s, &w_);
            window_features(&tb, &w_, 0, e0);
            for (int k = 0; k < q; k++) {
                int64_t nt = gt + off[3 * k] / s, ni = gi + off[3 * k + 1] / s, nx = gx + off[3 * k + 2] / s;
                if (nt < 0 || nt >= Tg || ni < 0 || ni >= ILg || nx < 0 || nx >= XLg) continue;
                window_spectrum(V, T, IL, XL, &tb, nt * s, ni * s, nx * s, &w_);
                window_features(&tb, &w_, 0, e1);
                for (int m = 0; m < 3; m++) acc[m] += literal ? fabs(e0[m] - w[k] * e1[m]) : w[k] * fabs(e0[m] - e1[m]);
                Q++;
            }
            for (int m = 0; m < 3; m++) {
                Sm[3 * j + m] = Q ? acc[m] / (double)Q : 0.0;
                if (E) E[3 * j + m] = e0[m];
            }
        }
        work_free(&w_);
    }
    tables_free(&tb);
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Cholesky solve of the 3x3 system A x = b.  Returns 0 and x on success, 1 if
 * A is not numerically positive definite (a pivot at or below 1e-12 times the
 * largest diagonal entry, or a non-finite entry). */
static int chol3_solve(const double A[9], const double b[3], double x[3]) {
    double dmax = 0.0;
    for (int i = 0; i < 3; i++) {
        if (!isfinite(A[4 * i])) return 1;
        if (A[4 * i] > dmax) dmax = A[4 * i];
    }
    if (!(dmax > 0.0)) return 1;
    double L[9] = {0};
    for (int j = 0; j < 3; j++) {
        double d = A[3 * j + j];
        for (int k = 0; k < j; k++) d -= L[3 * j + k] * L[3 * j + k];
        if (!(d > 1e-12 * dmax) || !isfinite(d)) return 1;
        L[3 * j + j] = sqrt(d);
        for (int i = j + 1; i < 3; i++) {
            double v = A[3 * i + j];
            for (int k = 0; k < j; k++) v -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = v / L[3 * j + j];
        }
    }
    double y[3];
    for (int i = 0; i < 3; i++) {
        double v = b[i];
        for (int k = 0; k < i; k++) v -= L[3 * i + k] * y[k];
        y[i] = v / L[3 * i + i];
    }
    for (int i = 2; i >= 0; i--) {
        double v = y[i];
        for (int k = i + 1; k < 3; k++) v -= L[3 * k + i] * x[k];
        x[i] = v / L[3 * i + i];
    }
    return 0;
}

/* Fusion weights (Sec. 2, Eq. 4).  mode 0 = equal, 1 = fixed, 2 = adapted
 * least squares against the desired map D over the mask.  stats (optional,
 * [11]) receives G00 G01 G02 G11 G12 G22 p0 p1 p2 sum(D^2) count. */
int orc_fusion_weights(const double* Sm, int64_t G, const float* D, const uint8_t* mask, int mode,
                       const double* wfix, double delta, double* W, int* fallback, double* stats) {
    *fallback = 0;
    if (mode == 0) {
        W[0] = W[1] = W[2] = 1.0 / 3.0;
        return ORC_OK;
    }
    if (mode == 1) {
        if (!wfix) return ORC_EARG;
        W[0] = wfix[0]; W[1] = wfix[1]; W[2] = wfix[2];
        return ORC_OK;
    }
    if (mode != 2 || !D || !(delta >= 0.0)) return ORC_EARG;
    double st[11] = {0};
    for (int64_t j = 0; j < G; j++) {
        if (mask && !mask[j]) continue;
        double u0 = Sm[j], u1 = Sm[G + j], u2 = Sm[2 * G + j], d = (double)D[j];
        st[0] += u0 * u0; st[1] += u0 * u1; st[2] += u0 * u2;
        st[3] += u1 * u1; st[4] += u1 * u2; st[5] += u2 * u2;
        st[6] += u0 * d; st[7] += u1 * d; st[8] += u2 * d;
        st[9] += d * d; st[10] += 1.0;
    }
    if (stats) memcpy(stats, st, sizeof(st));
    double A[9] = {st[0] + delta, st[1], st[2], st[1], st[3] + delta, st[4], st[2], st[4], st[5] + delta};
    double b[3] = {st[6], st[7], st[8]};
    if (chol3_solve(A, b, W)) {
        W[0] = W[1] = W[2] = 1.0 / 3.0;
        *fallback = 1;
    }
    return ORC_OK;
}

/* Nearest grid index of voxel v (ties to the lower centre), clamped. */
static int64_t cell_of(int64_t v, int s, int64_t Ng) {
    int64_t g = (v + (s - 1) / 2) / s;
    return g < Ng - 1 ? g : Ng - 1;
}

/* S(v) = sum_m W_m S_m(g(v)) at full resolution (Sec. 2, Eq. 4). */
int orc_combine(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const double* W, int64_t T, int64_t IL,
                int64_t XL, int s, double* S) {
    if (s < 1 || ceil_div(T, s) != Tg || ceil_div(IL, s) != ILg || ceil_div(XL, s) != XLg) return ORC_EARG;
    int64_t G = Tg * ILg * XLg;
    for (int64_t t = 0; t < T; t++)
        for (int64_t i = 0; i < IL; i++)
            for (int64_t x = 0; x < XL; x++) {
                int64_t j = (cell_of(t, s, Tg) * ILg + cell_of(i, s, ILg)) * XLg + cell_of(x, s, XLg);
                S[(t * IL + i) * XL + x] = W[0] * Sm[j] + W[1] * Sm[G + j] + W[2] * Sm[2 * G + j];
            }
    return ORC_OK;
}

/* Re-adaptation every N inline sections (Sec. 2, last paragraph).  Reading:
 * the grid's inline planes are cut into K = ceil(ILg / N) groups
 * [kN, kN + N) (N = 0: one group), and group k's weights are those of Eq. 4
 * fitted on the masked points of that group alone.  W: [K][3], fallback: [K],
 * stats: [K][11] or NULL. */
int64_t orc_fuse_groups(int64_t ILg, int64_t N) { return N > 0 ? ceil_div(ILg, N) : 1; }

int orc_fusion_weights_sections(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const float* D,
                                const uint8_t* mask, int mode, const double* wfix, double delta, int64_t N,
                                double* W, int* fallback, double* stats) {
    if (N < 0) return ORC_EARG;
    int64_t G = Tg * ILg * XLg, K = orc_fuse_groups(ILg, N);
    uint8_t* mk = (uint8_t*)malloc((size_t)(G > 0 ? G : 1));
    if (!mk) return ORC_ENOMEM;
    int rc = ORC_OK;
    for (int64_t k = 0; k < K && rc == ORC_OK; k++) {
        for (int64_t j = 0; j < G; j++) {
            int64_t gi = (j / XLg) % ILg;
            int in = N > 0 ? (gi >= k * N && gi < (k + 1) * N) : 1;
            mk[j] = (uint8_t)(in && (!mask || mask[j]));
        }
        rc = orc_fusion_weights(Sm, G, D, mk, mode, wfix, delta, W + 3 * k, fallback + k,
                                stats ? stats + 11 * k : NULL);
    }
    free(mk);
    return rc;
}

/* Sequential weight adaptation (Sec. 2, fusion paragraph, and Fig. 6: the
 * weights are adapted with LMS, NLMS or RLS towards the desired map).  The
 * samples are the masked grid points of each weight group in memory order,
 * u = (S_t, S_x, S_y), swept `passes` times; starting weights w0.  At every
 * sample, with the a priori error e = D - w.u:
 *   rule 0 (LMS):  w += mu e u;
 *   rule 1 (NLMS): w += mu e u / (eps + u.u);
 *   rule 2 (RLS):  P0 = I / delta (per group), k = P u / (lambda + u.P u),
 *                  w += k e, P = (P - k (P u)^T) / lambda.
 * W: [K][3]; count: [K] samples per pass; err2: [K][cap] squared a priori
 * errors in update order (the learning curve; the first cap kept), or NULL. */
int orc_adapt_sequential(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const float* D,
                         const uint8_t* mask, int rule, double mu, double eps, double lambda, double delta,
                         const double* w0, int passes, int64_t N, double* W, int64_t* count, double* err2,
                         int64_t cap) {
    if (rule < 0 || rule > 2 || passes < 1 || N < 0 || !D) return ORC_EARG;
    if (rule == 2 && (!(lambda > 0.0) || lambda > 1.0 || !(delta > 0.0))) return ORC_EARG;
    int64_t G = Tg * ILg * XLg, K = orc_fuse_groups(ILg, N);
    for (int64_t k = 0; k < K; k++) {
        double w[3] = {w0[0], w0[1], w0[2]};
        double P[9] = {1.0 / delta, 0, 0, 0, 1.0 / delta, 0, 0, 0, 1.0 / delta};
        int64_t it = 0, cnt = 0;
        for (int pass = 0; pass < passes; pass++) {
            cnt = 0;
            for (int64_t j = 0; j < G; j++) {
                int64_t gi = (j / XLg) % ILg;
                if (N > 0 && (gi < k * N || gi >= (k + 1) * N)) continue;
                if (mask && !mask[j]) continue;
                double u[3] = {Sm[j], Sm[G + j], Sm[2 * G + j]};
                double e = (double)D[j] - (w[0] * u[0] + w[1] * u[1] + w[2] * u[2]);
                if (err2 && it < cap) err2[k * cap + it] = e * e;
                if (rule == 0) {
                    for (int m = 0; m < 3; m++) w[m] += mu * e * u[m];
                } else if (rule == 1) {
                    double g = mu * e / (eps + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    for (int m = 0; m < 3; m++) w[m] += g * u[m];
                } else {
                    double Pu[3];
                    for (int a = 0; a < 3; a++) Pu[a] = P[3 * a] * u[0] + P[3 * a + 1] * u[1] + P[3 * a + 2] * u[2];
                    double den = lambda + u[0] * Pu[0] + u[1] * Pu[1] + u[2] * Pu[2];
                    double kg[3] = {Pu[0] / den, Pu[1] / den, Pu[2] / den};
                    for (int m = 0; m < 3; m++) w[m] += kg[m] * e;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++) P[3 * a + b] = (P[3 * a + b] - kg[a] * Pu[b]) / lambda;
                }
                it++;
                cnt++;
            }
        }
        W[3 * k] = w[0]; W[3 * k + 1] = w[1]; W[3 * k + 2] = w[2];
        count[k] = cnt;
    }
    return ORC_OK;
}

/* S(v) = sum_m W_m S_m(g(v)) with the weights of g(v)'s group. */
int orc_combine_sections(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const double* W, int64_t N,
                         int64_t T, int64_t IL, int64_t XL, int s, double* S) {
    if (s < 1 || N < 0 || ceil_div(T, s) != Tg || ceil_div(IL, s) != ILg || ceil_div(XL, s) != XLg) return ORC_EARG;
    int64_t G = Tg * ILg * XLg;
    for (int64_t t = 0; t < T; t++)
        for (int64_t i = 0; i < IL; i++)
            for (int64_t x = 0; x < XL; x++) {
                int64_t gi = cell_of(i, s, ILg);
                const double* Wk = W + 3 * (N > 0 ? gi / N : 0);
                int64_t j = (cell_of(t, s, Tg) * ILg + gi) * XLg + cell_of(x, s, XLg);
                S[(t * IL + i) * XL + x] = Wk[0] * Sm[j] + Wk[1] * Sm[G + j] + Wk[2] * Sm[2 * G + j];
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint.  Loss L = sum_v gS(v) S(v); all routines return dL/d(input).    */
/* ------------------------------------------------------------------------ */

static double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

/* Spectral adjoint of one window: given gE (3 values) and the window's
 * spectrum F in (w->xr, w->xi), form Y(k) = c(k) F(k)/|F(k)| with
 * c(k) = sum_m gE_m alpha_m(k) / n^3 (zero at DC and where |F| = 0) for the
 * magnitude feature, or Y(k) = 2 c(k) F(k) with c(k) = sum_m gE_m
 * alpha_m(k)^2 / n^3 for the energy feature, and the tapered real field
 * H(a) Re sum_k Y(k) e^{+2 pi i k.a/n} into w->yr. */
static void window_adjoint(const orc_tables* tb, const double gE[3], int feature, orc_work* w) {
    int n = tb->n;
    int64_t n3 = (int64_t)n * n * n;
    for (int64_t k = 0; k < n3; k++) {
        if (feature == 1) {
            double c = (gE[0] * tb->at[k] * tb->at[k] + gE[1] * tb->ax[k] * tb->ax[k] +
                        gE[2] * tb->ay[k] * tb->ay[k]) / (double)n3;
            w->xr[k] = 2.0 * c * w->xr[k];
            w->xi[k] = 2.0 * c * w->xi[k];
            continue;
        }
        double mag = sqrt(w->xr[k] * w->xr[k] + w->xi[k] * w->xi[k]);
        double c = (gE[0] * tb->at[k] + gE[1] * tb->ax[k] + gE[2] * tb->ay[k]) / (double)n3;
        if (mag > 0.0) {
            w->xr[k] = c * w->xr[k] / mag;
            w->xi[k] = c * w->xi[k] / mag;
        } else {
            w->xr[k] = 0.0;
            w->xi[k] = 0.0;
        }
    }
    dft_pass(tb, 0, +1, w->xr, w->xi, w->yr, w->yi);
    dft_pass(tb, 1, +1, w->yr, w->yi, w->xr, w->xi);
    dft_pass(tb, 2, +1, w->xr, w->xi, w->yr, w->yi);
    for (int at = 0; at < n; at++)
        for (int ai = 0; ai < n; ai++)
            for (int ax = 0; ax < n; ax++) {
                int64_t idx = ((int64_t)at * n + ai) * n + ax;
                w->yr[idx] *= tb->h[at] * tb->h[ai] * tb->h[ax];
            }
}

/* Adjoint of the center-surround: gE from gSm (both planar on the grid);
 * plane m's stencil as in orc_dcs_planes. */
static void dcs_adjoint(const double* E, const double* gSm, int64_t Tg, int64_t ILg, int64_t XLg, int s,
                        const int* q3, const int32_t* off_all, const double* w_all, int literal, double* gE) {
    int64_t G = Tg * ILg * XLg;
    memset(gE, 0, sizeof(double) * 3 * G);
    for (int m = 0; m < 3; m++) {
        int base = 0;
        for (int l = 0; l < m; l++) base += q3[l];
        const int q = q3[m];
        const int32_t* off = off_all + 3 * base;
        const double* w = w_all + base;
        const double* Em = E + m * G;
        double* gEm = gE + m * G;
        for (int64_t j = 0; j < G; j++) {
            int64_t gt = j / (ILg * XLg), gi = (j / XLg) % ILg, gx = j % XLg;
            int Q = 0;
            for (int k = 0; k < q; k++) {
                int64_t nt = gt + off[3 * k] / s, ni = gi + off[3 * k + 1] / s, nx = gx + off[3 * k + 2] / s;
                if (nt < 0 || nt >= Tg || ni < 0 || ni >= ILg || nx < 0 || nx >= XLg) continue;
                Q++;
            }
            if (!Q) continue;
            double coef = gSm[m * G + j] / (double)Q;
            for (int k = 0; k < q; k++) {
                int64_t nt = gt + off[3 * k] / s, ni = gi + off[3 * k + 1] / s, nx = gx + off[3 * k + 2] / s;
                if (nt < 0 || nt >= Tg || ni < 0 || ni >= ILg || nx < 0 || nx >= XLg) continue;
                int64_t jn = (nt * ILg + ni) * XLg + nx;
                if (literal) {
                    double sg = sgn(Em[j] - w[k] * Em[jn]);
                    gEm[j] += coef * sg;
                    gEm[jn] -= coef * w[k] * sg;
                } else {
                    double sg = sgn(Em[j] - Em[jn]);
                    gEm[j] += coef * w[k] * sg;
                    gEm[jn] -= coef * w[k] * sg;
                }
            }
        }
    }
}

/* Full backward: gV = dL/dV for L = sum gS * S, recomputing every forward
 * quantity from V, with a stencil per plane (as in orc_dcs_planes) and the
 * weights re-adapted every N inline sections (as in
 * orc_fusion_weights_sections; N = 0: one fit).  Also returns the forward's
 * W [K][3] and fallback flags [K]. */
int orc_backward_ex(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int feature,
                    const int* q3,
                    const int32_t* off_all, const double* w_all, int literal, int mode, const double* wfix,
                    double delta, const float* D, const uint8_t* mask, int64_t N, const float* gS, double* gV,
                    double* W_out, int* fallback_out, int nthreads) {
    int rc = check_spec(T, IL, XL, n, s, window);
    if (rc) return rc;
    if (N < 0 || (feature != 0 && feature != 1)) return ORC_EARG;
    {
        int base = 0;
        for (int m = 0; m < 3; m++) {
            if (check_stencil(s, q3[m], off_all + 3 * base)) return ORC_EARG;
            base += q3[m];
        }
    }
    int64_t Tg = ceil_div(T, s), ILg = ceil_div(IL, s), XLg = ceil_div(XL, s);
    int64_t G = Tg * ILg * XLg, NV = T * IL * XL, K = orc_fuse_groups(ILg, N);
    double* E = (double*)malloc(sizeof(double) * 3 * G);
    double* Sm = (double*)malloc(sizeof(double) * 3 * G);
    double* gSm = (double*)malloc(sizeof(double) * 3 * G);
    double* gE = (double*)malloc(sizeof(double) * 3 * G);
    double* cell = (double*)calloc((size_t)G, sizeof(double));
    double* W = (double*)malloc(sizeof(double) * 3 * K);
    double* st = (double*)malloc(sizeof(double) * 11 * K);
    double* gW = (double*)calloc((size_t)(3 * K), sizeof(double));
    int* fb = (int*)malloc(sizeof(int) * K);
    if (!E || !Sm || !gSm || !gE || !cell || !W || !st || !gW || !fb) { rc = ORC_ENOMEM; goto done; }
    rc = orc_features_ex(V, T, IL, XL, n, s, window, feature, E, nthreads);
    if (rc) goto done;
    orc_dcs_planes(E, Tg, ILg, XLg, s, q3, off_all, w_all, literal, Sm);
    rc = orc_fusion_weights_sections(Sm, Tg, ILg, XLg, D, mask, mode, wfix, delta, N, W, fb, st);
    if (rc) goto done;
    if (W_out) memcpy(W_out, W, sizeof(double) * 3 * K);
    if (fallback_out) memcpy(fallback_out, fb, sizeof(int) * K);
    /* adjoint of the combine step: per-cell sums of gS */
    for (int64_t t = 0; t < T; t++)
        for (int64_t i = 0; i < IL; i++)
            for (int64_t x = 0; x < XL; x++)
                cell[(cell_of(t, s, Tg) * ILg + cell_of(i, s, ILg)) * XLg + cell_of(x, s, XLg)] +=
                    (double)gS[(t * IL + i) * XL + x];
    for (int m = 0; m < 3; m++)
        for (int64_t j = 0; j < G; j++) {
            int64_t k = N > 0 ? ((j / XLg) % ILg) / N : 0;
            gSm[m * G + j] = W[3 * k + m] * cell[j];
            gW[3 * k + m] += Sm[m * G + j] * cell[j];
        }
    if (mode == 2) {
        /* adjoint of each group's W = (G + delta I)^{-1} p through G and p (D held fixed) */
        for (int64_t k = 0; k < K; k++) {
            if (fb[k]) continue;
            const double* a = st + 11 * k;
            double A[9] = {a[0] + delta, a[1], a[2], a[1], a[3] + delta, a[4], a[2], a[4], a[5] + delta};
            double lam[3];
            chol3_solve(A, gW + 3 * k, lam);
            const double* Wk = W + 3 * k;
            for (int64_t j = 0; j < G; j++) {
                int64_t gi = (j / XLg) % ILg;
                if (N > 0 && (gi < k * N || gi >= (k + 1) * N)) continue;
                if (mask && !mask[j]) continue;
                double u[3] = {Sm[j], Sm[G + j], Sm[2 * G + j]};
                double r = (double)D[j] - (Wk[0] * u[0] + Wk[1] * u[1] + Wk[2] * u[2]);
                double lu = lam[0] * u[0] + lam[1] * u[1] + lam[2] * u[2];
                for (int m = 0; m < 3; m++) gSm[m * G + j] += lam[m] * r - Wk[m] * lu;
            }
        }
    }
    dcs_adjoint(E, gSm, Tg, ILg, XLg, s, q3, off_all, w_all, literal, gE);
    /* spectral adjoint with overlap-add into per-thread copies of gV */
    {
        orc_tables tb;
        if (tables_init(&tb, n, window)) { tables_free(&tb); rc = ORC_ENOMEM; goto done; }
        int nt_ = 1;
        set_threads(nthreads);
#ifdef _OPENMP
        nt_ = omp_get_max_threads();
#endif
        double* part = (double*)calloc((size_t)nt_ * (size_t)NV, sizeof(double));
        if (!part) { tables_free(&tb); rc = ORC_ENOMEM; goto done; }
        int fail = 0;
#pragma omp parallel num_threads(nt_)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* acc = part + (size_t)tid * (size_t)NV;
            orc_work wk;
            int ok = work_init(&wk, n) == ORC_OK;
            if (!ok) {
#pragma omp atomic write
                fail = 1;
            }
#pragma omp for schedule(static)
            for (int64_t j = 0; j < G; j++) {
                if (!ok) continue;
                int64_t gt = j / (ILg * XLg), gi = (j / XLg) % ILg, gx = j % XLg;
                double ge[3] = {gE[j], gE[G + j], gE[2 * G + j]};
                if (ge[0] == 0.0 && ge[1] == 0.0 && ge[2] == 0.0) continue;
                window_spectrum(V, T, IL, XL, &tb, gt * s, gi * s, gx * s, &wk);
                window_adjoint(&tb, ge, feature, &wk);
                int half = n / 2;
                for (int at = 0; at < n; at++) {
                    int64_t pt = reflect_index(gt * s - half + at, T);
                    for (int ai = 0; ai < n; ai++) {
                        int64_t pi = reflect_index(gi * s - half + ai, IL);
                        for (int ax = 0; ax < n; ax++) {
                            int64_t px = reflect_index(gx * s - half + ax, XL);
                            acc[(pt * IL + pi) * XL + px] += wk.yr[((int64_t)at * n + ai) * n + ax];
                        }
                    }
                }
            }
            work_free(&wk);
        }
        for (int64_t v = 0; v < NV; v++) {
            double sacc = 0.0;
            for (int t = 0; t < nt_; t++) sacc += part[(size_t)t * (size_t)NV + v];
            gV[v] = sacc;
        }
        free(part);
        tables_free(&tb);
        if (fail) rc = ORC_ENOMEM;
    }
done:
    free(E); free(Sm); free(gSm); free(gE); free(cell); free(W); free(st); free(gW); free(fb);
    return rc;
}

/* orc_backward_ex with one stencil shared by the three planes and one fit. */
int orc_backward(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int q,
                 const int32_t* off, const double* w, int literal, int mode, const double* wfix, double delta,
                 const float* D, const uint8_t* mask, const float* gS, double* gV, double* W_out,
                 int* fallback_out, int nthreads) {
    if (q <= 0) return ORC_EARG;
    int q3[3] = {q, q, q};
    int32_t* off3 = (int32_t*)malloc(sizeof(int32_t) * 9 * q);
    double* w3 = (double*)malloc(sizeof(double) * 3 * q);
    if (!off3 || !w3) { free(off3); free(w3); return ORC_ENOMEM; }
    for (int m = 0; m < 3; m++) {
        memcpy(off3 + 3 * q * m, off, sizeof(int32_t) * 3 * q);
        memcpy(w3 + q * m, w, sizeof(double) * q);
    }
    int rc = orc_backward_ex(V, T, IL, XL, n, s, window, 0, q3, off3, w3, literal, mode, wfix, delta, D, mask, 0, gS,
                             gV, W_out, fallback_out, nthreads);
    free(off3);
    free(w3);
    return rc;
}

/* gV at a list of voxels p[cnt][3] for equal (mode 0) or fixed (mode 1)
 * fusion, where the weights do not depend on V.  Only the windows that cover
 * each voxel, and the features of their stencil neighbourhoods, are computed. */
int orc_backward_at(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int q,
                    const int32_t* off, const double* w, int literal, int mode, const double* wfix,
                    const float* gS, const int64_t* pts, int64_t cnt, double* gV, int nthreads) {
    int rc = check_spec(T, IL, XL, n, s, window);
    if (rc) return rc;
    if (check_stencil(s, q, off)) return ORC_EARG;
    if (mode != 0 && mode != 1) return ORC_EARG;
    if (mode == 1 && !wfix) return ORC_EARG;
    double W[3];
    if (mode == 0) W[0] = W[1] = W[2] = 1.0 / 3.0;
    else { W[0] = wfix[0]; W[1] = wfix[1]; W[2] = wfix[2]; }
    int64_t N3[3] = {T, IL, XL};
    int64_t Ng[3] = {ceil_div(T, s), ceil_div(IL, s), ceil_div(XL, s)};
    for (int64_t j = 0; j < cnt; j++)
        for (int a = 0; a < 3; a++)
            if (pts[3 * j + a] < 0 || pts[3 * j + a] >= N3[a]) return ORC_EARG;
    int reach = 0; /* stencil reach in grid units */
    for (int k = 0; k < 3 * q; k++) {
        int v = abs(off[k]) / s;
        if (v > reach) reach = v;
    }
    orc_tables tb;
    if (tables_init(&tb, n, window)) { tables_free(&tb); return ORC_ENOMEM; }
    int fail = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        orc_work wk;
        int ok = work_init(&wk, n) == ORC_OK;
        /* per axis: the (grid index, window sample) pairs whose reflected position is the voxel */
        int64_t* gl[3];
        int* al[3];
        int cntl[3];
        for (int a = 0; a < 3; a++) {
            gl[a] = (int64_t*)malloc(sizeof(int64_t) * (size_t)(Ng[a] * n));
            al[a] = (int*)malloc(sizeof(int) * (size_t)(Ng[a] * n));
            if (!gl[a] || !al[a]) ok = 0;
        }
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < cnt; j++) {
            if (!ok) continue;
            int64_t lo[3], hi[3], bx[3];
            for (int a = 0; a < 3; a++) {
                cntl[a] = 0;
                lo[a] = Ng[a];
                hi[a] = -1;
                for (int64_t g = 0; g < Ng[a]; g++)
                    for (int s_ = 0; s_ < n; s_++)
                        if (reflect_index(g * s - n / 2 + s_, N3[a]) == pts[3 * j + a]) {
                            gl[a][cntl[a]] = g;
                            al[a][cntl[a]] = s_;
                            cntl[a]++;
                            if (g < lo[a]) lo[a] = g;
                            if (g > hi[a]) hi[a] = g;
                        }
                /* features are needed at covering windows and their neighbours, and at the
                   neighbours' neighbours' centres through Q and sgn terms of g - o */
                lo[a] -= reach;
                hi[a] += reach;
                if (lo[a] < 0) lo[a] = 0;
                if (hi[a] > Ng[a] - 1) hi[a] = Ng[a] - 1;
                bx[a] = hi[a] - lo[a] + 1;
            }
            int64_t nb = bx[0] * bx[1] * bx[2];
            double* Eb = (double*)malloc(sizeof(double) * 3 * (size_t)nb);
            if (!Eb) {
#pragma omp atomic write
                fail = 1;
                continue;
            }
            for (int64_t b = 0; b < nb; b++) {
                int64_t bt = b / (bx[1] * bx[2]), bi = (b / bx[2]) % bx[1], bxx = b % bx[2];
                window_spectrum(V, T, IL, XL, &tb, (lo[0] + bt) * s, (lo[1] + bi) * s, (lo[2] + bxx) * s, &wk);
                window_features(&tb, &wk, 0, Eb + 3 * b);
            }
#define EB(gt_, gi_, gx_, m_) Eb[3 * ((((gt_) - lo[0]) * bx[1] + ((gi_) - lo[1])) * bx[2] + ((gx_) - lo[2])) + (m_)]
            double total = 0.0;
            /* visit each covering window once; sum over its matching samples */
            for (int it = 0; it < cntl[0]; it++) {
                if (it > 0 && gl[0][it] == gl[0][it - 1]) continue;
                for (int ii = 0; ii < cntl[1]; ii++) {
                    if (ii > 0 && gl[1][ii] == gl[1][ii - 1]) continue;
                    for (int ix = 0; ix < cntl[2]; ix++) {
                        if (ix > 0 && gl[2][ix] == gl[2][ix - 1]) continue;
                        int64_t gt = gl[0][it], gi = gl[1][ii], gx = gl[2][ix];
                        /* gE at window g: own term and the terms where g is the neighbour of g - o */
                        double ge[3] = {0, 0, 0};
                        int Qg = 0;
                        for (int k = 0; k < q; k++) {
                            int64_t nt = gt + off[3 * k] / s, ni = gi + off[3 * k + 1] / s, nx = gx + off[3 * k + 2] / s;
                            if (nt >= 0 && nt < Ng[0] && ni >= 0 && ni < Ng[1] && nx >= 0 && nx < Ng[2]) Qg++;
                        }
                        /* cell sum of gS at a grid point */
#define CELLSUM(ct_, ci_, cx_, out_)                                                                  \
    do {                                                                                              \
        double cs_ = 0.0;                                                                             \
        int64_t c3_[3] = {(ct_), (ci_), (cx_)};                                                       \
        int64_t vl_[3], vh_[3];                                                                       \
        for (int a_ = 0; a_ < 3; a_++) {                                                              \
            vl_[a_] = c3_[a_] * s - s;                                                                \
            vh_[a_] = c3_[a_] * s + s;                                                                \
            if (vl_[a_] < 0) vl_[a_] = 0;                                                             \
            if (vh_[a_] > N3[a_] - 1) vh_[a_] = N3[a_] - 1;                                           \
        }                                                                                             \
        for (int64_t vt_ = vl_[0]; vt_ <= vh_[0]; vt_++) {                                            \
            if (cell_of(vt_, s, Ng[0]) != c3_[0]) continue;                                           \
            for (int64_t vi_ = vl_[1]; vi_ <= vh_[1]; vi_++) {                                        \
                if (cell_of(vi_, s, Ng[1]) != c3_[1]) continue;                                       \
                for (int64_t vx_ = vl_[2]; vx_ <= vh_[2]; vx_++) {                                    \
                    if (cell_of(vx_, s, Ng[2]) != c3_[2]) continue;                                   \
                    cs_ += (double)gS[(vt_ * IL + vi_) * XL + vx_];                                   \
                }                                                                                     \
            }                                                                                         \
        }                                                                                             \
        (out_) = cs_;                                                                                 \
    } while (0)
                        double cg;
                        CELLSUM(gt, gi, gx, cg);
                        if (Qg) {
                            for (int k = 0; k < q; k++) {
                                int64_t nt = gt + off[3 * k] / s, ni = gi + off[3 * k + 1] / s, nx = gx + off[3 * k + 2] / s;
                                if (nt < 0 || nt >= Ng[0] || ni < 0 || ni >= Ng[1] || nx < 0 || nx >= Ng[2]) continue;
                                for (int m = 0; m < 3; m++) {
                                    double e0 = EB(gt, gi, gx, m), e1 = EB(nt, ni, nx, m);
                                    double sg = literal ? sgn(e0 - w[k] * e1) : sgn(e0 - e1);
                                    ge[m] += W[m] * cg / Qg * (literal ? 1.0 : w[k]) * sg;
                                }
                            }
                        }
                        for (int k = 0; k < q; k++) {
                            /* g is the neighbour o of p = g - o */
                            int64_t pt_ = gt - off[3 * k] / s, pi_ = gi - off[3 * k + 1] / s, px_ = gx - off[3 * k + 2] / s;
                            if (pt_ < 0 || pt_ >= Ng[0] || pi_ < 0 || pi_ >= Ng[1] || px_ < 0 || px_ >= Ng[2]) continue;
                            int Qp = 0;
                            for (int k2 = 0; k2 < q; k2++) {
                                int64_t nt = pt_ + off[3 * k2] / s, ni = pi_ + off[3 * k2 + 1] / s, nx = px_ + off[3 * k2 + 2] / s;
                                if (nt >= 0 && nt < Ng[0] && ni >= 0 && ni < Ng[1] && nx >= 0 && nx < Ng[2]) Qp++;
                            }
                            double cp;
                            CELLSUM(pt_, pi_, px_, cp);
                            for (int m = 0; m < 3; m++) {
                                double e0 = EB(pt_, pi_, px_, m), e1 = EB(gt, gi, gx, m);
                                double sg = literal ? sgn(e0 - w[k] * e1) : sgn(e0 - e1);
                                ge[m] -= W[m] * cp / Qp * w[k] * sg;
                            }
                        }
#undef CELLSUM
                        if (ge[0] == 0.0 && ge[1] == 0.0 && ge[2] == 0.0) continue;
                        window_spectrum(V, T, IL, XL, &tb, gt * s, gi * s, gx * s, &wk);
                        window_adjoint(&tb, ge, 0, &wk);
                        for (int jt = 0; jt < cntl[0]; jt++) {
                            if (gl[0][jt] != gt) continue;
                            for (int ji = 0; ji < cntl[1]; ji++) {
                                if (gl[1][ji] != gi) continue;
                                for (int jx = 0; jx < cntl[2]; jx++) {
                                    if (gl[2][jx] != gx) continue;
                                    total += wk.yr[((int64_t)al[0][jt] * n + al[1][ji]) * n + al[2][jx]];
                                }
                            }
                        }
                    }
                }
            }
#undef EB
            gV[j] = total;
            free(Eb);
        }
        for (int a = 0; a < 3; a++) { free(gl[a]); free(al[a]); }
        work_free(&wk);
    }
    tables_free(&tb);
    return fail ? ORC_ENOMEM : ORC_OK;
}
