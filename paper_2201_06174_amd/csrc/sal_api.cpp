// sal_api.cpp -- the C ABI of libsal: argument validation on the host, then launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "sal_aux.h"
#include "sal_internal.h"

namespace sal {

static sal_status check_grid(int64_t T, int64_t IL, int64_t XL, int s, int64_t Tg, int64_t ILg, int64_t XLg) {
    if (s < 1) return fail(SAL_ERR_ARG, "stride must be >= 1");
    if (ceil_div(T, s) != Tg || ceil_div(IL, s) != ILg || ceil_div(XL, s) != XLg)
        return fail(SAL_ERR_SHAPE, "grid extents must equal ceil(N / s) of the volume extents");
    return SAL_OK;
}

// Offsets in grid units and resolved weights of one stencil (no per-plane part).
static sal_status resolve_stencil(const sal_stencil* st, int s, int (*o)[3], float* w) {
    if (st->q < 1 || st->q > SAL_MAX_STENCIL) return fail(SAL_ERR_ARG, "stencil size must be 1..SAL_MAX_STENCIL");
    if (!st->offsets) return fail(SAL_ERR_ARG, "stencil offsets are NULL");
    int d = 0;
    for (int k = 0; k < st->q; k++) {
        for (int a = 0; a < 3; a++) {
            const int v = st->offsets[3 * k + a];
            if (v % s != 0) return fail(SAL_ERR_ARG, "stencil offsets must be multiples of the stride");
            if (std::abs(v) > (1 << 24)) return fail(SAL_ERR_ARG, "stencil offset too large");
            o[k][a] = v / s;
            d = std::abs(v) > d ? std::abs(v) : d;
        }
    }
    if (d == 0) return fail(SAL_ERR_ARG, "stencil offsets are all zero");
    if (st->weights) {
        for (int k = 0; k < st->q; k++) {
            if (!std::isfinite(st->weights[k])) return fail(SAL_ERR_ARG, "stencil weights must be finite");
            w[k] = st->weights[k];
        }
    } else {
        // Gaussian in the offset length, sigma = the stencil's Chebyshev reach, mean 1
        double g[SAL_MAX_STENCIL], sum = 0.0;
        for (int k = 0; k < st->q; k++) {
            double r2 = 0.0;
            for (int a = 0; a < 3; a++) r2 += double(st->offsets[3 * k + a]) * st->offsets[3 * k + a];
            g[k] = std::exp(-r2 / (2.0 * double(d) * d));
            sum += g[k];
        }
        for (int k = 0; k < st->q; k++) w[k] = float(g[k] * st->q / sum);
    }
    return SAL_OK;
}

// Stencil in grid units with resolved weights; per-plane stencils become the union of their
// offsets with a plane mask and per-plane weights per union entry.
sal_status make_stencil(const sal_stencil* st, int s, DcsStencil* out) {
    if (!st) return fail(SAL_ERR_ARG, "stencil is NULL");
    if (s < 1) return fail(SAL_ERR_ARG, "stride must be >= 1");
    std::memset(out, 0, sizeof(*out));
    out->literal = st->literal ? 1 : 0;
    sal_status rc;
    if (!st->per_plane) {
        out->planes = 0;
        out->q = st->q;
        if ((rc = resolve_stencil(st, s, out->o, out->w))) return rc;
        for (int k = 0; k < out->q; k++) {
            out->member[k] = 7;
            for (int m = 0; m < 3; m++) out->wp[k][m] = out->w[k];
        }
    } else {
        out->planes = 1;
        int q = 0;
        for (int m = 0; m < 3; m++) {
            const sal_stencil& pm = st->per_plane[m];
            if (pm.per_plane) return fail(SAL_ERR_ARG, "a per-plane stencil cannot nest further stencils");
            int o[SAL_MAX_STENCIL][3];
            float w[SAL_MAX_STENCIL];
            if ((rc = resolve_stencil(&pm, s, o, w))) return rc;
            for (int k = 0; k < pm.q; k++) {
                // the first union entry with this offset that plane m does not use yet (an offset
                // listed twice in one plane's stencil counts twice, as it does in a shared stencil)
                int u = -1;
                for (int e = 0; e < q && u < 0; e++)
                    if (out->o[e][0] == o[k][0] && out->o[e][1] == o[k][1] && out->o[e][2] == o[k][2] &&
                        !((out->member[e] >> m) & 1u))
                        u = e;
                if (u < 0) {
                    if (q == SAL_MAX_STENCIL)
                        return fail(SAL_ERR_ARG, "the per-plane stencils hold more than SAL_MAX_STENCIL distinct offsets");
                    u = q++;
                    for (int a = 0; a < 3; a++) out->o[u][a] = o[k][a];
                }
                out->member[u] |= (unsigned char)(1u << m);
                out->wp[u][m] = w[k];
            }
        }
        out->q = q;
    }
    for (int k = 0; k < out->q; k++)
        for (int a = 0; a < 3; a++) out->reach[a] = std::max(out->reach[a], std::abs(out->o[k][a]));
    // one-to-one pairing of each offset with an unused copy of its negation that belongs to the
    // same planes; equal offsets are interchangeable, so the greedy pairing succeeds whenever
    // every plane's stencil equals its reflection as a multiset
    bool used[SAL_MAX_STENCIL] = {};
    out->symmetric = 1;
    for (int k = 0; k < out->q && out->symmetric; k++) {
        int m = -1;
        for (int k2 = 0; k2 < out->q && m < 0; k2++)
            if (!used[k2] && out->o[k2][0] == -out->o[k][0] && out->o[k2][1] == -out->o[k][1] &&
                out->o[k2][2] == -out->o[k][2] && out->member[k2] == out->member[k])
                m = k2;
        if (m < 0) {
            out->symmetric = 0;
        } else {
            used[m] = true;
            out->mirror[k] = m;
        }
    }
    if (!out->symmetric)
        for (int k = 0; k < out->q; k++) out->mirror[k] = 0;
    return SAL_OK;
}

static sal_status check_fusion(const sal_fusion* f, const float* D) {
    if (!f) return fail(SAL_ERR_ARG, "fusion is NULL");
    if (f->mode != SAL_FUSE_EQUAL && f->mode != SAL_FUSE_FIXED && f->mode != SAL_FUSE_ADAPT_LS &&
        !fuse_sequential(f->mode))
        return fail(SAL_ERR_ARG, "unknown fusion mode");
    if (fuse_sequential(f->mode)) {
        if (!D) return fail(SAL_ERR_ARG, "LMS / NLMS / RLS need a desired map D");
        for (int m = 0; m < 3; m++)
            if (!std::isfinite(f->w_fixed[m])) return fail(SAL_ERR_ARG, "starting weights must be finite");
        if (f->passes < 1) return fail(SAL_ERR_ARG, "passes must be >= 1");
        if (f->mode != SAL_FUSE_RLS && (!(f->mu > 0.0) || !std::isfinite(f->mu)))
            return fail(SAL_ERR_ARG, "mu must be finite and > 0");
        if (f->mode == SAL_FUSE_NLMS && (!(f->eps >= 0.0) || !std::isfinite(f->eps)))
            return fail(SAL_ERR_ARG, "eps must be finite and >= 0");
        if (f->mode == SAL_FUSE_RLS && (!(f->lambda > 0.0) || f->lambda > 1.0))
            return fail(SAL_ERR_ARG, "lambda must lie in (0, 1]");
        if (f->mode == SAL_FUSE_RLS && (!(f->delta > 0.0) || !std::isfinite(f->delta)))
            return fail(SAL_ERR_ARG, "RLS needs a finite delta > 0 (P0 = I / delta)");
    }
    if (f->mode == SAL_FUSE_ADAPT_LS) {
        if (!D) return fail(SAL_ERR_ARG, "ADAPT_LS needs a desired map D");
        if (!(f->delta >= 0.0) || !std::isfinite(f->delta)) return fail(SAL_ERR_ARG, "delta must be finite and >= 0");
    }
    if (f->mode == SAL_FUSE_FIXED)
        for (int m = 0; m < 3; m++)
            if (!std::isfinite(f->w_fixed[m])) return fail(SAL_ERR_ARG, "fixed weights must be finite");
    if (f->sections < 0) return fail(SAL_ERR_ARG, "sections must be >= 0");
    return SAL_OK;
}

sal_status check_fusion_args(const sal_fusion* f, const float* D) { return check_fusion(f, D); }

}  // namespace sal

using namespace sal;

extern "C" {

static sal_status sal_local_spectra_body(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                             const int32_t* centers, int64_t cnt, float* F_out, sal_stream stream) {
    if (!spec) return fail(SAL_ERR_ARG, "spec is NULL");
    sal_spec sp = *spec;
    sp.s = 1;
    sp.precision = SAL_PREC_FP32;
    sp.feature = SAL_FEATURE_MAGNITUDE;
    sal_status st = check_spec(&sp, T, IL, XL);
    if (st) return st;
    if (cnt < 0) return fail(SAL_ERR_ARG, "negative centre count");
    if (cnt > 0 && (!V || !centers || !F_out)) return fail(SAL_ERR_ARG, "NULL buffer");
    return launch_local_spectra(V, T, IL, XL, sp.n, sp.window, centers, cnt, F_out, (hipStream_t)stream);
}

sal_status sal_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                             const int32_t* centers, int64_t cnt, float* F_out, sal_stream stream) {
    CallScope cs("sal_local_spectra");
    return cs.done(sal_local_spectra_body(V, T, IL, XL, spec, centers, cnt, F_out, stream));
}

static sal_status sal_project_body(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec, float* E_out,
                       sal_stream stream) {
    sal_status st = check_spec(spec, T, IL, XL);
    if (st) return st;
    if (!V || !E_out) return fail(SAL_ERR_ARG, "NULL buffer");
    const Tables* tb = nullptr;
    if ((st = get_tables((hipStream_t)stream, spec->n, spec->window, &tb))) return st;
    switch (spec->precision) {
        case SAL_PREC_FP32:
            return launch_project_fp32(V, T, IL, XL, spec->n, spec->s, spec->feature, tb, E_out, (hipStream_t)stream);
        default:
            return launch_project_lowp(V, T, IL, XL, spec->n, spec->s, spec->precision, tb, E_out,
                                       (hipStream_t)stream);
    }
}

sal_status sal_project(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec, float* E_out,
                       sal_stream stream) {
    CallScope cs("sal_project");
    return cs.done(sal_project_body(V, T, IL, XL, spec, E_out, stream));
}

static sal_status sal_center_surround_body(const float* E, int64_t Tg, int64_t ILg, int64_t XLg, int32_t s,
                               const sal_stencil* stencil, float* Sm_out, sal_stream stream) {
    if (!E || !Sm_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (E == Sm_out) return fail(SAL_ERR_ARG, "Sm_out must not alias E");
    if (Tg < 0 || ILg < 0 || XLg < 0) return fail(SAL_ERR_SHAPE, "negative grid extent");
    DcsStencil ds;
    sal_status st = make_stencil(stencil, s, &ds);
    if (st) return st;
    return launch_dcs(E, Sm_out, Tg, ILg, XLg, ds, (hipStream_t)stream);
}

sal_status sal_center_surround(const float* E, int64_t Tg, int64_t ILg, int64_t XLg, int32_t s,
                               const sal_stencil* stencil, float* Sm_out, sal_stream stream) {
    CallScope cs("sal_center_surround");
    return cs.done(sal_center_surround_body(E, Tg, ILg, XLg, s, stencil, Sm_out, stream));
}

int64_t sal_fuse_groups(const sal_fusion* fusion, int64_t ILg) {
    if (!fusion || ILg < 0 || fusion->sections < 0) return 0;
    return fuse_groups(fusion->sections, ILg);
}

static size_t fuse_ws_bytes(const sal_fusion* f, int64_t Tg, int64_t ILg, int64_t XLg) {
    const int64_t K = f && f->sections > 0 ? fuse_groups(f->sections, ILg) : 1;
    if (f && fuse_sequential(f->mode)) return seq_workspace_bytes(Tg * ILg * XLg, K);
    return fuse_workspace_bytes(K);
}

size_t sal_fuse_workspace_size(int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion) {
    if (Tg < 0 || ILg < 0 || XLg < 0) return 0;
    return fuse_ws_bytes(fusion, Tg, ILg, XLg);
}

sal_status sal_line_template(const int32_t* dir, int32_t length, double sigma, int32_t* offsets_out,
                             float* weights_out) {
    if (!dir || !offsets_out || !weights_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (length < 1 || length > SAL_MAX_STENCIL / 2) return fail(SAL_ERR_ARG, "length must be 1..SAL_MAX_STENCIL/2");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(SAL_ERR_ARG, "sigma must be finite and > 0");
    if (dir[0] == 0 && dir[1] == 0 && dir[2] == 0) return fail(SAL_ERR_ARG, "direction is zero");
    for (int a = 0; a < 3; a++)
        if (std::abs((int64_t)dir[a]) * length > (1 << 24)) return fail(SAL_ERR_ARG, "template reach too large");
    double g[SAL_MAX_STENCIL], sum = 0.0;
    int k = 0;
    for (int side = -1; side <= 1; side += 2)
        for (int i = 1; i <= length; i++) {
            const int j = side < 0 ? -(length + 1 - i) : i;  // -length .. -1, then 1 .. length
            for (int a = 0; a < 3; a++) offsets_out[3 * k + a] = j * dir[a];
            g[k] = std::exp(-double(j) * j / (2.0 * sigma * sigma));
            sum += g[k];
            k++;
        }
    for (int e = 0; e < k; e++) weights_out[e] = float(g[e] * k / sum);
    return SAL_OK;
}

static sal_status sal_fuse_body(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion, const float* D,
                    const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s, double* W_out, float* S_out,
                    void* ws, size_t ws_bytes, sal_stream stream) {
    sal_status st = check_fusion(fusion, D);
    if (st) return st;
    if (!Sm || !W_out || !S_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (T < 1 || IL < 1 || XL < 1) return fail(SAL_ERR_SHAPE, "empty volume");
    if ((st = check_grid(T, IL, XL, s, Tg, ILg, XLg))) return st;
    const bool needs_ws = fusion->mode == SAL_FUSE_ADAPT_LS || fuse_sequential(fusion->mode);
    if (needs_ws && (!ws || ws_bytes < fuse_ws_bytes(fusion, Tg, ILg, XLg)))
        return fail(SAL_ERR_NOMEM, "workspace smaller than sal_fuse_workspace_size()");
    if (fuse_sequential(fusion->mode)) {
        const int64_t K = fuse_groups(fusion->sections, ILg);
        if ((st = launch_seq_adapt(Sm, Tg, ILg, XLg, *fusion, D, mask, W_out, nullptr, 0, nullptr, ws,
                                   (hipStream_t)stream)))
            return st;
        return launch_combine(Sm, Tg, ILg, XLg, K > 1 ? fusion->sections : 0, T, IL, XL, s, W_out, S_out,
                              (hipStream_t)stream);
    }
    return launch_fuse(Sm, Tg, ILg, XLg, *fusion, D, mask, T, IL, XL, s, W_out, S_out, (double*)ws,
                       (hipStream_t)stream);
}

sal_status sal_fuse(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion, const float* D,
                    const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s, double* W_out, float* S_out,
                    void* ws, size_t ws_bytes, sal_stream stream) {
    CallScope cs("sal_fuse");
    return cs.done(sal_fuse_body(Sm, Tg, ILg, XLg, fusion, D, mask, T, IL, XL, s, W_out, S_out, ws, ws_bytes, stream));
}

static sal_status sal_adapt_weights_body(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion,
                             const float* D, const uint8_t* mask, double* W_out, float* err2_out, int64_t cap,
                             int64_t* count_out, void* ws, size_t ws_bytes, sal_stream stream) {
    sal_status st = check_fusion(fusion, D);
    if (st) return st;
    if (!fuse_sequential(fusion->mode)) return fail(SAL_ERR_ARG, "sal_adapt_weights takes the LMS, NLMS and RLS modes");
    if (!Sm || !W_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (Tg < 0 || ILg < 0 || XLg < 0) return fail(SAL_ERR_SHAPE, "negative grid extent");
    if (cap < 0 || (cap > 0 && !err2_out)) return fail(SAL_ERR_ARG, "err2_out must hold cap >= 0 values");
    if (!ws || ws_bytes < fuse_ws_bytes(fusion, Tg, ILg, XLg))
        return fail(SAL_ERR_NOMEM, "workspace smaller than sal_fuse_workspace_size()");
    return launch_seq_adapt(Sm, Tg, ILg, XLg, *fusion, D, mask, W_out, cap > 0 ? err2_out : nullptr, cap, count_out,
                            ws, (hipStream_t)stream);
}

sal_status sal_adapt_weights(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion,
                             const float* D, const uint8_t* mask, double* W_out, float* err2_out, int64_t cap,
                             int64_t* count_out, void* ws, size_t ws_bytes, sal_stream stream) {
    CallScope cs("sal_adapt_weights");
    return cs.done(sal_adapt_weights_body(Sm, Tg, ILg, XLg, fusion, D, mask, W_out, err2_out, cap, count_out, ws, ws_bytes, stream));
}

}  // extern "C"
