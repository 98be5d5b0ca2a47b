// sal_api.cpp -- the C ABI of libsal: argument validation on the host, then launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
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

// Stencil in grid units with resolved weights.
sal_status make_stencil(const sal_stencil* st, int s, DcsStencil* out) {
    if (!st) return fail(SAL_ERR_ARG, "stencil is NULL");
    if (st->q < 1 || st->q > SAL_MAX_STENCIL) return fail(SAL_ERR_ARG, "stencil size must be 1..SAL_MAX_STENCIL");
    if (!st->offsets) return fail(SAL_ERR_ARG, "stencil offsets are NULL");
    if (s < 1) return fail(SAL_ERR_ARG, "stride must be >= 1");
    out->q = st->q;
    out->literal = st->literal ? 1 : 0;
    out->reach[0] = out->reach[1] = out->reach[2] = 0;
    int d = 0;
    for (int k = 0; k < st->q; k++) {
        for (int a = 0; a < 3; a++) {
            const int v = st->offsets[3 * k + a];
            if (v % s != 0) return fail(SAL_ERR_ARG, "stencil offsets must be multiples of the stride");
            if (std::abs(v) > (1 << 24)) return fail(SAL_ERR_ARG, "stencil offset too large");
            out->o[k][a] = v / s;
            out->reach[a] = std::max(out->reach[a], std::abs(v / s));
            d = std::abs(v) > d ? std::abs(v) : d;
        }
    }
    if (d == 0) return fail(SAL_ERR_ARG, "stencil offsets are all zero");
    if (st->weights) {
        for (int k = 0; k < st->q; k++) out->w[k] = st->weights[k];
    } else {
        // Gaussian in the offset length, sigma = the stencil's Chebyshev reach, mean 1
        double w[SAL_MAX_STENCIL], sum = 0.0;
        for (int k = 0; k < st->q; k++) {
            double r2 = 0.0;
            for (int a = 0; a < 3; a++) r2 += double(st->offsets[3 * k + a]) * st->offsets[3 * k + a];
            w[k] = std::exp(-r2 / (2.0 * double(d) * d));
            sum += w[k];
        }
        for (int k = 0; k < st->q; k++) out->w[k] = float(w[k] * st->q / sum);
    }
    for (int k = st->q; k < SAL_MAX_STENCIL; k++) {
        out->o[k][0] = out->o[k][1] = out->o[k][2] = 0;
        out->w[k] = 0.f;
        out->mirror[k] = 0;
    }
    // one-to-one pairing of each offset with an unused copy of its negation; equal offsets
    // are interchangeable, so the greedy pairing succeeds whenever the stencil equals its
    // reflection as a multiset
    bool used[SAL_MAX_STENCIL] = {};
    out->symmetric = 1;
    for (int k = 0; k < st->q && out->symmetric; k++) {
        int m = -1;
        for (int k2 = 0; k2 < st->q && m < 0; k2++)
            if (!used[k2] && out->o[k2][0] == -out->o[k][0] && out->o[k2][1] == -out->o[k][1] &&
                out->o[k2][2] == -out->o[k][2])
                m = k2;
        if (m < 0) {
            out->symmetric = 0;
        } else {
            used[m] = true;
            out->mirror[k] = m;
        }
    }
    if (!out->symmetric)
        for (int k = 0; k < st->q; k++) out->mirror[k] = 0;
    return SAL_OK;
}

static sal_status check_fusion(const sal_fusion* f, const float* D) {
    if (!f) return fail(SAL_ERR_ARG, "fusion is NULL");
    if (f->mode != SAL_FUSE_EQUAL && f->mode != SAL_FUSE_FIXED && f->mode != SAL_FUSE_ADAPT_LS)
        return fail(SAL_ERR_ARG, "unknown fusion mode");
    if (f->mode == SAL_FUSE_ADAPT_LS) {
        if (!D) return fail(SAL_ERR_ARG, "ADAPT_LS needs a desired map D");
        if (!(f->delta >= 0.0) || !std::isfinite(f->delta)) return fail(SAL_ERR_ARG, "delta must be finite and >= 0");
    }
    if (f->mode == SAL_FUSE_FIXED)
        for (int m = 0; m < 3; m++)
            if (!std::isfinite(f->w_fixed[m])) return fail(SAL_ERR_ARG, "fixed weights must be finite");
    return SAL_OK;
}

sal_status check_fusion_args(const sal_fusion* f, const float* D) { return check_fusion(f, D); }

}  // namespace sal

using namespace sal;

extern "C" {

sal_status sal_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec,
                             const int32_t* centers, int64_t cnt, float* F_out, sal_stream stream) {
    if (!spec) return fail(SAL_ERR_ARG, "spec is NULL");
    sal_spec sp = *spec;
    sp.s = 1;
    sp.precision = SAL_PREC_FP32;
    sal_status st = check_spec(&sp, T, IL, XL);
    if (st) return st;
    if (cnt < 0) return fail(SAL_ERR_ARG, "negative centre count");
    if (cnt > 0 && (!V || !centers || !F_out)) return fail(SAL_ERR_ARG, "NULL buffer");
    return launch_local_spectra(V, T, IL, XL, sp.n, sp.window, centers, cnt, F_out, (hipStream_t)stream);
}

sal_status sal_project(const float* V, int64_t T, int64_t IL, int64_t XL, const sal_spec* spec, float* E_out,
                       sal_stream stream) {
    sal_status st = check_spec(spec, T, IL, XL);
    if (st) return st;
    if (!V || !E_out) return fail(SAL_ERR_ARG, "NULL buffer");
    const Tables* tb = nullptr;
    if ((st = get_tables(spec->n, spec->window, &tb))) return st;
    switch (spec->precision) {
        case SAL_PREC_FP32:
            return launch_project_fp32(V, T, IL, XL, spec->n, spec->s, tb, E_out, (hipStream_t)stream);
        default:
            return launch_project_lowp(V, T, IL, XL, spec->n, spec->s, spec->precision, tb, E_out,
                                       (hipStream_t)stream);
    }
}

sal_status sal_center_surround(const float* E, int64_t Tg, int64_t ILg, int64_t XLg, int32_t s,
                               const sal_stencil* stencil, float* Sm_out, sal_stream stream) {
    if (!E || !Sm_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (E == Sm_out) return fail(SAL_ERR_ARG, "Sm_out must not alias E");
    if (Tg < 0 || ILg < 0 || XLg < 0) return fail(SAL_ERR_SHAPE, "negative grid extent");
    DcsStencil ds;
    sal_status st = make_stencil(stencil, s, &ds);
    if (st) return st;
    return launch_dcs(E, Sm_out, Tg, ILg, XLg, ds, (hipStream_t)stream);
}

size_t sal_fuse_workspace_size(int64_t, int64_t, int64_t) { return fuse_adjoint_workspace_bytes(); }

sal_status sal_fuse(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion, const float* D,
                    const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s, double* W_out, float* S_out,
                    void* ws, size_t ws_bytes, sal_stream stream) {
    sal_status st = check_fusion(fusion, D);
    if (st) return st;
    if (!Sm || !W_out || !S_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (T < 1 || IL < 1 || XL < 1) return fail(SAL_ERR_SHAPE, "empty volume");
    if ((st = check_grid(T, IL, XL, s, Tg, ILg, XLg))) return st;
    if (fusion->mode == SAL_FUSE_ADAPT_LS && (!ws || ws_bytes < fuse_workspace_bytes()))
        return fail(SAL_ERR_NOMEM, "workspace smaller than sal_fuse_workspace_size()");
    return launch_fuse(Sm, Tg, ILg, XLg, *fusion, D, mask, T, IL, XL, s, W_out, S_out, (double*)ws,
                       (hipStream_t)stream);
}

}  // extern "C"
