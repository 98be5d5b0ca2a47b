/* Every routine of the FP64 oracle on small inputs (borders, strides, per-plane stencils,
 * sections, the energy feature, the sequential rules), built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitize.py: any out-of-bounds access, leak or
 * undefined operation aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_window(int n, int window, double* h);
int orc_local_spectra(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int window, const int64_t* centers,
                      int64_t cnt, double* F);
int orc_features_ex(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int feature,
                    double* E, int nthreads);
int orc_features_at_ex(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int feature,
                       const int64_t* g, int64_t cnt, double* E, int nthreads);
int orc_default_weights(int q, const int32_t* off, double* w);
int orc_dcs(const double* E, int64_t Tg, int64_t ILg, int64_t XLg, int s, int q, const int32_t* off, const double* w,
            int literal, double* S);
int orc_dcs_planes(const double* E, int64_t Tg, int64_t ILg, int64_t XLg, int s, const int* q3, const int32_t* off_all,
                   const double* w_all, int literal, double* S);
int orc_line_template(const int32_t* dir, int L, double sigma, int32_t* off, double* w);
int orc_saliency_at(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int q,
                    const int32_t* off, const double* w, int literal, const int64_t* g, int64_t cnt, double* Sm,
                    double* E, int nthreads);
int orc_fusion_weights(const double* Sm, int64_t G, const float* D, const uint8_t* mask, int mode, const double* wfix,
                       double delta, double* W, int* fallback, double* stats);
int orc_fusion_weights_sections(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const float* D,
                                const uint8_t* mask, int mode, const double* wfix, double delta, int64_t N, double* W,
                                int* fallback, double* stats);
int orc_combine(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const double* W, int64_t T, int64_t IL,
                int64_t XL, int s, double* S);
int orc_combine_sections(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const double* W, int64_t N,
                         int64_t T, int64_t IL, int64_t XL, int s, double* S);
int orc_adapt_sequential(const double* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const float* D, const uint8_t* mask,
                         int rule, double mu, double eps, double lambda, double delta, const double* w0, int passes,
                         int64_t N, double* W, int64_t* count, double* err2, int64_t cap);
int orc_backward_ex(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int feature,
                    const int* q3, const int32_t* off_all, const double* w_all, int literal, int mode,
                    const double* wfix, double delta, const float* D, const uint8_t* mask, int64_t N, const float* gS,
                    double* gV, double* W_out, int* fallback_out, int nthreads);
int orc_backward_at(const float* V, int64_t T, int64_t IL, int64_t XL, int n, int s, int window, int q,
                    const int32_t* off, const double* w, int literal, int mode, const double* wfix, const float* gS,
                    const int64_t* pts, int64_t cnt, double* gV, int nthreads);

#define CHECK(x)                                                   \
    do {                                                           \
        int rc_ = (x);                                             \
        if (rc_) {                                                 \
            fprintf(stderr, "%s failed: %d\n", #x, rc_);           \
            return 1;                                              \
        }                                                          \
    } while (0)

static float frand(unsigned* st) {
    *st = *st * 1664525u + 1013904223u;
    return (float)((*st >> 8) & 0xffff) / 32768.0f - 1.0f;
}

int main(void) {
    const int64_t T = 9, IL = 8, XL = 7;
    unsigned st = 12345u;
    float* V = malloc(sizeof(float) * T * IL * XL);
    float* gS = malloc(sizeof(float) * T * IL * XL);
    for (int64_t i = 0; i < T * IL * XL; i++) { V[i] = frand(&st); gS[i] = 0.5f + 0.5f * frand(&st); }
    double h[16];
    CHECK(orc_window(8, 0, h));
    int64_t c[6] = {0, 0, 0, T - 1, IL - 1, XL - 1};
    double* F = malloc(sizeof(double) * 2 * 8 * 8 * 8 * 2);
    CHECK(orc_local_spectra(V, T, IL, XL, 8, 1, c, 2, F));
    for (int s = 1; s <= 3; s++)
        for (int feature = 0; feature < 2; feature++) {
            const int n = 8;
            int64_t Tg = (T + s - 1) / s, ILg = (IL + s - 1) / s, XLg = (XL + s - 1) / s, G = Tg * ILg * XLg;
            double* E = malloc(sizeof(double) * 3 * G);
            double* S = malloc(sizeof(double) * 3 * G);
            double* Sv = malloc(sizeof(double) * T * IL * XL);
            double* gV = malloc(sizeof(double) * T * IL * XL);
            float* D = malloc(sizeof(float) * G);
            uint8_t* mask = malloc(G);
            for (int64_t j = 0; j < G; j++) { D[j] = frand(&st); mask[j] = (uint8_t)(j % 3 != 0); }
            CHECK(orc_features_ex(V, T, IL, XL, n, s, 0, feature, E, 2));
            int64_t g[6] = {0, 0, 0, Tg - 1, ILg - 1, XLg - 1};
            double Eg[6], Sg[6];
            CHECK(orc_features_at_ex(V, T, IL, XL, n, s, 1, feature, g, 2, Eg, 1));
            int32_t off[18] = {s, 0, 0, -s, 0, 0, 0, s, 0, 0, -s, 0, 0, 0, s, 0, 0, -s};
            double w[6];
            CHECK(orc_default_weights(6, off, w));
            CHECK(orc_dcs(E, Tg, ILg, XLg, s, 6, off, w, s == 2, S));
            CHECK(orc_saliency_at(V, T, IL, XL, n, s, 0, 6, off, w, 0, g, 2, Sg, Eg, 1));
            int32_t tmpl[3][3] = {{s, 0, 0}, {0, 0, s}, {s, 0, s}};
            int32_t offp[3 * 4 * 3];
            double wp[12];
            for (int m = 0; m < 3; m++) CHECK(orc_line_template(tmpl[m], 2, 1.0, offp + 12 * m, wp + 4 * m));
            int q3[3] = {4, 4, 4};
            CHECK(orc_dcs_planes(E, Tg, ILg, XLg, s, q3, offp, wp, 0, S));
            double W[3 * 8], stats[11 * 8];
            int fb[8];
            CHECK(orc_fusion_weights(S, G, D, mask, 2, NULL, 1e-6, W, fb, stats));
            CHECK(orc_fusion_weights_sections(S, Tg, ILg, XLg, D, mask, 2, NULL, 1e-6, 1, W, fb, stats));
            CHECK(orc_combine(S, Tg, ILg, XLg, W, T, IL, XL, s, Sv));
            CHECK(orc_combine_sections(S, Tg, ILg, XLg, W, 1, T, IL, XL, s, Sv));
            double w0[3] = {0.1, 0.2, 0.3};
            int64_t cnt[8];
            double* err = malloc(sizeof(double) * 8 * 64);
            for (int rule = 0; rule < 3; rule++)
                CHECK(orc_adapt_sequential(S, Tg, ILg, XLg, D, mask, rule, 0.1, 1e-6, 0.99, 1.0, w0, 2, 2, W, cnt, err,
                                           64));
            CHECK(orc_backward_ex(V, T, IL, XL, n, s, 0, feature, q3, offp, wp, 0, 2, NULL, 1e-4, D, mask, 2, gS, gV, W,
                                  fb, 2));
            int64_t pts[6] = {0, 0, 0, T - 1, IL - 1, XL - 1};
            double gp[2];
            double wf[3] = {0.2, 0.5, 0.3};
            CHECK(orc_backward_at(V, T, IL, XL, n, s, 0, 6, off, w, 1, 1, wf, gS, pts, 2, gp, 1));
            free(E); free(S); free(Sv); free(gV); free(D); free(mask); free(err);
        }
    free(V); free(gS); free(F);
    printf("ORACLE_SANITIZE_OK\n");
    return 0;
}
