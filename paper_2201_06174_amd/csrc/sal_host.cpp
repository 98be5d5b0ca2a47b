// sal_host.cpp -- error state, argument checks and the constant tables of libsal.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sal_internal.h"

namespace sal {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

sal_status fail(sal_status code, const std::string& msg) {
    g_error = msg;
    return code;
}

sal_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return SAL_OK;
    return fail(SAL_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

sal_status check_spec(const sal_spec* spec, int64_t T, int64_t IL, int64_t XL) {
    if (!spec) return fail(SAL_ERR_ARG, "spec is NULL");
    const int n = spec->n, s = spec->s;
    if (n < 2 || (n & 1)) return fail(SAL_ERR_ARG, "window side n must be even and >= 2");
    if (n != 4 && n != 8 && n != 12 && n != 16)
        return fail(SAL_ERR_UNSUPPORTED, "window side n must be 4, 8, 12 or 16 (the sides with kernels)");
    if (s < 1 || 2 * s >= n) return fail(SAL_ERR_ARG, "stride must satisfy 1 <= s < n/2 (more than 50% overlap)");
    if (spec->window != SAL_WINDOW_HANN && spec->window != SAL_WINDOW_RECT) return fail(SAL_ERR_ARG, "unknown window");
    if (spec->precision != SAL_PREC_FP32 && spec->precision != SAL_PREC_SPLIT_BF16 && spec->precision != SAL_PREC_FP16)
        return fail(SAL_ERR_ARG, "unknown precision");
    if (T < n / 2 || IL < n / 2 || XL < n / 2)
        return fail(SAL_ERR_SHAPE, "every volume axis must hold at least n/2 voxels (single reflection at borders)");
    if (T > (int64_t(1) << 31) || IL > (int64_t(1) << 31) || XL > (int64_t(1) << 31))
        return fail(SAL_ERR_SHAPE, "volume axis too long");
    return SAL_OK;
}

// ---------------------------------------------------------------- tables

static double taper(int a, int n, int window) {
    if (window == SAL_WINDOW_RECT) return 1.0;
    double v = std::sin(M_PI * a / n);
    return v * v;
}

// cos / sin of 2 pi k a / n, exact at multiples of a quarter turn
static double cos_k(int k, int a, int n) {
    int64_t r = (int64_t(k) * a) % n;
    if (r == 0) return 1.0;
    if (2 * r == n) return -1.0;
    if (4 * r == n || 4 * r == 3 * n) return 0.0;
    return std::cos(2.0 * M_PI * double(r) / n);
}
static double sin_k(int k, int a, int n) {
    int64_t r = (int64_t(k) * a) % n;
    if (r == 0 || 2 * r == n) return 0.0;
    if (4 * r == n) return 1.0;
    if (4 * r == 3 * n) return -1.0;
    return std::sin(2.0 * M_PI * double(r) / n);
}

static int signed_freq(int u, int n) { return u <= n / 2 ? u : u - n; }

static uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return uint16_t(r >> 16);
}
static float from_bf16(uint16_t h) {
    uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
static uint16_t to_f16(float f) {
    _Float16 h = (_Float16)f;
    uint16_t r;
    std::memcpy(&r, &h, 2);
    return r;
}

struct DevTables {
    Tables t;
    void* base = nullptr;
};

static std::mutex g_mu;
static std::map<std::tuple<int, int, int>, DevTables> g_tables;

sal_status get_tables(int n, int window, const Tables** out) {
    int dev = 0;
    sal_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_tuple(dev, n, window);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) {
        *out = &it->second.t;
        return SAL_OK;
    }
    const int KH = n / 2 + 1;
    std::vector<float> passA(size_t(KH) * n * 2), mat(16 * size_t(n)), wts(size_t(KH) * n * 16 * 4, 0.f),
        inv(16 * 16, 0.f);
    for (int k = 0; k < KH; k++)
        for (int a = 0; a < n; a++) {
            double h = taper(a, n, window);
            passA[(size_t(k) * n + a) * 2 + 0] = float(h * cos_k(k, a, n));
            passA[(size_t(k) * n + a) * 2 + 1] = float(-h * sin_k(k, a, n));
        }
    for (int r = 0; r < 16; r++) {
        int q, is_sin, valid;
        packed_row(r, n, &q, &is_sin, &valid);
        for (int a = 0; a < n; a++) {
            double h = taper(a, n, window);
            double v = valid ? h * (is_sin ? sin_k(q, a, n) : cos_k(q, a, n)) : 0.0;
            mat[size_t(r) * n + a] = float(v);
            // adjoint matrix [a][r]: transpose of the packed rows, taper included, both
            // dimensions padded to 16
            inv[size_t(a) * 16 + r] = float(v);
        }
    }
    const double n3 = double(n) * n * n;
    for (int kx = 0; kx < KH; kx++) {
        double mult = (kx == 0 || kx == n / 2) ? 1.0 : 2.0;
        for (int u = 0; u < n; u++) {
            double ki = signed_freq(u, n);
            for (int r = 0; r < 16; r++) {
                int q, is_sin, valid;
                packed_row(r, n, &q, &is_sin, &valid);
                if (!valid) continue;
                double kt = q;
                double k2 = kt * kt + ki * ki + double(kx) * kx;
                if (k2 == 0.0) continue;  // DC bin carries no weight
                double kn = std::sqrt(k2);
                float* w = &wts[((size_t(kx) * n + u) * 16 + r) * 4];
                w[0] = float(mult * std::sqrt(ki * ki + double(kx) * kx) / kn / n3);
                w[1] = float(mult * std::sqrt(kt * kt + ki * ki) / kn / n3);
                w[2] = float(mult * std::sqrt(kt * kt + double(kx) * kx) / kn / n3);
            }
        }
    }
    // natural-order bin weights and the complex DFT operands of the reduced-precision passes
    std::vector<float> wnat(size_t(KH) * n * 16 * 4, 0.f);
    for (int kx = 0; kx < KH; kx++) {
        double mult = (kx == 0 || kx == n / 2) ? 1.0 : 2.0;
        for (int u = 0; u < n; u++) {
            double ki = signed_freq(u, n);
            for (int r = 0; r < n; r++) {
                double kt = signed_freq(r, n);
                double k2 = kt * kt + ki * ki + double(kx) * kx;
                if (k2 == 0.0) continue;
                double kn = std::sqrt(k2);
                float* w = &wnat[((size_t(kx) * n + u) * 16 + r) * 4];
                w[0] = float(mult * std::sqrt(ki * ki + double(kx) * kx) / kn / n3);
                w[1] = float(mult * std::sqrt(kt * kt + ki * ki) / kn / n3);
                w[2] = float(mult * std::sqrt(kt * kt + double(kx) * kx) / kn / n3);
            }
        }
    }
    // the same with the Hermitian mirror folded in: on the planes kx = 0 and kx = n/2 only the ki
    // slots [0, n/2] are visited, and a slot whose mirror n - u is skipped counts twice
    std::vector<float> wnat_h(wnat);
    for (int kx = 0; kx < KH; kx++) {
        if (kx != 0 && 2 * kx != n) continue;
        for (int u = 1; u < n; u++)
            for (int c = 0; c < 16 * 4; c++) {
                float& w = wnat_h[(size_t(kx) * n + u) * 64 + c];
                w = u < n / 2 ? 2.f * w : (u == n / 2 ? w : 0.f);
            }
    }
    std::vector<uint16_t> chi(2 * 16 * 32, 0), clo(2 * 16 * 32, 0), ch16(2 * 16 * 32, 0);
    for (int c = 0; c < 2; c++)
        for (int r = 0; r < 16; r++)
            for (int k = 0; k < 32; k++) {
                const int half = k / 16, b = k % 16;
                double v = 0.0;
                if (r < n && b < n) {
                    const int kf = ((r % n) + n) % n;  // bin r as a non-negative frequency mod n
                    const double h = taper(b, n, window);
                    const double cs = cos_k(kf, b, n), sn = sin_k(kf, b, n);
                    if (c == 0) v = half == 0 ? h * cs : h * sn;
                    else v = half == 0 ? -h * sn : h * cs;
                }
                const float f = float(v);
                const uint16_t bh = to_bf16(f);
                chi[(c * 16 + r) * 32 + k] = bh;
                clo[(c * 16 + r) * 32 + k] = to_bf16(f - from_bf16(bh));
                ch16[(c * 16 + r) * 32 + k] = to_f16(f);
            }
    size_t bytes = (passA.size() + mat.size() + wts.size() + inv.size() + 2 * wnat.size()) * 4 + 3 * 1024 * 2 + 11 * 256;
    void* base = nullptr;
    st = check_hip(hipMalloc(&base, bytes), "hipMalloc(tables)");
    if (st) return st;
    char* p = (char*)base;
    auto put = [&](const void* src, size_t nb) -> char* {
        char* dst = p;
        p += (nb + 255) / 256 * 256;  // keep every table 256-byte aligned
        return (hipMemcpy(dst, src, nb, hipMemcpyHostToDevice) == hipSuccess) ? dst : nullptr;
    };
    DevTables dt;
    dt.base = base;
    dt.t.n = n;
    dt.t.window = window;
    dt.t.passA = (const float*)put(passA.data(), passA.size() * 4);
    dt.t.mat = (const float*)put(mat.data(), mat.size() * 4);
    dt.t.wts = (const float*)put(wts.data(), wts.size() * 4);
    dt.t.inv = (const float*)put(inv.data(), inv.size() * 4);
    dt.t.wts_nat = (const float*)put(wnat.data(), wnat.size() * 4);
    dt.t.wts_nat_h = (const float*)put(wnat_h.data(), wnat_h.size() * 4);
    dt.t.cpx_hi = (const uint16_t*)put(chi.data(), chi.size() * 2);
    dt.t.cpx_lo = (const uint16_t*)put(clo.data(), clo.size() * 2);
    dt.t.cpx_h16 = (const uint16_t*)put(ch16.data(), ch16.size() * 2);
    if (!dt.t.passA || !dt.t.mat || !dt.t.wts || !dt.t.inv || !dt.t.wts_nat || !dt.t.wts_nat_h || !dt.t.cpx_hi ||
        !dt.t.cpx_lo || !dt.t.cpx_h16) {
        (void)hipFree(base);  // already failing; the upload error is the one reported
        return fail(SAL_ERR_DEVICE, "uploading constant tables failed");
    }
    auto res = g_tables.emplace(key, dt);
    *out = &res.first->second.t;
    return SAL_OK;
}

static std::map<std::tuple<int, int, int, int>, void*> g_pa_ops;

sal_status get_pass_a_ops(int n, int s, int window, const uint16_t** out) {
    int dev = 0;
    sal_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_tuple(dev, n, s, window);
    auto it = g_pa_ops.find(key);
    if (it != g_pa_ops.end()) {
        *out = (const uint16_t*)it->second;
        return SAL_OK;
    }
    const int KH = n / 2 + 1;
    std::vector<uint16_t> ops(size_t(KH) * 3 * 16 * 32, 0);
    for (int kx = 0; kx < KH; kx++)
        for (int c = 0; c < 8; c++) {
            const int h = c >> 2, xc = c & 3;
            for (int x = 0; x < 32; x++) {
                const int a = x - xc * s;
                if (a < 0 || a >= n) continue;
                const double t = taper(a, n, window);
                const float f = float(h == 0 ? t * cos_k(kx, a, n) : -t * sin_k(kx, a, n));
                const uint16_t bh = to_bf16(f);
                uint16_t* o = &ops[(size_t(kx) * 3 * 16 + c) * 32 + x];
                o[0] = bh;
                o[16 * 32] = to_bf16(f - from_bf16(bh));
                o[2 * 16 * 32] = to_f16(f);
            }
        }
    void* d = nullptr;
    if ((st = check_hip(hipMalloc(&d, ops.size() * 2), "hipMalloc(pass A operands)"))) return st;
    if ((st = check_hip(hipMemcpy(d, ops.data(), ops.size() * 2, hipMemcpyHostToDevice), "hipMemcpy(pass A operands)"))) {
        (void)hipFree(d);  // already failing; the copy error is the one reported
        return st;
    }
    g_pa_ops.emplace(key, d);
    *out = (const uint16_t*)d;
    return SAL_OK;
}

}  // namespace sal

extern "C" {

const char* sal_last_error(void) { return sal::g_error.c_str(); }

const char* sal_version(void) { return "libsal 0.1 (gfx950)"; }

int64_t sal_grid_extent(int64_t N, int32_t s) { return s > 0 && N > 0 ? sal::ceil_div(N, s) : 0; }

}  // extern "C"
