// sal_host.cpp -- error state, argument checks and the constant tables of libsal.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
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

static bool log_enabled() {
    static const bool on = [] {
        const char* v = std::getenv("SAL_LOG");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    return on;
}

CallScope::CallScope(const char* name) : name_(name) { roctxRangePushA(name); }

CallScope::~CallScope() { roctxRangePop(); }

sal_status CallScope::done(sal_status st) {
    if (log_enabled()) {
        static const char* names[] = {"SAL_OK", "SAL_ERR_ARG", "SAL_ERR_SHAPE", "SAL_ERR_UNSUPPORTED",
                                      "SAL_ERR_NOMEM", "SAL_ERR_DEVICE", "SAL_ERR_STATE"};
        const char* sn = (int)st >= 0 && (int)st < 7 ? names[(int)st] : "?";
        if (st == SAL_OK) std::fprintf(stderr, "[libsal] %s -> %s\n", name_, sn);
        else std::fprintf(stderr, "[libsal] %s -> %s: %s\n", name_, sn, g_error.c_str());
    }
    return st;
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
    if (spec->feature != SAL_FEATURE_MAGNITUDE && spec->feature != SAL_FEATURE_ENERGY)
        return fail(SAL_ERR_ARG, "unknown feature");
    if (spec->feature == SAL_FEATURE_ENERGY && spec->precision != SAL_PREC_FP32)
        return fail(SAL_ERR_UNSUPPORTED, "the energy feature is built for the fp32 path only");
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

// ---------------------------------------------------------------- device-resident tables

// Every constant table the kernels read lives in static device memory, one slot per
// (n, window) and one per (n, s, window) for the reduced-precision pass-A operands, so no
// call ever allocates for them.  They are built on the host in double and uploaded once per
// device, by sal_init() or by the first call on the device that needs them (which must then
// not be inside a stream capture).
constexpr int kSides[4] = {4, 8, 12, 16};
constexpr int kTableSlots = 4 * 2;                  // (n, window)
constexpr size_t kTableSlotBytes = 240 * 1024;      // 233,472 B at n = 16
constexpr int kStridesPerWindow = 1 + 3 + 5 + 7;    // 1 <= s < n/2 for n = 4, 8, 12, 16
constexpr int kPassASlots = kStridesPerWindow * 2;  // (n, s, window)
constexpr size_t kPassASlotBytes = 27648;           // (n/2 + 1) x 3 x 16 x 32 x 2 B at n = 16

__device__ __align__(256) unsigned char g_const_tables[kTableSlots * kTableSlotBytes];
__device__ __align__(256) unsigned char g_pass_a_tables[kPassASlots * kPassASlotBytes];

static int side_index(int n) {
    for (int k = 0; k < 4; k++)
        if (kSides[k] == n) return k;
    return -1;
}
static int table_slot(int n, int window) { return side_index(n) * 2 + window; }
static int pass_a_slot(int n, int s, int window) {
    int base = 0;
    for (int k = 0; k < 4 && kSides[k] != n; k++) base += kSides[k] / 2 - 1;
    return window * kStridesPerWindow + base + (s - 1);
}

// Host image of one (n, window) table slot; fills `t` with offsets relative to the slot start.
static std::vector<unsigned char> build_table_slot(int n, int window, Tables* t) {
    const int KH = n / 2 + 1;
    std::vector<float> passA(size_t(KH) * n * 2), mat(16 * size_t(n)), wts(size_t(KH) * n * 16 * 4, 0.f),
        wts_e(size_t(KH) * n * 16 * 4, 0.f), inv(16 * 16, 0.f);
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
                // energy: the squared projection weights alpha_m^2 = P_m^2 / |k|^2
                float* we = &wts_e[((size_t(kx) * n + u) * 16 + r) * 4];
                we[0] = float(mult * (ki * ki + double(kx) * kx) / k2 / n3);
                we[1] = float(mult * (kt * kt + ki * ki) / k2 / n3);
                we[2] = float(mult * (kt * kt + double(kx) * kx) / k2 / n3);
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
    // the projection operand of the reduced-precision pass C: bf16 pairs of the weights, split
    // into hi = bf16(w) (columns m) and lo = bf16(w - hi) (columns 4 + m)
    std::vector<uint32_t> wproj(size_t(KH) * n * 64 * 2, 0u);
    for (int kx = 0; kx < KH; kx++)
        for (int u = 0; u < n; u++)
            for (int lane = 0; lane < 64; lane++) {
                const int col = lane & 15, g = lane >> 4, m = col & 3;
                if (m == 3 || col >= 8) continue;
                uint16_t v[4];
                for (int i = 0; i < 4; i++) {
                    const int r = 4 * g + i;
                    const float w = r < n ? wnat_h[((size_t(kx) * n + u) * 16 + r) * 4 + m] : 0.f;
                    const uint16_t h = to_bf16(w);
                    v[i] = col < 4 ? h : to_bf16(w - from_bf16(h));
                }
                uint32_t* o = &wproj[((size_t(kx) * n + u) * 64 + lane) * 2];
                o[0] = uint32_t(v[0]) | uint32_t(v[1]) << 16;
                o[1] = uint32_t(v[2]) | uint32_t(v[3]) << 16;
            }
    std::vector<unsigned char> img(kTableSlotBytes, 0);
    size_t off = 0;
    auto put = [&](const void* src, size_t nb) -> size_t {
        const size_t at = off;
        if (at + nb > img.size()) return SIZE_MAX;
        std::memcpy(img.data() + at, src, nb);
        off += (nb + 255) / 256 * 256;  // keep every table 256-byte aligned
        return at;
    };
    size_t o[11];
    o[9] = 0;
    o[0] = put(passA.data(), passA.size() * 4);
    o[1] = put(mat.data(), mat.size() * 4);
    o[2] = put(wts.data(), wts.size() * 4);
    o[3] = put(inv.data(), inv.size() * 4);
    o[4] = put(wnat.data(), wnat.size() * 4);
    o[5] = put(wnat_h.data(), wnat_h.size() * 4);
    o[6] = put(chi.data(), chi.size() * 2);
    o[7] = put(clo.data(), clo.size() * 2);
    o[8] = put(ch16.data(), ch16.size() * 2);
    o[9] = put(wts_e.data(), wts_e.size() * 4);
    o[10] = put(wproj.data(), wproj.size() * 4);
    for (size_t v : o)
        if (v == SIZE_MAX) return {};  // cannot happen for n <= 16 (the slot is sized for n = 16)
    t->n = n;
    t->window = window;
    // offsets for now; rebased onto the device slot by the caller
    t->passA = (const float*)o[0];
    t->mat = (const float*)o[1];
    t->wts = (const float*)o[2];
    t->inv = (const float*)o[3];
    t->wts_nat = (const float*)o[4];
    t->wts_nat_h = (const float*)o[5];
    t->cpx_hi = (const uint16_t*)o[6];
    t->cpx_lo = (const uint16_t*)o[7];
    t->cpx_h16 = (const uint16_t*)o[8];
    t->wts_e = (const float*)o[9];
    t->wproj = (const uint32_t*)o[10];
    return img;
}

// Host image of the reduced-precision pass-A operands of one (n, s, window).
static void build_pass_a_slot(int n, int s, int window, uint16_t* ops) {
    const int KH = n / 2 + 1;
    std::memset(ops, 0, kPassASlotBytes);
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
}

constexpr int kMaxDevices = 64;

struct DeviceTables {
    std::atomic<bool> ready{false};
    Tables t[kTableSlots];
    const uint16_t* pa[kPassASlots] = {};
};

static std::mutex g_mu;
static DeviceTables g_dev[kMaxDevices];

// Builds and uploads every table for device `dev` (current); idempotent.
static sal_status init_device_tables(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SAL_ERR_DEVICE, "device id out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceTables& d = g_dev[dev];
    if (d.ready.load(std::memory_order_acquire)) return SAL_OK;
    unsigned char* tab = nullptr;
    unsigned char* pas = nullptr;
    sal_status st = check_hip(hipGetSymbolAddress((void**)&tab, HIP_SYMBOL(g_const_tables)),
                              "hipGetSymbolAddress(constant tables)");
    if (!st) st = check_hip(hipGetSymbolAddress((void**)&pas, HIP_SYMBOL(g_pass_a_tables)),
                            "hipGetSymbolAddress(pass A operands)");
    if (st) return st;
    std::vector<unsigned char> img(size_t(kTableSlots) * kTableSlotBytes);
    for (int k = 0; k < 4; k++)
        for (int w = 0; w < 2; w++) {
            const int n = kSides[k], slot = table_slot(n, w);
            Tables t;
            std::vector<unsigned char> one = build_table_slot(n, w, &t);
            if (one.empty()) return fail(SAL_ERR_DEVICE, "constant table slot too small");
            std::memcpy(img.data() + size_t(slot) * kTableSlotBytes, one.data(), kTableSlotBytes);
            unsigned char* b = tab + size_t(slot) * kTableSlotBytes;
            t.passA = (const float*)(b + (size_t)t.passA);
            t.mat = (const float*)(b + (size_t)t.mat);
            t.wts = (const float*)(b + (size_t)t.wts);
            t.inv = (const float*)(b + (size_t)t.inv);
            t.wts_nat = (const float*)(b + (size_t)t.wts_nat);
            t.wts_nat_h = (const float*)(b + (size_t)t.wts_nat_h);
            t.cpx_hi = (const uint16_t*)(b + (size_t)t.cpx_hi);
            t.cpx_lo = (const uint16_t*)(b + (size_t)t.cpx_lo);
            t.cpx_h16 = (const uint16_t*)(b + (size_t)t.cpx_h16);
            t.wts_e = (const float*)(b + (size_t)t.wts_e);
            t.wproj = (const uint32_t*)(b + (size_t)t.wproj);
            d.t[slot] = t;
        }
    std::vector<uint16_t> pimg(size_t(kPassASlots) * kPassASlotBytes / 2);
    for (int w = 0; w < 2; w++)
        for (int k = 0; k < 4; k++)
            for (int s = 1; 2 * s < kSides[k]; s++) {
                const int slot = pass_a_slot(kSides[k], s, w);
                build_pass_a_slot(kSides[k], s, w, pimg.data() + size_t(slot) * kPassASlotBytes / 2);
                d.pa[slot] = (const uint16_t*)(pas + size_t(slot) * kPassASlotBytes);
            }
    // blocking uploads: nothing reads these slots before `ready` is published below
    st = check_hip(hipMemcpy(tab, img.data(), img.size(), hipMemcpyHostToDevice), "hipMemcpy(constant tables)");
    if (!st) st = check_hip(hipMemcpy(pas, pimg.data(), pimg.size() * 2, hipMemcpyHostToDevice),
                            "hipMemcpy(pass A operands)");
    if (st) return st;
    d.ready.store(true, std::memory_order_release);
    return SAL_OK;
}

sal_status init_device(int dev) {
    sal_status st = init_device_tables(dev);
    if (st) return st;
    return init_noalloc_scratch(dev);
}

// The tables of the current device, uploading them first if `stream` is not capturing.
static sal_status device_tables(hipStream_t stream, DeviceTables** out) {
    int dev = 0;
    sal_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev < 0 || dev >= kMaxDevices) return fail(SAL_ERR_DEVICE, "device id out of range");
    DeviceTables& d = g_dev[dev];
    if (!d.ready.load(std::memory_order_acquire)) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const hipError_t e = hipStreamIsCapturing(stream, &cs);
        if (e != hipSuccess || cs != hipStreamCaptureStatusNone)
            return fail(SAL_ERR_STATE, "the constant tables of this device are not uploaded yet and the stream is "
                                       "being captured: call sal_init() on the device before capturing");
        if ((st = init_device(dev))) return st;
    }
    *out = &d;
    return SAL_OK;
}

sal_status get_tables(hipStream_t stream, int n, int window, const Tables** out) {
    if (side_index(n) < 0 || (window != SAL_WINDOW_HANN && window != SAL_WINDOW_RECT))
        return fail(SAL_ERR_UNSUPPORTED, "no tables for this window side");
    DeviceTables* d = nullptr;
    sal_status st = device_tables(stream, &d);
    if (st) return st;
    *out = &d->t[table_slot(n, window)];
    return SAL_OK;
}

sal_status get_pass_a_ops(hipStream_t stream, int n, int s, int window, const uint16_t** out) {
    if (side_index(n) < 0 || s < 1 || 2 * s >= n || (window != SAL_WINDOW_HANN && window != SAL_WINDOW_RECT))
        return fail(SAL_ERR_UNSUPPORTED, "no pass A operands for this window side and stride");
    DeviceTables* d = nullptr;
    sal_status st = device_tables(stream, &d);
    if (st) return st;
    *out = d->pa[pass_a_slot(n, s, window)];
    return SAL_OK;
}

}  // namespace sal

extern "C" {

sal_status sal_init(void) {
    int dev = 0;
    sal_status st = sal::check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    return sal::init_device(dev);
}

const char* sal_last_error(void) { return sal::g_error.c_str(); }

const char* sal_version(void) { return "libsal 0.1 (gfx950)"; }

int64_t sal_grid_extent(int64_t N, int32_t s) { return s > 0 && N > 0 ? sal::ceil_div(N, s) : 0; }

}  // extern "C"
