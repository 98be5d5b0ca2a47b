// sal_internal.h -- shared host/device helpers of libsal (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>

#include "../../include/sal.h"

namespace sal {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
sal_status fail(sal_status code, const std::string& msg);
sal_status check_hip(hipError_t e, const char* what);

// Raises the dynamic-LDS limit of `kernel` to `bytes` on the current device, once per device
// (`done` holds a bit per device id below 64).  The attribute call is idempotent, so two
// threads racing on the first launch only repeat it.
inline sal_status lds_limit_once(const void* kernel, int bytes, std::atomic<uint64_t>& done, const char* what) {
    int dev = 0;
    sal_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    const uint64_t bit = dev >= 0 && dev < 64 ? uint64_t(1) << dev : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return SAL_OK;
    st = check_hip(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes), what);
    if (!st && bit) done.fetch_or(bit, std::memory_order_release);
    return st;
}

// ---------------------------------------------------------------- observability

// Opened by every C-ABI entry point that enqueues device work: a roctx range named after the
// call (recorded by rocprofv3 --marker-trace), and with SAL_LOG=1 in the environment one line
// per call on stderr with its status and, on failure, the message of sal_last_error().
class CallScope {
  public:
    explicit CallScope(const char* name);
    ~CallScope();
    sal_status done(sal_status st);

  private:
    const char* name_;
};

// ---------------------------------------------------------------- shapes

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Validates n, s, window, precision and the volume extents; returns SAL_OK or an error
// (with the message set).
sal_status check_spec(const sal_spec* spec, int64_t T, int64_t IL, int64_t XL);

// ---------------------------------------------------------------- constant tables

// Per (device, n, window) device tables, built once on the host in double and uploaded into
// static device memory by sal_init() (or by the first call on a device outside a capture).
struct Tables {
    int n = 0;
    int window = 0;
    const float* passA = nullptr;   // [KH][n][2]: h(a) cos(2 pi k a/n), -h(a) sin(2 pi k a/n)
    const float* mat = nullptr;     // [16][n]: packed taper*DFT rows c0, c_{n/2}, c1, s1, c2, s2, ...
    const float* wts = nullptr;     // [KH][n][16][4]: bin weights mult(kx) alpha_m / n^3 per packed row
    const float* wts_e = nullptr;   // the same with alpha_m^2 (energy feature)
    const float* inv = nullptr;     // [16 a][16 r]: h(a) * trig row r at sample a (transpose of `mat`), zero padded
    const float* wts_nat = nullptr; // [KH][n][16][4]: bin weights for natural-order rows (row r = bin r)
    const float* wts_nat_h = nullptr; // the same, with ki slots (n/2, n) of the planes kx = 0, n/2 folded into
                                      // their Hermitian mirrors (doubled slots 1 .. n/2-1, zero beyond n/2)
    // complex DFT operands of the reduced-precision passes, [2 (re, im)][16 rows][32 K]:
    // row r is bin r (signed frequency), K = [real part samples 0..15 | imaginary part samples 0..15],
    // re rows h cos | h sin, im rows -h sin | h cos; bf16 hi and lo parts and fp16
    const uint16_t* cpx_hi = nullptr;
    const uint16_t* cpx_lo = nullptr;
    const uint16_t* cpx_h16 = nullptr;
    // projection operand of the reduced-precision pass C, [KH][n slots u][64 lanes][2 words]: lane
    // col + 16 g holds four bf16 values, the weights (wts_nat_h) of plane m for the bins
    // r = 4g .. 4g + 3 of slot u: their hi parts in column m, their lo parts in column 4 + m
    // (m = 0, 1, 2), zero in the other columns
    const uint32_t* wproj = nullptr;
};

// The tables of the current device.  If they are not uploaded yet and `stream` is not being
// captured, uploads them (blocking); inside a capture fails with SAL_ERR_STATE.
sal_status get_tables(hipStream_t stream, int n, int window, const Tables** out);

// Uploads every table of device `dev` (current) and resolves its no-allocation scratch.
sal_status init_device(int dev);
// Resolves the device address of sal_fuse_noalloc's static scratch on `dev` (current).
sal_status init_noalloc_scratch(int dev);
// Fusion argument checks shared by sal_fuse, sal_fuse_noalloc and the plans.
sal_status check_fusion_args(const sal_fusion* f, const float* D);

// Per (device, n, s, window) B operands of the reduced-precision pass A, [KH][3][16 cols][32 K]:
// planes bf16 hi, bf16 lo, fp16; column c < 8 is (c >> 2: h cos | -h sin, c & 3: window column
// xc), K = sample x of a staged row, holding the taper*twiddle of tap x - xc*s (zero outside
// the window and for columns 8..15).
sal_status get_pass_a_ops(hipStream_t stream, int n, int s, int window, const uint16_t** out);

// Packed row r of an n-point transform: its frequency q and whether it is a sine row.
// Rows: 0 -> cos 0, 1 -> cos n/2, 2q -> cos q, 2q+1 -> sin q (1 <= q < n/2), r >= n -> zero.
inline void packed_row(int r, int n, int* q, int* is_sin, int* valid) {
    *valid = r < n;
    if (r == 0) { *q = 0; *is_sin = 0; }
    else if (r == 1) { *q = n / 2; *is_sin = 0; }
    else { *q = r / 2; *is_sin = r & 1; }
}

// ---------------------------------------------------------------- launch configuration of the fused feature kernel

struct ProjTile {
    int CT;     // t-centres per tile (<= 8 * CTW)
    int RT, RI, RX, RXp;
    size_t lds_bytes;
};

}  // namespace sal
