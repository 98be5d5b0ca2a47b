// sal_noalloc.hip -- sal_fuse_noalloc: sal_fuse with its workspace in a static device array,
// for callers that cannot allocate (code under graph capture, tight serving loops).
//
// The scratch holds the partial sums and reduced statistics of the adapted fit (Eq. 4) for at
// most kNoAllocMaxGroups weight groups.  Each device the library runs on holds its own copy
// until the process ends; its address is resolved once per device (sal_init, else the first
// call on the device outside a capture).  Every call on a device shares that device's array:
// calls that overlap on one device (two streams, two threads) race on it.  Nothing in it has
// to start at zero: the statistics kernel writes every partial sum it later reads.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>

#include "sal_aux.h"

namespace sal {

constexpr int64_t kNoAllocMaxGroups = 64;
constexpr size_t kScratchDoubles = (size_t)kNoAllocMaxGroups * (kFuseParts * kStats + 16);

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
std::atomic<double*> g_scratch[kMaxDevices];
}  // namespace

sal_status init_noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SAL_ERR_DEVICE, "device id out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[dev].load(std::memory_order_acquire)) return SAL_OK;
    double* ptr = nullptr;
    sal_status st = check_hip(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st) return st;
    if (!ptr) return fail(SAL_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev].store(ptr, std::memory_order_release);
    return SAL_OK;
}

}  // namespace sal

using namespace sal;

extern "C" {

size_t sal_fuse_noalloc_max_bytes(void) { return sizeof(double) * kScratchDoubles; }

static sal_status sal_fuse_noalloc_body(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion,
                            const float* D, const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s,
                            double* W_out, float* S_out, sal_stream stream) {
    sal_status st = check_fusion_args(fusion, D);
    if (st) return st;
    if (!Sm || !W_out || !S_out) return fail(SAL_ERR_ARG, "NULL buffer");
    if (T < 1 || IL < 1 || XL < 1) return fail(SAL_ERR_SHAPE, "empty volume");
    if (s < 1) return fail(SAL_ERR_ARG, "stride must be >= 1");
    if (ceil_div(T, s) != Tg || ceil_div(IL, s) != ILg || ceil_div(XL, s) != XLg)
        return fail(SAL_ERR_SHAPE, "grid extents must equal ceil(N / s) of the volume extents");
    if (fuse_sequential(fusion->mode))
        return fail(SAL_ERR_UNSUPPORTED, "sal_fuse_noalloc: the LMS / NLMS / RLS rules need a workspace of the grid's "
                                         "size (use sal_fuse)");
    const int64_t K = fuse_groups(fusion->sections, ILg);
    if (fusion->mode == SAL_FUSE_ADAPT_LS && fuse_workspace_bytes(K) > sal_fuse_noalloc_max_bytes())
        return fail(SAL_ERR_NOMEM, "sal_fuse_noalloc: " + std::to_string(K) + " weight groups need " +
                                       std::to_string(fuse_workspace_bytes(K)) + " bytes of scratch; the static scratch "
                                       "holds " + std::to_string(sal_fuse_noalloc_max_bytes()) + " (at most " +
                                       std::to_string(kNoAllocMaxGroups) + " groups): use sal_fuse with a workspace");
    int dev = 0;
    if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice"))) return st;
    if (dev < 0 || dev >= 64) return fail(SAL_ERR_DEVICE, "device id out of range");
    double* ws = g_scratch[dev].load(std::memory_order_acquire);
    if (!ws) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const hipError_t e = hipStreamIsCapturing((hipStream_t)stream, &cs);
        if (e != hipSuccess || cs != hipStreamCaptureStatusNone)
            return fail(SAL_ERR_STATE, "the static scratch of this device is not resolved yet and the stream is being "
                                       "captured: call sal_init() on the device before capturing");
        if ((st = init_noalloc_scratch(dev))) return st;
        ws = g_scratch[dev].load(std::memory_order_acquire);
    }
    return launch_fuse(Sm, Tg, ILg, XLg, *fusion, D, mask, T, IL, XL, s, W_out, S_out, ws, (hipStream_t)stream);
}

sal_status sal_fuse_noalloc(const float* Sm, int64_t Tg, int64_t ILg, int64_t XLg, const sal_fusion* fusion,
                            const float* D, const uint8_t* mask, int64_t T, int64_t IL, int64_t XL, int32_t s,
                            double* W_out, float* S_out, sal_stream stream) {
    CallScope cs("sal_fuse_noalloc");
    return cs.done(sal_fuse_noalloc_body(Sm, Tg, ILg, XLg, fusion, D, mask, T, IL, XL, s, W_out, S_out, stream));
}

}  // extern "C"
