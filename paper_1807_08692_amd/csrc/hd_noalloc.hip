// hd_rank_noalloc: the ranking of hd_rank without any device allocation, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc). Its top-K scratch (the sampled
// thresholds, per-block candidate lists and counts) lives in a fixed device
// array of this library, `scratch`, of kScratchBytes. The code object holds
// one copy of the array on every GPU it is loaded on, for the life of the
// process. In host code the array's name is not a device address: its
// address on each device is taken once, with that device current, by
// hipGetSymbolAddress (from hd_create, the library's set-up call) and kept
// per device; only that address is ever passed to kernels.
#include <mutex>

#include "hd_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

namespace hdi {

// Take the device address of `scratch` on `device` once (with that device
// current). Called by hd_create; thread-safe.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(HD_EINVAL, "hd_create: device %d above %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return HD_OK;
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
        return fail(HD_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_ptr[device] = p;
    return HD_OK;
}

}  // namespace hdi

extern "C" {

size_t hd_rank_noalloc_scratch_bytes(int32_t B, int64_t n, int32_t K) {
    if (B < 1 || n < 1 || K < 1) return 0;
    return hd::topk_scratch_bytes(B, n, K);
}

int hd_rank_noalloc(hd_ctx *c, int32_t B, int64_t n, const float *x, int64_t ldx, int32_t K,
                    int32_t *ids_out, float *scores_out, void *stream) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_rank_noalloc: NULL context");
    if (B < 1 || n < 1 || ldx < n || !x) return fail(HD_EINVAL, "hd_rank_noalloc: bad B, n, ldx or x");
    if (K < 1 || K > n || K > hd::kTopkMax)
        return fail(HD_EINVAL, "hd_rank_noalloc: K=%d not in [1, min(n, %d)]", K, hd::kTopkMax);
    const size_t need = hd::topk_scratch_bytes(B, n, K);
    if (need > kScratchBytes)
        return fail(HD_EINVAL, "hd_rank_noalloc: B=%d rows of n=%lld need %zu bytes of scratch, above the fixed %zu",
                    B, (long long)n, need, kScratchBytes);
    if (!ids_out && !scores_out) return HD_OK;
    void *p = c->device >= 0 && c->device < kMaxDevices ? g_ptr[c->device] : nullptr;
    if (!p) return fail(HD_ESTATE, "hd_rank_noalloc: scratch of device %d not set up", c->device);
    HIP_TRY(hipSetDevice(c->device));
    // every scratch field the kernels read is written earlier in the same
    // call, so the previous call's contents need no clearing
    HIP_TRY(hd::launch_topk(B, n, x, ldx, K, p, ids_out, scores_out, 0, (hipStream_t)stream));
    return HD_OK;
}

}  // extern "C"
