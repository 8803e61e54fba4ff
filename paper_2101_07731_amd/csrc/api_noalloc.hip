// tc_dtw_banded_noalloc: tc_dtw_banded for callers that cannot allocate
// device memory.  The scratch that the direct call plans into (for pairs of
// uneven shapes: 32 class counters and one 48-byte descriptor per pair) is
// a file-scope device array of fixed size instead of a caller workspace,
// and the plan's classes run one after another on the caller's stream, so
// the call creates no streams or events either.
//
// Each GPU holds its own copy of the array at its own address, found once
// per device with hipGetSymbolAddress on the first call with that device
// current; host code only ever passes that address, never the array's name
// (which in host code is a host-side stand-in).  The class counters are
// cleared by a kernel at the start of every call; the descriptors are
// rewritten by every call.  Calls that overlap on one GPU (other streams or
// threads) share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "api_common.h"

namespace tcdtw {

static constexpr size_t kScratchBytes = (size_t)8 << 20;
static constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// The current device's copy of `scratch`.
static tc_dtw_status device_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TC_DTW_ERR_DEVICE, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TC_DTW_OK;
}

static tc_dtw_status scratch_buffer(size_t need, void*, void** buf, size_t* bytes) {
    if (need > kScratchBytes)
        return fail(TC_DTW_ERR_UNSUPPORTED, "the batch's pair plan needs " + std::to_string(need) +
                                                " bytes; tc_dtw_banded_noalloc's static scratch holds " +
                                                std::to_string(kScratchBytes) + " bytes");
    *bytes = 0;
    *buf = nullptr;
    if (need == 0) return TC_DTW_OK;   // uniform pairs use no scratch
    tc_dtw_status st = check_device();
    if (st != TC_DTW_OK) return st;
    if ((st = device_scratch(buf)) != TC_DTW_OK) return st;
    *bytes = kScratchBytes;
    return TC_DTW_OK;
}

}  // namespace tcdtw

using namespace tcdtw;

extern "C" {

size_t tc_dtw_noalloc_scratch_bytes(void) { return kScratchBytes; }

tc_dtw_status tc_dtw_banded_noalloc(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                                    uint32_t flags, float* dist, void* saved, tc_dtw_stream stream) {
    return banded_direct(x, y, win, flags, dist, saved, nullptr, 0, false, scratch_buffer, nullptr,
                         reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
