// The device status word: one 32-bit word per device into which kernels OR
// conditions they detect but cannot report through a return value
// (non-finite inputs, an expired bounded wait).  tc_dtw_sync_status waits for
// a stream, reads the word and clears it.
//
// Each GPU holds its own copy of the word at its own address, found once per
// device with hipGetSymbolAddress; host code passes that address to the
// kernels, never the variable's name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "api_common.h"

namespace tcdtw {

static constexpr int kMaxStatusDevices = 64;
static __device__ __align__(16) uint32_t status_words[4];
static std::mutex g_status_mu;
static uint32_t* g_status_ptr[kMaxStatusDevices];

uint32_t* status_word() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxStatusDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_status_mu);
    if (!g_status_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(status_words)) != hipSuccess) return nullptr;
        g_status_ptr[dev] = static_cast<uint32_t*>(p);
    }
    return g_status_ptr[dev];
}

}  // namespace tcdtw

using namespace tcdtw;

extern "C" tc_dtw_status tc_dtw_sync_status(tc_dtw_stream stream) {
    tc_dtw_status st = check_device();
    if (st != TC_DTW_OK) return st;
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "stream");
    uint32_t* w = status_word();
    if (!w) return fail(TC_DTW_ERR_DEVICE, "the device status word cannot be located");
    uint32_t h = 0;
    if ((e = hipMemcpy(&h, w, sizeof h, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "status read");
    if (h == 0) return ok();
    const uint32_t zero = 0;
    if ((e = hipMemcpy(w, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "status clear");
    std::string msg = "device status:";
    if (h & kStatusNonFiniteRef) msg += " a reference value is not finite (index build);";
    if (h & kStatusNonFiniteQuery) msg += " a query value is not finite;";
    if (h & kStatusWaitExpired) msg += " a bounded wait between the waves of a pair ran out (its distance is NaN);";
    return fail(TC_DTW_ERR_DEVICE, msg);
}
