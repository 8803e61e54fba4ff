// Host-side helpers of the C ABI.
#include "api_common.h"

#include <cstdlib>
#include <cstring>
#include <mutex>

namespace tcdtw {

static thread_local std::string g_last_error;

tc_dtw_status fail(tc_dtw_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

tc_dtw_status ok() {
    g_last_error.clear();
    return TC_DTW_OK;
}

tc_dtw_status hip_fail(hipError_t e, const char* what) {
    return fail(TC_DTW_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

tc_dtw_status check_device() {
    // test hook: behave as on a machine without a usable device
    const char* fake = std::getenv("TC_DTW_FAKE_NO_DEVICE");
    if (fake && *fake && std::strcmp(fake, "0") != 0)
        return fail(TC_DTW_ERR_DEVICE, "no usable device (TC_DTW_FAKE_NO_DEVICE is set)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    static std::mutex mu;
    static std::vector<int> ok_devices, bad_devices;
    std::lock_guard<std::mutex> lk(mu);
    for (int d : ok_devices)
        if (d == dev) return TC_DTW_OK;
    for (int d : bad_devices)
        if (d == dev) return fail(TC_DTW_ERR_DEVICE, "current device is not a gfx950 (MI355X)");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        bad_devices.push_back(dev);
        return fail(TC_DTW_ERR_DEVICE, std::string("current device is ") + prop.gcnArchName +
                                           ", this library is built for gfx950 (MI355X)");
    }
    ok_devices.push_back(dev);
    return TC_DTW_OK;
}

tc_dtw_status read_set(const tc_dtw_batch* b, const char* what, HostSet& out) {
    const std::string w(what);
    if (!b) return fail(TC_DTW_ERR_INVALID, w + ": null batch");
    if (!b->data) return fail(TC_DTW_ERR_INVALID, w + ": null data pointer");
    if (b->count < 1) return fail(TC_DTW_ERR_INVALID, w + ": count must be >= 1");
    out = HostSet();
    out.count = b->count;
    out.data = b->data;
    if (b->dims) {
        out.mixed = true;
        out.dims.assign(b->dims, b->dims + b->count);
        for (int s = 0; s < b->count; ++s) {
            if (out.dims[s] < 1) return fail(TC_DTW_ERR_INVALID, w + ": every dims[s] must be >= 1");
            if (out.dims[s] > 64) return fail(TC_DTW_ERR_UNSUPPORTED, w + ": dim > 64 is not supported");
            if (out.dims[s] > out.dim) out.dim = out.dims[s];
        }
    } else {
        if (b->dim < 1) return fail(TC_DTW_ERR_INVALID, w + ": dim must be >= 1");
        if (b->dim > 64) return fail(TC_DTW_ERR_UNSUPPORTED, w + ": dim > 64 is not supported");
        out.dim = b->dim;
    }
    if (!b->len && !b->offset && !b->dims) {
        if (b->uniform_len < 1) return fail(TC_DTW_ERR_INVALID, w + ": uniform_len must be >= 1");
        out.uniform = true;
        out.ulen = b->uniform_len;
        out.maxlen = b->uniform_len;
        return TC_DTW_OK;
    }
    out.len.resize(b->count);
    out.off.resize(b->count);
    int64_t next = 0;
    for (int s = 0; s < b->count; ++s) {
        const int L = b->len ? b->len[s] : b->uniform_len;
        if (L < 1) return fail(TC_DTW_ERR_INVALID, w + ": every length must be >= 1");
        out.len[s] = L;
        out.off[s] = b->offset ? b->offset[s] : next;
        if (out.off[s] < 0) return fail(TC_DTW_ERR_INVALID, w + ": negative offset");
        next = out.off[s] + (int64_t)L * out.dimension(s);
        if (L > out.maxlen) out.maxlen = L;
    }
    return TC_DTW_OK;
}

tc_dtw_status check_window(tc_dtw_window w) {
    if (w.window < 0) return fail(TC_DTW_ERR_INVALID, "window must be >= 0");
    if (w.frac_den < 0 || w.frac_num < 0) return fail(TC_DTW_ERR_INVALID, "window fraction must be >= 0");
    return TC_DTW_OK;
}

int window_eff(int m, int n, tc_dtw_window w) {
    const int longer = m > n ? m : n;
    long long W = w.frac_den > 0 ? ((long long)longer * w.frac_num) / w.frac_den : w.window;
    const int diff = m > n ? m - n : n - m;
    if (W < diff) W = diff;
    if (W > longer - 1) W = longer - 1;   // every cell has |i-j| <= max(m,n)-1 anyway
    return (int)W;
}

int64_t band_cells(int m, int n, int W) {
    int64_t c = 0;
    for (int i = 0; i < m; ++i) {
        const int lo = i - W > 0 ? i - W : 0;
        const int hi = i + W < n - 1 ? i + W : n - 1;
        if (hi >= lo) c += hi - lo + 1;
    }
    return c;
}

}  // namespace tcdtw

extern "C" {

int tc_dtw_abi_version(void) { return TC_DTW_ABI_VERSION; }

const char* tc_dtw_last_error(void) { return tcdtw::g_last_error.c_str(); }

const char* tc_dtw_status_string(tc_dtw_status s) {
    switch (s) {
        case TC_DTW_OK: return "ok";
        case TC_DTW_ERR_INVALID: return "invalid argument";
        case TC_DTW_ERR_WORKSPACE: return "buffer too small";
        case TC_DTW_ERR_UNSUPPORTED: return "unsupported";
        case TC_DTW_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

}  // extern "C"
