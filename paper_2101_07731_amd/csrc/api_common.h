// Host-side helpers of the C ABI: error reporting, argument checks, the
// device check and workspace carving.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/tc_dtw.h"
#include "internal.h"

namespace tcdtw {

tc_dtw_status fail(tc_dtw_status st, const std::string& msg);
tc_dtw_status ok();
tc_dtw_status hip_fail(hipError_t e, const char* what);
// 0 if the current device is a gfx950, else an error status with a message.
tc_dtw_status check_device();

// Host view of a batch: lengths and float offsets of every series.
struct HostSet {
    int count = 0, dim = 0;       // dim: the largest D of the set
    bool uniform = false;         // one length and one D, packed densely
    bool mixed = false;           // per-series D given
    int ulen = 0;
    int maxlen = 0;
    const float* data = nullptr;
    std::vector<int32_t> len;
    std::vector<int64_t> off;
    std::vector<int32_t> dims;
    int length(int s) const { return uniform ? ulen : len[s]; }
    int dimension(int s) const { return mixed ? dims[s] : dim; }
    int64_t offset(int s) const { return uniform ? (int64_t)s * ulen * dim : off[s]; }
};

// Validates a batch and fills `out`; `what` names it in messages.
tc_dtw_status read_set(const tc_dtw_batch* b, const char* what, HostSet& out);
tc_dtw_status check_window(tc_dtw_window w);
int window_eff(int m, int n, tc_dtw_window w);

// Bump allocator over a caller workspace (256-byte aligned pieces).
struct Carve {
    char* base;
    size_t used = 0;
    size_t cap;
    explicit Carve(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <typename T> T* take(size_t count) {
        used = (used + 255) & ~(size_t)255;
        T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
    size_t need() const { return (used + 255) & ~(size_t)255; }
};

// tc_dtw_banded's body: pairs of uneven shapes are planned into `ws` (class
// counters and pair descriptors) on every call.  With `fork` the plan's
// classes run concurrently on the library's streams, else all on `s`.
// `buffer` (may be null), called after the host-side checks with the plan
// size, may supply the plan buffer in place of ws (or refuse with a status).
tc_dtw_status banded_direct(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win, uint32_t flags,
                            float* dist, void* saved, void* ws, size_t ws_bytes, bool fork,
                            tc_dtw_status (*buffer)(size_t need, void* ctx, void** buf, size_t* bytes),
                            void* ctx, hipStream_t s);

}  // namespace tcdtw
