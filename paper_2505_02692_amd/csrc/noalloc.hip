// fabx_score_noalloc: the score of fabx_score for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Every device buffer of the score -- the
// task tables, the fused kernel's column plan, the workspace -- is laid out in
// one file-scope device array, `scratch`, that each GPU holds from the
// library's load until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (when
// a context is created on the device, or on the entry point's first call
// there) and only that address is handed to copies and kernels.
#include <mutex>

#include "kernels.h"

namespace fabx {
namespace {

constexpr size_t kScratchBytes = size_t(FABX_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
    std::mutex mu;             // held by a call for its whole duration (calls are synchronous)
    char *ptr = nullptr;       // device address of this device's copy of `scratch`
};

ScratchSlot g_slots[kMaxDevices];
std::mutex g_setup_mu;

}  // namespace

// Device address of `scratch` on `device`, looked up on first use with that
// device current.
char *scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) fail(FABX_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_setup_mu);
    ScratchSlot &s = g_slots[device];
    if (!s.ptr) {
        int cur = -1;
        FABX_HIP(hipGetDevice(&cur));
        if (cur != device) FABX_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(FABX_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        }
        s.ptr = static_cast<char *>(p);
    }
    return s.ptr;
}

}  // namespace fabx

using namespace fabx;

extern "C" int fabx_score_noalloc(fabx_task *task, const fabx_score_opts *opts, int64_t *half_units,
                                  fabx_stats *stats) {
    try {
        if (!task || !half_units) fail(FABX_EINVAL, "null argument");
        TaskImpl &t = *task->p;
        const ScoreParams p = resolve_opts(opts, *t.ds);
        if (p.keep_pairs) fail(FABX_EINVAL, "keep_pairs is not available without allocation");
        const int device = t.ds->ctx->device;
        if (device < 0) fail(FABX_EINVAL, "context has no device (host-only context)");
        char *base = scratch_setup(device);
        std::lock_guard<std::mutex> lk(g_slots[device].mu);
        score_in_scratch(t, p, base, kScratchBytes, t.ds->ctx->stream, half_units, stats);
        set_last_error("");
        return FABX_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FABX_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return FABX_EINVAL;
    }
}
