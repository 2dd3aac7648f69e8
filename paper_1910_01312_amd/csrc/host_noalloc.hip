// ssnalm_project_noalloc: the projection onto {y^T x = 0, 0 <= x <= C}
// (Section 3.2.1) with no context and no device allocation, for callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc).
//
// The kernels are the ones ssnalm_op_project runs (multisection passes, the
// final clip); their scratch (the search state, the block partials and the
// two counts) lives in one file-scope device array instead of a context's
// workspace.  Each GPU holds its own copy of the array until the process
// ends; its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels and copies
// (the array's name is a host-side stand-in in host code).
//
// Calls that overlap on one GPU share the array and race: the caller
// serialises them (one stream, or its own ordering between streams).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "ssn_internal.h"

using namespace ssn;

namespace {

// Layout of the scratch array, in doubles: the search state, the reduction
// results, then the block partials of the passes (the projection grid is
// capped, so their size does not depend on n).
constexpr size_t kStateDoubles = (sizeof(ProjState) + 7) / 8;
constexpr size_t kScalarDoubles = (sizeof(Scalars) + 7) / 8;
constexpr size_t kPartDoubles = 8 * 4096;            // same capacity as a context's
constexpr size_t kScratchDoubles = 32 + kStateDoubles + kScalarDoubles + kPartDoubles;
constexpr int kMaxDevices = 64;

}  // namespace

// 256-byte aligned; about 260 KB per GPU.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
ssnalm_status scratch_ptr(double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(SSNALM_E_HIP, "no HIP device");
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(SSNALM_E_HIP, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(SSNALM_E_HIP, "hipGetSymbolAddress(scratch) failed: %s",
                             hipGetErrorString(e));
        g_ptr[dev] = (double*)p;
    }
    *out = g_ptr[dev];
    return SSNALM_OK;
}

}  // namespace

extern "C" ssnalm_status ssnalm_project_noalloc(const double* v, const int8_t* y, int64_t n,
                                                double C, double* x, uint8_t* free_mask,
                                                double* lam, int64_t* p, void* stream) {
    if (!v || !y || !x) return set_error(SSNALM_E_BADARG, "null argument");
    if (n < 1 || n > ssnalm_noalloc_max_n())
        return set_error(SSNALM_E_BADARG, "n must be in [1, %lld]", (long long)ssnalm_noalloc_max_n());
    if (!(C > 0.0) || !std::isfinite(C)) return set_error(SSNALM_E_BADARG, "C must be finite and > 0");
    double* base = nullptr;
    const ssnalm_status s0 = scratch_ptr(&base);
    if (s0 != SSNALM_OK) return s0;
    hipStream_t st = (hipStream_t)stream;
    ProjState* ps = reinterpret_cast<ProjState*>(base);
    Scalars* sc = reinterpret_cast<Scalars*>(base + kStateDoubles);
    double* part = base + kStateDoubles + kScalarDoubles;
    // Every scratch field that a kernel reads is written earlier in this call
    // (the init kernel sets the whole search state, the clip's finishing
    // kernel both counts), so nothing left by an earlier call is used.
    launch_proj_init(v, nullptr, 0.0, nullptr, y, n, C, ps, part, nullptr, st, nullptr);
    for (int i = 0; i < 5; ++i) launch_proj_pass(v, y, n, C, ps, part, nullptr, st);
    ProjState h;
    if (hipMemcpyAsync(&h, ps, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_error(SSNALM_E_HIP, "reading the projection state failed");
    if (!h.done)
        for (int i = 0; i < proj_max_passes(); ++i) launch_proj_pass(v, y, n, C, ps, part, nullptr, st);
    launch_proj_apply(v, y, n, C, ps, x, free_mask, sc, part, nullptr, st);
    if (hipGetLastError() != hipSuccess) return set_error(SSNALM_E_HIP, "kernel launch failed");
    Scalars hs;
    if (hipMemcpyAsync(&h, ps, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&hs, sc, sizeof hs, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_error(SSNALM_E_HIP, "reading the projection results failed");
    if (lam) *lam = h.lam;
    if (p) *p = hs.p;
    return SSNALM_OK;
}

extern "C" int64_t ssnalm_noalloc_max_n(void) { return (int64_t)INT32_MAX - 1; }

extern "C" int64_t ssnalm_noalloc_scratch_bytes(void) {
    return (int64_t)(kScratchDoubles * sizeof(double));
}
