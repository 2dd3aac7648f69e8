// C ABI of the warm-start network (include/ssnalm.h): parameter and
// workspace sizes, forward, backward and Adam.  The kernels are in
// kernels_mlp.hip; the feature and initial-point entries, which need a
// solver context, are in host.hip.
#include <hip/hip_runtime.h>

#include "ssn_internal.h"

using namespace ssn;

namespace {
constexpr int64_t kMaxRows = 4194304;     // 65536 row tiles of 64

ssnalm_status hip_status(const char* where) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(SSNALM_E_HIP, "%s: %s", where, hipGetErrorString(e));
    return SSNALM_OK;
}
}  // namespace

extern "C" int64_t ssnalm_mlp_param_count(void) {
    return (int64_t)MLP_IN * MLP_HID + MLP_HID + (int64_t)MLP_HID * MLP_HID + MLP_HID +
           (int64_t)MLP_HID * MLP_OUT + MLP_OUT;
}

extern "C" int64_t ssnalm_mlp_work_floats(int64_t n) {
    return 4 * n * MLP_HID + 4 * n;
}

extern "C" int64_t ssnalm_mlp_scratch_floats(int64_t n) {
    const int64_t nb = (n + 255) / 256;
    return 4 * n + 2 * n * MLP_HID + (int64_t)64 * MLP_HID * MLP_HID + 2 * nb + 64;
}

extern "C" ssnalm_status ssnalm_mlp_forward(const float* theta, const float* Z, int64_t n,
                                            float* out, float* work, void* stream) {
    if (!theta || !Z || !out || !work) return set_error(SSNALM_E_BADARG, "null argument");
    if (n < 1 || n > kMaxRows) return set_error(SSNALM_E_BADARG, "n must be in [1, %lld]", (long long)kMaxRows);
    float* O = work + 4 * n * MLP_HID;
    launch_mlp_forward(theta, Z, n, work, O, out, (hipStream_t)stream);
    return hip_status("ssnalm_mlp_forward");
}

extern "C" ssnalm_status ssnalm_mlp_backward(const float* theta, const float* Z, int64_t n,
                                             const float* work, const float* out,
                                             const int32_t* status, const float* target,
                                             float w_mse, float* grad, float* loss, float* scratch,
                                             void* stream) {
    if (!theta || !Z || !work || !out || !status || !target || !grad || !loss || !scratch)
        return set_error(SSNALM_E_BADARG, "null argument");
    if (n < 1 || n > kMaxRows) return set_error(SSNALM_E_BADARG, "n must be in [1, %lld]", (long long)kMaxRows);
    launch_mlp_backward(theta, Z, n, work, out, status, target, w_mse, grad, loss, scratch,
                        (hipStream_t)stream);
    return hip_status("ssnalm_mlp_backward");
}

extern "C" ssnalm_status ssnalm_mlp_adam(float* theta, const float* grad, float* m, float* v,
                                         int64_t count, float lr, float beta1, float beta2,
                                         float eps, int32_t step, void* stream) {
    if (!theta || !grad || !m || !v) return set_error(SSNALM_E_BADARG, "null argument");
    if (count < 1 || step < 1) return set_error(SSNALM_E_BADARG, "count and step must be >= 1");
    launch_adam(theta, grad, m, v, count, lr, beta1, beta2, eps, step, (hipStream_t)stream);
    return hip_status("ssnalm_mlp_adam");
}
