// C ABI of the RBF feature maps of Section 4 (random Fourier features and
// Nystroem features); the kernels are in kernels_features.hip.  The feature
// matrix Z is then an ordinary dense problem for ssnalm_create.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ssn_internal.h"

using namespace ssn;

namespace {

struct DevBufs {
    std::vector<void*> v;
    ~DevBufs() {
        for (void* p : v) (void)hipFree(p);
    }
    template <typename T>
    ssnalm_status get(T** p, int64_t count) {
        void* q = nullptr;
        const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(SSNALM_E_OOM, "feature workspace: allocation of %zu bytes failed", bytes);
        }
        v.push_back(q);
        *p = (T*)q;
        return SSNALM_OK;
    }
};

#define FCHK(expr)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_error(SSNALM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)
#define FST(expr)                          \
    do {                                   \
        ssnalm_status s_ = (expr);         \
        if (s_ < 0) return s_;             \
    } while (0)

ssnalm_status check_common(const void* X, int32_t dtype, int64_t n, int64_t q, const void* Z,
                           int32_t z_dtype) {
    if (!X || !Z) return set_error(SSNALM_E_BADARG, "null argument");
    if (n < 1 || q < 1 || n >= INT32_MAX || q >= INT32_MAX)
        return set_error(SSNALM_E_BADARG, "n and q must be in [1, 2^31)");
    if (dtype < SSNALM_F64 || dtype > SSNALM_BF16) return set_error(SSNALM_E_BADARG, "unknown dtype");
    if (z_dtype != SSNALM_F64 && z_dtype != SSNALM_F32)
        return set_error(SSNALM_E_BADARG, "z_dtype must be F64 or F32");
    return SSNALM_OK;
}

}  // namespace

extern "C" ssnalm_status ssnalm_rff_features(const void* X, int32_t dtype, int64_t n, int64_t q,
                                             const double* W, int64_t N, void* Z, int32_t z_dtype,
                                             void* stream) {
    FST(check_common(X, dtype, n, q, Z, z_dtype));
    if (!W) return set_error(SSNALM_E_BADARG, "null argument");
    if (N < 1 || N > 65535LL * 64) return set_error(SSNALM_E_BADARG, "N must be in [1, %lld]", 65535LL * 64);
    hipStream_t s = (hipStream_t)stream;
    launch_rff(dtype, X, n, q, W, N, Z, z_dtype == SSNALM_F64, s);
    FCHK(hipGetLastError());
    FCHK(hipStreamSynchronize(s));
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_nystroem_features(const void* X, int32_t dtype, int64_t n, int64_t q,
                                                  const int32_t* landmarks, int64_t r, double alpha,
                                                  double shift, void* Z, int32_t z_dtype,
                                                  void* stream) {
    FST(check_common(X, dtype, n, q, Z, z_dtype));
    if (!landmarks) return set_error(SSNALM_E_BADARG, "null argument");
    if (r < 1 || r > chol_blocked_max())
        return set_error(SSNALM_E_BADARG, "r must be in [1, %d]", chol_blocked_max());
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return set_error(SSNALM_E_BADARG, "alpha must be finite and > 0");
    if (!(shift >= 0.0) || !std::isfinite(shift)) return set_error(SSNALM_E_BADARG, "shift must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    // landmark indices are read on the host after the caller's stream wrote them
    FCHK(hipStreamSynchronize(s));
    {
        std::vector<int32_t> lh(r);
        FCHK(hipMemcpy(lh.data(), landmarks, sizeof(int32_t) * r, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < r; ++j)
            if (lh[j] < 0 || lh[j] >= n)
                return set_error(SSNALM_E_BADARG, "landmark %lld is %d, outside [0, n)", (long long)j, lh[j]);
    }
    DevBufs B;
    double *xn = nullptr, *ln = nullptr, *Krr = nullptr, *inv = nullptr, *Knr = nullptr;
    Scalars* sc = nullptr;
    FST(B.get(&xn, n));
    FST(B.get(&ln, r));
    FST(B.get(&Krr, r * r));
    FST(B.get(&inv, chol_inv_size(r)));
    FST(B.get(&Knr, n * r));
    FST(B.get(&sc, 1));
    double* Zw = (double*)Z;
    if (z_dtype != SSNALM_F64) FST(B.get(&Zw, n * r));
    FCHK(hipMemsetAsync(sc, 0, sizeof(Scalars), s));
    launch_row_norms(dtype, X, nullptr, n, q, xn, s);
    launch_row_norms(dtype, X, landmarks, r, q, ln, s);
    // K_rr + shift I, factored in place (L in the lower triangle)
    launch_rbf_block(dtype, X, q, landmarks, r, ln, landmarks, r, ln, alpha, shift, Krr, s);
    launch_chol_factor_blocked(Krr, r, inv, sc, s);
    launch_rbf_block(dtype, X, q, nullptr, n, xn, landmarks, r, ln, alpha, 0.0, Knr, s);
    launch_nys_solve(Knr, n, r, Krr, inv, Zw, s);
    if (z_dtype != SSNALM_F64) launch_copy_z(Zw, n * r, Z, 0, s);
    FCHK(hipGetLastError());
    int fail = 0;
    FCHK(hipMemcpyAsync(&fail, &sc->chol_fail, sizeof(int), hipMemcpyDeviceToHost, s));
    FCHK(hipStreamSynchronize(s));
    if (fail)
        return set_error(SSNALM_E_BADARG,
                         "K_rr + shift I is not positive definite (repeated landmarks need shift > 0)");
    return SSNALM_OK;
}
