// Low-rank update of the dense Newton step (Algorithm 3, step 1, with the
// Cholesky factor of an earlier step at the same sigma).  Between two Newton
// steps at one sigma the Newton matrix M = I + sigma (X_J^T X_J - s s^T / p)
// changes by the rows that enter or leave J and by the two centring terms:
//   M = M0 + U S U^T,  U = [x_i (entering) | x_i (leaving) | s0/sqrt(p0) | s/sqrt(p)],
//   S = diag(+sigma | -sigma | +sigma | -sigma),
// so by the Woodbury identity, with the factor of M0,
//   -M^{-1} g = d0 + Z' T^{-1} (U^T d0),  d0 = -M0^{-1} g,  Z' = -M0^{-1} U,
//   T = S^{-1} + U^T M0^{-1} U = S^{-1} - U^T Z'.
// T is symmetric but indefinite (S has both signs); it is factored by LU
// with partial pivoting in one workgroup.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

// out[i] = (a[i] != b[i])
__global__ void k_mask_diff(const uint8_t* __restrict__ a, const uint8_t* __restrict__ b, int64_t n,
                            uint8_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] != b[i] ? 1 : 0;
}
void launch_mask_diff(const uint8_t* a, const uint8_t* b, int64_t n, uint8_t* out, hipStream_t s) {
    SSN_LAUNCH(k_mask_diff, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n, out);
}

// Column c of U (q doubles, column-major) and its weight: c < nchg: row
// chg[c] of X, +sigma when it is in the new J (entering), -sigma otherwise;
// then s0 / sqrt(p0) (+sigma) when p0 > 0, then s / sqrt(p) (-sigma) when p > 0.
template <typename T>
__global__ __launch_bounds__(SSN_BLOCK) void k_lr_build(const T* __restrict__ X, int64_t q,
                                                        const int32_t* __restrict__ chg, int nchg,
                                                        const uint8_t* __restrict__ mask, double sigma,
                                                        const double* __restrict__ s0, double p0,
                                                        const double* __restrict__ s1, double p1,
                                                        double* __restrict__ U, double* __restrict__ wgt) {
    const int c = blockIdx.x;
    double* col = U + (int64_t)c * q;
    if (c < nchg) {
        const int64_t row = chg[c];
        const T* xr = X + row * q;
        for (int64_t j = threadIdx.x; j < q; j += blockDim.x) col[j] = to_f64(xr[j]);
        if (threadIdx.x == 0) wgt[c] = mask[row] ? sigma : -sigma;
        return;
    }
    const bool old = (c == nchg) && p0 > 0.0;
    const double* sv = old ? s0 : s1;
    const double sc = 1.0 / sqrt(old ? p0 : p1);
    for (int64_t j = threadIdx.x; j < q; j += blockDim.x) col[j] = sv[j] * sc;
    if (threadIdx.x == 0) wgt[c] = old ? sigma : -sigma;
}
void launch_lr_build(int dtype, const void* X, int64_t q, const int32_t* chg, int nchg, const uint8_t* mask,
                     double sigma, const double* s0, int64_t p0, const double* s1, int64_t p1, double* U,
                     double* wgt, int k, hipStream_t s) {
    if (k <= 0) return;
#define LRB(T) SSN_LAUNCH((k_lr_build<T>), dim3((unsigned)k), dim3(SSN_BLOCK), 0, s, (const T*)X, q, chg, nchg, \
                          mask, sigma, s0, (double)p0, s1, (double)p1, U, wgt)
    if (dtype == SSNALM_F64) LRB(double);
    else if (dtype == SSNALM_F32) LRB(float);
    else LRB(bf16_t);
#undef LRB
}

// T[a][b] = (a == b ? 1 / wgt[a] : 0) - U[:, a] . Zn[:, b]  (one block per entry)
__global__ __launch_bounds__(SSN_BLOCK) void k_lr_gram(const double* __restrict__ U,
                                                       const double* __restrict__ Zn, int64_t q, int k,
                                                       const double* __restrict__ wgt,
                                                       double* __restrict__ Tm) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int a = blockIdx.x, b = blockIdx.y;
    const double* ua = U + (int64_t)a * q;
    const double* zb = Zn + (int64_t)b * q;
    double t = 0.0;
    for (int64_t j = threadIdx.x; j < q; j += blockDim.x) t = fma(ua[j], zb[j], t);
    t = block_sum(t, sh);
    if (threadIdx.x == 0) Tm[a * k + b] = (a == b ? 1.0 / wgt[a] : 0.0) - t;
}

// LU with partial pivoting of T (k x k, row-major) in place, in LDS; piv[r]
// = the original row now at position r.  One workgroup.
constexpr int LR_MAX = 96;
__global__ __launch_bounds__(SSN_BLOCK) void k_lr_lu(double* __restrict__ Tm, int k, int32_t* __restrict__ piv,
                                                     Scalars* sc) {
    __shared__ double A[LR_MAX][LR_MAX + 1];
    __shared__ int P[LR_MAX];
    __shared__ int pr;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) A[e / k][e % k] = Tm[e];
    for (int r = threadIdx.x; r < k; r += blockDim.x) P[r] = r;
    __syncthreads();
    bool bad = false;
    for (int c = 0; c < k; ++c) {
        if (threadIdx.x == 0) {
            int best = c;
            double bv = fabs(A[c][c]);
            for (int r = c + 1; r < k; ++r)
                if (fabs(A[r][c]) > bv) { bv = fabs(A[r][c]); best = r; }
            pr = best;
        }
        __syncthreads();
        const int r0 = pr;
        if (r0 != c) {
            for (int j = threadIdx.x; j < k; j += blockDim.x) {
                const double t = A[c][j];
                A[c][j] = A[r0][j];
                A[r0][j] = t;
            }
            if (threadIdx.x == 0) { const int t = P[c]; P[c] = P[r0]; P[r0] = t; }
        }
        __syncthreads();
        const double pv = A[c][c];
        if (!(fabs(pv) > 0.0)) bad = true;
        // multipliers, then the trailing update (row r, column j > c)
        for (int r = c + 1 + threadIdx.x; r < k; r += blockDim.x) A[r][c] = pv != 0.0 ? A[r][c] / pv : 0.0;
        __syncthreads();
        const int w = k - c - 1;
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
            const int r = c + 1 + e / w, j = c + 1 + e % w;
            A[r][j] = fma(-A[r][c], A[c][j], A[r][j]);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) Tm[e] = A[e / k][e % k];
    for (int r = threadIdx.x; r < k; r += blockDim.x) piv[r] = P[r];
    if (bad && threadIdx.x == 0) sc->chol_fail = 1;
}

// out = d0 + Zn c,  c = T^{-1} (U^T d0), with T's LU and pivots; out may be d0.
__global__ __launch_bounds__(SSN_BLOCK) void k_lr_apply(const double* __restrict__ U,
                                                        const double* __restrict__ Zn, int64_t q, int k,
                                                        const double* __restrict__ LU,
                                                        const int32_t* __restrict__ piv,
                                                        const double* d0, double* out) {
    __shared__ double wv[LR_MAX], cv[LR_MAX];
    const int lane = threadIdx.x & (SSN_WAVE - 1), wid = threadIdx.x / SSN_WAVE;
    // w = U^T d0, one wave per column
    for (int a = wid; a < k; a += SSN_WAVES_PER_BLOCK) {
        const double* ua = U + (int64_t)a * q;
        double t = 0.0;
        for (int64_t j = lane; j < q; j += SSN_WAVE) t = fma(ua[j], d0[j], t);
        t = wave_sum(t);
        if (lane == 0) wv[a] = t;
    }
    __syncthreads();
    // L y = P w, U c = y: one row per step, summed by wave 0; every wave
    // takes part in the step's barrier
    for (int r = 0; r < k; ++r) {
        if (wid == 0) {
            double t = 0.0;
            for (int j = lane; j < r; j += SSN_WAVE) t = fma(LU[r * k + j], cv[j], t);
            t = wave_sum(t);
            if (lane == 0) cv[r] = wv[piv[r]] - t;
        }
        __syncthreads();
    }
    for (int r = k - 1; r >= 0; --r) {
        if (wid == 0) {
            double t = 0.0;
            for (int j = r + 1 + lane; j < k; j += SSN_WAVE) t = fma(LU[r * k + j], cv[j], t);
            t = wave_sum(t);
            if (lane == 0) cv[r] = (cv[r] - t) / LU[r * k + r];
        }
        __syncthreads();
    }
    for (int64_t j = threadIdx.x; j < q; j += blockDim.x) {
        double t = d0[j];
        for (int a = 0; a < k; ++a) t = fma(Zn[(int64_t)a * q + j], cv[a], t);
        out[j] = t;
    }
}

int lowrank_max() { return LR_MAX; }

void launch_lr_factor(const double* U, const double* Zn, int64_t q, int k, const double* wgt, double* Tm,
                      int32_t* piv, Scalars* sc, hipStream_t s) {
    SSN_LAUNCH(k_lr_gram, dim3((unsigned)k, (unsigned)k), dim3(SSN_BLOCK), 0, s, U, Zn, q, k, wgt, Tm);
    SSN_LAUNCH(k_lr_lu, dim3(1), dim3(SSN_BLOCK), 0, s, Tm, k, piv, sc);
}
void launch_lr_apply(const double* U, const double* Zn, int64_t q, int k, const double* LU, const int32_t* piv,
                     const double* d0, double* out, hipStream_t s) {
    SSN_LAUNCH(k_lr_apply, dim3(1), dim3(SSN_BLOCK), 0, s, U, Zn, q, k, LU, piv, d0, out);
}

}  // namespace ssn
