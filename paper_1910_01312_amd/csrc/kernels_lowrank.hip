// Low-rank update of the dense Newton step (Algorithm 3, step 1, with the
// Cholesky factor of an earlier step at the same sigma).  Between two Newton
// steps at one sigma the Newton matrix M = I + sigma (X_J^T X_J - s s^T / p)
// changes by the rows that enter or leave J and by the two centring terms:
//   M = M0 + U S U^T,  U = [x_i (entering) | x_i (leaving) | s0/sqrt(p0) | s/sqrt(p)],
//   S = diag(+sigma | -sigma | +sigma | -sigma),
// so by the Woodbury identity, with the factor of M0,
//   -M^{-1} g = d0 + Z' T^{-1} (U^T d0),  d0 = -M0^{-1} g,  Z' = -M0^{-1} U,
//   T = S^{-1} + U^T M0^{-1} U = S^{-1} - U^T Z'.
// T is symmetric but indefinite (S has both signs).  With M0 and M both
// positive definite, the inertia of T equals that of S^{-1} (Haynsworth's
// inertia additivity on [[M0, U], [U^T, -S^{-1}]]), so after ordering the
// columns with S > 0 first, the leading block S_+^{-1} + U_+^T M0^{-1} U_+ is
// positive definite and its Schur complement negative definite: T = L D L^T
// exists in that order without pivoting, with D > 0 on the first block and
// D < 0 on the second.  A pivot of the wrong sign (rounding) is reported as a
// factorisation failure and the step falls back to -g.
#include "dev_common.h"
#include "lane_ops.h"
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

constexpr int LR_MAX = 96;
constexpr int LR_TG = 16;                   // thread grid 16 x 16 over T
constexpr int LR_TT = LR_MAX / LR_TG;       // each thread holds a 6 x 6 register tile
static_assert(LR_TG * LR_TG == SSN_BLOCK, "one thread per tile");

// T = L D L^T in the order perm (columns with wgt > 0 first, each group in
// its original order); perm[r] = the column of T at position r.  Output in Tm
// (k x k, row-major, positions after perm): L[i][c] below the diagonal, D on
// it.  Thread (tr, tc) holds rows tr + 16a and columns tc + 16b of the
// permuted T; step c broadcasts column c through LDS (double-buffered, one
// barrier per column) and every thread applies the rank-one update to its
// tile; L and D collect in LDS and go to Tm at the end, so no global store is
// outstanding at a barrier.
__global__ __launch_bounds__(SSN_BLOCK) void k_lr_ldl(double* __restrict__ Tm, int k,
                                                      const double* __restrict__ wgt,
                                                      int32_t* __restrict__ perm, Scalars* sc) {
    __shared__ double colb[2][LR_MAX];
    __shared__ double Lsh[LR_MAX][LR_MAX + 1];   // L below the diagonal, D on it
    __shared__ int pm[LR_MAX];
    __shared__ int npos_s;
    const int tid = threadIdx.x, lane = tid & (SSN_WAVE - 1);
    const int tr = tid / LR_TG, tc = tid % LR_TG;
    if (tid < SSN_WAVE) {
        // stable partition by the sign of wgt with two ballots (k <= 128)
        const bool v0 = lane < k, v1 = lane + SSN_WAVE < k;
        const bool f0 = v0 && wgt[lane] > 0.0, f1 = v1 && wgt[lane + SSN_WAVE] > 0.0;
        const unsigned long long b0 = __ballot(f0), b1 = __ballot(f1);
        const unsigned long long lt = (1ull << lane) - 1ull;
        const int n0 = __popcll(b0), npos = n0 + __popcll(b1);
        const int r0 = __popcll(b0 & lt), r1 = __popcll(b1 & lt);
        if (v0) pm[f0 ? r0 : npos + (lane - r0)] = lane;
        if (v1) pm[f1 ? n0 + r1 : npos + (SSN_WAVE - n0) + (lane - r1)] = lane + SSN_WAVE;
        if (lane == 0) npos_s = npos;
    }
    __syncthreads();
    const int npos = npos_s;
    double A[LR_TT][LR_TT];
#pragma unroll
    for (int a = 0; a < LR_TT; ++a) {
        const int i = tr + LR_TG * a;
#pragma unroll
        for (int b = 0; b < LR_TT; ++b) {
            const int j = tc + LR_TG * b;
            A[a][b] = (i < k && j < k) ? Tm[pm[i] * k + pm[j]] : 0.0;
        }
    }
    __syncthreads();                 // every read of Tm before its overwrite
    bool bad = false;
    for (int c = 0; c < k; ++c) {
        double* cb = colb[c & 1];
        if (tc == (c % LR_TG)) {
            const int bc = c / LR_TG;
#pragma unroll
            for (int b = 0; b < LR_TT; ++b)
                if (b == bc) {
#pragma unroll
                    for (int a = 0; a < LR_TT; ++a) cb[tr + LR_TG * a] = A[a][b];
                }
        }
        __syncthreads();
        const double d = cb[c];
        if (!(c < npos ? d > 0.0 : d < 0.0)) bad = true;
        const double inv = d != 0.0 ? 1.0 / d : 0.0;
        double li[LR_TT], vj[LR_TT];
#pragma unroll
        for (int a = 0; a < LR_TT; ++a) {
            const int i = tr + LR_TG * a;
            li[a] = i > c && i < k ? cb[i] * inv : 0.0;
        }
#pragma unroll
        for (int b = 0; b < LR_TT; ++b) {
            const int j = tc + LR_TG * b;
            vj[b] = j > c && j < k ? cb[j] : 0.0;
        }
        if (tc == (c % LR_TG)) {
#pragma unroll
            for (int a = 0; a < LR_TT; ++a) {
                const int i = tr + LR_TG * a;
                if (i > c && i < k) Lsh[i][c] = li[a];
            }
            if (tr == 0) Lsh[c][c] = d;
        }
#pragma unroll
        for (int a = 0; a < LR_TT; ++a)
#pragma unroll
            for (int b = 0; b < LR_TT; ++b) A[a][b] = fma(-li[a], vj[b], A[a][b]);
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        if (j <= i) Tm[e] = Lsh[i][j];
    }
    for (int r = tid; r < k; r += blockDim.x) perm[r] = pm[r];
    if (bad && tid == 0) sc->chol_fail = 1;
}

// out = d0 + Zn c,  c = T^{-1} (U^T d0) with T = P^T L D L^T P from k_lr_ldl;
// out may be d0.  One workgroup of 1024 threads, so that the k x q reads of U
// and Zn have many loads in flight: U^T d0 with LR_CG columns per wave at a
// time; L (strictly lower, zero elsewhere) staged in LDS; the two triangular
// solves in wave 0 in column (axpy) form with the right-hand side in
// registers (lane l holds entries l and l + 64) and each solved entry
// broadcast by readlane, so no reduction and no barrier per row; then Zn c
// with the columns split in two halves summed through LDS.
constexpr int LR_APPLY_BLOCK = 1024;
constexpr int LR_APPLY_WAVES = LR_APPLY_BLOCK / SSN_WAVE;
constexpr int LR_CG = 6;
__global__ __launch_bounds__(LR_APPLY_BLOCK) void k_lr_apply(const double* __restrict__ U,
                                                             const double* __restrict__ Zn, int64_t q, int k,
                                                             const double* __restrict__ LD,
                                                             const int32_t* __restrict__ perm,
                                                             const double* d0, double* out) {
    __shared__ double Ls[LR_MAX][LR_MAX + 1];
    __shared__ double wv[LR_MAX], cv[LR_MAX], dv[LR_MAX];
    __shared__ int pm[LR_MAX];
    __shared__ double part[LR_APPLY_BLOCK / 2];
    const int tid = threadIdx.x, lane = tid & (SSN_WAVE - 1), wid = tid / SSN_WAVE;
    for (int e = tid; e < LR_MAX * LR_MAX; e += blockDim.x) {
        const int i = e / LR_MAX, j = e % LR_MAX;
        Ls[i][j] = (i < k && j < i) ? LD[i * k + j] : 0.0;
    }
    for (int r = tid; r < k; r += blockDim.x) {
        dv[r] = LD[r * k + r];
        pm[r] = perm[r];
    }
    // w = U^T d0 in the original column order; wave w takes columns
    // w, w + 16, ... in groups of LR_CG
    for (int a0 = wid; a0 < k; a0 += LR_APPLY_WAVES * LR_CG) {
        double t[LR_CG];
#pragma unroll
        for (int g = 0; g < LR_CG; ++g) t[g] = 0.0;
        for (int64_t j = lane; j < q; j += SSN_WAVE) {
            const double dj = d0[j];
#pragma unroll
            for (int g = 0; g < LR_CG; ++g) {
                const int a = a0 + g * LR_APPLY_WAVES;
                if (a < k) t[g] = fma(U[(int64_t)a * q + j], dj, t[g]);
            }
        }
#pragma unroll
        for (int g = 0; g < LR_CG; ++g) {
            const int a = a0 + g * LR_APPLY_WAVES;
            const double v = wave_sum(t[g]);
            if (a < k && lane == 0) wv[a] = v;
        }
    }
    __syncthreads();
    if (wid == 0) {
        const int l1 = lane + SSN_WAVE;
        double y0 = lane < k ? wv[pm[lane]] : 0.0;
        double y1 = l1 < k ? wv[pm[l1]] : 0.0;
        for (int r = 0; r < k; ++r) {                // L y = P w
            const double cr = r < SSN_WAVE ? readlane_f64(y0, r) : readlane_f64(y1, r - SSN_WAVE);
            y0 = fma(-Ls[lane][r], cr, y0);
            if (l1 < LR_MAX) y1 = fma(-Ls[l1][r], cr, y1);
        }
        if (lane < k) y0 /= dv[lane];                // D z = y
        if (l1 < k) y1 /= dv[l1];
        for (int r = k - 1; r >= 0; --r) {           // L^T (P c) = z
            const double cr = r < SSN_WAVE ? readlane_f64(y0, r) : readlane_f64(y1, r - SSN_WAVE);
            y0 = fma(-Ls[r][lane], cr, y0);
            if (l1 < LR_MAX) y1 = fma(-Ls[r][l1], cr, y1);
        }
        if (lane < k) cv[pm[lane]] = y0;
        if (l1 < k) cv[pm[l1]] = y1;
    }
    __syncthreads();
    // out = d0 + Zn c: threads [0, 512) take columns [0, kh), the others [kh, k)
    const int half = tid / (LR_APPLY_BLOCK / 2), ht = tid % (LR_APPLY_BLOCK / 2);
    const int kh = (k + 1) / 2, a_lo = half ? kh : 0, a_hi = half ? k : kh;
    for (int64_t j0 = 0; j0 < q; j0 += LR_APPLY_BLOCK / 2) {
        const int64_t j = j0 + ht;
        double t = 0.0;
        if (j < q) {
#pragma unroll 8
            for (int a = a_lo; a < a_hi; ++a) t = fma(Zn[(int64_t)a * q + j], cv[a], t);
        }
        if (half) part[ht] = t;
        __syncthreads();
        if (!half && j < q) out[j] = d0[j] + t + part[ht];
        __syncthreads();
    }
}

int lowrank_max() { return LR_MAX; }

void launch_lr_factor(const double* U, const double* Zn, int64_t q, int k, const double* wgt, double* Tm,
                      int32_t* perm, Scalars* sc, hipStream_t s) {
    SSN_LAUNCH(k_lr_gram, dim3((unsigned)k, (unsigned)k), dim3(SSN_BLOCK), 0, s, U, Zn, q, k, wgt, Tm);
    SSN_LAUNCH(k_lr_ldl, dim3(1), dim3(SSN_BLOCK), 0, s, Tm, k, wgt, perm, sc);
}
void launch_lr_apply(const double* U, const double* Zn, int64_t q, int k, const double* LD, const int32_t* perm,
                     const double* d0, double* out, hipStream_t s) {
    SSN_LAUNCH(k_lr_apply, dim3(1), dim3(LR_APPLY_BLOCK), 0, s, U, Zn, q, k, LD, perm, d0, out);
}

}  // namespace ssn
