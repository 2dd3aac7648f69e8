// Feature maps that turn the RBF-kernel C-SVC into a linear one (Section 4):
// random Fourier features and Nystroem features.  The linear solver then
// runs unchanged on the feature matrix Z (Q ~ diag(y) Z Z^T diag(y)).
// Also the exact kernel matrix Q of the nonlinear C-SVC (Section 1, eq.
// Def_Dual_of_C_SVM_Problem), formed once for the w-space solver.
//
// RBF kernel (Section 1): k(x, z) = exp(-|x - z|^2 / (2 alpha)).
//   Random Fourier features: frequencies w_1..w_N drawn by the caller from
//   the Gaussian with covariance I / alpha (the spectral density of k by
//   Bochner's theorem); Z[i][2k] = cos(w_k^T x_i) / sqrt(N),
//   Z[i][2k+1] = sin(w_k^T x_i) / sqrt(N), so Z Z^T averages the N sampled
//   kernels.
//   Nystroem: r landmark rows l_j; K_nr[i][j] = k(x_i, l_j), K_rr + s I =
//   L L^T, Z = K_nr L^{-T} (n x r), so Z Z^T = K_nr (K_rr + s I)^{-1} K_nr^T.
//
// Every product is a 64 x 64 tile of an "A B^T" contraction over the
// feature dimension, staged through LDS in 16-wide slices, accumulated in
// fp64 (4 x 4 outputs per thread), with the map applied in the epilogue
// (cos / sin, the kernel's exp, or the triangular-solve steps).
#include <cmath>

#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int FT = 64;          // tile rows / columns
constexpr int FK = 16;          // contraction slice

// acc[a][b] += sum_k A(r0 + 4 ty + a, k) B(c0 + 4 tx + b, k) for k < K,
// with A(i, k), B(j, k) fetched by the loaders (which return 0 out of range).
template <class LA, class LB>
__device__ __forceinline__ void tile_nt(const LA& la, const LB& lb, int64_t r0, int64_t c0, int64_t K,
                                        double (&acc)[4][4], double (*sA)[FT + 1],
                                        double (*sB)[FT + 1]) {
    const int t = threadIdx.x;
    const int tx = t % 16, ty = t / 16;
    for (int64_t k0 = 0; k0 < K; k0 += FK) {
        // 64 x 16 of each operand: 4 elements per thread, stored k-major
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + e * SSN_BLOCK;         // 0 .. 1023
            const int rr = idx / FK, kk = idx % FK;
            sA[kk][rr] = la(r0 + rr, k0 + kk);
            sB[kk][rr] = lb(c0 + rr, k0 + kk);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < FK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sA[kk][4 * ty + u];
                b[u] = sB[kk][4 * tx + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
}

// Row i, column k of a dense row-major matrix of any storage type (0 outside).
template <typename T>
struct RowLoader {
    const T* X;
    const int32_t* rows;        // optional row indirection (landmarks)
    int64_t n, q;
    __device__ __forceinline__ double operator()(int64_t i, int64_t k) const {
        if (i >= n || k >= q) return 0.0;
        const int64_t r = rows ? (int64_t)rows[i] : i;
        return to_f64(X[r * q + k]);
    }
};

template <typename ZT>
__device__ __forceinline__ void store_z(ZT* Z, int64_t idx, double v) { Z[idx] = (ZT)v; }

// ---------------------------------------------------------------- RFF
// One 64 x 64 tile of P = X W^T (rows of X, frequencies), then the cos / sin
// pairs of P written to Z (n x 2N).
template <typename T, typename ZT>
__global__ __launch_bounds__(SSN_BLOCK) void k_rff(const T* __restrict__ X, int64_t n, int64_t q,
                                                   const double* __restrict__ W, int64_t N,
                                                   ZT* __restrict__ Z, double scale) {
    __shared__ double sA[FK][FT + 1];
    __shared__ double sB[FK][FT + 1];
    const int64_t r0 = (int64_t)blockIdx.x * FT, c0 = (int64_t)blockIdx.y * FT;
    double acc[4][4] = {};
    RowLoader<T> la{X, nullptr, n, q};
    RowLoader<double> lb{W, nullptr, N, q};
    tile_nt(la, lb, r0, c0, q, acc, sA, sB);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 4 * ty + u;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t k = c0 + 4 * tx + v;
            if (k >= N) continue;
            double s, c;
            sincos(acc[u][v], &s, &c);
            store_z(Z, i * 2 * N + 2 * k, c * scale);
            store_z(Z, i * 2 * N + 2 * k + 1, s * scale);
        }
    }
}

// ---------------------------------------------------------------- Nystroem
// Squared norms of rows (optionally through a row list).
template <typename T>
__global__ __launch_bounds__(SSN_BLOCK) void k_row_norms(const T* __restrict__ X, const int32_t* rows,
                                                         int64_t n, int64_t q, double* __restrict__ out) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t i = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (i >= n) return;
    const int64_t r = rows ? (int64_t)rows[i] : i;
    double s = 0.0;
    for (int64_t k = lane; k < q; k += SSN_WAVE) {
        const double v = to_f64(X[r * q + k]);
        s = fma(v, v, s);
    }
    s = wave_sum(s);
    if (lane == 0) out[i] = s;
}

// K[i][j] = exp(-max(|a_i|^2 + |b_j|^2 - 2 a_i . b_j, 0) / (2 alpha)) for
// rows a of X (all, or the landmarks) and landmark rows b; plus `shift` on
// the diagonal when the two row sets are the same (K_rr + s I).
template <typename T>
__global__ __launch_bounds__(SSN_BLOCK) void k_rbf_block(const T* __restrict__ X, int64_t q,
                                                         const int32_t* arows, int64_t na,
                                                         const double* __restrict__ anorm,
                                                         const int32_t* __restrict__ lm, int64_t r,
                                                         const double* __restrict__ lnorm,
                                                         double inv2a, double shift,
                                                         double* __restrict__ K) {
    __shared__ double sA[FK][FT + 1];
    __shared__ double sB[FK][FT + 1];
    const int64_t r0 = (int64_t)blockIdx.x * FT, c0 = (int64_t)blockIdx.y * FT;
    double acc[4][4] = {};
    RowLoader<T> la{X, arows, na, q};
    RowLoader<T> lb{X, lm, r, q};
    tile_nt(la, lb, r0, c0, q, acc, sA, sB);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 4 * ty + u;
        if (i >= na) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t j = c0 + 4 * tx + v;
            if (j >= r) continue;
            const double d2 = fmax(anorm[i] + lnorm[j] - 2.0 * acc[u][v], 0.0);
            double kv = exp(-d2 * inv2a);
            if (arows && i == j) kv += shift;
            K[i * r + j] = kv;
        }
    }
}

// Q_ij = y_i y_j k(x_i, x_j) for the kernel C-SVC (all n x n entries, row
// stride ld, columns n .. ld-1 set to zero): one 64 x 64 tile per block,
// blockIdx.x the column tile, blockIdx.y the row tile.  Both (i, j) and
// (j, i) sum their products in the same order, so Q is exactly symmetric;
// the RBF diagonal is exactly 1.
template <typename T>
__global__ __launch_bounds__(SSN_BLOCK) void k_kernel_q(const T* __restrict__ X, int64_t n, int64_t q,
                                                        const double* __restrict__ norms,
                                                        const int8_t* __restrict__ y, int rbf,
                                                        double inv2a, double* __restrict__ Q,
                                                        int64_t ld) {
    __shared__ double sA[FK][FT + 1];
    __shared__ double sB[FK][FT + 1];
    const int64_t r0 = (int64_t)blockIdx.y * FT, c0 = (int64_t)blockIdx.x * FT;
    double acc[4][4] = {};
    RowLoader<T> la{X, nullptr, n, q};
    if (c0 < n) tile_nt(la, la, r0, c0, q, acc, sA, sB);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 4 * ty + u;
        if (i >= n) continue;
        const double yi = (double)y[i];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t j = c0 + 4 * tx + v;
            if (j >= ld) continue;
            double kv = 0.0;
            if (j < n) {
                if (rbf) {
                    const double d2 = i == j ? 0.0 : fmax(norms[i] + norms[j] - 2.0 * acc[u][v], 0.0);
                    kv = exp(-d2 * inv2a);
                } else {
                    kv = acc[u][v];
                }
                kv *= yi * (double)y[j];
            }
            Q[i * ld + j] = kv;
        }
    }
}

// Block column b of Z = K L^{-T} (64 rows of Z per workgroup):
//   Y = K[:, b] - Z[:, <b] L[b, <b]^T,   Z[:, b] = Y X_b^T,  X_b = L_bb^{-1},
// with the factor L in the lower triangle of F (r x r, row-major) and X_b
// row-major in inv (per 64 x 64 block: X_b then X_b^T).  Z is written in
// fp64 to Zw (n x r, the working copy read by later block columns).
__global__ __launch_bounds__(SSN_BLOCK) void k_nys_solve_block(const double* __restrict__ K, int64_t n,
                                                               int64_t r, const double* __restrict__ F,
                                                               const double* __restrict__ inv, int b,
                                                               double* __restrict__ Zw) {
    __shared__ double sA[FK][FT + 1];
    __shared__ double sB[FK][FT + 1];
    __shared__ double sY[FT][FT + 1];
    const int64_t r0 = (int64_t)blockIdx.x * FT;
    const int64_t o = (int64_t)b * FT;
    const int m = (int)min<int64_t>(FT, r - o);
    double acc[4][4] = {};
    struct ZLoad {
        const double* Zw; int64_t n, r, cmax;
        __device__ double operator()(int64_t i, int64_t k) const {
            return (i < n && k < cmax) ? Zw[i * r + k] : 0.0;
        }
    } lz{Zw, n, r, o};
    struct LLoad {
        const double* F; int64_t r, o, m, cmax;
        __device__ double operator()(int64_t j, int64_t k) const {   // L[o + j][k]
            return (j < m && k < cmax) ? F[(o + j) * r + k] : 0.0;
        }
    } ll{F, r, o, m, o};
    if (o > 0) tile_nt(lz, ll, r0, 0, o, acc, sA, sB);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 4 * ty + u;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = 4 * tx + v;
            const double kv = (i < n && j < m) ? K[i * r + o + j] : 0.0;
            sY[4 * ty + u][j] = kv - acc[u][v];
        }
    }
    __syncthreads();
    // Z[i][o + k'] = sum_k Y[i][k] X_b[k'][k]
    const double* Xb = inv + (int64_t)b * 2 * FT * FT;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = r0 + 4 * ty + u;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kp = 4 * tx + v;
            double z = 0.0;
            for (int k = 0; k < FT; ++k) z = fma(sY[4 * ty + u][k], Xb[kp * FT + k], z);
            if (i < n && kp < m) Zw[i * r + o + kp] = z;
        }
    }
}

template <typename ZT>
__global__ void k_copy_z(const double* __restrict__ Zw, int64_t count, ZT* __restrict__ Z) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride)
        Z[k] = (ZT)Zw[k];
}

// ---------------------------------------------------------------- launchers
#define FEAT_DISPATCH_X(dtype, FN, ...)                                    \
    do {                                                                  \
        if ((dtype) == SSNALM_F64) FN<double>(__VA_ARGS__);               \
        else if ((dtype) == SSNALM_F32) FN<float>(__VA_ARGS__);           \
        else FN<bf16_t>(__VA_ARGS__);                                     \
    } while (0)

template <typename T>
static void rff_t(const void* X, int64_t n, int64_t q, const double* W, int64_t N, void* Z,
                  int z_f64, hipStream_t s) {
    const dim3 grid((unsigned)((n + FT - 1) / FT), (unsigned)((N + FT - 1) / FT));
    const double scale = 1.0 / std::sqrt((double)N);
    if (z_f64)
        SSN_LAUNCH((k_rff<T, double>), grid, dim3(SSN_BLOCK), 0, s, (const T*)X, n, q, W, N,
                   (double*)Z, scale);
    else
        SSN_LAUNCH((k_rff<T, float>), grid, dim3(SSN_BLOCK), 0, s, (const T*)X, n, q, W, N,
                   (float*)Z, scale);
}
void launch_rff(int dtype, const void* X, int64_t n, int64_t q, const double* W, int64_t N, void* Z,
                int z_f64, hipStream_t s) {
    FEAT_DISPATCH_X(dtype, rff_t, X, n, q, W, N, Z, z_f64, s);
}

template <typename T>
static void norms_t(const void* X, const int32_t* rows, int64_t n, int64_t q, double* out,
                    hipStream_t s) {
    SSN_LAUNCH((k_row_norms<T>), dim3((unsigned)((n + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK)),
               dim3(SSN_BLOCK), 0, s, (const T*)X, rows, n, q, out);
}
void launch_row_norms(int dtype, const void* X, const int32_t* rows, int64_t n, int64_t q,
                      double* out, hipStream_t s) {
    FEAT_DISPATCH_X(dtype, norms_t, X, rows, n, q, out, s);
}

template <typename T>
static void rbf_t(const void* X, int64_t q, const int32_t* arows, int64_t na, const double* anorm,
                  const int32_t* lm, int64_t r, const double* lnorm, double alpha, double shift,
                  double* K, hipStream_t s) {
    const dim3 grid((unsigned)((na + FT - 1) / FT), (unsigned)((r + FT - 1) / FT));
    SSN_LAUNCH((k_rbf_block<T>), grid, dim3(SSN_BLOCK), 0, s, (const T*)X, q, arows, na, anorm, lm, r,
               lnorm, 0.5 / alpha, shift, K);
}
void launch_rbf_block(int dtype, const void* X, int64_t q, const int32_t* arows, int64_t na,
                      const double* anorm, const int32_t* lm, int64_t r, const double* lnorm,
                      double alpha, double shift, double* K, hipStream_t s) {
    FEAT_DISPATCH_X(dtype, rbf_t, X, q, arows, na, anorm, lm, r, lnorm, alpha, shift, K, s);
}

template <typename T>
static void kernel_q_t(const void* X, int64_t n, int64_t q, const double* norms, const int8_t* y,
                       int rbf, double alpha, double* Q, int64_t ld, hipStream_t s) {
    const dim3 grid((unsigned)((ld + FT - 1) / FT), (unsigned)((n + FT - 1) / FT));
    SSN_LAUNCH((k_kernel_q<T>), grid, dim3(SSN_BLOCK), 0, s, (const T*)X, n, q, norms, y, rbf,
               rbf ? 0.5 / alpha : 0.0, Q, ld);
}
void launch_kernel_q(int dtype, const void* X, int64_t n, int64_t q, const double* norms,
                     const int8_t* y, int rbf, double alpha, double* Q, int64_t ld, hipStream_t s) {
    FEAT_DISPATCH_X(dtype, kernel_q_t, X, n, q, norms, y, rbf, alpha, Q, ld, s);
}

void launch_nys_solve(const double* K, int64_t n, int64_t r, const double* F, const double* inv,
                      double* Zw, hipStream_t s) {
    const unsigned gb = (unsigned)((n + FT - 1) / FT);
    const int nb = (int)((r + FT - 1) / FT);
    for (int b = 0; b < nb; ++b)
        SSN_LAUNCH(k_nys_solve_block, dim3(gb), dim3(SSN_BLOCK), 0, s, K, n, r, F, inv, b, Zw);
}

void launch_copy_z(const double* Zw, int64_t count, void* Z, int z_f64, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>((count + SSN_BLOCK - 1) / SSN_BLOCK, 8192);
    if (z_f64)
        SSN_LAUNCH((k_copy_z<double>), dim3(g), dim3(SSN_BLOCK), 0, s, Zw, count, (double*)Z);
    else
        SSN_LAUNCH((k_copy_z<float>), dim3(g), dim3(SSN_BLOCK), 0, s, Zw, count, (float*)Z);
}

}  // namespace ssn
