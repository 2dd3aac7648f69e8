// Small vector kernels of the Newton loop: fixed-order dot products,
// axpy-type updates and the elementwise pieces of u(omega).
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

static inline unsigned vec_grid(int64_t len) {
    int64_t b = (len + 2047) / 2048;
    if (b > 256) b = 256;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Sums of up to four columns of block partials (part[b * stride + c],
// b < nb) in block order, by one block, into the destinations of d.
__global__ __launch_bounds__(SSN_BLOCK) void k_colsum_fin(const double* __restrict__ part, int nb,
                                                          int stride, int ncols, ColSumDst d) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    if (d.skip && ld_grid(d.skip)) return;
    for (int c = 0; c < ncols; ++c) {
        const double t = grid_colsum(part, nb, stride, c, shd);
        if (threadIdx.x == 0 && d.p[c]) {
            if (d.as_ll[c]) *(long long*)d.p[c] = (long long)t;
            else *(double*)d.p[c] = t * d.scale[c];
        }
    }
}
void launch_colsum_fin(const double* part, int nb, int stride, int ncols, const ColSumDst& d,
                       hipStream_t s) {
    SSN_LAUNCH(k_colsum_fin, dim3(1), dim3(SSN_BLOCK), 0, s, part, nb, stride, ncols, d);
}
ColSumDst colsum_dst() {
    ColSumDst d;
    for (int c = 0; c < 4; ++c) {
        d.p[c] = nullptr;
        d.as_ll[c] = 0;
        d.scale[c] = 1.0;
    }
    d.skip = nullptr;
    return d;
}

// r_k = a_k . b_k for up to three pairs.  Block partials in part[3*b + k],
// combined in block order by a one-block finishing kernel.
__global__ __launch_bounds__(SSN_BLOCK) void k_dots(int npair, const double* __restrict__ a0,
                                                    const double* __restrict__ b0,
                                                    const double* __restrict__ a1,
                                                    const double* __restrict__ b1,
                                                    const double* __restrict__ a2,
                                                    const double* __restrict__ b2, int64_t len,
                                                    double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
        s0 = fma(a0[i], b0[i], s0);
        if (npair > 1) s1 = fma(a1[i], b1[i], s1);
        if (npair > 2) s2 = fma(a2[i], b2[i], s2);
    }
    const double t0 = block_sum(s0, shd);
    const double t1 = npair > 1 ? block_sum(s1, shd) : 0.0;
    const double t2 = npair > 2 ? block_sum(s2, shd) : 0.0;
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = t0;
        part[blockIdx.x * 3 + 1] = t1;
        part[blockIdx.x * 3 + 2] = t2;
    }
}

void launch_dots(int npair, const double* a0, const double* b0, double* r0, const double* a1,
                 const double* b1, double* r1, const double* a2, const double* b2, double* r2,
                 int64_t len, double* part, unsigned* counter, hipStream_t s) {
    (void)counter;
    const unsigned g = vec_grid(len);
    SSN_LAUNCH(k_dots, dim3(g), dim3(SSN_BLOCK), 0, s, npair, a0, b0, a1, b1, a2, b2, len,
                       part);
    ColSumDst d = colsum_dst();
    d.p[0] = r0;
    d.p[1] = npair > 1 ? r1 : nullptr;
    d.p[2] = npair > 2 ? r2 : nullptr;
    launch_colsum_fin(part, (int)g, 3, npair, d, s);
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) y[i] = fma(a, x[i], y[i]);
}
void launch_axpy(double* y, const double* x, double a, int64_t len, hipStream_t s) {
    SSN_LAUNCH(k_axpy, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, y, x, a, len);
}

__global__ void k_scale_copy(double* __restrict__ y, const double* __restrict__ x, double a,
                             int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) y[i] = a * x[i];
}
void launch_scale_copy(double* y, const double* x, double a, int64_t len, hipStream_t s) {
    SSN_LAUNCH(k_scale_copy, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, y, x, a,
                       len);
}

// u = x^k + sigma (e - A omega)   (u(w) of eq. Def_psi with c = -e, Q w = A omega)
// u = x^k - sigma (A omega + c) (eq. Def_psi); c = -e when lin is null
__global__ void k_u_from(const double* __restrict__ xk, const double* __restrict__ aw, double sigma,
                         const double* __restrict__ lin, double* __restrict__ u, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = fma(sigma, (lin ? -lin[i] : 1.0) - aw[i], xk[i]);
}
void launch_u_from(const double* xk, const double* aw, double sigma, double* u, int64_t n,
                   hipStream_t s, const double* lin) {
    SSN_LAUNCH(k_u_from, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xk, aw, sigma,
                       lin, u, n);
}

// ---------------------------------------------------------------- eps-SVR
// The eps-SVR dual (eq. Def_Dual_of_SVR_Problem) as an instance of (P) over
// the 2n variables [x; z]: B = [X; -X] = diag(a) [X; X] with a = [e; -e],
// c = [eps e + y; eps e - y].  Labels a and linear term c from the targets.
__global__ void k_svr_setup(const double* __restrict__ yr, int64_t n, double eps,
                            int8_t* __restrict__ a, double* __restrict__ lin) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = yr[i];
    a[i] = 1;
    a[n + i] = -1;
    lin[i] = eps + v;
    lin[n + i] = eps - v;
}
void launch_svr_setup(const double* yr, int64_t n, double eps, int8_t* a, double* lin, hipStream_t s) {
    SSN_LAUNCH(k_svr_setup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, yr, n, eps, a, lin);
}
// B v from X v (first n entries of t): t[n + i] = -t[i]
__global__ void k_svr_expand(double* __restrict__ t, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) t[n + i] = -t[i];
}
void launch_svr_expand(double* t, int64_t n, hipStream_t s) {
    SSN_LAUNCH(k_svr_expand, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, n);
}
// B^T z = X^T (z_top - z_bot); B_J^T a_J = X^T (mask_top + mask_bot)
__global__ void k_svr_fold(const double* __restrict__ z, const uint8_t* __restrict__ mask, int64_t n,
                           double* __restrict__ zc, uint8_t* __restrict__ mc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (zc) zc[i] = z ? z[i] - z[n + i] : 0.0;
    if (mask) mc[i] = (uint8_t)(mask[i] + mask[n + i]);
}
void launch_svr_fold(const double* z, const uint8_t* mask, int64_t n, double* zc, uint8_t* mc,
                     hipStream_t s) {
    SSN_LAUNCH(k_svr_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, mask, n, zc, mc);
}
// rows of the free list that index the second copy of X map to their row of X
__global__ void k_list_mod(int32_t* __restrict__ list, int64_t p, int32_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < p && list[k] >= n) list[k] -= n;
}
void launch_list_mod(int32_t* list, int64_t p, int64_t n, hipStream_t s) {
    if (p <= 0) return;
    SSN_LAUNCH(k_list_mod, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, list, p, (int32_t)n);
}

__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ o, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) o[i] = a[i] - b[i];
}
void launch_sub(const double* a, const double* b, double* out, int64_t len, hipStream_t s) {
    SSN_LAUNCH(k_sub, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, a, b, out, len);
}

// o = y .* z (the coefficients of X^T (y .* z), gathered once per entry)
__global__ void k_mul_y(const double* __restrict__ z, const int8_t* __restrict__ y,
                        double* __restrict__ o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = (double)y[i] * z[i];
}
void launch_mul_y(const double* z, const int8_t* y, double* out, int64_t n, hipStream_t s) {
    SSN_LAUNCH(k_mul_y, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, y, out, n);
}

// Column relabelling at the boundary: internal index perm[j] holds
// original column j.  to_internal: dst[perm[j]] = src[j]; otherwise
// dst[j] = src[perm[j]].
__global__ void k_permute(const double* __restrict__ src, const int32_t* __restrict__ perm,
                          double* __restrict__ dst, int64_t q, int to_internal) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    if (to_internal) dst[perm[j]] = src[j];
    else dst[j] = src[perm[j]];
}
void launch_permute(const double* src, const int32_t* perm, double* dst, int64_t q, bool to_internal,
                    hipStream_t s) {
    if (q <= 0) return;
    SSN_LAUNCH(k_permute, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, src, perm, dst,
                       q, to_internal ? 1 : 0);
}

__global__ void k_fill(double* __restrict__ p, double v, int64_t len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) p[i] = v;
}
void launch_fill(double* p, double v, int64_t len, hipStream_t s) {
    SSN_LAUNCH(k_fill, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, p, v, len);
}

}  // namespace ssn
