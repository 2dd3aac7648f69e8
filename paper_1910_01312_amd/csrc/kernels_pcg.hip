// Matrix-free preconditioned conjugate gradients for step 1 of Algorithm 3
// (the paper solves the Newton system by CG to the residual tolerance
// min(eta, |grad psi|^{1+tau})):
//     M d = -g,  M = I + sigma X_J^T (I - 1 1^T / p) X_J,
// with the Jacobi preconditioner diag(M)_j = 1 + sigma (sum_J X_ij^2 - s_j^2 / p).
// The CG scalars live in device memory; the host only polls |r|^2 every few
// iterations.  Once |r|^2 <= tol^2 the kernels stop updating (cg_done).
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

static inline unsigned grid_for(int64_t len) {
    int64_t b = (len + 2047) / 2048;
    if (b > 256) b = 256;
    if (b < 1) b = 1;
    return (unsigned)b;
}

__global__ void k_jacobi_diag(const double* __restrict__ sq, const double* __restrict__ sv,
                              double sigma, double inv_p, double* __restrict__ diag, int64_t q) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < q) diag[j] = fmax(1.0 + sigma * (sq[j] - sv[j] * sv[j] * inv_p), 1.0);
}
void launch_jacobi_diag(const double* sq, const double* sv, double sigma, int64_t p, double* diag,
                        int64_t q, hipStream_t s) {
    SSN_LAUNCH(k_jacobi_diag, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, sq, sv,
                       sigma, p > 0 ? 1.0 / (double)p : 0.0, diag, q);
}

// x = 0, r = -g, z = r / diag, p = z; rz = r.z, rr = r.r
__global__ __launch_bounds__(SSN_BLOCK) void k_pcg_init(const double* __restrict__ g,
                                                        const double* __restrict__ diag,
                                                        double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        double* __restrict__ z,
                                                        double* __restrict__ pd, int64_t q,
                                                        double tol2, Scalars* sc,
                                                        double* __restrict__ part,
                                                        unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    double rz = 0.0, rr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
        const double rj = -g[j];
        const double zj = rj / diag[j];
        x[j] = 0.0;
        r[j] = rj;
        z[j] = zj;
        pd[j] = zj;
        rz = fma(rj, zj, rz);
        rr = fma(rj, rj, rr);
    }
    const double a = block_sum(rz, shd), b = block_sum(rr, shd);
    if (threadIdx.x == 0) { part[blockIdx.x * 2] = a; part[blockIdx.x * 2 + 1] = b; }
    if (last_block_arrives(counter)) {
        const double s0 = grid_colsum(part, gridDim.x, 2, 0, shd);
        const double s1 = grid_colsum(part, gridDim.x, 2, 1, shd);
        if (threadIdx.x == 0) {
            sc->cg_rz = s0;
            sc->cg_rr = s1;
            sc->cg_done = s1 <= tol2 ? 1 : 0;       // x = 0 may already meet the tolerance
            sc->cg_count = 0;
        }
    }
}
void launch_pcg_init(const double* g, const double* diag, double* x, double* r, double* z, double* pd,
                     int64_t q, double tol2, Scalars* sc, double* part, unsigned* counter,
                     hipStream_t s) {
    SSN_LAUNCH(k_pcg_init, dim3(grid_for(q)), dim3(SSN_BLOCK), 0, s, g, diag, x, r, z, pd, q,
                       tol2, sc, part, counter);
}

// pap = p . Ap
__global__ __launch_bounds__(SSN_BLOCK) void k_pcg_pap(const double* __restrict__ pd,
                                                       const double* __restrict__ Ap, int64_t q,
                                                       Scalars* sc, double* __restrict__ part,
                                                       unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    if (ld_grid(&sc->cg_done)) return;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride)
        s = fma(pd[j], Ap[j], s);
    const double a = block_sum(s, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
    if (last_block_arrives(counter)) {
        const double t = grid_colsum(part, gridDim.x, 1, 0, shd);
        if (threadIdx.x == 0) sc->cg_pap = t;
    }
}
void launch_pcg_pap(const double* pd, const double* Ap, int64_t q, Scalars* sc, double* part,
                    unsigned* counter, hipStream_t s) {
    SSN_LAUNCH(k_pcg_pap, dim3(grid_for(q)), dim3(SSN_BLOCK), 0, s, pd, Ap, q, sc, part,
                       counter);
}

// alpha = rz / pap; x += alpha p; r -= alpha Ap; z = r / diag; then
// rz_new, rr, beta = rz_new / rz.  Sets cg_done when rr <= tol2.
__global__ __launch_bounds__(SSN_BLOCK) void k_pcg_step(double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        const double* __restrict__ pd,
                                                        const double* __restrict__ Ap,
                                                        const double* __restrict__ diag,
                                                        double* __restrict__ z, int64_t q,
                                                        Scalars* sc, double tol2,
                                                        double* __restrict__ part,
                                                        unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    if (ld_grid(&sc->cg_done)) return;
    const double pap = sc->cg_pap, rz = sc->cg_rz;
    const double alpha = (pap > 0.0 && rz > 0.0) ? rz / pap : 0.0;
    double a = 0.0, b = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
        x[j] = fma(alpha, pd[j], x[j]);
        const double rj = fma(-alpha, Ap[j], r[j]);
        r[j] = rj;
        const double zj = rj / diag[j];
        z[j] = zj;
        a = fma(rj, zj, a);
        b = fma(rj, rj, b);
    }
    const double sa = block_sum(a, shd), sb = block_sum(b, shd);
    if (threadIdx.x == 0) { part[blockIdx.x * 2] = sa; part[blockIdx.x * 2 + 1] = sb; }
    if (last_block_arrives(counter)) {
        const double s0 = grid_colsum(part, gridDim.x, 2, 0, shd);
        const double s1 = grid_colsum(part, gridDim.x, 2, 1, shd);
        if (threadIdx.x == 0) {
            sc->cg_beta = rz > 0.0 ? s0 / rz : 0.0;
            sc->cg_rz = s0;
            sc->cg_rr = s1;
            sc->cg_count += 1;                       // an iteration that changed x
            if (s1 <= tol2 || !(alpha > 0.0)) sc->cg_done = 1;
        }
    }
}
void launch_pcg_step(double* x, double* r, double* pd, const double* Ap, const double* diag,
                     double* z, int64_t q, Scalars* sc, double tol2, double* part,
                     unsigned* counter, hipStream_t s) {
    SSN_LAUNCH(k_pcg_step, dim3(grid_for(q)), dim3(SSN_BLOCK), 0, s, x, r, pd, Ap, diag, z,
                       q, sc, tol2, part, counter);
}

__global__ void k_pcg_dir(double* __restrict__ pd, const double* __restrict__ z, int64_t q,
                          const Scalars* sc) {
    if (ld_grid(&sc->cg_done)) return;
    const double beta = sc->cg_beta;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < q) pd[j] = fma(beta, pd[j], z[j]);
}
void launch_pcg_dir(double* pd, const double* z, int64_t q, Scalars* sc, hipStream_t s) {
    SSN_LAUNCH(k_pcg_dir, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, pd, z, q, sc);
}

// mean over J of w_i = y_i t_i (t = y .* X p): stored in *mean_out
__global__ __launch_bounds__(SSN_BLOCK) void k_masked_mean(const double* __restrict__ t,
                                                           const int8_t* __restrict__ y,
                                                           const uint8_t* __restrict__ mask,
                                                           int64_t n, double inv_p,
                                                           double* mean_out,
                                                           double* __restrict__ part,
                                                           unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (mask[i]) s += (double)y[i] * t[i];
    const double a = block_sum(s, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
    if (last_block_arrives(counter)) {
        const double tot = grid_colsum(part, gridDim.x, 1, 0, shd);
        if (threadIdx.x == 0) *mean_out = tot * inv_p;
    }
}
void launch_masked_mean(const double* t, const int8_t* y, const uint8_t* mask, int64_t n, int64_t p,
                        double* mean_out, double* part, unsigned* counter, hipStream_t s) {
    SSN_LAUNCH(k_masked_mean, dim3(grid_for(n)), dim3(SSN_BLOCK), 0, s, t, y, mask, n,
                       p > 0 ? 1.0 / (double)p : 0.0, mean_out, part, counter);
}

// z_i = y_i * mask_i * (y_i t_i - mean): the transposed product of A then
// yields X_J^T (w - mean 1) because y_i^2 = 1.
__global__ void k_masked_center(const double* __restrict__ t, const int8_t* __restrict__ y,
                                const uint8_t* __restrict__ mask, int64_t n,
                                const double* __restrict__ mean, double* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double yi = (double)y[i];
    z[i] = mask[i] ? yi * (yi * t[i] - *mean) : 0.0;
}
void launch_masked_center_t(double* t, const int8_t* y, const uint8_t* mask, int64_t n,
                            const double* mean, double* z, hipStream_t s) {
    SSN_LAUNCH(k_masked_center, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, y,
                       mask, n, mean, z);
}

// Ap = p + sigma * z
__global__ void k_mop_finish(const double* __restrict__ pd, const double* __restrict__ z,
                             double sigma, double* __restrict__ Ap, int64_t q) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < q) Ap[j] = fma(sigma, z[j], pd[j]);
}
void launch_mop_finish(const double* pd, const double* z, double sigma, const double*, const double*,
                       int64_t, double* Ap, int64_t q, hipStream_t s) {
    SSN_LAUNCH(k_mop_finish, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, pd, z, sigma,
                       Ap, q);
}

// count p = #{0 < x_i < C}, nsv = #{x_i > 0} and e^T x of a feasible x
__global__ __launch_bounds__(SSN_BLOCK) void k_count_x(const double* __restrict__ x, int64_t n,
                                                       double C, Scalars* sc,
                                                       double* __restrict__ part,
                                                       unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    long long p = 0, ns = 0;
    double sx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i];
        p += (xi > 0.0 && xi < C) ? 1 : 0;
        ns += xi > 0.0 ? 1 : 0;
        sx += xi;
    }
    const long long bp = block_sum_ll(p, shl), bn = block_sum_ll(ns, shl);
    const double bs = block_sum(sx, shd);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3] = (double)bp;
        part[blockIdx.x * 3 + 1] = (double)bn;
        part[blockIdx.x * 3 + 2] = bs;
    }
    if (last_block_arrives(counter)) {
        const double a = grid_colsum(part, gridDim.x, 3, 0, shd);
        const double b = grid_colsum(part, gridDim.x, 3, 1, shd);
        const double c = grid_colsum(part, gridDim.x, 3, 2, shd);
        if (threadIdx.x == 0) {
            sc->p = (long long)a;
            sc->nsv = (long long)b;
            sc->sumx = c;
        }
    }
}
void launch_count_x(const double* x, int64_t n, double C, Scalars* sc, double* part,
                    unsigned* counter, hipStream_t s) {
    SSN_LAUNCH(k_count_x, dim3(grid_for(n)), dim3(SSN_BLOCK), 0, s, x, n, C, sc, part,
                       counter);
}

}  // namespace ssn
