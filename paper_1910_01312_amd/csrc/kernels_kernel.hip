// Kernels of the w-space solver for the kernel C-SVC (Section 1, eq.
// Def_Dual_of_C_SVM_Problem with a nonlinear kernel; Proposition 5 for the
// Newton step).  Q (n x n, fp64, row stride ld, symmetric) is resident in
// device memory; every product reads whole rows of Q, which are contiguous.
//
//   Q v for a v with support S:   (Q v)_j = sum_{k in S} v_k Q[k][j]
//     (symmetry: the rows of Q at the support stand in for its columns).
//     Column tiles of 256 entries x chunks of S: each wave owns every fourth
//     row of its chunk, every lane two adjacent columns per 128-column half,
//     so one row is read as 1 KB runs of 16-byte loads; the four waves are
//     summed through LDS and each block writes its partial row, summed in a
//     fixed order afterwards (deterministic).
//   Q_JJ v:                        one wave per row J_a, lanes over J_b.
//   The p x p Newton matrix I + sigma Pi Q_JJ Pi, Pi = I - a a^T / p
//   (a = y_J, p = a^T a): entries
//     delta_ab + sigma (Q_{J_a J_b} - (a_a r_b + r_a a_b) / p + a_a a_b rho / p^2),
//   r = Q_JJ a, rho = a^T r.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int QC_NCH = 2;                         // 128-column halves per tile
constexpr int QC_COLS = SSN_WAVE * 2 * QC_NCH;    // 256 columns per block

// mask[i] = (v[i] != 0)
__global__ void k_nz_mask(const double* __restrict__ v, int64_t n, uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mask[i] = v[i] != 0.0 ? 1 : 0;
}
void launch_nz_mask(const double* v, int64_t n, uint8_t* mask, hipStream_t s) {
    SSN_LAUNCH(k_nz_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, mask);
}

// part[c * n + j] = sum over k in chunk c of coef(k) Q[list[k]][j], with
// coef(k) = by_row ? v[list[k]] : v[k].  Chunk c covers [c * chunk, ...) of
// the m listed rows.
__global__ __launch_bounds__(SSN_BLOCK) void k_qcols(const double* __restrict__ Q, int64_t n, int64_t ld,
                                                     const int32_t* __restrict__ list, int64_t m,
                                                     int64_t chunk, const double* __restrict__ v,
                                                     int by_row, double* __restrict__ part) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK][QC_COLS];
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int w = threadIdx.x / SSN_WAVE;
    const int64_t c0 = (int64_t)blockIdx.x * QC_COLS;
    const int64_t k0 = (int64_t)blockIdx.y * chunk;
    const int64_t k1 = min(m, k0 + chunk);
    double acc[QC_NCH][2] = {};
    // a lane loads columns col, col + 1 only when col < ld (ld is a multiple
    // of 32, so col + 1 < ld too); Q is zero in columns [n, ld)
    const int64_t col[QC_NCH] = {c0 + 2 * lane, c0 + 2 * lane + 2 * SSN_WAVE};
    bool ok[QC_NCH];
#pragma unroll
    for (int h = 0; h < QC_NCH; ++h) ok[h] = col[h] < ld;
    int64_t k = k0 + w;
    // four rows of this wave per round: 8 loads of 16 bytes in flight
    for (; k + 3 * SSN_WAVES_PER_BLOCK < k1; k += 4 * SSN_WAVES_PER_BLOCK) {
        double2 x[4][QC_NCH];
        double cf[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t kk = k + r * SSN_WAVES_PER_BLOCK;
            const int64_t row = list[kk];
            cf[r] = by_row ? v[row] : v[kk];
            const double* base = Q + row * ld;
#pragma unroll
            for (int h = 0; h < QC_NCH; ++h)
                x[r][h] = ok[h] ? *reinterpret_cast<const double2*>(base + col[h]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int h = 0; h < QC_NCH; ++h) {
                acc[h][0] = fma(cf[r], x[r][h].x, acc[h][0]);
                acc[h][1] = fma(cf[r], x[r][h].y, acc[h][1]);
            }
    }
    for (; k < k1; k += SSN_WAVES_PER_BLOCK) {
        const int64_t row = list[k];
        const double cf = by_row ? v[row] : v[k];
        const double* base = Q + row * ld;
#pragma unroll
        for (int h = 0; h < QC_NCH; ++h) {
            const double2 x = ok[h] ? *reinterpret_cast<const double2*>(base + col[h]) : make_double2(0.0, 0.0);
            acc[h][0] = fma(cf, x.x, acc[h][0]);
            acc[h][1] = fma(cf, x.y, acc[h][1]);
        }
    }
#pragma unroll
    for (int h = 0; h < QC_NCH; ++h) {
        sh[w][2 * lane + 2 * SSN_WAVE * h] = acc[h][0];
        sh[w][2 * lane + 2 * SSN_WAVE * h + 1] = acc[h][1];
    }
    __syncthreads();
    // thread t sums column c0 + t over the four waves in wave order
    const int64_t j = c0 + threadIdx.x;
    if (j < n) {
        double t = 0.0;
#pragma unroll
        for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) t += sh[ww][threadIdx.x];
        part[blockIdx.y * n + j] = t;
    }
}

int qcols_chunks(int64_t n, int64_t m) {
    // enough blocks to fill the chip (about 4096) without chunks of fewer
    // than 16 rows
    const int64_t tiles = (n + QC_COLS - 1) / QC_COLS;
    int64_t c = (4096 + tiles - 1) / tiles;
    c = std::min<int64_t>(c, (m + 15) / 16);
    c = std::min<int64_t>(c, kQcolsMaxChunks);
    return (int)std::max<int64_t>(c, 1);
}

void launch_qcols(const double* Q, int64_t n, int64_t ld, const int32_t* list, int64_t m, const double* v,
                  int by_row, double* part, int nchunk, hipStream_t s) {
    const int64_t chunk = std::max<int64_t>((m + nchunk - 1) / nchunk, 1);
    const dim3 grid((unsigned)((n + QC_COLS - 1) / QC_COLS), (unsigned)nchunk);
    SSN_LAUNCH(k_qcols, grid, dim3(SSN_BLOCK), 0, s, Q, n, ld, list, m, chunk, v, by_row, part);
}

// out[a] = sum_b Q[J_a][J_b] v_b (one wave per row a)
__global__ __launch_bounds__(SSN_BLOCK) void k_qjj_mv(const double* __restrict__ Q, int64_t ld,
                                                      const int32_t* __restrict__ J, int64_t p,
                                                      const double* __restrict__ v,
                                                      double* __restrict__ out) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t a = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (a >= p) return;
    const double* row = Q + (int64_t)J[a] * ld;
    double s0 = 0.0, s1 = 0.0;
    int64_t b = lane;
    for (; b + SSN_WAVE < p; b += 2 * SSN_WAVE) {
        s0 = fma(row[J[b]], v[b], s0);
        s1 = fma(row[J[b + SSN_WAVE]], v[b + SSN_WAVE], s1);
    }
    if (b < p) s0 = fma(row[J[b]], v[b], s0);
    const double t = wave_sum(s0 + s1);
    if (lane == 0) out[a] = t;
}
void launch_qjj_mv(const double* Q, int64_t ld, const int32_t* J, int64_t p, const double* v, double* out,
                   hipStream_t s) {
    const unsigned nb = (unsigned)((p + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
    SSN_LAUNCH(k_qjj_mv, dim3(nb), dim3(SSN_BLOCK), 0, s, Q, ld, J, p, v, out);
}

// M (p x p, row-major) = I + sigma Pi Q_JJ Pi with r = Q_JJ a, rho = a^T r
// (device scalar), a_b = y[J_b].
__global__ __launch_bounds__(SSN_BLOCK) void k_qjj_form(const double* __restrict__ Q, int64_t ld,
                                                        const int32_t* __restrict__ J, int64_t p,
                                                        const double* __restrict__ aJ,
                                                        const double* __restrict__ r,
                                                        const double* __restrict__ rho, double sigma,
                                                        double* __restrict__ M) {
    const int64_t a = blockIdx.y;
    const int64_t b = (int64_t)blockIdx.x * SSN_BLOCK + threadIdx.x;
    if (b >= p) return;
    const double inv_p = 1.0 / (double)p;
    const double qab = Q[(int64_t)J[a] * ld + J[b]];
    const double aa = aJ[a], ab = aJ[b];
    const double c = qab - (aa * r[b] + r[a] * ab) * inv_p + aa * ab * (*rho) * inv_p * inv_p;
    M[a * p + b] = (a == b ? 1.0 : 0.0) + sigma * c;
}
void launch_qjj_form(const double* Q, int64_t ld, const int32_t* J, int64_t p, const double* aJ,
                     const double* r, const double* rho, double sigma, double* M, hipStream_t s) {
    const dim3 grid((unsigned)((p + SSN_BLOCK - 1) / SSN_BLOCK), (unsigned)p);
    SSN_LAUNCH(k_qjj_form, grid, dim3(SSN_BLOCK), 0, s, Q, ld, J, p, aJ, r, rho, sigma, M);
}

// Jacobi preconditioner of the same matrix: its diagonal, floored at 1.
__global__ void k_qjj_diag(const double* __restrict__ Q, int64_t ld, const int32_t* __restrict__ J, int64_t p,
                           const double* __restrict__ aJ, const double* __restrict__ r,
                           const double* __restrict__ rho, double sigma, double* __restrict__ diag) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p) return;
    const double inv_p = 1.0 / (double)p;
    const double ab = aJ[b];
    const double c = Q[(int64_t)J[b] * ld + J[b]] - 2.0 * ab * r[b] * inv_p + ab * ab * (*rho) * inv_p * inv_p;
    diag[b] = fmax(1.0 + sigma * c, 1.0);
}
void launch_qjj_diag(const double* Q, int64_t ld, const int32_t* J, int64_t p, const double* aJ,
                     const double* r, const double* rho, double sigma, double* diag, hipStream_t s) {
    SSN_LAUNCH(k_qjj_diag, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, Q, ld, J, p, aJ, r, rho,
               sigma, diag);
}

// aJ[b] = y[J_b], gJ[b] = g[J_b]
__global__ void k_kgather(const int32_t* __restrict__ J, int64_t p, const int8_t* __restrict__ y,
                          const double* __restrict__ g, double* __restrict__ aJ, double* __restrict__ gJ) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p) return;
    const int32_t i = J[b];
    aJ[b] = (double)y[i];
    gJ[b] = g[i];
}
void launch_kgather(const int32_t* J, int64_t p, const int8_t* y, const double* g, double* aJ, double* gJ,
                    hipStream_t s) {
    SSN_LAUNCH(k_kgather, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, J, p, y, g, aJ, gJ);
}

// out[b] = (base ? base[b] : 0) + scale (u[b] - aJ[b] dot / p): Pi u scaled,
// with dot = a^T u already in device memory.
__global__ void k_kcenter(const double* __restrict__ u, const double* __restrict__ aJ,
                          const double* __restrict__ dot, int64_t p, double scale,
                          const double* __restrict__ base, double* __restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p) return;
    const double c = *dot / (double)p;
    const double t = scale * (u[b] - aJ[b] * c);
    out[b] = base ? base[b] + t : t;
}
void launch_kcenter(const double* u, const double* aJ, const double* dot, int64_t p, double scale,
                    const double* base, double* out, hipStream_t s) {
    SSN_LAUNCH(k_kcenter, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, u, aJ, dot, p, scale, base,
               out);
}

// d[J_b] += z_b
__global__ void k_scatter_add(const int32_t* __restrict__ J, int64_t p, const double* __restrict__ z,
                              double* __restrict__ d) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < p) d[J[b]] += z[b];
}
void launch_scatter_add(const int32_t* J, int64_t p, const double* z, double* d, hipStream_t s) {
    SSN_LAUNCH(k_scatter_add, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, J, p, z, d);
}

}  // namespace ssn
