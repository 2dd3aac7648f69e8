// Blocked fp64 Cholesky of the reduced Newton matrix
//     M = I + sigma (X_J^T X_J - s s^T / p)   (q x q, symmetric positive definite)
// for q above the LDS-resident kernel's limit, and the two triangular solves
// giving d = -M^{-1} g.  Right-looking with 64 x 64 blocks: for each block
// column kb, factor the diagonal block in LDS, solve the panel below it, and
// update the trailing lower tiles.  The factor is kept in the lower triangle
// of M and mirrored into the upper triangle (row j of the upper part holds
// column j of L), so both solves read contiguous rows.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int NB = 64;
constexpr int CHOL_BLOCKED_MAX = 2048;

int chol_blocked_max() { return CHOL_BLOCKED_MAX; }

// Factor the diagonal block kb in LDS.  A non-positive pivot is replaced by 1
// and reported through sc->chol_fail.
__global__ __launch_bounds__(SSN_BLOCK) void k_chol_diag(double* __restrict__ M, int q, int kb,
                                                         Scalars* sc) {
    __shared__ double A[NB][NB + 1];
    if (kb == 0 && threadIdx.x == 0) sc->chol_fail = 0;
    const int o = kb * NB;
    const int m = min(NB, q - o);
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        A[i][j] = (i < m && j < m) ? M[(int64_t)(o + i) * q + o + j] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        double akk = A[k][k];
        if (!(akk > 0.0)) {
            if (threadIdx.x == 0) sc->chol_fail = 1;
            akk = 1.0;
        }
        const double lkk = sqrt(akk);
        __syncthreads();
        for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) A[i][k] /= lkk;
        if (threadIdx.x == 0) A[k][k] = lkk;
        __syncthreads();
        const int r = m - k - 1;
        for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
            const int a = e / r, b = e % r;
            if (b <= a) A[k + 1 + a][k + 1 + b] -= A[k + 1 + a][k] * A[k + 1 + b][k];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e % m;
        if (j <= i) {
            const double v = A[i][j];
            M[(int64_t)(o + i) * q + o + j] = v;
            M[(int64_t)(o + j) * q + o + i] = v;
        }
    }
}

// Panel solve: rows below the diagonal block, L_ib,kb = A_ib,kb L_kb,kb^{-T}.
// One block per row block, one thread per row.
__global__ __launch_bounds__(NB) void k_chol_trsm(double* __restrict__ M, int q, int kb) {
    __shared__ double L[NB][NB + 1];
    const int o = kb * NB;
    const int m = min(NB, q - o);
    const int ib = kb + 1 + blockIdx.x;
    const int ro = ib * NB;
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        L[i][j] = (i < m && j < m && j <= i) ? M[(int64_t)(o + i) * q + o + j] : 0.0;
    }
    __syncthreads();
    const int r = ro + threadIdx.x;
    if (r >= q) return;
    double x[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = j < m ? M[(int64_t)r * q + o + j] : 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j < m) {
            double a = x[j];
#pragma unroll
            for (int k = 0; k < j; ++k) a -= x[k] * L[j][k];
            x[j] = a / L[j][j];
        }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j < m) {
            M[(int64_t)r * q + o + j] = x[j];
            M[(int64_t)(o + j) * q + r] = x[j];
        }
    }
}

// Trailing update of the lower tiles (ib >= jb > kb):
// A_ib,jb -= L_ib,kb L_jb,kb^T.  One 64 x 64 tile per block, 4 x 4 per thread.
__global__ __launch_bounds__(SSN_BLOCK) void k_chol_update(double* __restrict__ M, int q, int kb) {
    __shared__ double Li[NB][NB + 1];
    __shared__ double Lj[NB][NB + 1];
    const int nt = (q + NB - 1) / NB - kb - 1;      // trailing block count
    // blockIdx.x -> (a, b), a >= b, over the nt x nt lower triangle
    int t = blockIdx.x, a = 0;
    while (t > a) { t -= a + 1; ++a; }
    const int b = t;
    const int ib = kb + 1 + a, jb = kb + 1 + b;
    (void)nt;
    const int o = kb * NB, io = ib * NB, jo = jb * NB;
    const int m = min(NB, q - o);
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, k = e % NB;
        Li[i][k] = (io + i < q && k < m) ? M[(int64_t)(io + i) * q + o + k] : 0.0;
        Lj[i][k] = (jo + i < q && k < m) ? M[(int64_t)(jo + i) * q + o + k] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int k = 0; k < m; ++k) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = Li[ty * 4 + u][k];
            y[u] = Lj[tx * 4 + u][k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(x[u], y[v], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = io + ty * 4 + u, j = jo + tx * 4 + v;
            if (i < q && j < q && j <= i) M[(int64_t)i * q + j] -= acc[u][v];
        }
}

// d = -M^{-1} g with the factor in M, by 64-row blocks in one workgroup.
// Forward L w = -g: for block B, subtract L[B, <B] w[<B] (rows of L, all
// waves, one wave-reduction per row), then wave 0 solves the 64 x 64 lower
// triangular block with lane i owning row i.  Backward L^T d = w: for block
// B from the last, subtract L[>B, B]^T d[>B] (row j of the upper triangle
// holds column j of L), then wave 0 solves the upper triangular L_BB^T.
__global__ __launch_bounds__(SSN_BLOCK) void k_chol_solve2(const double* __restrict__ M,
                                                           const double* __restrict__ g,
                                                           double* __restrict__ d, int q) {
    extern __shared__ double z[];                  // q doubles
    __shared__ double Lb[NB][NB + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < q; i += blockDim.x) z[i] = -g[i];
    const int nblk = (q + NB - 1) / NB;
    // ---- forward
    for (int B = 0; B < nblk; ++B) {
        const int o = B * NB, m = min(NB, q - o);
        __syncthreads();
        // z[o+r] -= sum_{c < o} L[o+r][c] z[c]
        for (int r = wv; r < m; r += SSN_WAVES_PER_BLOCK) {
            const double* row = M + (int64_t)(o + r) * q;
            double acc = 0.0;
            for (int c = lane; c < o; c += SSN_WAVE) acc = fma(row[c], z[c], acc);
            acc = wave_sum(acc);
            if (lane == 0) z[o + r] -= acc;
        }
        for (int e = tid; e < NB * NB; e += blockDim.x) {
            const int i = e / NB, j = e % NB;
            Lb[i][j] = (i < m && j < m && j <= i) ? M[(int64_t)(o + i) * q + o + j] : 0.0;
        }
        __syncthreads();
        if (wv == 0) {
            double ri = lane < m ? z[o + lane] : 0.0;
            for (int j = 0; j < m; ++j) {
                const double wj = __shfl(ri, j, SSN_WAVE) / Lb[j][j];
                if (lane == j) ri = wj;
                if (lane > j) ri -= Lb[lane][j] * wj;
            }
            if (lane < m) z[o + lane] = ri;
        }
    }
    // ---- backward
    for (int B = nblk - 1; B >= 0; --B) {
        const int o = B * NB, m = min(NB, q - o), e0 = o + m;
        __syncthreads();
        // z[o+r] -= sum_{c >= e0} L[c][o+r] d[c] = sum upper[o+r][c] d[c]
        for (int r = wv; r < m; r += SSN_WAVES_PER_BLOCK) {
            const double* row = M + (int64_t)(o + r) * q;
            double acc = 0.0;
            for (int c = e0 + lane; c < q; c += SSN_WAVE) acc = fma(row[c], z[c], acc);
            acc = wave_sum(acc);
            if (lane == 0) z[o + r] -= acc;
        }
        for (int e = tid; e < NB * NB; e += blockDim.x) {
            const int i = e / NB, j = e % NB;
            Lb[i][j] = (i < m && j < m && j <= i) ? M[(int64_t)(o + i) * q + o + j] : 0.0;
        }
        __syncthreads();
        if (wv == 0) {
            double ri = lane < m ? z[o + lane] : 0.0;
            for (int j = m - 1; j >= 0; --j) {
                const double dj = __shfl(ri, j, SSN_WAVE) / Lb[j][j];
                if (lane == j) ri = dj;
                if (lane < j) ri -= Lb[j][lane] * dj;
            }
            if (lane < m) z[o + lane] = ri;
        }
    }
    __syncthreads();
    for (int i = tid; i < q; i += blockDim.x) d[i] = z[i];
}

void launch_chol_factor_blocked(double* M, int64_t q, Scalars* sc, hipStream_t s) {
    const int nblk = (int)((q + NB - 1) / NB);
    for (int kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(SSN_BLOCK), 0, s, M, (int)q, kb, sc);
        const int nt = nblk - kb - 1;
        if (nt > 0) {
            hipLaunchKernelGGL(k_chol_trsm, dim3(nt), dim3(NB), 0, s, M, (int)q, kb);
            hipLaunchKernelGGL(k_chol_update, dim3(nt * (nt + 1) / 2), dim3(SSN_BLOCK), 0, s, M,
                               (int)q, kb);
        }
    }
}

void launch_chol_solve_factored(const double* M, const double* g, double* d, int64_t q,
                                double* work, hipStream_t s) {
    (void)work;
    hipLaunchKernelGGL(k_chol_solve2, dim3(1), dim3(SSN_BLOCK), (size_t)q * sizeof(double), s, M, g,
                       d, (int)q);
}

void launch_chol_solve_blocked(double* M, const double* g, double* d, int64_t q, double* work,
                               Scalars* sc, hipStream_t s) {
    launch_chol_factor_blocked(M, q, sc, s);
    launch_chol_solve_factored(M, g, d, q, work, s);
}

}  // namespace ssn
