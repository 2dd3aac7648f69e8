// Reduced Newton system of Algorithm 3 (step 1) in omega-space:
//     (I + sigma (X_J^T X_J - s s^T / p)) d = -g,   s = X_J^T 1,  p = |J|,
// which is the system of eq. Newton_Linear_System written in the L = A
// coordinates of Proposition 5 (the labels cancel in A^T P A because
// y_i^2 = 1).  Kernels: gather-SYRK of X_J^T X_J over the compacted row
// list, the rank-one centering, and an fp64 Cholesky factor/solve.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

// ------------------------------------------------------------------ SYRK
// Tile TS x TS of G (lower-triangular tiles only), split over the row list
// into nsplit chunks.  Rows of X_J are gathered through the index list and
// staged in LDS as fp64 (exact widening of fp32/bf16).  Each thread owns a
// 4 x 4 block of the tile.  Partial tiles are summed in split order by
// k_syrk_reduce, which also mirrors the lower triangle.
constexpr int TS = 64;
constexpr int TR = 16;        // rows staged per step

template <typename T>
__global__ __launch_bounds__(SSN_BLOCK) void k_syrk_gather(const T* __restrict__ X, int64_t q,
                                                           const int32_t* __restrict__ list,
                                                           int64_t p, int64_t rows_per_split,
                                                           const int2* __restrict__ tiles,
                                                           double* __restrict__ part) {
    __shared__ double As[TR][TS + 1];
    __shared__ double Bs[TR][TS + 1];
    const int2 tl = tiles[blockIdx.x];
    const int64_t i0 = (int64_t)tl.x * TS, j0 = (int64_t)tl.y * TS;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < p ? r0 + rows_per_split : p;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;    // 16 x 16 threads, 4x4 each
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += TR) {
        // stage TR rows x TS columns of both column blocks
        for (int e = threadIdx.x; e < TR * TS; e += SSN_BLOCK) {
            const int rr = e / TS, cc = e % TS;
            const int64_t r = rb + rr;
            double va = 0.0, vb = 0.0;
            if (r < r1) {
                const T* xr = X + (int64_t)list[r] * q;
                if (i0 + cc < q) va = to_f64(xr[i0 + cc]);
                if (j0 + cc < q) vb = to_f64(xr[j0 + cc]);
            }
            As[rr][cc] = va;
            Bs[rr][cc] = vb;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < TR; ++rr) {
            double a[4], b[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                a[k] = As[rr][ty * 4 + k];
                b[k] = Bs[rr][tx * 4 + k];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
    double* out = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * TS * TS;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(ty * 4 + u) * TS + tx * 4 + v] = acc[u][v];
}

__global__ void k_syrk_reduce(const double* __restrict__ part, int ntile, int nsplit,
                              const int2* __restrict__ tiles, double* __restrict__ G, int64_t q) {
    const int tile = blockIdx.x;
    const int2 tl = tiles[tile];
    for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
        const int a = e / TS, b = e % TS;
        const int64_t i = (int64_t)tl.x * TS + a, j = (int64_t)tl.y * TS + b;
        if (i >= q || j >= q || j > i) continue;
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[((int64_t)k * ntile + tile) * TS * TS + e];
        G[i * q + j] = s;
        G[j * q + i] = s;
    }
}

struct SyrkTiles {
    int2* dev = nullptr;
    int64_t q = -1;
    int ntile = 0;
};
static SyrkTiles g_tiles_cache[8];

static const int2* syrk_tiles(int64_t q, int* ntile_out, hipStream_t s) {
    const int nt = (int)((q + TS - 1) / TS);
    const int ntile = nt * (nt + 1) / 2;
    for (auto& c : g_tiles_cache)
        if (c.q == q && c.dev) { *ntile_out = c.ntile; return c.dev; }
    int2* host = (int2*)malloc(sizeof(int2) * ntile);
    int k = 0;
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j <= i; ++j) host[k++] = make_int2(i, j);
    int2* dev = nullptr;
    if (hipMalloc(&dev, sizeof(int2) * ntile) != hipSuccess) { free(host); return nullptr; }
    hipMemcpyAsync(dev, host, sizeof(int2) * ntile, hipMemcpyHostToDevice, s);
    hipStreamSynchronize(s);
    free(host);
    for (auto& c : g_tiles_cache)
        if (!c.dev) { c.dev = dev; c.q = q; c.ntile = ntile; break; }
    *ntile_out = ntile;
    return dev;
}

int64_t syrk_part_size(int64_t q, int64_t p) {
    const int nt = (int)((q + TS - 1) / TS);
    const int64_t ntile = (int64_t)nt * (nt + 1) / 2;
    int64_t nsplit = (1024 + ntile - 1) / ntile;
    const int64_t maxsplit = (p + 255) / 256;
    if (nsplit > maxsplit) nsplit = maxsplit;
    if (nsplit < 1) nsplit = 1;
    return nsplit * ntile * TS * TS;
}

void launch_syrk_gather(int dtype, const void* X, int64_t q, const int32_t* list, int64_t p,
                        double* G, double* part, int64_t part_cap, hipStream_t s) {
    int ntile = 0;
    const int2* tiles = syrk_tiles(q, &ntile, s);
    int64_t nsplit = (1024 + ntile - 1) / ntile;
    const int64_t maxsplit = (p + 255) / 256;
    if (nsplit > maxsplit) nsplit = maxsplit;
    if (nsplit < 1) nsplit = 1;
    while (nsplit > 1 && nsplit * ntile * TS * TS > part_cap) --nsplit;
    const int64_t rps = (p + nsplit - 1) / nsplit;
    dim3 grid((unsigned)ntile, (unsigned)nsplit);
    if (dtype == SSNALM_F64)
        SSN_LAUNCH((k_syrk_gather<double>), grid, dim3(SSN_BLOCK), 0, s, (const double*)X,
                           q, list, p, rps, tiles, part);
    else if (dtype == SSNALM_F32)
        SSN_LAUNCH((k_syrk_gather<float>), grid, dim3(SSN_BLOCK), 0, s, (const float*)X, q,
                           list, p, rps, tiles, part);
    else
        SSN_LAUNCH((k_syrk_gather<bf16_t>), grid, dim3(SSN_BLOCK), 0, s, (const bf16_t*)X,
                           q, list, p, rps, tiles, part);
    SSN_LAUNCH(k_syrk_reduce, dim3((unsigned)ntile), dim3(SSN_BLOCK), 0, s, part, ntile,
                       (int)nsplit, tiles, G, q);
}

// ------------------------------------------------------------------ M
__global__ void k_form_M(const double* __restrict__ G, const double* __restrict__ sv, double sigma,
                         double inv_p, double* __restrict__ M, int64_t q) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q * q) return;
    const int64_t i = e / q, j = e % q;
    const double c = G[e] - sv[i] * sv[j] * inv_p;
    M[e] = (i == j ? 1.0 : 0.0) + sigma * c;
}

void launch_form_M_inv(const double* G, const double* sv, double sigma, double inv_den, double* M,
                       int64_t q, hipStream_t s) {
    const int64_t tot = q * q;
    SSN_LAUNCH(k_form_M, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, G, sv, sigma, inv_den,
               M, q);
}
void launch_form_M(const double* G, const double* sv, double sigma, int64_t p, double* M, int64_t q,
                   hipStream_t s) {
    const int64_t tot = q * q;
    SSN_LAUNCH(k_form_M, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, G, sv, sigma,
                       p > 0 ? 1.0 / (double)p : 0.0, M, q);
}

// ------------------------------------------------------------------ Cholesky (LDS)
// Whole factorisation and both triangular solves in one workgroup with the
// matrix resident in LDS (q <= 128: 128 KiB).  Right-looking, column by
// column.  A non-positive pivot sets sc->chol_fail and d = -g.
constexpr int CHOL_SMALL_MAX = 128;
int chol_small_max() { return CHOL_SMALL_MAX; }

__global__ __launch_bounds__(1024) void k_chol_solve_small(const double* __restrict__ M,
                                                           const double* __restrict__ g,
                                                           double* __restrict__ d, int q,
                                                           Scalars* sc) {
    extern __shared__ double L[];         // q*q, row-major
    __shared__ double z[CHOL_SMALL_MAX];
    __shared__ int fail;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < q * q; e += nt) L[e] = M[e];
    for (int i = tid; i < q; i += nt) z[i] = -g[i];
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int k = 0; k < q; ++k) {
        const double akk = L[k * q + k];
        if (!(akk > 0.0)) {
            if (tid == 0) fail = 1;
            break;                                     // uniform: all threads read the same value
        }
        const double lkk = sqrt(akk);
        __syncthreads();
        for (int i = k + 1 + tid; i < q; i += nt) L[i * q + k] /= lkk;
        if (tid == 0) L[k * q + k] = lkk;
        __syncthreads();
        const int m = q - k - 1;
        for (int e = tid; e < m * m; e += nt) {
            const int a = e / m, b = e % m;
            if (b <= a) {
                const int i = k + 1 + a, j = k + 1 + b;
                L[i * q + j] -= L[i * q + k] * L[j * q + k];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (fail) {
        for (int i = tid; i < q; i += nt) d[i] = -g[i];
        if (tid == 0) sc->chol_fail = 1;
        return;
    }
    // forward: L w = z
    for (int j = 0; j < q; ++j) {
        if (tid == 0) z[j] /= L[j * q + j];
        __syncthreads();
        const double zj = z[j];
        for (int i = j + 1 + tid; i < q; i += nt) z[i] -= L[i * q + j] * zj;
        __syncthreads();
    }
    // backward: L^T d = w
    for (int j = q - 1; j >= 0; --j) {
        if (tid == 0) z[j] /= L[j * q + j];
        __syncthreads();
        const double zj = z[j];
        for (int i = tid; i < j; i += nt) z[i] -= L[j * q + i] * zj;
        __syncthreads();
    }
    for (int i = tid; i < q; i += nt) d[i] = z[i];
    if (tid == 0) sc->chol_fail = 0;
}

void launch_chol_solve_small(const double* M, const double* g, double* d, int64_t q, Scalars* sc,
                             hipStream_t s) {
    const size_t shm = (size_t)q * q * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
        hipFuncSetAttribute((const void*)k_chol_solve_small,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            CHOL_SMALL_MAX * CHOL_SMALL_MAX * (int)sizeof(double));
        attr_set = true;
    }
    SSN_LAUNCH(k_chol_solve_small, dim3(1), dim3(q <= 64 ? 256 : 1024), shm, s, M, g, d,
                       (int)q, sc);
}

}  // namespace ssn
