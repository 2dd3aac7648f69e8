// Mixed-precision pieces of the dense Newton step.
//
// Gather-SYRK  G = X_J^T X_J  on the matrix cores: bf16 operands, fp32
// accumulation (v_mfma_f32_32x32x16_bf16), 128 x 128 output tiles of the
// lower triangle, split over the row list J.  A block stages gathered rows x
// 128 columns of each column block in LDS, stored transposed (column major,
// 8 consecutive rows contiguous) so that each lane's MFMA operand is one
// 16-byte LDS read.  Four waves each own a 64 x 64 sub-tile (2 x 2 MFMA
// tiles).  When q is a multiple of 8, k_syrk_mfma16 stages 64 rows per step
// with the next step's loads in flight; otherwise k_syrk_mfma stages 32 rows
// per step with per-element column checks.  The per-split fp32 partial tiles
// are summed in split order in fp64.
//
// Dense X_J v over a row list (one wave per row, fp64 accumulation), used by
// the exact Newton operator of the iterative refinement.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int MT = 128;          // output tile
constexpr int KC = 32;           // rows staged per step
constexpr int KP = KC + 8;       // padded row count in the transposed LDS tile

bool syrk_mfma_supported(int dtype, int64_t q) { return dtype == SSNALM_BF16 && q >= 1; }

static inline int mfma_ntile(int64_t q) {
    const int nt = (int)((q + MT - 1) / MT);
    return nt * (nt + 1) / 2;
}
static inline int64_t mfma_nsplit(int64_t q, int64_t p) {
    const int ntile = mfma_ntile(q);
    int64_t ns = (512 + ntile - 1) / ntile;
    const int64_t maxs = (p + 2 * KC - 1) / (2 * KC);
    if (ns > maxs) ns = maxs;
    if (ns > 32) ns = 32;
    if (ns < 1) ns = 1;
    return ns;
}
int64_t syrk_mfma_part_size(int64_t q, int64_t p) {
    return mfma_nsplit(q, p) * (int64_t)mfma_ntile(q) * MT * MT;
}

// stage rows [rb, rb+KC) of the list, columns [c0, c0+MT) into s (transposed)
__device__ __forceinline__ void stage_tile(const bf16_t* __restrict__ X, int64_t q,
                                           const int32_t* __restrict__ list, int64_t rb,
                                           int64_t r1, int64_t c0, bf16_t (*s)[KP]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = (t >> 4) + 16 * h;            // 0..31
        const int cg = t & 15;                      // 16 groups of 8 columns
        const int64_t row = rb + r;
        const int64_t col = c0 + cg * 8;
        bf16_t v[8];
        if (row < r1) {
            const bf16_t* src = X + (int64_t)list[row] * q + col;
            if (col + 8 <= q && ((q & 7) == 0)) {
                const uint4 u = *reinterpret_cast<const uint4*>(src);
                v[0] = (bf16_t)(u.x & 0xffff); v[1] = (bf16_t)(u.x >> 16);
                v[2] = (bf16_t)(u.y & 0xffff); v[3] = (bf16_t)(u.y >> 16);
                v[4] = (bf16_t)(u.z & 0xffff); v[5] = (bf16_t)(u.z >> 16);
                v[6] = (bf16_t)(u.w & 0xffff); v[7] = (bf16_t)(u.w >> 16);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = (col + e < q) ? src[e] : (bf16_t)0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = 0;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) s[cg * 8 + e][r] = v[e];
    }
}

__global__ __launch_bounds__(SSN_BLOCK) void k_syrk_mfma(const bf16_t* __restrict__ X, int64_t q,
                                                         const int32_t* __restrict__ list,
                                                         int64_t p, int64_t rows_per_split,
                                                         float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) bf16_t sA[MT][KP];
    __shared__ __attribute__((aligned(16))) bf16_t sB[MT][KP];
    // lower-triangle tile (ti >= tj) from blockIdx.x
    int t = blockIdx.x, ti = 0;
    while (t > ti) { t -= ti + 1; ++ti; }
    const int tj = t;
    const bool diag = ti == tj;
    const int64_t i0 = (int64_t)ti * MT, j0 = (int64_t)tj * MT;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < p ? r0 + rows_per_split : p;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m = lane & 31, kg = lane >> 5;
    f32x16_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.f;
    bf16_t (*sBp)[KP] = diag ? sA : sB;
    for (int64_t rb = r0; rb < r1; rb += KC) {
        stage_tile(X, q, list, rb, r1, i0, sA);
        if (!diag) stage_tile(X, q, list, rb, r1, j0, sB);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8_t fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                fa[a] = *reinterpret_cast<const bf16x8_t*>(&sA[wm * 64 + a * 32 + m][ks * 16 + kg * 8]);
#pragma unroll
            for (int b = 0; b < 2; ++b)
                fb[b] = *reinterpret_cast<const bf16x8_t*>(&sBp[wn * 64 + b * 32 + m][ks * 16 + kg * 8]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    float* out = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * MT * MT;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = wm * 64 + a * 32 + 8 * (e >> 2) + 4 * kg + (e & 3);
                const int col = wn * 64 + b * 32 + m;
                out[row * MT + col] = acc[a][b][e];
            }
}

// Same product when q is a multiple of 8 (every 8-column piece is one 16-byte
// load).  64 gathered rows per step; the next step's rows are loaded into
// registers while the current step's MFMAs run, and the list entries one step
// further ahead, so a step waits for one memory round trip at most.  Loads are
// issued unconditionally (row index clamped to the split, column to the last
// piece) and the values masked afterwards.  Each thread holds 4 consecutive
// rows of one 8-column piece and writes them to the transposed LDS tile as one
// 8-byte store per column.  LDS element (col, r) sits at
//   col * KP2 + (((r >> 3) ^ ((col >> 4) & 7)) << 3) + (r & 7):
// the 8-row blocks of a column are permuted by bits of the column index so that
// both the 8-byte stores of a wave and the 16-byte MFMA operand reads of a wave
// spread over all banks; an operand (8 consecutive rows of one column) stays one
// aligned 16-byte read.
constexpr int KC2 = 64;
constexpr int KP2 = KC2 + 8;     // 144-byte column stride

__device__ __forceinline__ int sw_off(int col, int r) {
    return col * KP2 + ((((r >> 3) ^ ((col >> 4) & 7))) << 3) + (r & 7);
}

// rows 4*rq .. 4*rq+3 of piece cg (masked by the validity bits in mk) -> LDS
__device__ __forceinline__ void put_rows(const uint4 (&u)[4], unsigned mk, int cg, int rq,
                                         bf16_t* __restrict__ sT) {
    uint32_t w[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool ok = (mk >> k) & 1u;
        w[k][0] = ok ? u[k].x : 0u;
        w[k][1] = ok ? u[k].y : 0u;
        w[k][2] = ok ? u[k].z : 0u;
        w[k][3] = ok ? u[k].w : 0u;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint2 ev, od;
        ev.x = (w[0][c] & 0xffffu) | (w[1][c] << 16);
        ev.y = (w[2][c] & 0xffffu) | (w[3][c] << 16);
        od.x = (w[0][c] >> 16) | (w[1][c] & 0xffff0000u);
        od.y = (w[2][c] >> 16) | (w[3][c] & 0xffff0000u);
        const int col = cg * 8 + 2 * c;
        *reinterpret_cast<uint2*>(sT + sw_off(col, 4 * rq)) = ev;
        *reinterpret_cast<uint2*>(sT + sw_off(col + 1, 4 * rq)) = od;
    }
}

template <bool DIAG>
__device__ __forceinline__ void syrk16_body(const bf16_t* __restrict__ X, int64_t q,
                                            const int32_t* __restrict__ list, int64_t r0,
                                            int64_t r1, int64_t i0, int64_t j0,
                                            bf16_t* __restrict__ sA, bf16_t* __restrict__ sB,
                                            f32x16_t (&acc)[2][2]) {
    const int t = threadIdx.x;
    const int cg = t & 15, rq = t >> 4;
    const int lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m = lane & 31, kg = lane >> 5;
    const int64_t ca = i0 + 8 * cg, cb = j0 + 8 * cg;
    const bool va = ca < q, vb = cb < q;
    const bf16_t* Xa = X + (va ? ca : q - 8);
    const bf16_t* Xb = X + (vb ? cb : q - 8);
    const int64_t last = r1 - 1;
    int li[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t row = r0 + 4 * rq + k;
        li[k] = list[row < last ? row : last];
    }
    uint4 ua[4], ub[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ua[k] = *reinterpret_cast<const uint4*>(Xa + (int64_t)li[k] * q);
        if (!DIAG) ub[k] = *reinterpret_cast<const uint4*>(Xb + (int64_t)li[k] * q);
    }
    for (int64_t rb = r0; rb < r1; rb += KC2) {
        const int64_t rn = rb + KC2;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t row = rn + 4 * rq + k;
            li[k] = list[row < last ? row : last];
        }
        unsigned mk = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) mk |= (rb + 4 * rq + k < r1 ? 1u : 0u) << k;
        put_rows(ua, va ? mk : 0u, cg, rq, sA);
        if (!DIAG) put_rows(ub, vb ? mk : 0u, cg, rq, sB);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ua[k] = *reinterpret_cast<const uint4*>(Xa + (int64_t)li[k] * q);
            if (!DIAG) ub[k] = *reinterpret_cast<const uint4*>(Xb + (int64_t)li[k] * q);
        }
        const bf16_t* sBp = DIAG ? sA : sB;
#pragma unroll
        for (int ks = 0; ks < KC2 / 16; ++ks) {
            const int r = ks * 16 + kg * 8;
            bf16x8_t fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                fa[a] = *reinterpret_cast<const bf16x8_t*>(sA + sw_off(wm * 64 + a * 32 + m, r));
#pragma unroll
            for (int b = 0; b < 2; ++b)
                fb[b] = *reinterpret_cast<const bf16x8_t*>(sBp + sw_off(wn * 64 + b * 32 + m, r));
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(SSN_BLOCK) void k_syrk_mfma16(const bf16_t* __restrict__ X, int64_t q,
                                                           const int32_t* __restrict__ list,
                                                           int64_t p, int64_t rows_per_split,
                                                           float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) bf16_t sA[MT * KP2];
    __shared__ __attribute__((aligned(16))) bf16_t sB[MT * KP2];
    int t = blockIdx.x, ti = 0;
    while (t > ti) { t -= ti + 1; ++ti; }
    const int tj = t;
    const int64_t i0 = (int64_t)ti * MT, j0 = (int64_t)tj * MT;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < p ? r0 + rows_per_split : p;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m = lane & 31, kg = lane >> 5;
    f32x16_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.f;
    if (r0 < r1) {
        if (ti == tj) syrk16_body<true>(X, q, list, r0, r1, i0, j0, sA, sB, acc);
        else syrk16_body<false>(X, q, list, r0, r1, i0, j0, sA, sB, acc);
    }
    float* out = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * MT * MT;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = wm * 64 + a * 32 + 8 * (e >> 2) + 4 * kg + (e & 3);
                const int col = wn * 64 + b * 32 + m;
                out[row * MT + col] = acc[a][b][e];
            }
}

// G[i][j] (lower tiles, mirrored) = sum over splits, in split order, in fp64;
// one element per thread, RED_BLOCKS blocks per 128 x 128 tile
constexpr int RED_BLOCKS = MT * MT / SSN_BLOCK;
__global__ __launch_bounds__(SSN_BLOCK) void k_syrk_mfma_reduce(const float* __restrict__ part,
                                                                int ntile, int nsplit,
                                                                double* __restrict__ G, int64_t q) {
    const int tile = blockIdx.x / RED_BLOCKS;
    const int e = (blockIdx.x % RED_BLOCKS) * SSN_BLOCK + threadIdx.x;
    int t = tile, ti = 0;
    while (t > ti) { t -= ti + 1; ++ti; }
    const int tj = t;
    const int a = e / MT, b = e % MT;
    const int64_t i = (int64_t)ti * MT + a, j = (int64_t)tj * MT + b;
    if (i >= q || j >= q || j > i) return;
    const float* src = part + (int64_t)tile * MT * MT + e;
    const int64_t stride = (int64_t)ntile * MT * MT;
    double s = 0.0;
    int k = 0;
    for (; k + 8 <= nsplit; k += 8) {
        float v[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) v[h] = src[(k + h) * stride];
#pragma unroll
        for (int h = 0; h < 8; ++h) s += (double)v[h];
    }
    for (; k < nsplit; ++k) s += (double)src[k * stride];
    G[i * q + j] = s;
    G[j * q + i] = s;
}

void launch_syrk_mfma(const void* X, int dtype, int64_t q, const int32_t* list, int64_t p,
                      double* G, float* part, int64_t part_cap, hipStream_t s) {
    (void)dtype;
    const int ntile = mfma_ntile(q);
    int64_t ns = mfma_nsplit(q, p);
    while (ns > 1 && ns * ntile * MT * MT > part_cap) --ns;
    int64_t rps = (p + ns - 1) / ns;
    if (q % 8 == 0) {
        rps = (rps + KC2 - 1) / KC2 * KC2;
        SSN_LAUNCH(k_syrk_mfma16, dim3((unsigned)ntile, (unsigned)ns), dim3(SSN_BLOCK), 0, s,
                           (const bf16_t*)X, q, list, p, rps, part);
    } else {
        rps = (rps + KC - 1) / KC * KC;
        SSN_LAUNCH(k_syrk_mfma, dim3((unsigned)ntile, (unsigned)ns), dim3(SSN_BLOCK), 0, s,
                           (const bf16_t*)X, q, list, p, rps, part);
    }
    SSN_LAUNCH(k_syrk_mfma_reduce, dim3((unsigned)(ntile * RED_BLOCKS)), dim3(SSN_BLOCK), 0, s,
                       part, ntile, (int)ns, G, q);
}

// ------------------------------------------------------------------ X_J v (dense)
// w[k] = X[list[k]] . v (fp64 accumulation); Pw[b] = block sum of w (for the mean)
template <typename T, int VEC>
__global__ __launch_bounds__(SSN_BLOCK) void k_dense_rows(const T* __restrict__ X, int64_t q,
                                                          const int32_t* __restrict__ list,
                                                          int64_t p, const double* __restrict__ v,
                                                          double* __restrict__ w,
                                                          double* __restrict__ Pw) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t wave = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    const int64_t nwave = (int64_t)gridDim.x * SSN_WAVES_PER_BLOCK;
    double loc = 0.0;
    for (int64_t k = wave; k < p; k += nwave) {
        const T* xr = X + (int64_t)list[k] * q;
        double acc = 0.0;
        for (int64_t c0 = (int64_t)lane * VEC; c0 < q; c0 += (int64_t)SSN_WAVE * VEC) {
            double xv[VEC];
            if (c0 + VEC <= q) {
                VecLoad<T, VEC>::load(xr + c0, xv);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) xv[e] = (c0 + e < q) ? to_f64(xr[c0 + e]) : 0.0;
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (c0 + e < q) acc = fma(xv[e], v[c0 + e], acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            w[k] = acc;
            loc += acc;
        }
    }
    const double bs = block_sum(loc, sh);
    if (threadIdx.x == 0) Pw[blockIdx.x] = bs;
}

// The same for rows that fit one 16-byte piece per lane (q <= 64 VEC, q a
// multiple of VEC): v stays in registers (each lane's VEC entries, loaded once),
// and a wave takes its rows R at a time, the R row indices loaded by lanes
// 0..R-1 at once and the R row pieces in flight together.  Rows go to waves,
// and the per-lane products and wave sums run, in the same order as above, so
// w and Pw are bit-identical to it.
template <typename T, int VEC, int R>
__global__ __launch_bounds__(SSN_BLOCK) void k_dense_rows_r(const T* __restrict__ X, int64_t q,
                                                            const int32_t* __restrict__ list,
                                                            int64_t p, const double* __restrict__ v,
                                                            double* __restrict__ w,
                                                            double* __restrict__ Pw) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t wave = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    const int64_t nwave = (int64_t)gridDim.x * SSN_WAVES_PER_BLOCK;
    const int64_t c0 = (int64_t)lane * VEC;
    const bool on = c0 < q;
    double vl[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) vl[e] = on ? v[c0 + e] : 0.0;
    double loc = 0.0;
    for (int64_t k0 = wave; k0 < p; k0 += (int64_t)R * nwave) {
        int li = 0;
        {
            const int64_t kr = k0 + (int64_t)(lane & (R - 1)) * nwave;
            if (lane < R && kr < p) li = list[kr];
        }
        RawPiece<T, VEC> pc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t kr = k0 + (int64_t)r * nwave;
            const int row = __builtin_amdgcn_readlane(li, r);
            pc[r].u = make_uint4(0u, 0u, 0u, 0u);
            if (kr < p && on) pc[r].u = *reinterpret_cast<const uint4*>(X + (int64_t)row * q + c0);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t kr = k0 + (int64_t)r * nwave;
            if (kr >= p) break;                       // uniform across the wave
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc = fma(pc[r].get(e), vl[e], acc);
            acc = wave_sum(acc);
            if (lane == 0) {
                w[kr] = acc;
                loc += acc;
            }
        }
    }
    const double bs = block_sum(loc, sh);
    if (threadIdx.x == 0) Pw[blockIdx.x] = bs;
}

unsigned dense_rows_grid(int64_t p) {
    int64_t b = (p + 3) / 4;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_dense_rows(int dtype, const void* X, int64_t q, const int32_t* list, int64_t p,
                       const double* v, double* w, double* Pw, hipStream_t s) {
    const unsigned g = dense_rows_grid(p);
    const uintptr_t a = (uintptr_t)X;
    if (dtype == SSNALM_F64) {
        if ((q * 8) % 16 == 0 && a % 16 == 0 && q <= (int64_t)SSN_WAVE * 2)
            SSN_LAUNCH((k_dense_rows_r<double, 2, 8>), dim3(g), dim3(SSN_BLOCK), 0, s, (const double*)X, q, list, p, v, w, Pw);
        else if ((q * 8) % 16 == 0 && a % 16 == 0)
            SSN_LAUNCH((k_dense_rows<double, 2>), dim3(g), dim3(SSN_BLOCK), 0, s, (const double*)X, q, list, p, v, w, Pw);
        else
            SSN_LAUNCH((k_dense_rows<double, 1>), dim3(g), dim3(SSN_BLOCK), 0, s, (const double*)X, q, list, p, v, w, Pw);
    } else if (dtype == SSNALM_F32) {
        if ((q * 4) % 16 == 0 && a % 16 == 0 && q <= (int64_t)SSN_WAVE * 4)
            SSN_LAUNCH((k_dense_rows_r<float, 4, 8>), dim3(g), dim3(SSN_BLOCK), 0, s, (const float*)X, q, list, p, v, w, Pw);
        else if ((q * 4) % 16 == 0 && a % 16 == 0)
            SSN_LAUNCH((k_dense_rows<float, 4>), dim3(g), dim3(SSN_BLOCK), 0, s, (const float*)X, q, list, p, v, w, Pw);
        else
            SSN_LAUNCH((k_dense_rows<float, 1>), dim3(g), dim3(SSN_BLOCK), 0, s, (const float*)X, q, list, p, v, w, Pw);
    } else {
        if ((q * 2) % 16 == 0 && a % 16 == 0 && q <= (int64_t)SSN_WAVE * 8)
            SSN_LAUNCH((k_dense_rows_r<bf16_t, 8, 8>), dim3(g), dim3(SSN_BLOCK), 0, s, (const bf16_t*)X, q, list, p, v, w, Pw);
        else if ((q * 2) % 16 == 0 && a % 16 == 0)
            SSN_LAUNCH((k_dense_rows<bf16_t, 8>), dim3(g), dim3(SSN_BLOCK), 0, s, (const bf16_t*)X, q, list, p, v, w, Pw);
        else
            SSN_LAUNCH((k_dense_rows<bf16_t, 1>), dim3(g), dim3(SSN_BLOCK), 0, s, (const bf16_t*)X, q, list, p, v, w, Pw);
    }
}

// z[list[k]] = y_i (w_k - mean), mean = sum(Pw) / p (every block reduces the
// partials itself, fixed order); the transposed product of A then gives
// X_J^T (w - mean 1).
__global__ __launch_bounds__(SSN_BLOCK) void k_scatter_centered(const int32_t* __restrict__ list,
                                                                int64_t p, const double* __restrict__ w,
                                                                const double* __restrict__ Pw, int nbw,
                                                                const int8_t* __restrict__ y,
                                                                double* __restrict__ z) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    double a = 0.0;
    for (int b = threadIdx.x; b < nbw; b += blockDim.x) a += Pw[b];
    const double mean = p > 0 ? block_sum(a, sh) / (double)p : 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < p;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = list[k];
        z[i] = (double)y[i] * (w[k] - mean);
    }
}
void launch_scatter_centered(const int32_t* list, int64_t p, const double* w, const double* Pw,
                             int nbw, const int8_t* y, double* z, hipStream_t s) {
    int64_t b = (p + 255) / 256;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    SSN_LAUNCH(k_scatter_centered, dim3((unsigned)b), dim3(SSN_BLOCK), 0, s, list, p, w, Pw,
                       nbw, y, z);
}

// rn = g + d + sigma t  (= -(residual of M d = -g)), out for the next solve
__global__ void k_refine_res(const double* __restrict__ g, const double* __restrict__ d,
                             const double* __restrict__ t, double sigma, double* __restrict__ rn,
                             int64_t q) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < q) rn[j] = g[j] + d[j] + sigma * t[j];
}
void launch_refine_res(const double* g, const double* d, const double* t, double sigma, double* rn,
                       int64_t q, hipStream_t s) {
    SSN_LAUNCH(k_refine_res, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, g, d, t,
                       sigma, rn, q);
}

}  // namespace ssn
