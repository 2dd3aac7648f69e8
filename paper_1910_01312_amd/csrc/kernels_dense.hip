// Dense products with A = diag(y) X for row-major X (fp64 / fp32 / bf16
// storage, fp64 accumulation):
//   forward   t = A v = y .* (X v)           (Q w = A omega, eq. Def_psi)
//   transpose r = A^T z = X^T (y .* z)       (grad psi, eq. Def_differential_of_psi)
// Both stream X once from HBM.  A wave owns whole rows: its 64 lanes read
// one row in 16-byte pieces, so every load instruction of the wave covers a
// contiguous 1 KiB of the row.  The forward product reduces each row across
// the wave; the transpose keeps per-lane column accumulators and never
// reduces per row.  Rows whose coefficient is zero are skipped in the
// transpose, so it reads only the support-vector rows.
#include "dev_common.h"
#include "lane_ops.h"
#include "ssn_internal.h"

namespace ssn {

// ---------------------------------------------------------------- forward
// Each wave handles ROWS rows per iteration; lane l covers columns
// [c*64*VEC + l*VEC, +VEC) for chunk c.  v is staged in LDS when it fits.
template <typename T, int VEC, int ROWS>
__global__ __launch_bounds__(SSN_BLOCK) void k_amul_dense(const T* __restrict__ X,
                                                          const int8_t* __restrict__ y,
                                                          const double* __restrict__ v,
                                                          double* __restrict__ t,
                                                          int64_t n, int64_t q, int use_lds) {
    extern __shared__ double sv[];
    const double* vv = v;
    if (use_lds) {
        for (int64_t j = threadIdx.x; j < q; j += blockDim.x) sv[j] = v[j];
        __syncthreads();
        vv = sv;
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t wave = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    const int64_t nwave = (int64_t)gridDim.x * SSN_WAVES_PER_BLOCK;
    const int64_t span = (int64_t)SSN_WAVE * VEC;
    for (int64_t r0 = wave * ROWS; r0 < n; r0 += nwave * ROWS) {
        double acc[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;
        for (int64_t c0 = (int64_t)lane * VEC; c0 < q; c0 += span) {
            double vloc[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) vloc[e] = (c0 + e < q) ? vv[c0 + e] : 0.0;
            double xv[ROWS][VEC];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int64_t row = r0 + r;
                if (row < n) {
                    if (VEC == 1 || c0 + VEC <= q) {
                        VecLoad<T, VEC>::load(X + row * q + c0, xv[r]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            xv[r][e] = (c0 + e < q) ? to_f64(X[row * q + c0 + e]) : 0.0;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) xv[r][e] = 0.0;
                }
            }
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[r] = fma(xv[r][e], vloc[e], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            double s = wave_sum(acc[r]);
            const int64_t row = r0 + r;
            if (lane == r && row < n) t[row] = (double)y[row] * s;
        }
    }
}

// ---------------------------------------------------------------- forward, q <= 64 VEC
// Rows that fit one 16-byte piece per lane: lane l covers columns
// [l VEC, l VEC + VEC) of every row, so its slice of v stays in registers.
// A wave keeps R rows in flight as raw 16-byte pieces (widened only at the
// FMA), then a reduce-scatter over the R rows (log2 R exchange steps, each
// halving the live values) followed by plain xor sums leaves the total of
// row 4 b5 + 2 b4 + b3 (lane bits, for R = 8) in the lanes whose low bits
// are zero.  Fixed summation order: deterministic.
template <typename T, int VEC, int R>
__global__ __launch_bounds__(SSN_BLOCK) void k_amul_rows(const T* __restrict__ X,
                                                         const int8_t* __restrict__ y,
                                                         const double* __restrict__ v,
                                                         double* __restrict__ t, int64_t n,
                                                         int64_t q) {
    static_assert(R >= 1 && R <= SSN_WAVE && (R & (R - 1)) == 0, "R: power of two");
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t wave = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    const int64_t nwave = (int64_t)gridDim.x * SSN_WAVES_PER_BLOCK;
    const int64_t c0 = (int64_t)lane * VEC;
    double vloc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) vloc[e] = c0 + e < q ? v[c0 + e] : 0.0;
    // q is a multiple of VEC here; every load is issued: a lane past the row
    // end reads the row's last piece and a row past n reads row n - 1, and
    // both products are dropped (vloc is 0 there, the store is skipped), so
    // that no load sits under a branch
    const int64_t cc = c0 < q ? c0 : q - VEC;
    for (int64_t r0 = wave * R; r0 < n; r0 += nwave * R) {
        RawPiece<T, VEC> raw[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t row = r0 + u < n ? r0 + u : n - 1;
            raw[u].u = *reinterpret_cast<const uint4*>(X + row * q + cc);
        }
        double acc[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            double a = 0.0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) a = fma(raw[u].get(e), vloc[e], a);
            acc[u] = a;
        }
        // reduce-scatter over the R rows
#pragma unroll
        for (int h = SSN_WAVE / 2, live = R; live > 1; h >>= 1, live >>= 1) {
            const bool up = (lane & h) != 0;
#pragma unroll
            for (int j = 0; j < live / 2; ++j) {
                const double lo_v = acc[j], hi_v = acc[j + live / 2];
                const double send = up ? lo_v : hi_v;
                const double keep = up ? hi_v : lo_v;
                acc[j] = keep + __shfl_xor(send, h, SSN_WAVE);
            }
        }
        double sum = acc[0];
#pragma unroll
        for (int h = SSN_WAVE / (2 * R); h >= 1; h >>= 1) sum += __shfl_xor(sum, h, SSN_WAVE);
        // lane bits above log2(64 / R) name the row
        const int sub = SSN_WAVE / R;
        if ((lane & (sub - 1)) == 0) {
            int u = 0;
#pragma unroll
            for (int b = 0, h = SSN_WAVE / 2; (1 << b) < R; ++b, h >>= 1)
                if (lane & h) u |= (R >> (b + 1));
            const int64_t row = r0 + u;
            if (row < n) t[row] = (double)y[row] * sum;
        }
    }
}

template <typename T, int VEC>
static void amul_dispatch_rows(const T* X, const int8_t* y, const double* v, double* t,
                               int64_t n, int64_t q, hipStream_t s) {
    if constexpr (VEC * sizeof(T) == 16) {
      if (q <= (int64_t)SSN_WAVE * VEC) {
        constexpr int R = 8;
        int64_t blocks = (n + R * SSN_WAVES_PER_BLOCK - 1) / (R * SSN_WAVES_PER_BLOCK);
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        SSN_LAUNCH((k_amul_rows<T, VEC, R>), dim3((unsigned)blocks), dim3(SSN_BLOCK), 0, s,
                           X, y, v, t, n, q);
        return;
      }
    }
    const int use_lds = q <= 8192 ? 1 : 0;
    const size_t shm = use_lds ? (size_t)q * sizeof(double) : 0;
    // enough waves to keep every CU busy; each wave walks rows with a stride
    int64_t rows_per_wave = 4;
    int64_t blocks = (n + rows_per_wave * SSN_WAVES_PER_BLOCK - 1) / (rows_per_wave * SSN_WAVES_PER_BLOCK);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    SSN_LAUNCH((k_amul_dense<T, VEC, 4>), dim3((unsigned)blocks), dim3(SSN_BLOCK), shm, s,
                       X, y, v, t, n, q, use_lds);
}

void launch_amul_dense(int dtype, const void* X, const int8_t* y, const double* v, double* t,
                       int64_t n, int64_t q, hipStream_t s) {
    const uintptr_t a = (uintptr_t)X;
    if (dtype == SSNALM_F64) {
        if ((q * 8) % 16 == 0 && a % 16 == 0)
            amul_dispatch_rows<double, 2>((const double*)X, y, v, t, n, q, s);
        else
            amul_dispatch_rows<double, 1>((const double*)X, y, v, t, n, q, s);
    } else if (dtype == SSNALM_F32) {
        if ((q * 4) % 16 == 0 && a % 16 == 0)
            amul_dispatch_rows<float, 4>((const float*)X, y, v, t, n, q, s);
        else
            amul_dispatch_rows<float, 1>((const float*)X, y, v, t, n, q, s);
    } else {
        if ((q * 2) % 16 == 0 && a % 16 == 0)
            amul_dispatch_rows<bf16_t, 8>((const bf16_t*)X, y, v, t, n, q, s);
        else
            amul_dispatch_rows<bf16_t, 1>((const bf16_t*)X, y, v, t, n, q, s);
    }
}

// ---------------------------------------------------------------- transpose
// Block b owns rows [b*rows_per_blk, ...).  Column tile blockIdx.y covers
// NCH chunks of 64*VEC columns.  Every lane keeps NCH*VEC accumulators for
// the coefficient y.*z and (with a mask) NCH*VEC more for the 0/1 mask.
// At the end the four waves are summed through LDS in a fixed order and the
// block writes its partial row part[b*q + j].
template <typename T, int VEC, int NCH, int MM>
__global__ __launch_bounds__(SSN_BLOCK) void k_atmul_dense(const T* __restrict__ X,
                                                           const int8_t* __restrict__ y,
                                                           const double* __restrict__ z,
                                                           const uint8_t* __restrict__ mask,
                                                           int64_t n, int64_t q,
                                                           int64_t rows_per_blk,
                                                           double* __restrict__ part,
                                                           double* __restrict__ part2) {
    __shared__ double red[SSN_WAVES_PER_BLOCK][SSN_WAVE * VEC * NCH];
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int w = threadIdx.x / SSN_WAVE;
    const int64_t tile_cols = (int64_t)SSN_WAVE * VEC * NCH;
    const int64_t col0 = (int64_t)blockIdx.y * tile_cols;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t re = rb + rows_per_blk < n ? rb + rows_per_blk : n;

    double acc[NCH][VEC], acc2[NCH][VEC];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) { acc[c][e] = 0.0; acc2[c][e] = 0.0; }

    for (int64_t row = rb + w; row < re; row += SSN_WAVES_PER_BLOCK) {
        const double cf = z ? (double)y[row] * z[row] : 0.0;
        const double cm = MM ? (double)mask[row] : 0.0;
        if (cf == 0.0 && cm == 0.0) continue;     // uniform across the wave
        const T* xr = X + row * q;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int64_t j0 = col0 + (int64_t)c * SSN_WAVE * VEC + (int64_t)lane * VEC;
            double xv[VEC];
            if (j0 + VEC <= q) {
                VecLoad<T, VEC>::load(xr + j0, xv);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) xv[e] = (j0 + e < q) ? to_f64(xr[j0 + e]) : 0.0;
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                acc[c][e] = fma(cf, xv[e], acc[c][e]);
                if (MM == 1) acc2[c][e] = fma(cm, xv[e], acc2[c][e]);
                if (MM == 2) acc2[c][e] = fma(cm * xv[e], xv[e], acc2[c][e]);
            }
        }
    }
    // block reduction through LDS (fixed order), twice when masked
#pragma unroll
    for (int pass = 0; pass < (MM ? 2 : 1); ++pass) {
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                red[w][c * SSN_WAVE * VEC + lane * VEC + e] = pass == 0 ? acc[c][e] : acc2[c][e];
        __syncthreads();
        double* out = pass == 0 ? part : part2;
        for (int64_t k = threadIdx.x; k < tile_cols; k += SSN_BLOCK) {
            const int64_t j = col0 + k;
            if (j < q) {
                double sacc = 0.0;
#pragma unroll
                for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) sacc += red[ww][k];
                out[(int64_t)blockIdx.x * q + j] = sacc;
            }
        }
        __syncthreads();
    }
}

// The same sums for rows that fit one 16-byte piece per lane (q <= 64 VEC,
// q VEC-aligned).  A wave takes 64-row chunks: lane l loads row l's
// coefficients (those of the next chunk are loaded while this one is
// processed), a ballot marks the rows with a nonzero one, and the wave walks
// the marked rows R at a time, issuing all R row loads (raw pieces, widened
// at the FMA) before the first FMA, with each coefficient broadcast from its
// lane by readlane.  Rows with zero coefficients are never read, and every
// batch is R useful rows however sparse the coefficients are.  Then the block
// reduction as above.
template <typename T, int VEC, int R, int MM>
__global__ __launch_bounds__(SSN_BLOCK) void k_atmul_rows(const T* __restrict__ X,
                                                          const int8_t* __restrict__ y,
                                                          const double* __restrict__ z,
                                                          const uint8_t* __restrict__ mask,
                                                          int64_t n, int64_t q,
                                                          int64_t rows_per_blk,
                                                          double* __restrict__ part,
                                                          double* __restrict__ part2) {
    __shared__ double red[SSN_WAVES_PER_BLOCK][SSN_WAVE * VEC];
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int w = threadIdx.x / SSN_WAVE;
    const int64_t rb = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t re = rb + rows_per_blk < n ? rb + rows_per_blk : n;
    const bool on = (int64_t)lane * VEC < q;
    const int64_t cstep = (int64_t)SSN_WAVES_PER_BLOCK * SSN_WAVE;
    double acc[VEC], acc2[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) { acc[e] = 0.0; acc2[e] = 0.0; }
    auto coef = [&](int64_t row, double& mz, double& mm) {
        mz = 0.0;
        mm = 0.0;
        if (row < re) {
            if (z) mz = (double)y[row] * z[row];
            if (MM) mm = (double)mask[row];
        }
    };
    int64_t cb = rb + (int64_t)w * SSN_WAVE;
    double mzn, mmn;
    coef(cb + lane, mzn, mmn);
    for (; cb < re; cb += cstep) {
        const double mz = mzn, mm = mmn;
        coef(cb + cstep + lane, mzn, mmn);          // the next chunk's, in flight meanwhile
        unsigned long long bits = __ballot(mz != 0.0 || mm != 0.0);
        while (bits) {                              // uniform across the wave
            int rr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rr[r] = bits ? __ffsll((unsigned long long)bits) - 1 : -1;
                bits &= bits - 1;
            }
            RawPiece<T, VEC> pc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                pc[r].u = make_uint4(0u, 0u, 0u, 0u);
                if (rr[r] >= 0 && on)
                    pc[r].u = *reinterpret_cast<const uint4*>(X + (cb + rr[r]) * q + (int64_t)lane * VEC);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (rr[r] < 0) break;
                const double cf = readlane_f64(mz, rr[r]);
                const double cm = MM ? readlane_f64(mm, rr[r]) : 0.0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const double xv = pc[r].get(e);
                    acc[e] = fma(cf, xv, acc[e]);
                    if (MM == 1) acc2[e] = fma(cm, xv, acc2[e]);
                    if (MM == 2) acc2[e] = fma(cm * xv, xv, acc2[e]);
                }
            }
        }
    }
#pragma unroll
    for (int pass = 0; pass < (MM ? 2 : 1); ++pass) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) red[w][lane * VEC + e] = pass == 0 ? acc[e] : acc2[e];
        __syncthreads();
        double* out = pass == 0 ? part : part2;
        for (int64_t k = threadIdx.x; k < q; k += SSN_BLOCK) {
            double sacc = 0.0;
#pragma unroll
            for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) sacc += red[ww][k];
            out[(int64_t)blockIdx.x * q + k] = sacc;
        }
        __syncthreads();
    }
}

int atmul_dense_nblk(int64_t n) {
    int64_t nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    return (int)nb;
}

template <typename T, int VEC>
static void atmul_dispatch(const T* X, const int8_t* y, const double* z, const uint8_t* mask,
                           int64_t n, int64_t q, double* part, double* part2, hipStream_t s,
                           int mm) {
    const int nb = atmul_dense_nblk(n);
    const int64_t rows_per_blk = (n + nb - 1) / nb;
    if constexpr (VEC * sizeof(T) == 16) {
        if (q <= (int64_t)SSN_WAVE * VEC) {            // one piece per lane covers a row
            constexpr int R = 8;
            if (mask && mm == 2)
                SSN_LAUNCH((k_atmul_rows<T, VEC, R, 2>), dim3((unsigned)nb), dim3(SSN_BLOCK), 0,
                                   s, X, y, z, mask, n, q, rows_per_blk, part, part2);
            else if (mask)
                SSN_LAUNCH((k_atmul_rows<T, VEC, R, 1>), dim3((unsigned)nb), dim3(SSN_BLOCK), 0,
                                   s, X, y, z, mask, n, q, rows_per_blk, part, part2);
            else
                SSN_LAUNCH((k_atmul_rows<T, VEC, R, 0>), dim3((unsigned)nb), dim3(SSN_BLOCK), 0,
                                   s, X, y, z, mask, n, q, rows_per_blk, part, part2);
            return;
        }
    }
    constexpr int NCH = (VEC == 1) ? 4 : 2;     // columns per tile: 64*VEC*NCH
    const int64_t tile_cols = (int64_t)SSN_WAVE * VEC * NCH;
    const int64_t ty = (q + tile_cols - 1) / tile_cols;
    dim3 grid((unsigned)nb, (unsigned)ty);
    if (mask && mm == 2)
        SSN_LAUNCH((k_atmul_dense<T, VEC, NCH, 2>), grid, dim3(SSN_BLOCK), 0, s, X, y,
                           z, mask, n, q, rows_per_blk, part, part2);
    else if (mask)
        SSN_LAUNCH((k_atmul_dense<T, VEC, NCH, 1>), grid, dim3(SSN_BLOCK), 0, s, X, y,
                           z, mask, n, q, rows_per_blk, part, part2);
    else
        SSN_LAUNCH((k_atmul_dense<T, VEC, NCH, 0>), grid, dim3(SSN_BLOCK), 0, s, X, y,
                           z, mask, n, q, rows_per_blk, part, part2);
}

void launch_atmul_dense(int dtype, const void* X, const int8_t* y, const double* z,
                        const uint8_t* mask, int64_t n, int64_t q, double* part, double* part2,
                        hipStream_t s, int mm) {
    const uintptr_t a = (uintptr_t)X;
    if (dtype == SSNALM_F64) {
        if ((q * 8) % 16 == 0 && a % 16 == 0)
            atmul_dispatch<double, 2>((const double*)X, y, z, mask, n, q, part, part2, s, mm);
        else
            atmul_dispatch<double, 1>((const double*)X, y, z, mask, n, q, part, part2, s, mm);
    } else if (dtype == SSNALM_F32) {
        if ((q * 4) % 16 == 0 && a % 16 == 0)
            atmul_dispatch<float, 4>((const float*)X, y, z, mask, n, q, part, part2, s, mm);
        else
            atmul_dispatch<float, 1>((const float*)X, y, z, mask, n, q, part, part2, s, mm);
    } else {
        if ((q * 2) % 16 == 0 && a % 16 == 0)
            atmul_dispatch<bf16_t, 8>((const bf16_t*)X, y, z, mask, n, q, part, part2, s, mm);
        else
            atmul_dispatch<bf16_t, 1>((const bf16_t*)X, y, z, mask, n, q, part, part2, s, mm);
    }
}

// out[j] = base[j] + sign * sum_b part[b*q + j].  A block of 16 waves owns 64
// columns (one per lane); wave w sums the partial rows b = w, w+16, ... with
// eight loads in flight, and the 16 wave sums are added in wave order: a fixed
// order, so the result is deterministic.
constexpr int RC_WAVES = 16;
constexpr int RC_UNROLL = 8;
__global__ __launch_bounds__(RC_WAVES * SSN_WAVE) void k_reduce_cols(const double* __restrict__ part,
                                                                    int nblk, int64_t q,
                                                                    const double* __restrict__ base,
                                                                    double sign, double* __restrict__ out) {
    __shared__ double sh[RC_WAVES][SSN_WAVE];
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    const int64_t j = (int64_t)blockIdx.x * SSN_WAVE + lane;
    double s = 0.0;
    if (j < q) {
        int b = w;
        for (; b + (RC_UNROLL - 1) * RC_WAVES < nblk; b += RC_UNROLL * RC_WAVES) {
            double a[RC_UNROLL];
#pragma unroll
            for (int u = 0; u < RC_UNROLL; ++u) a[u] = part[(int64_t)(b + u * RC_WAVES) * q + j];
#pragma unroll
            for (int u = 0; u < RC_UNROLL; ++u) s += a[u];
        }
        for (; b < nblk; b += RC_WAVES) s += part[(int64_t)b * q + j];
    }
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < q) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < RC_WAVES; ++k) t += sh[k][lane];
        out[j] = (base ? base[j] : 0.0) + sign * t;
    }
}

void launch_reduce_cols(const double* part, int nblk, int64_t q, const double* base, double sign,
                        double* out, hipStream_t s) {
    const unsigned blocks = (unsigned)((q + SSN_WAVE - 1) / SSN_WAVE);
    SSN_LAUNCH(k_reduce_cols, dim3(blocks), dim3(RC_WAVES * SSN_WAVE), 0, s, part, nblk, q, base,
                       sign, out);
}

}  // namespace ssn
