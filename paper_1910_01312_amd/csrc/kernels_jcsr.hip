// Sparse products restricted to the free rows J (the rows that carry the
// second-order sparsity of Proposition 5), used by the matrix-free Newton
// operator M v = v + sigma X_J^T (I - 1 1^T / p) X_J v for CSR input.
//
//  * X_J v : one 16-lane group per row of the ordered J list (each row's
//            entries are contiguous in CSR), result as a p-vector.
//  * X_J^T z: a column-major copy of X_J, rebuilt once per Newton step by
//            filtering the full column-major copy (CSC) down to the entries
//            whose row is in J.  The filter keeps the full copy's 512-entry
//            tile boundaries, so a compact tile t holds exactly the J entries
//            of full tile t and the full plan's per-tile first/last columns
//            and its list of tile-spanning columns stay valid; the product
//            then runs the same segmented reduction as the full operator on
//            far fewer entries.  Each kept entry stores (rank of its row in
//            J, column, value); the rank indexes the p-vector directly.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int JE = 8;                       // entries per lane, as the full plan
constexpr int JTILE = JE * SSN_WAVE;        // entries per full tile

// ------------------------------------------------------------------ ranks
__global__ void k_rank_from_list(const int32_t* __restrict__ list, const long long* __restrict__ pdev,
                                 int32_t* __restrict__ rank) {
    const long long p = *pdev;
    for (long long k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < p;
         k += (int64_t)gridDim.x * blockDim.x)
        rank[list[k]] = (int32_t)k;
}
void launch_rank_from_list(const int32_t* list, const long long* pdev, int64_t n, int32_t* rank,
                           hipStream_t s) {
    int64_t b = (n + 255) / 256;
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(k_rank_from_list, dim3((unsigned)b), dim3(256), 0, s, list, pdev, rank);
}

// ------------------------------------------------------------------ X_J v
// w[k] = sum_{e in row list[k]} val[e] v[col[e]] for k < p; the block sums of
// w go to part[], and the last block stores mean = sum w / p in *mean_out.
template <typename V>
__global__ __launch_bounds__(SSN_BLOCK) void k_rows_fwd(const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const V* __restrict__ val,
                                                        const int32_t* __restrict__ list,
                                                        int64_t p, const double* __restrict__ v,
                                                        double* __restrict__ w,
                                                        double* mean_out,
                                                        double* __restrict__ part,
                                                        unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int grp = lane >> 4, sub = lane & 15;
    const int64_t wave = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    const int64_t nwave = (int64_t)gridDim.x * SSN_WAVES_PER_BLOCK;
    double local = 0.0;
    for (int64_t base = wave * 4; base < p; base += nwave * 4) {
        const int64_t k = base + grp;
        double acc = 0.0;
        if (k < p) {
            const int32_t r = list[k];
            const int32_t e0 = rp[r], e1 = rp[r + 1];
            for (int32_t e = e0 + sub; e < e1; e += 16) acc = fma((double)val[e], v[ci[e]], acc);
        }
        acc += __shfl_xor(acc, 8, SSN_WAVE);
        acc += __shfl_xor(acc, 4, SSN_WAVE);
        acc += __shfl_xor(acc, 2, SSN_WAVE);
        acc += __shfl_xor(acc, 1, SSN_WAVE);
        if (k < p && sub == 0) {
            w[k] = acc;
            local += acc;
        }
    }
    const double bs = block_sum(local, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
    if (last_block_arrives(counter)) {
        const double tot = grid_colsum(part, gridDim.x, 1, 0, shd);
        if (threadIdx.x == 0) *mean_out = p > 0 ? tot / (double)p : 0.0;
    }
}

unsigned rows_fwd_grid(int64_t p) {
    int64_t b = (p + 15) / 16;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_rows_fwd(const SegPlan& F, const int32_t* list, int64_t p, const double* v, double* w,
                     double* mean_out, double* part, unsigned* counter, hipStream_t s) {
    const unsigned g = rows_fwd_grid(p);
    if (F.val_f64)
        hipLaunchKernelGGL((k_rows_fwd<double>), dim3(g), dim3(SSN_BLOCK), 0, s, F.ptr, F.idx,
                           (const double*)F.val, list, p, v, w, mean_out, part, counter);
    else
        hipLaunchKernelGGL((k_rows_fwd<float>), dim3(g), dim3(SSN_BLOCK), 0, s, F.ptr, F.idx,
                           (const float*)F.val, list, p, v, w, mean_out, part, counter);
}

// ------------------------------------------------------------------ filter
// Per full tile: number of entries whose row is in J.
__global__ __launch_bounds__(SSN_BLOCK) void k_jcsc_count(const int32_t* __restrict__ ridx,
                                                          int64_t nnz, int64_t ntile,
                                                          const uint8_t* __restrict__ mask,
                                                          int* __restrict__ tcount) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t t = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (t >= ntile) return;
    const int64_t k0 = t * JTILE + (int64_t)lane * JE;
    int c = 0;
#pragma unroll
    for (int e = 0; e < JE; ++e) {
        const int64_t k = k0 + e;
        if (k < nnz) c += mask[ridx[k]] ? 1 : 0;
    }
    c = (int)wave_sum_ll(c);
    if (lane == 0) tcount[t] = c;
}

// Exclusive scan of tcount[0..ntile) into toff[0..ntile] by one block of
// 1024 threads, 8192 entries per round: a coalesced load into LDS, a
// sequential scan of 8 entries per thread, a wave scan and a scan of the 16
// wave totals.  Integer sums: exact.  *total = toff[ntile].
__global__ __launch_bounds__(1024) void k_scan_tiles(const int* __restrict__ tcount, int64_t ntile,
                                                     int* __restrict__ toff, long long* total) {
    __shared__ int buf[8192];
    __shared__ long long wtot[16];
    __shared__ long long round_tot;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    long long carry = 0;
    for (int64_t base = 0; base < ntile; base += 8192) {
        for (int i = tid; i < 8192; i += 1024) {
            const int64_t k = base + i;
            buf[i] = k < ntile ? tcount[k] : 0;
        }
        __syncthreads();
        int loc[8];
        long long s = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            loc[e] = (int)s;
            s += buf[tid * 8 + e];
        }
        long long incl = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wtot[wv] = incl;
        __syncthreads();
        if (tid == 0) {
            long long run = 0;
            for (int k = 0; k < 16; ++k) {
                const long long t = wtot[k];
                wtot[k] = run;
                run += t;
            }
            round_tot = run;
        }
        __syncthreads();
        const long long excl = carry + wtot[wv] + incl - s;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t k = base + tid * 8 + e;
            if (k < ntile) toff[k] = (int)(excl + loc[e]);
        }
        carry += round_tot;
        __syncthreads();
    }
    if (tid == 0) {
        toff[ntile] = (int)carry;
        *total = carry;
    }
}

// Write the kept entries of full tile t at toff[t] + (rank among the tile's
// kept entries), in the full copy's order (columns ascending).
template <typename V>
__global__ __launch_bounds__(SSN_BLOCK) void k_jcsc_write(
    const int32_t* __restrict__ cptr, const int32_t* __restrict__ ridx, const V* __restrict__ val,
    int64_t nnz, int64_t ntile, const int32_t* __restrict__ lane_seg,
    const uint8_t* __restrict__ mask, const int32_t* __restrict__ rank,
    const int* __restrict__ toff, int32_t* __restrict__ jr, int32_t* __restrict__ jc,
    V* __restrict__ jv) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t t = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (t >= ntile) return;
    const int64_t k0 = t * JTILE + (int64_t)lane * JE;
    bool keep[JE];
    int32_t row[JE];
    int c = 0;
#pragma unroll
    for (int e = 0; e < JE; ++e) {
        const int64_t k = k0 + e;
        row[e] = k < nnz ? ridx[k] : 0;
        keep[e] = k < nnz && mask[row[e]];
        c += keep[e] ? 1 : 0;
    }
    // exclusive prefix of c over the lanes of the wave
    int incl = c;
#pragma unroll
    for (int off = 1; off < SSN_WAVE; off <<= 1) {
        const int o = __shfl_up(incl, off, SSN_WAVE);
        if (lane >= off) incl += o;
    }
    int pos = toff[t] + incl - c;
    if (c == 0) return;
    int32_t seg = lane_seg[t * SSN_WAVE + lane];
    int64_t segend = cptr[seg + 1];
#pragma unroll
    for (int e = 0; e < JE; ++e) {
        const int64_t k = k0 + e;
        if (k >= nnz) break;
        while (k >= segend) {
            ++seg;
            segend = cptr[seg + 1];
        }
        if (keep[e]) {
            jr[pos] = rank[row[e]];
            jc[pos] = seg;
            jv[pos] = val[k];
            ++pos;
        }
    }
}

void launch_jcsc_build(const SegPlan& T, const uint8_t* mask, const int32_t* rank, int* tcount,
                       int* toff, long long* total, int32_t* jr, int32_t* jc, void* jv,
                       hipStream_t s) {
    const unsigned nb = (unsigned)((T.ntile + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
    if (T.ntile == 0) return;
    hipLaunchKernelGGL(k_jcsc_count, dim3(nb), dim3(SSN_BLOCK), 0, s, T.idx, T.nnz, T.ntile, mask,
                       tcount);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, tcount, T.ntile, toff, total);
    if (T.val_f64)
        hipLaunchKernelGGL((k_jcsc_write<double>), dim3(nb), dim3(SSN_BLOCK), 0, s, T.ptr, T.idx,
                           (const double*)T.val, T.nnz, T.ntile, T.lane_seg, mask, rank, toff, jr,
                           jc, (double*)jv);
    else
        hipLaunchKernelGGL((k_jcsc_write<float>), dim3(nb), dim3(SSN_BLOCK), 0, s, T.ptr, T.idx,
                           (const float*)T.val, T.nnz, T.ntile, T.lane_seg, mask, rank, toff, jr,
                           jc, (float*)jv);
}

// ------------------------------------------------------------------ X_J^T z
// out[c] (+ per-tile carries of tile-spanning columns) = sum over the kept
// entries of column c of coef(e) with
//   MODE 0: val * (w[rank] - mean)   (centred operator)
//   MODE 1: val                      (s = X_J^T 1)
//   MODE 2: val^2                    (Jacobi diagonal)
// Columns without kept entries are not written: out must be zeroed first.
template <typename V, int MODE>
__global__ __launch_bounds__(SSN_BLOCK) void k_jcsc_tr(
    const int* __restrict__ toff, const int32_t* __restrict__ jr, const int32_t* __restrict__ jc,
    const V* __restrict__ jv, int64_t ntile, int64_t nnz_full, const int32_t* __restrict__ cptr,
    const int32_t* __restrict__ tile_first, const double* __restrict__ w,
    const double* __restrict__ mean, double* __restrict__ carry, double* __restrict__ out) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t t = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (t >= ntile) return;
    const int64_t fb = t * JTILE;                                   // full tile range
    const int64_t fe = fb + JTILE < nnz_full ? fb + JTILE : nnz_full;
    const int cb = toff[t], ce = toff[t + 1];                       // compact range
    const int k0 = cb + lane * JE;
    const int k1 = k0 + JE < ce ? k0 + JE : ce;
    const bool active = k0 < ce;
    const double mu = (MODE == 0) ? *mean : 0.0;
    const int32_t INF = 0x7fffffff;
    int32_t F = INF, Lt = INF;
    double fsum = 0.0, lsum = 0.0;
    if (active) {
        int32_t key = jc[k0];
        F = key;
        double cur = 0.0;
        bool first_closed = false;
        for (int k = k0; k < k1; ++k) {
            const int32_t kk = jc[k];
            if (kk != key) {
                if (!first_closed) {
                    first_closed = true;
                    fsum = cur;               // run of F, may continue from the left
                } else {
                    out[key] = cur;           // middle run: complete, not tile-spanning
                }
                key = kk;
                cur = 0.0;
            }
            const double a = (double)jv[k];
            double cf;
            if (MODE == 0) cf = a * (w[jr[k]] - mu);
            else if (MODE == 1) cf = a;
            else cf = a * a;
            cur += cf;
        }
        Lt = key;
        lsum = cur;
        if (!first_closed) F = Lt;          // F == Lt: no separate head
    }
    // segmented inclusive scan of the tail sums keyed by Lt
    double S = lsum;
#pragma unroll
    for (int off = 1; off < SSN_WAVE; off <<= 1) {
        const double o = __shfl_up(S, off, SSN_WAVE);
        const int32_t ok = __shfl_up(Lt, off, SSN_WAVE);
        if (lane >= off && ok == Lt) S += o;
    }
    const double S_prev = __shfl_up(S, 1, SSN_WAVE);
    const int32_t Lt_prev = __shfl_up(Lt, 1, SSN_WAVE);
    const int32_t F_next = __shfl_down(F, 1, SSN_WAVE);
    const bool has_next = lane + 1 < SSN_WAVE && (k0 + JE) < ce;
    const int32_t tf = tile_first[t];
    int slot_written = 0;                  // bit 0: slot 0, bit 1: slot 1
    auto emit = [&](int32_t c, double v) {
        const int64_t a = cptr[c], b = cptr[c + 1];
        if (a >= fb && b <= fe) {
            out[c] = v;
        } else {
            const int slot = (c == tf) ? 0 : 1;
            carry[t * 2 + slot] = v;
            slot_written |= 1 << slot;
        }
    };
    if (active) {
        if (F < Lt) {
            double tot = fsum;
            if (lane > 0 && Lt_prev == F) tot += S_prev;
            emit(F, tot);
        }
        if (!has_next || F_next != Lt) emit(Lt, S);
    }
    // carries of spanning columns absent from this compact tile are zero
    const unsigned long long b0 = __ballot(slot_written & 1);
    const unsigned long long b1 = __ballot(slot_written & 2);
    if (lane == 0) {
        if (!b0) carry[t * 2 + 0] = 0.0;
        if (!b1) carry[t * 2 + 1] = 0.0;
    }
}

template <int MODE>
static void jcsc_tr_launch(const SegPlan& T, const int* toff, const int32_t* jr, const int32_t* jc,
                           const void* jv, const double* w, const double* mean, double* out,
                           hipStream_t s) {
    const unsigned nb = (unsigned)((T.ntile + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
    if (T.ntile == 0) return;
    if (T.val_f64)
        hipLaunchKernelGGL((k_jcsc_tr<double, MODE>), dim3(nb), dim3(SSN_BLOCK), 0, s, toff, jr, jc,
                           (const double*)jv, T.ntile, T.nnz, T.ptr, T.tile_first, w, mean, T.carry,
                           out);
    else
        hipLaunchKernelGGL((k_jcsc_tr<float, MODE>), dim3(nb), dim3(SSN_BLOCK), 0, s, toff, jr, jc,
                           (const float*)jv, T.ntile, T.nnz, T.ptr, T.tile_first, w, mean, T.carry,
                           out);
}

void launch_segsum_fix_only(const SegPlan& P, double* out, hipStream_t s);

// out = X_J^T (w - mean) (mode 0), X_J^T 1 (mode 1) or sum_J X_ij^2 (mode 2)
void launch_jcsc_tr(int mode, const SegPlan& T, const int* toff, const int32_t* jr,
                    const int32_t* jc, const void* jv, const double* w, const double* mean,
                    double* out, int64_t q, hipStream_t s) {
    launch_fill(out, 0.0, q, s);
    if (mode == 0) jcsc_tr_launch<0>(T, toff, jr, jc, jv, w, mean, out, s);
    else if (mode == 1) jcsc_tr_launch<1>(T, toff, jr, jc, jv, w, mean, out, s);
    else jcsc_tr_launch<2>(T, toff, jr, jc, jv, w, mean, out, s);
    launch_segsum_fix_only(T, out, s);
}

// ------------------------------------------------------------------ operator end
// Ap = p + sigma * z and pap = p . Ap (last block), skipped once CG is done.
__global__ __launch_bounds__(SSN_BLOCK) void k_mop_pap(const double* __restrict__ pd,
                                                       const double* __restrict__ z, double sigma,
                                                       double* __restrict__ Ap, int64_t q,
                                                       Scalars* sc, double* __restrict__ part,
                                                       unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    if (ld_grid(&sc->cg_done)) return;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
        const double a = fma(sigma, z[j], pd[j]);
        Ap[j] = a;
        s = fma(pd[j], a, s);
    }
    const double bs = block_sum(s, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
    if (last_block_arrives(counter)) {
        const double t = grid_colsum(part, gridDim.x, 1, 0, shd);
        if (threadIdx.x == 0) sc->cg_pap = t;
    }
}
void launch_mop_pap(const double* pd, const double* z, double sigma, double* Ap, int64_t q,
                    Scalars* sc, double* part, unsigned* counter, hipStream_t s) {
    int64_t b = (q + 2047) / 2048;
    if (b > 256) b = 256;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_mop_pap, dim3((unsigned)b), dim3(SSN_BLOCK), 0, s, pd, z, sigma, Ap, q, sc,
                       part, counter);
}

}  // namespace ssn
