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
// rank[list[k]] = k, and jrow[k] = (rp[list[k]], rp[list[k] + 1]): the entry
// range of the k-th row of J, so that X_J v reads it in one coalesced load.
__global__ void k_rank_from_list(const int32_t* __restrict__ list, const long long* __restrict__ pdev,
                                 int32_t* __restrict__ rank, const int32_t* __restrict__ rp,
                                 int2* __restrict__ jrow) {
    const long long p = *pdev;
    for (long long k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < p;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = list[k];
        rank[r] = (int32_t)k;
        jrow[k] = make_int2(rp[r], rp[r + 1]);
    }
}
void launch_rank_from_list(const int32_t* list, const long long* pdev, int64_t n, int32_t* rank,
                           const int32_t* rp, int2* jrow, hipStream_t s) {
    int64_t b = (n + 255) / 256;
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(k_rank_from_list, dim3((unsigned)b), dim3(256), 0, s, list, pdev, rank, rp,
                       jrow);
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

}  // namespace ssn
