// Sparse products restricted to the free rows J (the rows that carry the
// second-order sparsity of Proposition 5), used by the matrix-free Newton
// operator M v = v + sigma X_J^T (I - 1 1^T / p) X_J v for CSR input.
//
//  * X_J v : one 16-lane group per row of the ordered J list (each row's
//            entries are contiguous in CSR), result as a p-vector.
//  * X_J^T z: a column-major copy of X_J, rebuilt once per Newton step by
//            filtering the full column-major copy (CSC) down to the entries
//            whose row is in J: per 512-entry tile of the full copy a count,
//            a scan of the counts, then the kept entries of tile t written
//            from offset t, in order, so the copy stays sorted by column.
//            Each kept entry stores (rank of its row in J, column, value);
//            the rank indexes the p-vector directly.  The product itself
//            (kernels_cg.hip) is a keyed segmented sum over 256-entry chunks
//            of the copy.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int JE = 8;                       // entries per lane, as the full plan
constexpr int JTILE = JE * SSN_WAVE;        // entries per full tile
constexpr int JBLOCK = 1024;                // filter blocks: 16 waves, one mask copy in LDS
constexpr int JWAVES = JBLOCK / SSN_WAVE;

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
    SSN_LAUNCH(k_rank_from_list, dim3((unsigned)b), dim3(256), 0, s, list, pdev, rank, rp,
                       jrow);
}

// ------------------------------------------------------------------ filter
// The J mask as bits (word w holds rows 32w .. 32w+31), so that the filter
// kernels keep it in LDS: every membership test is an LDS read instead of a
// scattered global byte load.
constexpr int JBITS_MAX_WORDS = 40960;         // 160 KiB of LDS: n <= 1310720 rows
int jcsc_bits_words(int64_t n) { return (int)((n + 31) / 32); }
bool jcsc_bits_fit(int64_t n) { return jcsc_bits_words(n) <= JBITS_MAX_WORDS; }

__global__ void k_mask_bits(const uint8_t* __restrict__ mask, int64_t n, uint32_t* __restrict__ bits) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w * 32 >= n) return;
    uint32_t b = 0;
    const int64_t r0 = w * 32;
    if (r0 + 32 <= n) {
        const uint4* p = reinterpret_cast<const uint4*>(mask + r0);   // 32-byte aligned: r0 % 32 == 0
        const uint4 u0 = p[0], u1 = p[1];
        const uint32_t v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) b |= ((v[i] >> (8 * j)) & 0xffu ? 1u : 0u) << (4 * i + j);
    } else {
        for (int64_t r = r0; r < n; ++r) b |= (mask[r] ? 1u : 0u) << (r - r0);
    }
    bits[w] = b;
}

// Stage the bit mask in LDS (dynamic, nw words) by the whole block, or (for
// masks beyond the LDS) read it from global memory, where it is L2-resident.
template <bool LDS>
__device__ __forceinline__ const uint32_t* stage_bits(const uint32_t* __restrict__ bits, int nw,
                                                      uint32_t* sb) {
    if (!LDS) return bits;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) sb[i] = bits[i];
    __syncthreads();
    return sb;
}
__device__ __forceinline__ bool in_j(const uint32_t* mb, int32_t r) {
    return (mb[r >> 5] >> (r & 31)) & 1u;
}
// row r >= 0 and in J, without a branch (r < 0 marks entries past the end)
__device__ __forceinline__ bool keep_row(const uint32_t* mb, int32_t r) {
    return (r >= 0) & in_j(mb, r < 0 ? 0 : r);
}
// Wait for every outstanding global load.  Issued once after a loop's first
// prefetch so that the loop header starts with no load in flight: the
// compiler's wait placement at a loop header otherwise assumes the worst for
// the prefetch registers and waits for the next prefetch as well.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Row indices of entries k0 + 64 e (e < JE) of one lane, -1 past nnz
// (nnz >= 1).  Every load is issued: an index past the end reads the last
// entry instead, so that no load sits under a branch and the compiler can
// count the loads in flight exactly.
__device__ __forceinline__ void load_rows(const int32_t* __restrict__ ridx, int64_t k0, int64_t nnz,
                                          int32_t (&row)[JE]) {
#pragma unroll
    for (int e = 0; e < JE; ++e) {
        const int64_t k = k0 + (int64_t)e * SSN_WAVE;
        const int32_t r = ridx[k < nnz ? k : nnz - 1];
        row[e] = k < nnz ? r : -1;
    }
}

// Per full tile: number of entries whose row is in J.  Persistent blocks,
// each with the mask in LDS; one wave per tile, lane l reading entries
// 64 e + l, the next tile's loads issued before this tile's tests.
template <bool LDS>
__global__ __launch_bounds__(JBLOCK) void k_jcsc_count(const int32_t* __restrict__ ridx,
                                                          int64_t nnz, int64_t ntile,
                                                          const uint32_t* __restrict__ bits, int nw,
                                                          int* __restrict__ tcount) {
    extern __shared__ uint32_t sbuf[];
    const uint32_t* sb = stage_bits<LDS>(bits, nw, sbuf);
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t nwave = (int64_t)gridDim.x * JWAVES;
    int64_t t = (int64_t)blockIdx.x * JWAVES + threadIdx.x / SSN_WAVE;
    if (t >= ntile) return;
    int32_t row[JE];
    load_rows(ridx, t * JTILE + lane, nnz, row);
    wait_loads();
    for (; t < ntile; t += nwave) {
        int32_t nxt[JE];
        load_rows(ridx, (t + nwave) * JTILE + lane, nnz, nxt);   // all -1 past the last tile
        int c = 0;
#pragma unroll
        for (int e = 0; e < JE; ++e) c += __popcll(__ballot(keep_row(sb, row[e])));
        if (lane == 0) tcount[t] = c;
#pragma unroll
        for (int e = 0; e < JE; ++e) row[e] = nxt[e];
    }
}

// Exclusive scan of tcount[0..ntile) into toff[0..ntile]: block b scans tiles
// [8192 b, 8192 b + 8192) after summing every count before them itself (so
// no block waits on another), with 1024 threads: a coalesced load into LDS,
// a sequential scan of 8 entries per thread, a wave scan and a scan of the
// 16 wave totals.  Integer sums: exact.  The last block writes toff[ntile]
// and *total.
constexpr int SCAN_CHUNK = 8192;
__global__ __launch_bounds__(1024) void k_scan_tiles(const int* __restrict__ tcount, int64_t ntile,
                                                     int* __restrict__ toff, long long* total) {
    __shared__ int buf[SCAN_CHUNK];
    __shared__ long long wtot[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
#pragma unroll
    for (int i = tid; i < SCAN_CHUNK; i += 1024) {
        const int64_t k = base + i;
        buf[i] = k < ntile ? tcount[k] : 0;
    }
    // the sum of every count before this chunk (base is a multiple of 4:
    // 16-byte loads of the 16-byte aligned count array)
    long long pre = 0;
    {
        const int4* q4 = reinterpret_cast<const int4*>(tcount);
        const int64_t n4 = base / 4;
        for (int64_t i = tid; i < n4; i += 1024) {
            const int4 v = q4[i];
            pre += (long long)v.x + v.y + v.z + v.w;
        }
        pre = wave_sum_ll(pre);
        if (lane == 0) wtot[wv] = pre;
        __syncthreads();
        pre = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) pre += wtot[k];
        __syncthreads();
    }
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
    long long wbefore = 0, ctot = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < wv) wbefore += wtot[k];
        ctot += wtot[k];
    }
    const long long excl = pre + wbefore + incl - s;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = base + tid * 8 + e;
        if (k < ntile) toff[k] = (int)(excl + loc[e]);
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        toff[ntile] = (int)(pre + ctot);
        *total = pre + ctot;
    }
}

// Write the kept entries of full tile t from toff[t] on, in the full copy's
// order (columns ascending).  Lane l of the wave takes entries
// 64 e + l of the tile, so the kept entries of one step e are consecutive in
// the output: a ballot gives each its place and every store of the step
// lands in one contiguous run.  Persistent blocks with the mask in LDS, as
// the count; tcv gives the (column, value) of every entry of the full copy.
template <typename V, typename CV, bool LDS>
__global__ __launch_bounds__(JBLOCK) void k_jcsc_write(
    const CV* __restrict__ tcv, const int32_t* __restrict__ ridx,
    int64_t nnz, int64_t ntile, const uint32_t* __restrict__ bits, int nw,
    const int32_t* __restrict__ rank,
    const int* __restrict__ toff, int32_t* __restrict__ jr, int32_t* __restrict__ jc,
    V* __restrict__ jv) {
    extern __shared__ uint32_t sbuf[];
    const uint32_t* sb = stage_bits<LDS>(bits, nw, sbuf);
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nwave = (int64_t)gridDim.x * JWAVES;
    const int64_t t0 = (int64_t)blockIdx.x * JWAVES + threadIdx.x / SSN_WAVE;
    int32_t cur[JE];
    load_rows(ridx, t0 * JTILE + lane, nnz, cur);
    wait_loads();
    for (int64_t t = t0; t < ntile; t += nwave) {
        const int64_t k0 = t * JTILE + lane;
        int32_t row[JE];
#pragma unroll
        for (int e = 0; e < JE; ++e) row[e] = cur[e];
        int pos = toff[t];
        bool keep[JE];
        int at[JE];
#pragma unroll
        for (int e = 0; e < JE; ++e) {
            keep[e] = keep_row(sb, row[e]);
            const unsigned long long m = __ballot(keep[e]);
            at[e] = pos + __popcll(m & below);
            pos += __popcll(m);
        }
        // every gather of the tile in flight before the first store
        int32_t rk[JE], cl[JE];
        V vv[JE];
#pragma unroll
        for (int e = 0; e < JE; ++e) {
            const int64_t k = k0 + (int64_t)e * SSN_WAVE;
            rk[e] = keep[e] ? rank[row[e]] : 0;
            const CV cv = keep[e] ? tcv[k] : CV{};
            cl[e] = cv.col;
            vv[e] = cv.v;
        }
        // the next tile's row indices, issued after this tile's gathers so
        // that the stores below wait for the gathers only
        load_rows(ridx, (t + nwave) * JTILE + lane, nnz, cur);
#pragma unroll
        for (int e = 0; e < JE; ++e) {
            if (keep[e]) {
                jr[at[e]] = rk[e];
                jc[at[e]] = cl[e];
                jv[at[e]] = vv[e];
            }
        }
    }
}

template <bool LDS>
static void jcsc_build_t(const SegPlan& T, const void* tcv, const uint32_t* bits, int nw,
                         const int32_t* rank,
                         int* tcount, int* toff, long long* total, int32_t* jr, int32_t* jc, void* jv,
                         hipStream_t s) {
    const size_t shm = LDS ? (size_t)nw * sizeof(uint32_t) : 0;
    static bool attr = false;
    if (LDS && !attr) {
        const int mx = JBITS_MAX_WORDS * (int)sizeof(uint32_t);
        (void)hipFuncSetAttribute((const void*)k_jcsc_count<LDS>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
        (void)hipFuncSetAttribute((const void*)k_jcsc_write<float, ColValF, LDS>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
        (void)hipFuncSetAttribute((const void*)k_jcsc_write<double, ColValD, LDS>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
        attr = true;
    }
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // each block stages the mask once: as many blocks as fit the CUs at once
    // (two per CU by waves, fewer when the mask fills the LDS)
    int per_cu = 2;
    if (LDS && shm > 0) per_cu = std::max(1, std::min(2, (int)((160 * 1024) / shm)));
    int64_t nb = (T.ntile + JWAVES - 1) / JWAVES;
    if (nb > (int64_t)per_cu * ncu) nb = (int64_t)per_cu * ncu;
    SSN_LAUNCH((k_jcsc_count<LDS>), dim3((unsigned)nb), dim3(JBLOCK), shm, s, T.idx, T.nnz,
                       T.ntile, bits, nw, tcount);
    SSN_LAUNCH(k_scan_tiles, dim3((unsigned)((T.ntile + SCAN_CHUNK - 1) / SCAN_CHUNK)), dim3(1024),
                       0, s, tcount, T.ntile, toff, total);
    if (T.val_f64)
        SSN_LAUNCH((k_jcsc_write<double, ColValD, LDS>), dim3((unsigned)nb), dim3(JBLOCK), shm, s,
                           (const ColValD*)tcv, T.idx, T.nnz, T.ntile, bits, nw, rank, toff,
                           jr, jc, (double*)jv);
    else
        SSN_LAUNCH((k_jcsc_write<float, ColValF, LDS>), dim3((unsigned)nb), dim3(JBLOCK), shm, s,
                           (const ColValF*)tcv, T.idx, T.nnz, T.ntile, bits, nw, rank, toff,
                           jr, jc, (float*)jv);
}

void launch_jcsc_build(const SegPlan& T, const void* tcv, const uint8_t* mask, int64_t n,
                       uint32_t* bits,
                       const int32_t* rank, int* tcount, int* toff, long long* total, int32_t* jr,
                       int32_t* jc, void* jv, hipStream_t s) {
    if (T.ntile == 0) return;
    const int nw = jcsc_bits_words(n);
    SSN_LAUNCH(k_mask_bits, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, mask, n, bits);
    if (jcsc_bits_fit(n))
        jcsc_build_t<true>(T, tcv, bits, nw, rank, tcount, toff, total, jr, jc, jv, s);
    else
        jcsc_build_t<false>(T, tcv, bits, nw, rank, tcount, toff, total, jr, jc, jv, s);
}

}  // namespace ssn
