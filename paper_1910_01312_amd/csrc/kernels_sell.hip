// Forward sparse product t = y .* (X v) (the A omega of eq. Def_psi and the
// A d of the line search) on a sliced-ELL copy of the CSR rows, fp32 values.
//
// Rows are sorted by decreasing length inside windows of SELL_WINDOW rows;
// each run of 64 sorted rows is a slice, stored column-major: entry k of the
// slice's row l sits at ptr[s] + 64 k + l as a (column, value) pair, padded
// with (0, 0) up to the slice's length (its longest row, rounded up to
// SELL_PAD).  perm[64 s + l] is the original index of that row (-1 past n).
// One lane per row: a wave streams its slice with 512-byte coalesced loads,
// gathers v, sums its row in fp64 in entry order and writes y_i times the sum
// to the row's own place.
//
// What bounds this product is the gather of v, one random column per lane
// and entry, through the vector memory path: with the gathers taken out the
// same stream of entries runs in about 60% of the time.  Columns are
// numbered by decreasing entry count, so the first few thousand carry most
// entries of a text-like matrix (the first 16384 of 10^5 Zipf(1.1) columns:
// 88%); each workgroup keeps v over those columns in LDS and gathers only the
// rest from global memory.  The copy is built only when its padding and its
// longest row stay small (5% padding on Poisson(60) rows).
#include "dev_common.h"
#include "ssn_internal.h"

#include <algorithm>

namespace ssn {

constexpr int SELL_U = 8;                 // entries per lane per group
constexpr int SELL_HEAD = 16384;          // columns copied to LDS (128 KB: one workgroup per CU)
constexpr int SELL_THREADS = 1024;        // 16 waves per workgroup
constexpr int SELL_WPB = SELL_THREADS / SSN_WAVE;
static_assert(SELL_SLICE == SSN_WAVE, "one lane per row of a slice");
static_assert(SELL_HEAD % SELL_THREADS == 0, "the head is copied in whole rounds");

// Persistent workgroups: each first copies v[0, H) (the most frequent
// columns, since columns are numbered by decreasing entry count) into LDS,
// then its waves take slices in turn.  A gather reads the LDS copy for a
// column below H and global memory otherwise; both reads are issued for
// every entry, the one not needed pointed at a fixed address, so no load
// sits under a per-lane branch and the global read of a frequent column is
// the same line for every lane.
__global__ __launch_bounds__(SELL_THREADS) void k_sell_amul(
    int64_t nslice, const int64_t* __restrict__ ptr, const int32_t* __restrict__ len,
    const ColValF* __restrict__ cv, const int32_t* __restrict__ perm,
    const double* __restrict__ v, int32_t H, const int8_t* __restrict__ y,
    double* __restrict__ out) {
    __shared__ double vh[SELL_HEAD];
    {
        constexpr int PER = SELL_HEAD / SELL_THREADS;
        double t[PER];                           // every load issued before any store
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = (int)threadIdx.x + i * SELL_THREADS;
            t[i] = v[j < H ? j : 0];
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = (int)threadIdx.x + i * SELL_THREADS;
            if (j < H) vh[j] = t[i];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t w0 = (int64_t)blockIdx.x * SELL_WPB + __builtin_amdgcn_readfirstlane(threadIdx.x / SSN_WAVE);
    const int64_t wstride = (int64_t)gridDim.x * SELL_WPB;
    for (int64_t s = w0; s < nslice; s += wstride) {
        const int64_t base = ptr[s];
        const int L = len[s];                     // a multiple of SELL_PAD
        const int32_t row = perm[s * SSN_WAVE + lane];
        // each (column, value) pair as one 64-bit word: column in the low half
        const uint64_t* p = reinterpret_cast<const uint64_t*>(cv + base) + lane;
        const int ngrp = (L + SELL_U - 1) / SELL_U;
        double acc = 0.0;
        for (int gi = 0; gi < ngrp; ++gi) {
            const int k = gi * SELL_U;
            uint64_t e[SELL_U];
#pragma unroll
            for (int u = 0; u < SELL_U; ++u) {
                const int kk = k + u < L ? k + u : L - 1;   // past the end: reload, value zeroed
                e[u] = p[(int64_t)kk * SSN_WAVE];
            }
            double gl[SELL_U], gg[SELL_U];
#pragma unroll
            for (int u = 0; u < SELL_U; ++u) {
                const int32_t c = (int32_t)(uint32_t)e[u];
                gl[u] = vh[c < H ? c : 0];
                gg[u] = v[c < H ? 0 : c];
            }
#pragma unroll
            for (int u = 0; u < SELL_U; ++u) {
                const int32_t c = (int32_t)(uint32_t)e[u];
                const float a = __uint_as_float((uint32_t)(e[u] >> 32));
                acc = fma(k + u < L ? (double)a : 0.0, c < H ? gl[u] : gg[u], acc);
            }
        }
        const int8_t yi = y[row >= 0 ? row : 0];
        if (row >= 0) out[row] = (double)yi * acc;
    }
}

int device_cu_count() {
    static int ncu_of[64];                       // per device, read once
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!ncu_of[dev]) {
        int n = 0;
        ncu_of[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0
                          ? n : 256;
    }
    return ncu_of[dev];
}

void launch_sell_amul(const SellPlan& P, const double* v, int64_t q, const int8_t* y, double* out,
                      hipStream_t s) {
    if (P.nslice == 0) return;
    const int ncu = device_cu_count();
    const int per_cu = (160 * 1024) / (int)(SELL_HEAD * sizeof(double) + 1024);
    const int64_t want = (P.nslice + SELL_WPB - 1) / SELL_WPB;
    const int64_t nb = std::min<int64_t>(want, (int64_t)ncu * std::max(per_cu, 1));
    const int32_t H = (int32_t)std::min<int64_t>(q, SELL_HEAD);
    SSN_LAUNCH(k_sell_amul, dim3((unsigned)nb), dim3(SELL_THREADS), 0, s, P.nslice, P.ptr, P.len, P.cv,
               P.perm, v, H, y, out);
}

}  // namespace ssn
