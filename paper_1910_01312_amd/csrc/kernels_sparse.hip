// Sparse products with A = diag(y) X for CSR X:
//   forward    t = y .* (X v)        segments = rows of the CSR arrays
//   transpose  r = X^T (y .* z)      segments = columns of a CSC copy
// Both are one "segmented sum" out[s] = sum_{k in seg s} val[k] coef(idx[k])
// executed nnz-balanced (merge-path style): lane chunk c owns the E entries
// [c E, (c+1) E), a wave owns 64 consecutive chunks (a tile).  A lane sums
// its entries segment by segment; segments that lie inside the lane are
// final and written at once.  The partial sums at lane borders are combined
// across the wave with a segmented scan, and segments that cross a tile
// border leave one partial per tile in a carry array that a second kernel
// adds in tile order.  No floating-point atomics: results are deterministic
// whatever the segment-length distribution (a column present in nearly
// every row is simply spread over many tiles).
//
// For the transpose of a large X the gathered vector (one double per row)
// outgrows one XCD's L2, and each gather that misses fetches a whole line
// from HBM.  The transpose then runs over a CSC copy cut into row blocks
// (segment = (row block, column)) whose tiles are dealt to the XCDs block by
// block, so every XCD gathers from its own slice of the vector only; the
// per-block column sums are added in block order afterwards.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int SEG_E = 8;                       // entries per lane
constexpr int SEG_TILE = SEG_E * SSN_WAVE;     // entries per wave tile

// ends[j] for a run-time j < SEG_E without indexing a register array (which
// would place it in scratch memory)
__device__ __forceinline__ int32_t pick8(const int32_t (&a)[8], int j) {
    int32_t r = a[0];
#pragma unroll
    for (int m = 1; m < 8; ++m) r = (j == m) ? a[m] : r;
    return r;
}

// eight consecutive values from a 32-byte aligned address, as 16-byte loads
__device__ __forceinline__ void load8(const float* p, double (&a)[8]) {
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 u = q[0], v = q[1];
    a[0] = u.x; a[1] = u.y; a[2] = u.z; a[3] = u.w;
    a[4] = v.x; a[5] = v.y; a[6] = v.z; a[7] = v.w;
}
__device__ __forceinline__ void load8(const double* p, double (&a)[8]) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 u0 = q[0], u1 = q[1], u2 = q[2], u3 = q[3];
    a[0] = u0.x; a[1] = u0.y; a[2] = u1.x; a[3] = u1.y;
    a[4] = u2.x; a[5] = u2.y; a[6] = u3.x; a[7] = u3.y;
}

template <typename V>
__device__ __forceinline__ double segval(const V* val, int64_t k, bool sq) {
    const double a = (double)val[k];
    return sq ? a * a : a;
}

// coef(i) = vin[i] * (yin ? yin[i] : 1) * (mask ? mask[i] : 1), or mask[i]
// alone when vin == nullptr.  CM names the case at compile time, so that the
// gathers carry no run-time tests and are all in flight together:
// 0 = vin alone, 1 = mask alone, 2 = any other combination.
template <typename V, int CM>
__global__ __launch_bounds__(SSN_BLOCK) void k_segsum(
    int64_t nseg, int64_t nnz, const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
    const V* __restrict__ val, const int32_t* __restrict__ lane_seg, int64_t ntile,
    const int32_t* __restrict__ tile_first, double* __restrict__ carry,
    const double* __restrict__ vin, const int8_t* __restrict__ yin,
    const uint8_t* __restrict__ mask, const int8_t* __restrict__ yout,
    const uint8_t* __restrict__ out_mask, double* __restrict__ out, int parts, int64_t tpp) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    int64_t tile;
    if (parts > 1) {
        // block b runs on XCD b % parts: part k of the tiles (tpp of them) goes
        // to the blocks of XCD k
        const int64_t lt = (int64_t)(blockIdx.x / parts) * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
        if (lt >= tpp) return;
        tile = (int64_t)(blockIdx.x % parts) * tpp + lt;
    } else {
        tile = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    }
    if (tile >= ntile) return;                    // whole wave leaves together
    const int64_t tb = tile * SEG_TILE;
    const int64_t te = tb + SEG_TILE < nnz ? tb + SEG_TILE : nnz;
    const int64_t k0 = tb + (int64_t)lane * SEG_E;
    const int64_t k1 = k0 + SEG_E < te ? k0 + SEG_E : te;
    const bool active = k0 < te;
    const int32_t INF = 0x7fffffff;

    const int32_t tfirst = tile_first[tile];
    int32_t F = INF, Lt = INF;
    int64_t aF = 0, bF = 0, aL = 0, bL = 0;      // entry ranges of segments F and Lt
    double fsum = 0.0, lsum = 0.0;
    if (active) {
        const int32_t seg0 = lane_seg[tile * SSN_WAVE + lane];
        const int ne = (int)(k1 - k0);
        // all loads of the lane first: entry indices and values (vector
        // loads for a full, aligned chunk), the next segment ends, then the
        // gathered coefficients
        int32_t ii[SEG_E];
        double av[SEG_E];
        if (ne == SEG_E) {
            const int4* ip = reinterpret_cast<const int4*>(idx + k0);
            const int4 i0 = ip[0], i1 = ip[1];
            ii[0] = i0.x; ii[1] = i0.y; ii[2] = i0.z; ii[3] = i0.w;
            ii[4] = i1.x; ii[5] = i1.y; ii[6] = i1.z; ii[7] = i1.w;
            load8(val + k0, av);
        } else {
#pragma unroll
            for (int e = 0; e < SEG_E; ++e) {
                ii[e] = e < ne ? idx[k0 + e] : 0;
                av[e] = e < ne ? (double)val[k0 + e] : 0.0;
            }
        }
        // where segment seg0 starts and the next SEG_E segment ends; every load
        // issued (index clamped to nseg), so none sits under a branch
        const int64_t p0 = ptr[seg0];
        int32_t ends[SEG_E];
#pragma unroll
        for (int j = 0; j < SEG_E; ++j) {
            const int64_t sj = (int64_t)seg0 + 1 + j;
            const int32_t v = ptr[sj <= nseg ? sj : nseg];
            ends[j] = sj <= nseg ? v : 0x7fffffff;
        }
        double cfv[SEG_E];
#pragma unroll
        for (int e = 0; e < SEG_E; ++e) {
            double cf = 0.0;
            if constexpr (CM == 0) {
                cf = vin[ii[e]];                 // ii = 0, av = 0 past the lane's entries
            } else if constexpr (CM == 1) {
                cf = (double)mask[ii[e]];
            } else if (e < ne) {
                const int32_t i = ii[e];
                if (vin) {
                    cf = vin[i];
                    if (yin) cf *= (double)yin[i];
                    if (mask) cf *= (double)mask[i];
                } else {
                    cf = (double)mask[i];
                }
            }
            cfv[e] = cf * av[e];
        }
        // walk the lane's entries segment by segment
        int j = 0;                             // current segment = seg0 + j
        int64_t segend = ends[0], segbeg = p0;
        F = seg0;
        double cur = 0.0;
        bool have_head = false;
#pragma unroll
        for (int e = 0; e < SEG_E; ++e) {
            if (e >= ne) break;
            const int64_t k = k0 + e;
            while (k >= segend) {                 // close segment seg0 + j
                const int32_t sg = seg0 + j;
                const bool omask = out_mask && !out_mask[sg];
                if (sg == F && !have_head) {
                    have_head = true;
                    fsum = cur;
                    if (p0 >= k0) {                // complete inside the lane
                        out[sg] = omask ? 0.0 : (yout ? (double)yout[sg] : 1.0) * cur;
                        F = INF - 1;               // head already emitted
                    }
                } else {
                    out[sg] = omask ? 0.0 : (yout ? (double)yout[sg] : 1.0) * cur;
                }
                ++j;
                segbeg = segend;
                segend = j < SEG_E ? pick8(ends, j) : ptr[seg0 + 1 + j];
                cur = 0.0;
            }
            cur += cfv[e];
        }
        Lt = seg0 + j;
        aL = segbeg;
        bL = segend;
        aF = p0;
        bF = ends[0];
        lsum = (out_mask && !out_mask[Lt]) ? 0.0 : cur;
        if (!have_head) {           // the lane stayed inside one segment: it is the tail
            F = Lt;
        } else if (F == INF - 1) {
            F = Lt;                 // no pending head
        }
        // now: F == Lt  -> no separate head; F < Lt -> head (F, fsum) pending
    }
    // ---- segmented inclusive scan of the tail sums keyed by Lt
    double S = lsum;
#pragma unroll
    for (int off = 1; off < SSN_WAVE; off <<= 1) {
        const double o = __shfl_up(S, off, SSN_WAVE);
        const int32_t ok = __shfl_up(Lt, off, SSN_WAVE);
        // all lanes in between share the key iff the lane `off` below does
        // (keys are nondecreasing along the wave)
        if (lane >= off && ok == Lt) S += o;
    }
    const double S_prev = __shfl_up(S, 1, SSN_WAVE);
    const int32_t Lt_prev = __shfl_up(Lt, 1, SSN_WAVE);
    const int32_t F_next = __shfl_down(F, 1, SSN_WAVE);
    const bool has_next = lane + 1 < SSN_WAVE && (k0 + SEG_E) < te;

    // segment s = [a, b): final when it lies inside the tile, else a carry
    auto emit = [&](int32_t s, int64_t a, int64_t b, double v) {
        if (a >= tb && b <= te) {
            double scale = yout ? (double)yout[s] : 1.0;
            if (out_mask && !out_mask[s]) scale = 0.0;
            out[s] = scale * v;
        } else {
            carry[tile * 2 + (s == tfirst ? 0 : 1)] = v;
        }
    };
    if (active) {
        if (F < Lt) {                    // pending head segment F (= the lane's first)
            double tot = fsum;
            if (lane > 0 && Lt_prev == F) tot += S_prev;
            emit(F, aF, bF, tot);
        }
        if (!has_next || F_next != Lt) emit(Lt, aL, bL, S);
    }
}

// out[s] for segments that cross tile borders (and empty segments, t0 > t1):
// sum of their per-tile partials in tile order.  In every tile after t0 the
// segment is the tile's first one (slot 0); only t0 needs the test.  The
// span list holds the short spans (at most SEG_SHORT tiles) first: one
// thread each, in the first blocks; then the long ones: one wave each.
constexpr int SEG_SHORT = 4;
__device__ __forceinline__ void segsum_put(int32_t s, double acc, const int8_t* yout,
                                           const uint8_t* out_mask, double* out) {
    double scale = yout ? (double)yout[s] : 1.0;
    if (out_mask && !out_mask[s]) scale = 0.0;
    out[s] = scale * acc;
}
__global__ __launch_bounds__(SSN_BLOCK) void k_segsum_fix(
    const int32_t* __restrict__ span_seg, const int32_t* __restrict__ span_t0,
    const int32_t* __restrict__ span_t1, int64_t nspan, int64_t nshort,
    const int32_t* __restrict__ tile_first, const double* __restrict__ carry,
    const int8_t* __restrict__ yout, const uint8_t* __restrict__ out_mask, double* __restrict__ out) {
    const int64_t nbs = (nshort + SSN_BLOCK - 1) / SSN_BLOCK;
    if ((int64_t)blockIdx.x < nbs) {
        const int64_t w = (int64_t)blockIdx.x * SSN_BLOCK + threadIdx.x;
        if (w >= nshort) return;
        const int32_t s = span_seg[w], t0 = span_t0[w], t1 = span_t1[w];
        double acc = 0.0;
        if (t0 <= t1) {
            acc = carry[(int64_t)t0 * 2 + ((s == tile_first[t0]) ? 0 : 1)];
#pragma unroll
            for (int d = 1; d < SEG_SHORT; ++d)
                if (t0 + d <= t1) acc += carry[(int64_t)(t0 + d) * 2];
        }
        segsum_put(s, acc, yout, out_mask, out);
        return;
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t w = nshort + ((int64_t)blockIdx.x - nbs) * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (w >= nspan) return;
    const int32_t s = span_seg[w], t0 = span_t0[w], t1 = span_t1[w];
    // four independent loads per lane per round
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (lane == 0) a0 = carry[(int64_t)t0 * 2 + ((s == tile_first[t0]) ? 0 : 1)];
    int64_t t = (int64_t)t0 + 1 + lane;
    for (; t + 3 * SSN_WAVE <= t1; t += 4 * SSN_WAVE) {
        a0 += carry[t * 2];
        a1 += carry[(t + SSN_WAVE) * 2];
        a2 += carry[(t + 2 * SSN_WAVE) * 2];
        a3 += carry[(t + 3 * SSN_WAVE) * 2];
    }
    for (; t <= t1; t += SSN_WAVE) a0 += carry[t * 2];
    const double acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) segsum_put(s, acc, yout, out_mask, out);
}
int seg_short_tiles() { return SEG_SHORT; }

static void segsum_launch(const SegPlan& P, const double* vin, const int8_t* yin,
                          const uint8_t* mask, const int8_t* yout, const uint8_t* out_mask,
                          double* out, hipStream_t s, int parts = 1) {
    int64_t tpp = 0, nb = (P.ntile + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK;
    if (parts > 1) {
        tpp = (P.ntile + parts - 1) / parts;
        nb = (int64_t)parts * ((tpp + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
    }
    if (nb > 0) {
        const int cm = (vin && !yin && !mask) ? 0 : ((!vin && mask) ? 1 : 2);
#define SEGSUM(V, CM) SSN_LAUNCH((k_segsum<V, CM>), dim3((unsigned)nb), dim3(SSN_BLOCK), 0, \
                                         s, P.nseg, P.nnz, P.ptr, P.idx, (const V*)P.val, P.lane_seg, \
                                         P.ntile, P.tile_first, P.carry, vin, yin, mask, yout, \
                                         out_mask, out, parts, tpp)
        if (P.val_f64) {
            if (cm == 0) SEGSUM(double, 0); else if (cm == 1) SEGSUM(double, 1); else SEGSUM(double, 2);
        } else {
            if (cm == 0) SEGSUM(float, 0); else if (cm == 1) SEGSUM(float, 1); else SEGSUM(float, 2);
        }
#undef SEGSUM
    }
    if (P.nspan > 0) {
        const int64_t nbs = (P.nshort + SSN_BLOCK - 1) / SSN_BLOCK;
        const int64_t nbl = (P.nspan - P.nshort + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK;
        SSN_LAUNCH(k_segsum_fix, dim3((unsigned)(nbs + nbl)), dim3(SSN_BLOCK), 0, s,
                           P.span_seg, P.span_t0, P.span_t1, P.nspan, P.nshort, P.tile_first,
                           P.carry, yout, out_mask, out);
    }
}

void launch_segsum(const SegPlan& P, const double* vin, const int8_t* yin, const uint8_t* mask,
                   const int8_t* yout, const uint8_t* out_mask, double* out, hipStream_t s) {
    segsum_launch(P, vin, yin, mask, yout, out_mask, out, s);
}

void launch_segsum_parts(const SegPlan& P, int parts, const double* vin, double* out,
                         hipStream_t s) {
    segsum_launch(P, vin, nullptr, nullptr, nullptr, nullptr, out, s, parts);
}

int seg_entries_per_lane() { return SEG_E; }

// Row blocks of the transpose: one per XCD of the MI355X (8) once the
// gathered vector (8 bytes per row) passes 1 MiB, a quarter of an XCD's L2;
// segment ids (block * q + column) must stay within int32.
int atmul_row_parts(int64_t n, int64_t q, int64_t nnz) {
    const int parts = 8;
    if (n < (1 << 17) || nnz < (int64_t)parts * SEG_TILE) return 1;
    if ((int64_t)parts * q + 1 > 0x7fffffffLL) return 1;
    return parts;
}


}  // namespace ssn
