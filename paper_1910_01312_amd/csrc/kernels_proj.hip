// Projection onto K ∩ L = {y^T x = 0, 0 <= x <= C} (Section 3.2.1) and the
// n-vector reductions around it (line-search increments, KKT residual,
// ordered compaction of the free set J).
//
// Pi(v) = clip(v - lam y, 0, C) with lam a zero of the nondecreasing
// piecewise-linear function g(lam) = -y^T clip(v - lam y, 0, C) (the
// gradient of phi in Section 3.2.1 with a = y, d = 0).  Writing
// b_i = y_i v_i - C [y_i > 0], every term is
//     -y_i clip(v_i - lam y_i, 0, C) = clip(lam - b_i, 0, C) - C [y_i > 0],
// so g has the 2n breakpoints b_i and b_i + C.  Instead of sorting them
// (Algorithm 2) the GPU brackets the root by multisection: each pass
// evaluates g at PK+1 points of the current bracket [lo, hi]
// (g(lo) < 0 <= g(hi)) in one sweep over the data, keeps the sub-interval
// where g changes sign, and counts (integer histogram) the breakpoints
// strictly inside every sub-interval.  When the kept one holds none, g is
// affine on it and the zero is found by the same linear interpolation that
// Algorithm 2 performs between its two final breakpoints; the result is the
// smallest zero of g, the value Algorithm 2 returns.  The points are equally
// spaced, except in the first pass of a projection that has a nearby
// multiplier (a line-search trial next to the accepted point): there they
// lie at hint -/+ C 4^e, e = -15..15, plus the two ends.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int PK = 64;            // sub-intervals per pass (one per lane of a wave)
constexpr int PNV = PK + 1;       // partial values per block: PK+1 g-values
static_assert(PK == SSN_WAVE, "the pass decision takes one candidate per lane");
constexpr int PROJ_MAXPASS = 48;
constexpr int PROJ_GRID_MAX = 256;
constexpr int PASS_CAP = 4096;    // LDS list of elements evaluated at every candidate

int proj_max_passes() { return PROJ_MAXPASS; }

static inline unsigned proj_grid(int64_t n) {
    int64_t b = (n + 1023) / 1024;
    if (b > PROJ_GRID_MAX) b = PROJ_GRID_MAX;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ------------------------------------------------------------------ init
// v = u - as * td (or v = u), then lo = min b_i, hi = max b_i + 2C so that
// g(lo) = -C n_+ and g(hi) = C n_- exactly.
template <bool HAS_TD>
__global__ __launch_bounds__(SSN_BLOCK) void k_proj_init(const double* __restrict__ u,
                                                         const double* __restrict__ td,
                                                         double as, double* __restrict__ vout,
                                                         const int8_t* __restrict__ y, int64_t n,
                                                         double C, double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    double bmin = 1.0 / 0.0, bmax = -1.0 / 0.0;
    long long npos = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double v = u[i];
        if (HAS_TD) {
            v = fma(-as, td[i], v);
            vout[i] = v;
        }
        const bool pos = y[i] > 0;
        const double b = pos ? v - C : -v;
        bmin = fmin(bmin, b);
        bmax = fmax(bmax, b);
        npos += pos ? 1 : 0;
    }
    // block reductions (min, max, count)
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    bmin = wave_min(bmin);
    if (lane == 0) shd[w] = bmin;
    __syncthreads();
    double r = shd[0];
    for (int k = 1; k < SSN_WAVES_PER_BLOCK; ++k) r = fmin(r, shd[k]);
    __syncthreads();
    bmax = wave_max(bmax);
    if (lane == 0) shd[w] = bmax;
    __syncthreads();
    double r2 = shd[0];
    for (int k = 1; k < SSN_WAVES_PER_BLOCK; ++k) r2 = fmax(r2, shd[k]);
    long long c = block_sum_ll(npos, shl);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = r;
        part[blockIdx.x * 3 + 1] = r2;
        part[blockIdx.x * 3 + 2] = (double)c;
    }
}

// Part 2 of the init (one block): combine the nb block partials.
__global__ __launch_bounds__(SSN_BLOCK) void k_proj_init_fin(int64_t n, double C, ProjState* st,
                                                             const double* __restrict__ part, int nb,
                                                             const ProjState* hint) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    {
        // min / max are order-independent; the count is an exact integer
        double mn = 1.0 / 0.0, mx = -1.0 / 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            mn = fmin(mn, ld_grid(&part[b * 3 + 0]));
            mx = fmax(mx, ld_grid(&part[b * 3 + 1]));
        }
        mn = wave_min(mn);
        mx = wave_max(mx);
        __syncthreads();
        if (lane == 0) { shd[w] = mn; }
        __syncthreads();
        for (int k = 0; k < SSN_WAVES_PER_BLOCK; ++k) mn = fmin(mn, shd[k]);
        __syncthreads();
        if (lane == 0) { shd[w] = mx; }
        __syncthreads();
        for (int k = 0; k < SSN_WAVES_PER_BLOCK; ++k) mx = fmax(mx, shd[k]);
        const double cnt = grid_colsum(part, nb, 3, 2, shd);
        if (threadIdx.x == 0) {
            st->lo = mn;
            st->hi = mx + 2.0 * C;
            st->npos = (long long)cnt;
            st->passes = 0;
            st->approx = 0;
            st->inside = -1;
            st->mode = hint ? 1 : 0;
            st->hint = hint ? hint->lam : 0.0;
            st->glo = -C * cnt;
            st->ghi = C * ((double)n - cnt);
            if (cnt == 0.0) {          // g <= 0 everywhere: the search's left end
                st->lam = mn;
                st->done = 1;
            } else {
                st->lam = 0.0;
                st->done = 0;
            }
        }
    }
}

void launch_proj_init(const double* u, const double* td, double alpha_sigma, double* v_out,
                      const int8_t* y, int64_t n, double C, ProjState* st, double* part,
                      unsigned* counter, hipStream_t s, const ProjState* hint) {
    (void)counter;
    const unsigned g = proj_grid(n);
    if (td)
        SSN_LAUNCH((k_proj_init<true>), dim3(g), dim3(SSN_BLOCK), 0, s, u, td, alpha_sigma,
                           v_out, y, n, C, part);
    else
        SSN_LAUNCH((k_proj_init<false>), dim3(g), dim3(SSN_BLOCK), 0, s, u, td, 0.0,
                           v_out, y, n, C, part);
    SSN_LAUNCH(k_proj_init_fin, dim3(1), dim3(SSN_BLOCK), 0, s, n, C, st, part, (int)g, hint);
}

// ------------------------------------------------------------------ pass
__device__ __forceinline__ double cand_uniform(double lo, double hi, int k) {
    return k == PK ? hi : lo + (hi - lo) * ((double)k / (double)PK);
}
// geometric points around the hint: k = 1..31 -> hint - C 4^(16-k),
// k = 32 -> hint, k = 33..63 -> hint + C 4^(k-48); clamped to [lo, hi]
__device__ __forceinline__ double cand_geometric(double lo, double hi, double hint, double C, int k) {
    if (k == 0) return lo;
    if (k == PK) return hi;
    double v;
    if (k < 32) v = hint - C * ldexp(1.0, 2 * (16 - k));
    else if (k == 32) v = hint;
    else v = hint + C * ldexp(1.0, 2 * (k - 48));
    return fmin(fmax(v, lo), hi);
}

constexpr int PU = 8;                     // elements per thread per sweep step
constexpr int PCOL = PNV + 1;             // double columns per block: g partials, lin_s
constexpr int PICOL = PK + 2;             // int columns: histogram, constant count, lin count

// The candidates of the pass (both kernels of a pass compute the same ones).
__device__ __forceinline__ void pass_candidates(const ProjState* st, double C, double* lam_s) {
    const double lo = st->lo, hi = st->hi;
    const bool geo = st->mode == 1;
    const double hint = st->hint;
    if (threadIdx.x <= PK)
        lam_s[threadIdx.x] = geo ? cand_geometric(lo, hi, hint, C, threadIdx.x)
                                 : cand_uniform(lo, hi, threadIdx.x);
}

// One multisection pass, part 1: every block sweeps its share of the data
// and writes its partial g-values, histogram and closed-form counts.
__global__ __launch_bounds__(SSN_BLOCK) void k_proj_pass(const double* __restrict__ v,
                                                         const int8_t* __restrict__ y, int64_t n,
                                                         double C, const ProjState* st,
                                                         double* __restrict__ part,
                                                         int* __restrict__ hpart) {
    __shared__ double lam_s[PK + 1];
    __shared__ double red[SSN_WAVES_PER_BLOCK][PCOL];
    __shared__ long long redl[SSN_WAVES_PER_BLOCK][2];
    __shared__ int hist[PK];
    __shared__ double list[PASS_CAP];
    __shared__ int wsum[PU][SSN_WAVES_PER_BLOCK];
    if (ld_grid(&st->done)) return;         // uniform over the grid
    pass_candidates(st, C, lam_s);
    if (threadIdx.x < PK) hist[threadIdx.x] = 0;
    __syncthreads();
    // Each element adds clip(lam - b, 0, C) - C [y > 0] to g(lam).  With both
    // breakpoints b, b + C outside (lam_s[0], lam_s[PK]) that term is, over
    // the whole bracket, the constant C (b + C <= lo), 0 (b >= hi) or
    // exactly (lam - lo) + (lo - b) (b <= lo, b + C >= hi): summed in closed
    // form (counts and the sum of lo - b, combined once by the decision).
    // Only elements with a breakpoint strictly inside the bracket are
    // evaluated at every candidate; they are gathered (element order) into an
    // LDS list so that whole blocks work on them together.
    const double blo = lam_s[0], bhi = lam_s[PK];
    double acc[PK];
    double acc_hi = 0.0;
#pragma unroll
    for (int k = 0; k < PK; ++k) acc[k] = 0.0;
    // the constant part is C times an integer count, kept exact so that g is
    // exactly 0 on a flat stretch (no component strictly inside the box)
    long long kc = 0, lin_n = 0;
    double lin_s = 0.0;
    const int64_t step = (int64_t)gridDim.x * SSN_BLOCK * PU;
    int64_t base = (int64_t)blockIdx.x * SSN_BLOCK * PU;
    int cnt = 0, maxcnt = 0;
    for (;;) {
        const bool more = base < n;                    // uniform over the block
        if (more) {
            double vv[PU];
            int yy[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {             // every load of the step first
                // (an index past n reads element n - 1, unused below: no load
                // sits under a branch, so all of them are in flight together)
                const int64_t i = base + u * SSN_BLOCK + threadIdx.x;
                const int64_t ic = i < n ? i : n - 1;
                vv[u] = v[ic];
                yy[u] = (int)y[ic];
            }
            bool take[PU];
            double bb[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int64_t i = base + u * SSN_BLOCK + threadIdx.x;
                take[u] = false;
                bb[u] = 0.0;
                if (i < n) {
                    const bool pos = yy[u] > 0;
                    const double b = pos ? vv[u] - C : -vv[u];
                    const double bh = b + C;
                    kc -= pos ? 1 : 0;
                    if (bh <= blo) kc += 1;
                    else if (b >= bhi) {}
                    else if (b <= blo && bh >= bhi) { lin_n += 1; lin_s += blo - b; }
                    else { take[u] = true; bb[u] = b; }
                }
            }
            cnt += block_append_multi<PU>(take, bb, list, cnt, wsum);
            base += step;
        }
        if (!more || cnt > PASS_CAP - PU * SSN_BLOCK) {
            __syncthreads();
            maxcnt = max(maxcnt, cnt);
            for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
                const double b = list[e];
                const double bh = b + C;
#pragma unroll
                for (int k = 0; k < PK; ++k) acc[k] += clampd(lam_s[k] - b, 0.0, C);
                acc_hi += clampd(bhi - b, 0.0, C);
                // histogram of breakpoints strictly inside each sub-interval
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double t = h ? bh : b;
                    if (t > blo && t < bhi) {
                        int lo_k = 0, hi_k = PK;           // lam_s[lo_k] < t < lam_s[hi_k]
                        while (hi_k - lo_k > 1) {
                            const int mid = (lo_k + hi_k) >> 1;
                            if (lam_s[mid] < t) lo_k = mid; else hi_k = mid;
                        }
                        if (t < lam_s[lo_k + 1]) atomicAdd(&hist[lo_k], 1);
                    }
                }
            }
            __syncthreads();
            cnt = 0;
            if (!more) break;
        }
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    // a wave whose threads evaluated no list entry holds zeros in acc
    double gk = 0.0, ghi = 0.0;
    if (maxcnt > w * SSN_WAVE) {
        gk = wave_reduce_scatter64(acc);
        ghi = wave_sum(acc_hi);
    }
    const double ls = wave_sum(lin_s);
    const long long kw = wave_sum_ll(kc), lw = wave_sum_ll(lin_n);
    red[w][lane] = gk;
    if (lane == 0) {
        red[w][PK] = ghi;
        red[w][PK + 1] = ls;
        redl[w][0] = kw;
        redl[w][1] = lw;
    }
    __syncthreads();
    const int nb = gridDim.x;                   // <= PROJ_GRID_MAX
    if (threadIdx.x < PCOL) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) s += red[ww][threadIdx.x];
        part[(int64_t)threadIdx.x * PROJ_GRID_MAX + blockIdx.x] = s;   // [column][block]
    }
    if (threadIdx.x < PK) hpart[(int64_t)threadIdx.x * PROJ_GRID_MAX + blockIdx.x] = hist[threadIdx.x];
    if (blockIdx.x == 0) {
        // zero the slots of the blocks nb .. (next multiple of 64) - 1, which
        // the decision reads without masks
        const int nbp = (int)gridDim.x, top = (nbp + SSN_WAVE - 1) / SSN_WAVE * SSN_WAVE;
        for (int e = threadIdx.x; e < (top - nbp) * PCOL; e += blockDim.x) {
            const int cc = e / (top - nbp), bb = nbp + e % (top - nbp);
            part[(int64_t)cc * PROJ_GRID_MAX + bb] = 0.0;
            if (cc < PICOL) hpart[(int64_t)cc * PROJ_GRID_MAX + bb] = 0;
        }
    }
    if (threadIdx.x == 0) {
        long long k2 = 0, l2 = 0;
#pragma unroll
        for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) { k2 += redl[ww][0]; l2 += redl[ww][1]; }
        hpart[(int64_t)PK * PROJ_GRID_MAX + blockIdx.x] = (int)k2;
        hpart[(int64_t)(PK + 1) * PROJ_GRID_MAX + blockIdx.x] = (int)l2;
    }
}

// One multisection pass, part 2 (one block): fixed-order reduction of the
// partials of the nb blocks of part 1, then the decision.  Column c is summed
// by wave c mod 4: lane l owns blocks l, l+64, l+128, l+192.  A separate
// launch instead of a last-arriving block: the kernel boundary makes the
// partials visible without a device-wide fence in every block.
constexpr int DEC_THREADS = 1024;
constexpr int DEC_WAVES = DEC_THREADS / SSN_WAVE;
__global__ __launch_bounds__(DEC_THREADS) void k_proj_decide(double C, ProjState* st,
                                                             const double* __restrict__ part,
                                                             const int* __restrict__ hpart, int nb) {
    __shared__ double lam_s[PK + 1];
    __shared__ double fin[PNV];
    __shared__ int hfin[PK];
    __shared__ long long kfin, linn_fin;
    __shared__ double lins_fin;
    __shared__ double lred[PCOL][SSN_WAVE];
    __shared__ int lhred[PICOL][SSN_WAVE];
    __shared__ int jsel;
    if (ld_grid(&st->done)) return;
    pass_candidates(st, C, lam_s);
    const double blo = st->lo;
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    {
        // lane l of wave w sums blocks l, l+64, ... (slots up to the next
        // multiple of 64 past nb hold zeros) of columns w, w+16, ...; the
        // per-lane sums go through LDS and thread c adds the 64 of column c in
        // lane order.  Every load of a wave is issued before any sum.
        constexpr int CPW = (PCOL + DEC_WAVES - 1) / DEC_WAVES;
        constexpr int BPL = PROJ_GRID_MAX / SSN_WAVE;
        static_assert(PICOL <= CPW * DEC_WAVES, "int columns per wave");
        const int jmax = (nb + SSN_WAVE - 1) / SSN_WAVE;
        double vals[CPW][BPL];
        int hv[CPW][BPL];
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int c = w + i * DEC_WAVES;
#pragma unroll
            for (int j = 0; j < BPL; ++j) {
                vals[i][j] = 0.0;
                hv[i][j] = 0;
                if (j < jmax) {                         // uniform over the wave
                    if (c < PCOL) vals[i][j] = ld_grid(&part[(int64_t)c * PROJ_GRID_MAX + lane + j * SSN_WAVE]);
                    if (c < PICOL) hv[i][j] = ld_grid(&hpart[(int64_t)c * PROJ_GRID_MAX + lane + j * SSN_WAVE]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int c = w + i * DEC_WAVES;
            double sum = 0.0;
            int hsum = 0;
#pragma unroll
            for (int j = 0; j < BPL; ++j) {
                sum += vals[i][j];
                hsum += hv[i][j];
            }
            if (c < PCOL) lred[c][lane] = sum;
            if (c < PICOL) lhred[c][lane] = hsum;
        }
        __syncthreads();
        const int c = threadIdx.x;
        if (c < PCOL) {
            double sum = 0.0;
#pragma unroll 16
            for (int l = 0; l < SSN_WAVE; ++l) sum += lred[c][l];
            if (c < PNV) fin[c] = sum;
            else lins_fin = sum;
        }
        if (c < PICOL) {
            long long hsum = 0;
#pragma unroll 16
            for (int l = 0; l < SSN_WAVE; ++l) hsum += lhred[c][l];
            if (c < PK) hfin[c] = (int)hsum;
            else if (c == PK) kfin = hsum;
            else linn_fin = hsum;
        }
    }
    __syncthreads();
    if (threadIdx.x <= PK)
        fin[threadIdx.x] += C * (double)kfin + (double)linn_fin * (lam_s[threadIdx.x] - blo) + lins_fin;
    __syncthreads();
    // kept sub-interval: the last k < PK with g(lam_k) < 0 (0 if none)
    if (threadIdx.x < SSN_WAVE) {
        const unsigned long long neg = __ballot(fin[threadIdx.x] < 0.0);
        if (threadIdx.x == 0) jsel = neg ? SSN_WAVE - 1 - __clzll((long long)neg) : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int passes = st->passes + 1;
        st->passes = passes;
        st->mode = 0;
        const int j = jsel;
        const double nlo = lam_s[j], nhi = lam_s[j + 1];
        const double g0 = fin[j], g1 = fin[j + 1];
        const int ins = hfin[j];
        st->inside = ins;
        st->lo = nlo;
        st->hi = nhi;
        st->glo = g0;
        st->ghi = g1;
        // done: no breakpoint inside the kept sub-interval, the interval can
        // no longer be split, or the pass cap
        const bool tiny = !(nlo < nhi) || !(nlo + (nhi - nlo) / (double)PK > nlo);
        if (ins == 0 || tiny || passes >= PROJ_MAXPASS) {
            double lam;
            if (g1 == 0.0) lam = nhi;
            else if (g1 > g0) lam = nlo + (-g0) / (g1 - g0) * (nhi - nlo);
            else lam = nlo;
            lam = fmin(fmax(lam, nlo), nhi);
            st->lam = lam;
            // inexact only when the pass cap stopped a splittable bracket that
            // still holds breakpoints
            st->approx = (ins != 0 && !tiny) ? 1 : 0;
            st->done = 1;                        // read by later launches only
        }
    }
}

void launch_proj_pass(const double* v, const int8_t* y, int64_t n, double C, ProjState* st,
                      double* part, unsigned* counter, hipStream_t s) {
    (void)counter;
    // doubles for the g-values, then ints for the histogram, in one scratch
    int* hpart = reinterpret_cast<int*>(part + (int64_t)PCOL * PROJ_GRID_MAX);
    const unsigned g = proj_grid(n);
    SSN_LAUNCH(k_proj_pass, dim3(g), dim3(SSN_BLOCK), 0, s, v, y, n, C, st, part, hpart);
    SSN_LAUNCH(k_proj_decide, dim3(1), dim3(DEC_THREADS), 0, s, C, st, part, hpart, (int)g);
}

// ------------------------------------------------------------------ apply
// x = clip(v - lam y, 0, C); mask = 1 on the strict interior (the set J of
// Proposition 5; a component exactly at a bound is active).  Counts p and
// the number of support vectors.
__global__ __launch_bounds__(SSN_BLOCK) void k_proj_apply(const double* __restrict__ v,
                                                          const int8_t* __restrict__ y, int64_t n,
                                                          double C, const ProjState* st,
                                                          double* __restrict__ x,
                                                          uint8_t* __restrict__ mask,
                                                          double* __restrict__ part) {
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam;
    long long p = 0, nsv = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double t = v[i] - lam * (double)y[i];
        const double xi = clampd(t, 0.0, C);
        const bool fr = (t > 0.0) && (t < C);
        x[i] = xi;
        if (mask) mask[i] = fr ? 1 : 0;
        p += fr ? 1 : 0;
        nsv += xi > 0.0 ? 1 : 0;
    }
    const long long bp = block_sum_ll(p, shl);
    const long long bs = block_sum_ll(nsv, shl);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2 + 0] = (double)bp;
        part[blockIdx.x * 2 + 1] = (double)bs;
    }
}

void launch_proj_apply(const double* v, const int8_t* y, int64_t n, double C, const ProjState* st,
                       double* x, uint8_t* mask, Scalars* sc, double* part, unsigned* counter,
                       hipStream_t s) {
    (void)counter;
    const unsigned g = proj_grid(n);
    SSN_LAUNCH(k_proj_apply, dim3(g), dim3(SSN_BLOCK), 0, s, v, y, n, C, st, x, mask, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->p;
    d.as_ll[0] = 1;
    d.p[1] = &sc->nsv;
    d.as_ll[1] = 1;
    launch_colsum_fin(part, (int)g, 2, 2, d, s);
}

// ------------------------------------------------------------------ line search
// phi(t) = int_0^t clip(s, 0, C) ds; increment phi(t + dt) - phi(t) with
// the closed form of the piece when both ends lie on the same piece, so a
// large t never cancels against itself.
__device__ __forceinline__ double huber_piece(double t, double C) {
    return t <= 0.0 ? 0.0 : (t < C ? 0.5 * t * t : C * (t - 0.5 * C));
}
__device__ __forceinline__ double huber_inc(double t, double dt, double C) {
    const double b = t + dt;
    if (t >= C && b >= C) return C * dt;
    if (t <= 0.0 && b <= 0.0) return 0.0;
    if (t > 0.0 && t < C && b > 0.0 && b < C) return dt * (t + 0.5 * dt);
    return huber_piece(b, C) - huber_piece(t, C);
}

// v = u_base - as * td (already written by the init kernel).  The increment
// of component i is dt_i = -as td_i - (lam - lam_base) y_i.
__global__ __launch_bounds__(SSN_BLOCK) void k_ls_finalize(
    const double* __restrict__ v, const double* __restrict__ u_base,
    const double* __restrict__ td, double as, const int8_t* __restrict__ y, int64_t n, double C,
    const ProjState* st, const ProjState* st_base, const double* __restrict__ xk,
    double* __restrict__ x, uint8_t* __restrict__ mask, double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam, lamb = st_base->lam, dl = lam - lamb;
    double dh = 0.0, d2 = 0.0;
    long long p = 0, nsv = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // LSU elements per thread per step, every load of the step issued first
    // (an index past n reads element n - 1, unused); the elements are taken
    // in the order of a plain strided loop
    constexpr int LSU = 4;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; base < n; base += LSU * stride) {
        double vv[LSU], yv[LSU], xkv[LSU], ubv[LSU], tdv[LSU];
#pragma unroll
        for (int u = 0; u < LSU; ++u) {
            const int64_t i = base + u * stride;
            const int64_t ic = i < n ? i : n - 1;
            vv[u] = v[ic];
            yv[u] = (double)y[ic];
            xkv[u] = xk[ic];
            ubv[u] = u_base[ic];
            tdv[u] = td ? td[ic] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LSU; ++u) {
            const int64_t i = base + u * stride;
            if (i >= n) break;
            const double yi = yv[u];
            const double t = vv[u] - lam * yi;
            const double xi = clampd(t, 0.0, C);
            const bool fr = (t > 0.0) && (t < C);
            x[i] = xi;
            mask[i] = fr ? 1 : 0;
            p += fr ? 1 : 0;
            nsv += xi > 0.0 ? 1 : 0;
            const double dx = xi - xkv[u];
            d2 = fma(dx, dx, d2);
            const double tb = ubv[u] - lamb * yi;
            const double dt = td ? fma(-as, tdv[u], -dl * yi) : -dl * yi;
            dh += huber_inc(tb, dt, C);
        }
    }
    const double bdh = block_sum(dh, shd);
    const double bd2 = block_sum(d2, shd);
    const long long bp = block_sum_ll(p, shl);
    const long long bs = block_sum_ll(nsv, shl);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = bdh;
        part[blockIdx.x * 4 + 1] = bd2;
        part[blockIdx.x * 4 + 2] = (double)bp;
        part[blockIdx.x * 4 + 3] = (double)bs;
    }
}

void launch_ls_finalize(const double* v, const double* u_base, const double* td, double as,
                        const int8_t* y, int64_t n, double C, const ProjState* st,
                        const ProjState* st_base, const double* xk, double* x, uint8_t* mask,
                        Scalars* sc, double* part, unsigned* counter, hipStream_t s) {
    (void)counter;
    const unsigned g = proj_grid(n);
    SSN_LAUNCH(k_ls_finalize, dim3(g), dim3(SSN_BLOCK), 0, s, v, u_base, td, as, y, n, C, st,
                       st_base, xk, x, mask, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->dh;
    d.p[1] = &sc->dist2;
    d.p[2] = &sc->p;
    d.as_ll[2] = 1;
    d.p[3] = &sc->nsv;
    d.as_ll[3] = 1;
    launch_colsum_fin(part, (int)g, 4, 4, d, s);
}

// ------------------------------------------------------------------ KKT
// v = x - Q x - c (eq. Def_Rkkt); c = -e when lin is null
__global__ void k_kkt_prepare(const double* __restrict__ x, const double* __restrict__ Qx,
                              const double* __restrict__ lin, double* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = x[i] - Qx[i] - (lin ? lin[i] : -1.0);
}
void launch_kkt_prepare(const double* x, const double* Qx, double* v, int64_t n, hipStream_t s,
                        const double* lin) {
    SSN_LAUNCH(k_kkt_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, Qx, lin, v,
                       n);
}

// |x - Pi(v)|^2, |x|^2, e^T x (c^T x with a linear term) and the loss sum
// of the primal at the bias given by lam:
//   C-SVC  sum_i max(0, 1 - Qx_i - y_i lam) = sum_i max(0, 1 - y_i (x~_i^T w + lam))
//          (Qx = A w, so Qx_i = y_i x~_i^T w; b = lam);
//   eps-SVR (svr_n = n / 2 rows of X, lin = c): with w = X^T (z - x) the primal
//          weights, Qx_i = -x~_i^T w for i < svr_n, and b = -lam,
//          sum_{i < svr_n} max(0, |y_i - x~_i^T w - b| - eps)
//          = sum max(0, |c_i - eps + Qx_i + lam| - eps).
__global__ __launch_bounds__(SSN_BLOCK) void k_kkt_finalize(const double* __restrict__ v,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ Qx,
                                                            const int8_t* __restrict__ y,
                                                            int64_t n, double C,
                                                            const ProjState* st,
                                                            const double* __restrict__ lin,
                                                            int64_t svr_n, double eps,
                                                            double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam;
    double r2 = 0.0, x2 = 0.0, sx = 0.0, hs = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i];
        const double yi = (double)y[i];
        const double pi = clampd(v[i] - lam * yi, 0.0, C);
        const double r = xi - pi;
        r2 = fma(r, r, r2);
        x2 = fma(xi, xi, x2);
        if (lin) {
            sx = fma(lin[i], xi, sx);
            if (i < svr_n) hs += fmax(0.0, fabs(lin[i] - eps + Qx[i] + lam) - eps);
        } else {
            sx += xi;
            hs += fmax(0.0, 1.0 - Qx[i] - lam * yi);
        }
    }
    const double a = block_sum(r2, shd);
    const double b = block_sum(x2, shd);
    const double c = block_sum(sx, shd);
    const double h = block_sum(hs, shd);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = a;
        part[blockIdx.x * 4 + 1] = b;
        part[blockIdx.x * 4 + 2] = c;
        part[blockIdx.x * 4 + 3] = h;
    }
}

void launch_kkt_finalize(const double* v, const double* x, const double* Qx, const int8_t* y,
                         int64_t n, double C, const ProjState* st, Scalars* sc, double* part,
                         unsigned* counter, hipStream_t s, const double* lin, int64_t svr_n,
                         double eps) {
    (void)counter;
    const unsigned g = proj_grid(n);
    SSN_LAUNCH(k_kkt_finalize, dim3(g), dim3(SSN_BLOCK), 0, s, v, x, Qx, y, n, C, st, lin, svr_n,
               eps, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->res2;
    d.p[1] = &sc->x2;
    d.p[2] = &sc->sumx;
    d.p[3] = &sc->hinge;
    launch_colsum_fin(part, (int)g, 4, 4, d, s);
}

// ------------------------------------------------------------------ compaction
// Ordered list of the indices with mask[i] != 0.  Block b owns the chunk
// [b*CH, (b+1)*CH); thread t the 16 consecutive elements starting at
// b*CH + 16 t.  Pass 1 counts per block and the last block turns the
// counts into offsets (exclusive scan in block order); pass 2 writes.
constexpr int CMP_EPT = 16;
constexpr int CMP_CH = SSN_BLOCK * CMP_EPT;

__global__ __launch_bounds__(SSN_BLOCK) void k_compact_count(const uint8_t* __restrict__ mask,
                                                             int64_t n, int* blk) {
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * CMP_CH + (int64_t)threadIdx.x * CMP_EPT;
    long long c = 0;
#pragma unroll
    for (int e = 0; e < CMP_EPT; ++e)
        if (base + e < n) c += mask[base + e] ? 1 : 0;
    const long long bc = block_sum_ll(c, shl);
    if (threadIdx.x == 0) blk[blockIdx.x] = (int)bc;
}
// Every block sums the counts of the blocks before it (its offset; exact
// integers) and writes its indices there in order; the last block also
// writes the total.
__global__ __launch_bounds__(SSN_BLOCK) void k_compact_write(const uint8_t* __restrict__ mask,
                                                             int64_t n, const int* __restrict__ blk,
                                                             int32_t* __restrict__ list,
                                                             long long* total) {
    __shared__ int sh[SSN_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    long long before = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += blockDim.x) before += blk[b];
    const long long off = block_sum_ll(before, shl);
    const int64_t base = (int64_t)blockIdx.x * CMP_CH + (int64_t)threadIdx.x * CMP_EPT;
    int c = 0;
#pragma unroll
    for (int e = 0; e < CMP_EPT; ++e)
        if (base + e < n) c += mask[base + e] ? 1 : 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    // inclusive scan over the block (Hillis-Steele, fixed and exact: integers)
    for (int o = 1; o < SSN_BLOCK; o <<= 1) {
        const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t pos = off + sh[threadIdx.x] - c;
#pragma unroll
    for (int e = 0; e < CMP_EPT; ++e)
        if (base + e < n && mask[base + e]) list[pos++] = (int32_t)(base + e);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SSN_BLOCK - 1) *total = off + sh[SSN_BLOCK - 1];
}
void launch_compact(const uint8_t* mask, int64_t n, int32_t* list, long long* count, int* blk,
                    unsigned* counter, hipStream_t s) {
    (void)counter;
    const unsigned nb = (unsigned)((n + CMP_CH - 1) / CMP_CH);
    SSN_LAUNCH(k_compact_count, dim3(nb), dim3(SSN_BLOCK), 0, s, mask, n, blk);
    SSN_LAUNCH(k_compact_write, dim3(nb), dim3(SSN_BLOCK), 0, s, mask, n, blk, list, count);
}

int compact_blocks(int64_t n) { return (int)((n + CMP_CH - 1) / CMP_CH); }

}  // namespace ssn
