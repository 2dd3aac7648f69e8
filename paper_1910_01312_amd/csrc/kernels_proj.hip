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
// evaluates g at PK+1 equally spaced points of the current bracket
// [lo, hi] (g(lo) < 0 <= g(hi)) in one sweep over the data, keeps the
// sub-interval where g changes sign, and counts the breakpoints strictly
// inside the current bracket.  When none is inside, g is affine on the
// bracket and the zero is found by the same linear interpolation that
// Algorithm 2 performs between its two final breakpoints; the result is the
// smallest zero of g, the value Algorithm 2 returns.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int PK = 32;            // sub-intervals per pass
constexpr int PNV = PK + 2;       // partial values per block: PK+1 g-values, 1 count
constexpr int PROJ_MAXPASS = 48;
constexpr int PROJ_GRID_MAX = 256;

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
                                                         double C, ProjState* st,
                                                         double* __restrict__ part,
                                                         unsigned* counter) {
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
    if (last_block_arrives(counter)) {
        if (threadIdx.x == 0) {
            double mn = 1.0 / 0.0, mx = -1.0 / 0.0, cnt = 0.0;
            for (unsigned b = 0; b < gridDim.x; ++b) {
                mn = fmin(mn, ld_acquire(&part[b * 3 + 0]));
                mx = fmax(mx, ld_acquire(&part[b * 3 + 1]));
                cnt += ld_acquire(&part[b * 3 + 2]);
            }
            st->lo = mn;
            st->hi = mx + 2.0 * C;
            st->npos = (long long)cnt;
            st->passes = 0;
            st->approx = 0;
            st->inside = -1;
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
                      unsigned* counter, hipStream_t s) {
    const unsigned g = proj_grid(n);
    if (td)
        hipLaunchKernelGGL((k_proj_init<true>), dim3(g), dim3(SSN_BLOCK), 0, s, u, td, alpha_sigma,
                           v_out, y, n, C, st, part, counter);
    else
        hipLaunchKernelGGL((k_proj_init<false>), dim3(g), dim3(SSN_BLOCK), 0, s, u, td, 0.0,
                           v_out, y, n, C, st, part, counter);
}

// ------------------------------------------------------------------ pass
__device__ __forceinline__ double cand(double lo, double hi, int k) {
    return k == PK ? hi : lo + (hi - lo) * ((double)k / (double)PK);
}

__global__ __launch_bounds__(SSN_BLOCK) void k_proj_pass(const double* __restrict__ v,
                                                         const int8_t* __restrict__ y, int64_t n,
                                                         double C, ProjState* st,
                                                         double* __restrict__ part,
                                                         unsigned* counter) {
    __shared__ double lam_s[PK + 1];
    __shared__ double red[SSN_WAVES_PER_BLOCK][PNV];
    __shared__ double fin[8][PNV];
    if (ld_acquire(&st->done)) return;         // uniform over the grid
    const double lo = st->lo, hi = st->hi;
    if (threadIdx.x <= PK) lam_s[threadIdx.x] = cand(lo, hi, threadIdx.x);
    __syncthreads();
    double acc[PK + 1];
#pragma unroll
    for (int k = 0; k <= PK; ++k) acc[k] = 0.0;
    double inside = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double vi = v[i];
        const bool pos = y[i] > 0;
        const double b = pos ? vi - C : -vi;
        const double bh = b + C;
        const double cp = pos ? C : 0.0;
#pragma unroll
        for (int k = 0; k <= PK; ++k) acc[k] += clampd(lam_s[k] - b, 0.0, C) - cp;
        inside += (b > lo && b < hi) ? 1.0 : 0.0;
        inside += (bh > lo && bh < hi) ? 1.0 : 0.0;
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
#pragma unroll
    for (int k = 0; k <= PK; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[w][k] = s;
    }
    {
        const double s = wave_sum(inside);
        if (lane == 0) red[w][PK + 1] = s;
    }
    __syncthreads();
    if (threadIdx.x < PNV) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) s += red[ww][threadIdx.x];
        part[(int64_t)blockIdx.x * PNV + threadIdx.x] = s;
    }
    if (!last_block_arrives(counter)) return;
    // ---- last block: fixed-order reduction over blocks, then the decision
    const int nb = gridDim.x;
    for (int e = threadIdx.x; e < 8 * PNV; e += blockDim.x) {
        const int c = e % PNV, gi = e / PNV;
        double s = 0.0;
        for (int b = gi; b < nb; b += 8) s += ld_acquire(&part[(int64_t)b * PNV + c]);
        fin[gi][c] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double G[PK + 1];
        for (int c = 0; c <= PK; ++c) {
            double s = 0.0;
            for (int gi = 0; gi < 8; ++gi) s += fin[gi][c];
            G[c] = s;
        }
        double ins = 0.0;
        for (int gi = 0; gi < 8; ++gi) ins += fin[gi][PK + 1];
        const int passes = st->passes + 1;
        st->passes = passes;
        st->inside = (int)ins;
        st->glo = G[0];
        st->ghi = G[PK];
        bool finish = (ins == 0.0) || passes >= PROJ_MAXPASS;
        int j = 0;
        if (!finish) {
            for (int k = 0; k < PK; ++k)
                if (G[k] < 0.0) j = k;
            const double nlo = cand(lo, hi, j), nhi = cand(lo, hi, j + 1);
            if (!(nlo > lo || nhi < hi)) {
                finish = true;         // bracket cannot be split further
            } else {
                st->lo = nlo;
                st->hi = nhi;
            }
        }
        if (finish) {
            double lam;
            const double g0 = G[0], g1 = G[PK];
            if (g1 == 0.0) lam = hi;
            else if (g1 > g0) lam = lo + (-g0) / (g1 - g0) * (hi - lo);
            else lam = lo;
            lam = fmin(fmax(lam, lo), hi);
            st->lam = lam;
            st->approx = (ins == 0.0) ? 0 : 1;
            __threadfence();
            atomicExch(&st->done, 1);
        }
    }
}

void launch_proj_pass(const double* v, const int8_t* y, int64_t n, double C, ProjState* st,
                      double* part, unsigned* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_proj_pass, dim3(proj_grid(n)), dim3(SSN_BLOCK), 0, s, v, y, n, C, st, part,
                       counter);
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
                                                          Scalars* sc, double* __restrict__ part,
                                                          unsigned* counter) {
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
    if (last_block_arrives(counter) && threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (unsigned k = 0; k < gridDim.x; ++k) {
            a += ld_acquire(&part[k * 2 + 0]);
            b += ld_acquire(&part[k * 2 + 1]);
        }
        sc->p = (long long)a;
        sc->nsv = (long long)b;
    }
}

void launch_proj_apply(const double* v, const int8_t* y, int64_t n, double C, const ProjState* st,
                       double* x, uint8_t* mask, Scalars* sc, double* part, unsigned* counter,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_proj_apply, dim3(proj_grid(n)), dim3(SSN_BLOCK), 0, s, v, y, n, C, st, x,
                       mask, sc, part, counter);
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
    double* __restrict__ x, uint8_t* __restrict__ mask, Scalars* sc, double* __restrict__ part,
    unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam, lamb = st_base->lam, dl = lam - lamb;
    double dh = 0.0, d2 = 0.0;
    long long p = 0, nsv = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double yi = (double)y[i];
        const double t = v[i] - lam * yi;
        const double xi = clampd(t, 0.0, C);
        const bool fr = (t > 0.0) && (t < C);
        x[i] = xi;
        mask[i] = fr ? 1 : 0;
        p += fr ? 1 : 0;
        nsv += xi > 0.0 ? 1 : 0;
        const double dx = xi - xk[i];
        d2 = fma(dx, dx, d2);
        const double tb = u_base[i] - lamb * yi;
        const double dt = td ? fma(-as, td[i], -dl * yi) : -dl * yi;
        dh += huber_inc(tb, dt, C);
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
    if (last_block_arrives(counter) && threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
        for (unsigned k = 0; k < gridDim.x; ++k) {
            a += ld_acquire(&part[k * 4 + 0]);
            b += ld_acquire(&part[k * 4 + 1]);
            c += ld_acquire(&part[k * 4 + 2]);
            d += ld_acquire(&part[k * 4 + 3]);
        }
        sc->dh = a;
        sc->dist2 = b;
        sc->p = (long long)c;
        sc->nsv = (long long)d;
    }
}

void launch_ls_finalize(const double* v, const double* u_base, const double* td, double as,
                        const int8_t* y, int64_t n, double C, const ProjState* st,
                        const ProjState* st_base, const double* xk, double* x, uint8_t* mask,
                        Scalars* sc, double* part, unsigned* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_ls_finalize, dim3(proj_grid(n)), dim3(SSN_BLOCK), 0, s, v, u_base, td, as,
                       y, n, C, st, st_base, xk, x, mask, sc, part, counter);
}

// ------------------------------------------------------------------ KKT
__global__ void k_kkt_prepare(const double* __restrict__ x, const double* __restrict__ Qx,
                              double* __restrict__ v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = x[i] - Qx[i] + 1.0;
}
void launch_kkt_prepare(const double* x, const double* Qx, double* v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_kkt_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, Qx, v,
                       n);
}

__global__ __launch_bounds__(SSN_BLOCK) void k_kkt_finalize(const double* __restrict__ v,
                                                            const double* __restrict__ x,
                                                            const int8_t* __restrict__ y,
                                                            int64_t n, double C,
                                                            const ProjState* st, Scalars* sc,
                                                            double* __restrict__ part,
                                                            unsigned* counter) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam;
    double r2 = 0.0, x2 = 0.0, sx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i];
        const double pi = clampd(v[i] - lam * (double)y[i], 0.0, C);
        const double r = xi - pi;
        r2 = fma(r, r, r2);
        x2 = fma(xi, xi, x2);
        sx += xi;
    }
    const double a = block_sum(r2, shd);
    const double b = block_sum(x2, shd);
    const double c = block_sum(sx, shd);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = a;
        part[blockIdx.x * 3 + 1] = b;
        part[blockIdx.x * 3 + 2] = c;
    }
    if (last_block_arrives(counter) && threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (unsigned k = 0; k < gridDim.x; ++k) {
            s0 += ld_acquire(&part[k * 3 + 0]);
            s1 += ld_acquire(&part[k * 3 + 1]);
            s2 += ld_acquire(&part[k * 3 + 2]);
        }
        sc->res2 = s0;
        sc->x2 = s1;
        sc->sumx = s2;
    }
}

void launch_kkt_finalize(const double* v, const double* x, const int8_t* y, int64_t n, double C,
                         const ProjState* st, Scalars* sc, double* part, unsigned* counter,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_kkt_finalize, dim3(proj_grid(n)), dim3(SSN_BLOCK), 0, s, v, x, y, n, C, st,
                       sc, part, counter);
}

// ------------------------------------------------------------------ compaction
// Ordered list of the indices with mask[i] != 0.  Block b owns the chunk
// [b*CH, (b+1)*CH); thread t the 16 consecutive elements starting at
// b*CH + 16 t.  Pass 1 counts per block and the last block turns the
// counts into offsets (exclusive scan in block order); pass 2 writes.
constexpr int CMP_EPT = 16;
constexpr int CMP_CH = SSN_BLOCK * CMP_EPT;

__global__ __launch_bounds__(SSN_BLOCK) void k_compact_count(const uint8_t* __restrict__ mask,
                                                             int64_t n, int* blk,
                                                             long long* total,
                                                             unsigned* counter) {
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * CMP_CH + (int64_t)threadIdx.x * CMP_EPT;
    long long c = 0;
#pragma unroll
    for (int e = 0; e < CMP_EPT; ++e)
        if (base + e < n) c += mask[base + e] ? 1 : 0;
    const long long bc = block_sum_ll(c, shl);
    if (threadIdx.x == 0) blk[blockIdx.x] = (int)bc;
    if (last_block_arrives(counter) && threadIdx.x == 0) {
        long long run = 0;
        for (unsigned b = 0; b < gridDim.x; ++b) {
            const int cb = ld_acquire(&blk[b]);
            blk[b] = (int)run;
            run += cb;
        }
        *total = run;
    }
}

__global__ __launch_bounds__(SSN_BLOCK) void k_compact_write(const uint8_t* __restrict__ mask,
                                                             int64_t n, const int* __restrict__ blk,
                                                             int32_t* __restrict__ list) {
    __shared__ int sh[SSN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * CMP_CH + (int64_t)threadIdx.x * CMP_EPT;
    int c = 0;
#pragma unroll
    for (int e = 0; e < CMP_EPT; ++e)
        if (base + e < n) c += mask[base + e] ? 1 : 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    // inclusive scan over the block (Hillis-Steele, fixed and exact: integers)
    for (int off = 1; off < SSN_BLOCK; off <<= 1) {
        const int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int pos = blk[blockIdx.x] + sh[threadIdx.x] - c;
#pragma unroll
    for (int e = 0; e < CMP_EPT; ++e)
        if (base + e < n && mask[base + e]) list[pos++] = (int32_t)(base + e);
}

void launch_compact(const uint8_t* mask, int64_t n, int32_t* list, long long* count, int* blk,
                    unsigned* counter, hipStream_t s) {
    const unsigned nb = (unsigned)((n + CMP_CH - 1) / CMP_CH);
    hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(SSN_BLOCK), 0, s, mask, n, blk, count,
                       counter);
    hipLaunchKernelGGL(k_compact_write, dim3(nb), dim3(SSN_BLOCK), 0, s, mask, n, blk, list);
}

int compact_blocks(int64_t n) { return (int)((n + CMP_CH - 1) / CMP_CH); }

}  // namespace ssn
