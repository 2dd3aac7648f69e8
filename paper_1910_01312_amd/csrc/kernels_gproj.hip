// Projection onto K ∩ L = {l <= x <= u, a^T x = d} for general a, l, u, d
// (Section 3.2.1, problem (P) of Section 1), and the n-vector reductions of
// the general problem's line search and KKT residual.
//
// Pi(v) = clip(v - lam a, l, u) with lam the smallest zero of the
// nondecreasing piecewise-linear g(lam) = -a^T clip(v - lam a, l, u) + d.
// For a_i != 0 the term -a_i clip(v_i - lam a_i, l_i, u_i) equals
// K_i + a_i^2 clip(lam - e_i, 0, f_i - e_i), with breakpoints e_i < f_i (the
// two values (v_i - u_i)/a_i, (v_i - l_i)/a_i in order) and K_i = -a_i times
// the bound held left of e_i (u_i if a_i > 0, else l_i); a_i = 0 adds
// nothing.  So g = sum K_i + d + sum a_i^2 clip(lam - e_i, 0, w_i).
//
// The root is bracketed by multisection: each pass evaluates g at 65 equally
// spaced points of the bracket [lo, hi] (g(lo) < 0 <= g(hi)) in one sweep
// and counts the breakpoints strictly inside every sub-interval; it keeps
// the sub-interval where g changes sign, and once that holds no breakpoint,
// g is affine on it and the zero is its linear interpolation (the value
// Algorithm 2 returns).  Unlike the C-SVC kernels (a = y, one box) every
// element is evaluated at every point; this path is not the hot one.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int GK = 64;                 // sub-intervals per pass
constexpr int GMAXPASS = 48;
constexpr int GGRID = 256;

static inline unsigned ggrid(int64_t n) {
    int64_t b = (n + 1023) / 1024;
    if (b > GGRID) b = GGRID;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// breakpoints e <= f, slope weight a^2 and left constant K of element i
__device__ __forceinline__ bool gterm(double v, double a, double l, double u, double& e, double& f,
                                      double& a2, double& K) {
    if (a == 0.0) return false;
    const double b1 = (v - u) / a, b2 = (v - l) / a;
    e = fmin(b1, b2);
    f = fmax(b1, b2);
    a2 = a * a;
    K = -a * (a > 0.0 ? u : l);
    return true;
}

// ---------------------------------------------------------------- init
// v = u0 - as td (written to vout) or v = u0; per-block partials of
// min e, max f, sum K, sum a^2 (f - e).
template <bool HAS_TD>
__global__ __launch_bounds__(SSN_BLOCK) void k_gproj_init(const double* __restrict__ u0,
                                                          const double* __restrict__ td, double as,
                                                          double* __restrict__ vout, GBox box,
                                                          int64_t n, double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    double mn = 1.0 / 0.0, mx = -1.0 / 0.0, sk = 0.0, sw = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double v = u0[i];
        if (HAS_TD) {
            v = fma(-as, td[i], v);
            vout[i] = v;
        }
        double e, f, a2, K;
        if (gterm(v, box.a[i], box.l[i], box.u[i], e, f, a2, K)) {
            mn = fmin(mn, e);
            mx = fmax(mx, f);
            sk += K;
            sw = fma(a2, f - e, sw);
        }
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    mn = wave_min(mn);
    if (lane == 0) shd[w] = mn;
    __syncthreads();
    double r0 = shd[0];
    for (int k = 1; k < SSN_WAVES_PER_BLOCK; ++k) r0 = fmin(r0, shd[k]);
    __syncthreads();
    mx = wave_max(mx);
    if (lane == 0) shd[w] = mx;
    __syncthreads();
    double r1 = shd[0];
    for (int k = 1; k < SSN_WAVES_PER_BLOCK; ++k) r1 = fmax(r1, shd[k]);
    __syncthreads();
    const double r2 = block_sum(sk, shd);
    const double r3 = block_sum(sw, shd);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = r0;
        part[blockIdx.x * 4 + 1] = r1;
        part[blockIdx.x * 4 + 2] = r2;
        part[blockIdx.x * 4 + 3] = r3;
    }
}

// One block: the bracket [min e, max f] with g(lo) = sum K + d and g(hi) =
// sum K + sum a^2 w + d; the ends settle the degenerate cases as Algorithm 2
// does (g(lo) >= 0: lo; g(hi) < 0: hi; no a_i != 0: 0).
__global__ __launch_bounds__(SSN_BLOCK) void k_gproj_init_fin(ProjState* st, const double* __restrict__ part,
                                                              int nb, double d) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    double mn = 1.0 / 0.0, mx = -1.0 / 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        mn = fmin(mn, part[b * 4 + 0]);
        mx = fmax(mx, part[b * 4 + 1]);
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    mn = wave_min(mn);
    if (lane == 0) shd[w] = mn;
    __syncthreads();
    for (int k = 0; k < SSN_WAVES_PER_BLOCK; ++k) mn = fmin(mn, shd[k]);
    __syncthreads();
    mx = wave_max(mx);
    if (lane == 0) shd[w] = mx;
    __syncthreads();
    for (int k = 0; k < SSN_WAVES_PER_BLOCK; ++k) mx = fmax(mx, shd[k]);
    __syncthreads();
    const double sk = grid_colsum(part, nb, 4, 2, shd);
    const double sw = grid_colsum(part, nb, 4, 3, shd);
    if (threadIdx.x == 0) {
        const double base = sk + d;
        st->gbase = base;
        st->lo = mn;
        st->hi = mx;
        st->glo = base;
        st->ghi = base + sw;
        st->passes = 0;
        st->approx = 0;
        st->inside = -1;
        st->mode = 0;
        st->hint = 0.0;
        st->npos = 0;
        if (!(mn <= mx)) {                 // every a_i = 0: g is the constant d
            st->lam = 0.0;
            st->done = 1;
        } else if (base >= 0.0) {
            st->lam = mn;
            st->done = 1;
        } else if (base + sw < 0.0) {
            st->lam = mx;
            st->done = 1;
        } else {
            st->lam = 0.0;
            st->done = 0;
        }
    }
}

// ---------------------------------------------------------------- pass
__device__ __forceinline__ double gcand(double lo, double hi, int k) {
    return k == GK ? hi : lo + (hi - lo) * ((double)k / (double)GK);
}

// Part 1: every block sweeps its share, partial sum_i a^2 clip(lam_k - e, 0, w)
// for the 65 points (part[k * GGRID + b]) and the count of breakpoints
// strictly inside each sub-interval (hpart[k * GGRID + b]).
__global__ __launch_bounds__(SSN_BLOCK) void k_gproj_pass(const double* __restrict__ v, GBox box,
                                                          int64_t n, const ProjState* st,
                                                          double* __restrict__ part,
                                                          int* __restrict__ hpart) {
    __shared__ double lam_s[GK + 1];
    __shared__ int hist[GK];
    __shared__ double red[SSN_WAVES_PER_BLOCK][GK + 1];
    if (st->done) return;                           // uniform over the grid
    const double lo = st->lo, hi = st->hi;
    if (threadIdx.x <= GK) lam_s[threadIdx.x] = gcand(lo, hi, threadIdx.x);
    if (threadIdx.x < GK) hist[threadIdx.x] = 0;
    __syncthreads();
    double acc[GK];
    double acc_hi = 0.0;
#pragma unroll
    for (int k = 0; k < GK; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double e, f, a2, K;
        if (!gterm(v[i], box.a[i], box.l[i], box.u[i], e, f, a2, K)) continue;
        const double w = f - e;
        if (f <= lo) {
            // at its upper plateau over the whole bracket
#pragma unroll
            for (int k = 0; k < GK; ++k) acc[k] = fma(a2, w, acc[k]);
            acc_hi = fma(a2, w, acc_hi);
            continue;
        }
        if (e >= hi) continue;                       // zero over the bracket
#pragma unroll
        for (int k = 0; k < GK; ++k) acc[k] = fma(a2, clampd(lam_s[k] - e, 0.0, w), acc[k]);
        acc_hi = fma(a2, clampd(hi - e, 0.0, w), acc_hi);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double t = h ? f : e;
            if (t > lo && t < hi) {
                int a0 = 0, b0 = GK;                 // lam_s[a0] < t < lam_s[b0]
                while (b0 - a0 > 1) {
                    const int mid = (a0 + b0) >> 1;
                    if (lam_s[mid] < t) a0 = mid; else b0 = mid;
                }
                if (t < lam_s[a0 + 1]) atomicAdd(&hist[a0], 1);
            }
        }
    }
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    const double gk = wave_reduce_scatter64(acc);
    const double gh = wave_sum(acc_hi);
    red[w][lane] = gk;
    if (lane == 0) red[w][GK] = gh;
    __syncthreads();
    if (threadIdx.x <= GK) {
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) s += red[ww][threadIdx.x];
        part[(int64_t)threadIdx.x * GGRID + blockIdx.x] = s;
    }
    if (threadIdx.x < GK) hpart[(int64_t)threadIdx.x * GGRID + blockIdx.x] = hist[threadIdx.x];
}

// Part 2 (one block): fixed-order sums of the block partials, then the
// decision: the last k < 64 with g(lam_k) < 0 keeps [lam_k, lam_k+1].
__global__ __launch_bounds__(SSN_BLOCK) void k_gproj_decide(ProjState* st, const double* __restrict__ part,
                                                            const int* __restrict__ hpart, int nb) {
    __shared__ double fin[GK + 1];
    __shared__ int hfin[GK];
    __shared__ int jsel;
    if (st->done) return;
    const double lo = st->lo, hi = st->hi, base = st->gbase;
    if (threadIdx.x <= GK) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(int64_t)threadIdx.x * GGRID + b];
        fin[threadIdx.x] = s + base;
    }
    if (threadIdx.x < GK) {
        int h = 0;
        for (int b = 0; b < nb; ++b) h += hpart[(int64_t)threadIdx.x * GGRID + b];
        hfin[threadIdx.x] = h;
    }
    __syncthreads();
    if (threadIdx.x < SSN_WAVE) {
        const unsigned long long neg = __ballot(fin[threadIdx.x] < 0.0);
        if (threadIdx.x == 0) jsel = neg ? SSN_WAVE - 1 - __clzll((long long)neg) : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int passes = st->passes + 1;
        st->passes = passes;
        const int j = jsel;
        const double nlo = gcand(lo, hi, j), nhi = gcand(lo, hi, j + 1);
        const double g0 = fin[j], g1 = fin[j + 1];
        const int ins = hfin[j];
        st->inside = ins;
        st->lo = nlo;
        st->hi = nhi;
        st->glo = g0;
        st->ghi = g1;
        const bool tiny = !(nlo < nhi) || !(nlo + (nhi - nlo) / (double)GK > nlo);
        if (ins == 0 || tiny || passes >= GMAXPASS) {
            double lam;
            if (g1 == 0.0) lam = nhi;
            else if (g1 > g0) lam = nlo + (-g0) / (g1 - g0) * (nhi - nlo);
            else lam = nlo;
            lam = fmin(fmax(lam, nlo), nhi);
            st->lam = lam;
            st->approx = (ins != 0 && !tiny) ? 1 : 0;
            st->done = 1;
        }
    }
}

// ---------------------------------------------------------------- n-vector steps
// x = clip(v - lam a, l, u), J mask (l < t < u strictly), and partials of
// |x - x^k|^2 (when xk), the psi increment sum_i h_i(t_b + dt) - h_i(t_b)
// with h(t) = t clip(t) - clip(t)^2 / 2, t_b = u_b - lam_b a,
// dt = -as td - (lam - lam_b) a (when u_base), |J| and #(x_i > l_i).
__device__ __forceinline__ double gh_piece(double t, double l, double u) {
    const double x = clampd(t, l, u);
    return t * x - 0.5 * x * x;
}
__device__ __forceinline__ double gh_inc(double t, double dt, double l, double u) {
    const double b = t + dt;
    if (t >= u && b >= u) return u * dt;
    if (t <= l && b <= l) return l * dt;
    if (t > l && t < u && b > l && b < u) return dt * (t + 0.5 * dt);
    return gh_piece(b, l, u) - gh_piece(t, l, u);
}
__global__ __launch_bounds__(SSN_BLOCK) void k_gfinalize(const double* __restrict__ v,
                                                         const double* __restrict__ u_base,
                                                         const double* __restrict__ td, double as,
                                                         GBox box, int64_t n, const ProjState* st,
                                                         const ProjState* st_base,
                                                         const double* __restrict__ xk,
                                                         double* __restrict__ x,
                                                         uint8_t* __restrict__ mask,
                                                         double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam;
    const double lamb = u_base ? st_base->lam : 0.0, dl = lam - lamb;
    double dh = 0.0, d2 = 0.0;
    long long p = 0, nsv = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ai = box.a[i], li = box.l[i], ui = box.u[i];
        const double t = v[i] - lam * ai;
        const double xi = clampd(t, li, ui);
        const bool fr = (t > li) && (t < ui);
        x[i] = xi;
        if (mask) mask[i] = fr ? 1 : 0;
        p += fr ? 1 : 0;
        nsv += xi > li ? 1 : 0;
        if (xk) {
            const double dx = xi - xk[i];
            d2 = fma(dx, dx, d2);
        }
        if (u_base) {
            const double tb = u_base[i] - lamb * ai;
            const double dt = td ? fma(-as, td[i], -dl * ai) : -dl * ai;
            dh += gh_inc(tb, dt, li, ui);
        }
    }
    const double bdh = block_sum(dh, shd);
    const double bd2 = block_sum(d2, shd);
    const long long bp = block_sum_ll(p, shl);
    const long long bs = block_sum_ll(nsv, shl);
    if (threadIdx.x == 0) {
        // the lam d term of 1/2 (|u|^2 - |u - Pi(u)|^2) = sum h_i(t_i) + lam d
        part[blockIdx.x * 4 + 0] = bdh + (blockIdx.x == 0 && u_base ? dl * box.d : 0.0);
        part[blockIdx.x * 4 + 1] = bd2;
        part[blockIdx.x * 4 + 2] = (double)bp;
        part[blockIdx.x * 4 + 3] = (double)bs;
    }
}

// R_KKT pieces of a general problem: |x - Pi(v)|^2, |x|^2, c^T x
__global__ __launch_bounds__(SSN_BLOCK) void k_gkkt_finalize(const double* __restrict__ v,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ c, GBox box,
                                                             int64_t n, const ProjState* st,
                                                             double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    const double lam = st->lam;
    double r2 = 0.0, x2 = 0.0, cx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i];
        const double pi = clampd(v[i] - lam * box.a[i], box.l[i], box.u[i]);
        const double r = xi - pi;
        r2 = fma(r, r, r2);
        x2 = fma(xi, xi, x2);
        cx = fma(c[i], xi, cx);
    }
    const double a = block_sum(r2, shd);
    const double b = block_sum(x2, shd);
    const double cc = block_sum(cx, shd);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = a;
        part[blockIdx.x * 4 + 1] = b;
        part[blockIdx.x * 4 + 2] = cc;
        part[blockIdx.x * 4 + 3] = 0.0;
    }
}

// coefficients of s = B_J^T a_J (zc_i = a_i [i in J]) and partials of a_J^T a_J
__global__ __launch_bounds__(SSN_BLOCK) void k_gcoef(const double* __restrict__ a,
                                                     const uint8_t* __restrict__ mask, int64_t n,
                                                     double* __restrict__ zc, double* __restrict__ part) {
    __shared__ double shd[SSN_WAVES_PER_BLOCK];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ai = mask[i] ? a[i] : 0.0;
        zc[i] = ai;
        s = fma(ai, ai, s);
    }
    const double b = block_sum(s, shd);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// partials of #(l_i < x_i < u_i) and #(x_i > l_i) of a returned x
__global__ __launch_bounds__(SSN_BLOCK) void k_gcount(const double* __restrict__ x, GBox box, int64_t n,
                                                      double* __restrict__ part) {
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    long long p = 0, ns = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i], li = box.l[i];
        p += (xi > li && xi < box.u[i]) ? 1 : 0;
        ns += xi > li ? 1 : 0;
    }
    const long long bp = block_sum_ll(p, shl), bn = block_sum_ll(ns, shl);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2] = (double)bp;
        part[blockIdx.x * 2 + 1] = (double)bn;
    }
}

// ---------------------------------------------------------------- launchers
void launch_gcount(const double* x, const GBox& box, int64_t n, Scalars* sc, double* part,
                   hipStream_t s) {
    const unsigned g = ggrid(n);
    SSN_LAUNCH(k_gcount, dim3(g), dim3(SSN_BLOCK), 0, s, x, box, n, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->p;
    d.as_ll[0] = 1;
    d.p[1] = &sc->nsv;
    d.as_ll[1] = 1;
    launch_colsum_fin(part, (int)g, 2, 2, d, s);
}

void launch_gproj_init(const double* u0, const double* td, double as, double* vout, const GBox& box,
                       int64_t n, ProjState* st, double* part, hipStream_t s) {
    const unsigned g = ggrid(n);
    if (td)
        SSN_LAUNCH((k_gproj_init<true>), dim3(g), dim3(SSN_BLOCK), 0, s, u0, td, as, vout, box, n, part);
    else
        SSN_LAUNCH((k_gproj_init<false>), dim3(g), dim3(SSN_BLOCK), 0, s, u0, td, as, vout, box, n, part);
    SSN_LAUNCH(k_gproj_init_fin, dim3(1), dim3(SSN_BLOCK), 0, s, st, part, (int)g, box.d);
}

void launch_gproj_pass(const double* v, const GBox& box, int64_t n, ProjState* st, double* part,
                       hipStream_t s) {
    const unsigned g = ggrid(n);
    int* hpart = reinterpret_cast<int*>(part + (int64_t)(GK + 1) * GGRID);
    SSN_LAUNCH(k_gproj_pass, dim3(g), dim3(SSN_BLOCK), 0, s, v, box, n, st, part, hpart);
    SSN_LAUNCH(k_gproj_decide, dim3(1), dim3(SSN_BLOCK), 0, s, st, part, hpart, (int)g);
}
int gproj_max_passes() { return GMAXPASS; }

void launch_gfinalize(const double* v, const double* u_base, const double* td, double as,
                      const GBox& box, int64_t n, const ProjState* st, const ProjState* st_base,
                      const double* xk, double* x, uint8_t* mask, Scalars* sc, double* part,
                      hipStream_t s) {
    const unsigned g = ggrid(n);
    SSN_LAUNCH(k_gfinalize, dim3(g), dim3(SSN_BLOCK), 0, s, v, u_base, td, as, box, n, st, st_base,
               xk, x, mask, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->dh;
    d.p[1] = &sc->dist2;
    d.p[2] = &sc->p;
    d.as_ll[2] = 1;
    d.p[3] = &sc->nsv;
    d.as_ll[3] = 1;
    launch_colsum_fin(part, (int)g, 4, 4, d, s);
}

void launch_gkkt_finalize(const double* v, const double* x, const double* c, const GBox& box,
                          int64_t n, const ProjState* st, Scalars* sc, double* part, hipStream_t s) {
    const unsigned g = ggrid(n);
    SSN_LAUNCH(k_gkkt_finalize, dim3(g), dim3(SSN_BLOCK), 0, s, v, x, c, box, n, st, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->res2;
    d.p[1] = &sc->x2;
    d.p[2] = &sc->cx;
    launch_colsum_fin(part, (int)g, 4, 3, d, s);
}

void launch_gcoef(const double* a, const uint8_t* mask, int64_t n, double* zc, Scalars* sc,
                  double* part, hipStream_t s) {
    const unsigned g = ggrid(n);
    SSN_LAUNCH(k_gcoef, dim3(g), dim3(SSN_BLOCK), 0, s, a, mask, n, zc, part);
    ColSumDst d = colsum_dst();
    d.p[0] = &sc->aja;
    launch_colsum_fin(part, (int)g, 1, 1, d, s);
}

}  // namespace ssn
