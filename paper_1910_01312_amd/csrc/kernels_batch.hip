// Batched kernels: many independent C-SVC duals (dense, same q <= 128 and
// dtype, different n and C) advanced together, one launch per phase for all
// of them.
//
// Work decomposition.  The rows of problem k are cut into items of at most
// BRPI consecutive rows (a static list built once).  Before a phase, a
// one-block kernel compacts the items of the problems whose `active` flag is
// set into a work list and records, per problem, where its items start in it
// (ioff) and how many there are (icnt).  Row kernels are persistent: a grid of
// a tuned size strides over the work list.  Every per-problem sum is taken in
// two steps: one partial per item (fixed order inside the item), then a
// per-problem kernel adding that problem's item partials in item order.  No
// atomics on data, no cross-block fences; a problem's results depend only on
// its own data and on BRPI, not on the grid size or on the other problems.
//
// The per-problem arithmetic is that of the single-problem path: products
// with A = diag(y) X in fp64, the multisection projection onto
// {y^T x = 0, 0 <= x <= C} (Section 3.2.1), the line-search increments of
// psi, the ordered compaction of J, the Gram matrix X_J^T X_J, the centred
// Newton matrix I + sigma (X_J^T X_J - s s^T / p) with its Cholesky solve in
// LDS (Section 3.2.4), and the KKT residual of eq. Def_Rkkt.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int BPK = 64;            // multisection sub-intervals per pass
constexpr int BPNV = BPK + 1;      // g-values per pass
constexpr int BMAXPASS = 48;       // pass cap of one projection
constexpr int LPR = 16;            // lanes per row in the row products
constexpr int RPB = SSN_BLOCK / LPR;   // rows per block step (16)
constexpr int BSLOT = 8;           // columns per lane: 8 * 16 = 128 >= q
constexpr int GROWS = 512;         // J rows per Gram item (target)
constexpr int GMAXI = 32;          // Gram items per problem (cap)
constexpr int GST = 32;            // J rows staged in LDS per Gram step

int batch_rows_per_item() { return BRPI; }
int batch_qmax() { return BQMAX; }
int batch_gram_items_max(int64_t n) {
    const int64_t m = (n + GROWS - 1) / GROWS;
    return (int)(m < GMAXI ? m : GMAXI);
}
int batch_proj_max_passes() { return BMAXPASS; }

// ------------------------------------------------------------------ helpers
template <typename T>
struct BVec { static constexpr int V = 16 / (int)sizeof(T); };

// Column of slot s for lane j of a row group.  Vector layout: lane j loads V
// consecutive columns at g*16V + jV (g = s / V); scalar layout: j + 16 s.
template <typename T, bool VEC>
__device__ __forceinline__ int bcol(int s, int j) {
    constexpr int V = BVec<T>::V;
    return VEC ? (s / V) * (LPR * V) + j * V + (s % V) : j + LPR * s;
}

// The BSLOT elements of row xr that lane j owns (0 outside [0, q)).
template <typename T, bool VEC>
__device__ __forceinline__ void bload(const T* __restrict__ xr, int q, int j, double* e) {
    constexpr int V = BVec<T>::V;
    if (VEC) {
#pragma unroll
        for (int g = 0; g < BSLOT / V; ++g) {
            const int c = g * LPR * V + j * V;
            if (c < q) {
                VecLoad<T, V>::load(xr + c, e + g * V);
            } else {
#pragma unroll
                for (int t = 0; t < V; ++t) e[g * V + t] = 0.0;
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < BSLOT; ++s) {
            const int c = j + LPR * s;
            e[s] = c < q ? to_f64(xr[c]) : 0.0;
        }
    }
}

// sum_{i < n} p[i * stride] with 8 independent accumulators (loads in
// flight) combined in a fixed order: deterministic.
__device__ __forceinline__ double sum_items(const double* __restrict__ p, int64_t stride, int n) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 8 <= n; i += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += p[(int64_t)(i + u) * stride];
    }
    for (int u = 0; i < n; ++i, ++u) a[u] += p[(int64_t)i * stride];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}
__device__ __forceinline__ int isum_items(const int* __restrict__ p, int64_t stride, int n) {
    int a = 0, b = 0, c = 0, d = 0;
    int i = 0;
    for (; i + 4 <= n; i += 4) {
        a += p[(int64_t)i * stride];
        b += p[(int64_t)(i + 1) * stride];
        c += p[(int64_t)(i + 2) * stride];
        d += p[(int64_t)(i + 3) * stride];
    }
    for (; i < n; ++i) a += p[(int64_t)i * stride];
    return a + b + c + d;
}

// Sum over the 16 lanes of a row group (xor offsets stay inside the group).
__device__ __forceinline__ double group_sum(double v) {
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

// ------------------------------------------------------------------ work list
// One block: ioff / icnt per problem (icnt = 0 for inactive ones) in problem
// order and *wl_n = the length of the work list.
__global__ __launch_bounds__(1024) void kb_wl_scan(BArgs A) {
    __shared__ int sc[1024];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int k0 = 0; k0 < A.nprob; k0 += 1024) {
        const int k = k0 + threadIdx.x;
        const int c = (k < A.nprob && A.par[k].active) ? A.prob[k].nitem : 0;
        sc[threadIdx.x] = c;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
            __syncthreads();
            sc[threadIdx.x] += t;
            __syncthreads();
        }
        if (k < A.nprob) {
            A.ioff[k] = base + sc[threadIdx.x] - c;
            A.icnt[k] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) base += sc[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *A.wl_n = base;
}
// One block per problem: copy its items into the work list.
__global__ __launch_bounds__(256) void kb_wl_copy(BArgs A, const int4* __restrict__ items) {
    const int k = blockIdx.x;
    const int ck = A.icnt[k];
    if (ck == 0) return;
    const int ok = A.ioff[k], i0 = A.prob[k].item0;
    for (int i = threadIdx.x; i < ck; i += blockDim.x) A.wl[ok + i] = items[i0 + i];
}

// ------------------------------------------------------------------ A v
// t[off + r] = y_r X_k[r] . v_k for the rows of the active problems.
template <typename T, bool VEC, int UNR>
__global__ __launch_bounds__(SSN_BLOCK) void kb_amul(BArgs A, const double* __restrict__ V,
                                                     double* __restrict__ t) {
    __shared__ double vs[BQMAX];
    const int nw = *A.wl_n, q = A.q;
    const int j = threadIdx.x & (LPR - 1), grp = threadIdx.x / LPR;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int k = item.x;
        const BProb P = A.prob[k];
        __syncthreads();
        for (int c = threadIdx.x; c < q; c += blockDim.x) vs[c] = V[(int64_t)k * q + c];
        __syncthreads();
        const T* X = (const T*)P.X;
        for (int r = item.y + grp; r < item.z; r += RPB * UNR) {
            double e[UNR][BSLOT];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int rr = min(r + u * RPB, item.z - 1);
                bload<T, VEC>(X + (int64_t)rr * q, q, j, e[u]);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                double acc = 0.0;
#pragma unroll
                for (int s = 0; s < BSLOT; ++s) {
                    const int c = bcol<T, VEC>(s, j);
                    acc = fma(e[u][s], c < q ? vs[c] : 0.0, acc);
                }
                acc = group_sum(acc);
                const int rr = r + u * RPB;
                if (j == 0 && rr < item.z) t[P.off + rr] = (double)P.y[rr] * acc;
            }
        }
    }
}

// Rows of 16-byte-aligned data: P lanes (a power of two) cover a row in
// 16-byte pieces, G = 64 / P rows per load; a wave keeps R loads (R G rows)
// in flight as raw pieces, the lane's slice of v_k in registers.  Within each
// P-lane group a reduce-scatter over the R row sums (log2 R steps) and xor
// sums over the remaining lanes leave row u's total in the group's lanes
// whose position is a multiple of P / R.
template <typename T, int P, int R>
__global__ __launch_bounds__(SSN_BLOCK) void kb_amul2(BArgs A, const double* __restrict__ V,
                                                      double* __restrict__ t) {
    static_assert(R <= P && (P & (P - 1)) == 0 && (R & (R - 1)) == 0, "P, R: powers of two, R <= P");
    constexpr int VE = BVec<T>::V;
    constexpr int G = SSN_WAVE / P;
    const int nw = *A.wl_n, q = A.q;
    const int lane = threadIdx.x & (SSN_WAVE - 1), wv = threadIdx.x / SSN_WAVE;
    const int pl = lane & (P - 1), g = lane / P;
    const int c0 = pl * VE;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int k = item.x;
        const BProb Pr = A.prob[k];
        double vloc[VE];
#pragma unroll
        for (int e = 0; e < VE; ++e) vloc[e] = c0 + e < q ? V[(int64_t)k * q + c0 + e] : 0.0;
        const T* X = (const T*)Pr.X;
        // every load issued: a row past the item reads the item's last row and a
        // piece past the row end (P rounded up to a power of two) reads the last
        // piece; both products are dropped (vloc is 0 there, the store is
        // skipped).  q is a multiple of VE here, so a piece never straddles it.
        const int cc = c0 < q ? c0 : q - VE;
        for (int r0 = item.y + wv * R * G; r0 < item.z; r0 += SSN_WAVES_PER_BLOCK * R * G) {
            RawPiece<T, VE> raw[R];
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int row = r0 + u * G + g;
                const int rc = row < item.z ? row : item.z - 1;
                raw[u].u = *reinterpret_cast<const uint4*>(X + (int64_t)rc * q + cc);
            }
            double acc[R];
#pragma unroll
            for (int u = 0; u < R; ++u) {
                double a = 0.0;
#pragma unroll
                for (int e = 0; e < VE; ++e) a = fma(raw[u].get(e), vloc[e], a);
                acc[u] = a;
            }
#pragma unroll
            for (int h = P / 2, live = R; live > 1; h >>= 1, live >>= 1) {
                const bool up = (pl & h) != 0;
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
            for (int h = P / (2 * R); h >= 1; h >>= 1) sum += __shfl_xor(sum, h, SSN_WAVE);
            if ((pl & (P / R - 1)) == 0) {
                int u = 0;
#pragma unroll
                for (int b = 0; (1 << b) < R; ++b)
                    if (pl & (P >> (b + 1))) u |= R >> (b + 1);
                const int row = r0 + u * G + g;
                if (row < item.z) t[Pr.off + row] = (double)Pr.y[row] * sum;
            }
        }
    }
}

// ------------------------------------------------------------------ A^T z
// part[it*q + c] = sum over the item's rows of y_r z_r X_rc; part2 likewise
// with the 0/1 mask (X_J^T 1).  Rows with zero coefficients are skipped.
template <typename T, bool VEC, bool MASK>
__global__ __launch_bounds__(SSN_BLOCK) void kb_atmul(BArgs A, const double* __restrict__ z,
                                                      const uint8_t* __restrict__ mask,
                                                      double* __restrict__ part,
                                                      double* __restrict__ part2) {
    __shared__ double red[RPB][BQMAX];
    __shared__ double red2[MASK ? RPB : 1][BQMAX];
    const int nw = *A.wl_n, q = A.q;
    const int j = threadIdx.x & (LPR - 1), grp = threadIdx.x / LPR;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const BProb P = A.prob[item.x];
        const T* X = (const T*)P.X;
        double acc[BSLOT], accm[BSLOT];
#pragma unroll
        for (int s = 0; s < BSLOT; ++s) acc[s] = accm[s] = 0.0;
        if constexpr (VEC) {
            // RU rows per group at a time: their coefficients first (a row past
            // the item reads the item's last row and gets coefficient 0), then
            // the raw 16-byte pieces of every row with a nonzero coefficient,
            // widened at the FMA, so that all of a step's loads are in flight
            constexpr int V = BVec<T>::V, NP = BSLOT / V, RU = 4;
            for (int r0 = item.y + grp; r0 < item.z; r0 += RPB * RU) {
                double cf[RU], cm[RU];
                int rc[RU];
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int r = r0 + u * RPB;
                    const bool in = r < item.z;
                    rc[u] = in ? r : item.z - 1;
                    const int64_t gi = P.off + rc[u];
                    const double a = (double)P.y[rc[u]] * z[gi];
                    const double b = MASK ? (double)mask[gi] : 0.0;
                    cf[u] = in ? a : 0.0;
                    cm[u] = in ? b : 0.0;
                }
                // a row with coefficient 0 reads the item's first row instead (a
                // cache hit, dropped at the FMA), a piece past q the last piece:
                // the loads carry no branch
                RawPiece<T, V> pc[RU][NP];
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int rl = (cf[u] != 0.0 || cm[u] != 0.0) ? rc[u] : item.y;
#pragma unroll
                    for (int g = 0; g < NP; ++g) {
                        const int c = g * LPR * V + j * V;
                        pc[u][g].u = *reinterpret_cast<const uint4*>(X + (int64_t)rl * q + (c < q ? c : q - V));
                    }
                }
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int g = 0; g < NP; ++g)
#pragma unroll
                        for (int t = 0; t < V; ++t) {
                            const double xv = g * LPR * V + j * V < q ? pc[u][g].get(t) : 0.0;
                            acc[g * V + t] = fma(cf[u], xv, acc[g * V + t]);
                            if (MASK) accm[g * V + t] = fma(cm[u], xv, accm[g * V + t]);
                        }
            }
        } else {
            for (int r = item.y + grp; r < item.z; r += RPB) {
                const int64_t gi = P.off + r;
                const double cf = (double)P.y[r] * z[gi];
                const double cm = MASK ? (double)mask[gi] : 0.0;
                if (cf == 0.0 && cm == 0.0) continue;
                double e[BSLOT];
                bload<T, VEC>(X + (int64_t)r * q, q, j, e);
#pragma unroll
                for (int s = 0; s < BSLOT; ++s) {
                    acc[s] = fma(cf, e[s], acc[s]);
                    if (MASK) accm[s] = fma(cm, e[s], accm[s]);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < BSLOT; ++s) {
            const int c = bcol<T, VEC>(s, j);
            if (c < q) {
                red[grp][c] = acc[s];
                if (MASK) red2[grp][c] = accm[s];
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < q; c += blockDim.x) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int g = 0; g < RPB; ++g) {
                a += red[g][c];
                if (MASK) b += red2[g][c];
            }
            part[(int64_t)it * q + c] = a;
            if (MASK) part2[(int64_t)it * q + c] = b;
        }
    }
}

// out_k = (base ? base_k : 0) + sign * sum of problem k's item partials
// (item order); out2_k likewise from part2 without a base.  One block per
// problem.
__global__ __launch_bounds__(128) void kb_atmul_fin(BArgs A, const double* __restrict__ part,
                                                    const double* __restrict__ part2,
                                                    const double* __restrict__ base, double sign,
                                                    double* __restrict__ out,
                                                    double* __restrict__ out2) {
    const int k = blockIdx.x;
    if (!A.par[k].active) return;
    const int q = A.q, i0 = A.ioff[k], ni = A.icnt[k];
    for (int c = threadIdx.x; c < q; c += blockDim.x) {
        const double s = sum_items(part + (int64_t)i0 * q + c, q, ni);
        const double sm = part2 ? sum_items(part2 + (int64_t)i0 * q + c, q, ni) : 0.0;
        const int64_t o = (int64_t)k * q + c;
        out[o] = (base ? base[o] : 0.0) + sign * s;
        if (out2) out2[o] = sm;
    }
}

// ------------------------------------------------------------------ elementwise
// mode 0: o = a + sigma_k (1 - b)      (u = x^k + sigma (e - A omega))
// mode 1: o = a - b + 1                 (v = x - Qx + e, KKT)
// mode 2: o = a (copy)
__global__ __launch_bounds__(SSN_BLOCK) void kb_elem(BArgs A, int mode,
                                                     const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ o) {
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int64_t off = A.prob[item.x].off;
        const double sg = A.par[item.x].sigma;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) {
            const int64_t i = off + r;
            if (mode == 0) o[i] = fma(sg, 1.0 - b[i], a[i]);
            else if (mode == 1) o[i] = a[i] - b[i] + 1.0;
            else o[i] = a[i];
        }
    }
}

// accept of a line-search step on the n-side: aw += alpha td, u = ut,
// xt = xtt, jm = jmt
__global__ __launch_bounds__(SSN_BLOCK) void kb_accept_n(BArgs A, double* __restrict__ aw,
                                                         const double* __restrict__ td,
                                                         double* __restrict__ u,
                                                         const double* __restrict__ ut,
                                                         double* __restrict__ xt,
                                                         const double* __restrict__ xtt,
                                                         uint8_t* __restrict__ jm,
                                                         const uint8_t* __restrict__ jmt) {
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int64_t off = A.prob[item.x].off;
        const double al = A.par[item.x].alpha;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) {
            const int64_t i = off + r;
            aw[i] = fma(al, td[i], aw[i]);
            u[i] = ut[i];
            xt[i] = xtt[i];
            jm[i] = jmt[i];
        }
    }
}

// q-side per problem (one block each):
// mode 0: o = a + alpha_k b;  mode 1: o = a - b;  mode 2: o = 0;  mode 3: o = a
// mode 0 also copies the trial projection state into the base one.
__global__ __launch_bounds__(128) void kb_qvec(BArgs A, int mode, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ o) {
    const int k = blockIdx.x;
    if (!A.par[k].active) return;
    const double al = A.par[k].alpha;
    for (int c = threadIdx.x; c < A.q; c += blockDim.x) {
        const int64_t i = (int64_t)k * A.q + c;
        if (mode == 0) o[i] = fma(al, b[i], a[i]);
        else if (mode == 1) o[i] = a[i] - b[i];
        else if (mode == 2) o[i] = 0.0;
        else o[i] = a[i];
    }
    if (mode == 0 && threadIdx.x == 0) A.bs[k].ps[0] = A.bs[k].ps[1];
}

// per-problem dots of q-vectors into bs[k].r[f0 + t], t < npair
__global__ __launch_bounds__(128) void kb_qdots(BArgs A, int npair, const double* __restrict__ a0,
                                                const double* __restrict__ b0,
                                                const double* __restrict__ a1,
                                                const double* __restrict__ b1,
                                                const double* __restrict__ a2,
                                                const double* __restrict__ b2, int f0) {
    __shared__ double sh[2];
    const int k = blockIdx.x;
    if (!A.par[k].active) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int t = 0; t < npair; ++t) {
        const double* a = t == 0 ? a0 : (t == 1 ? a1 : a2);
        const double* b = t == 0 ? b0 : (t == 1 ? b1 : b2);
        double s = 0.0;
        for (int c = threadIdx.x; c < A.q; c += blockDim.x)
            s = fma(a[(int64_t)k * A.q + c], b[(int64_t)k * A.q + c], s);
        s = wave_sum(s);
        __syncthreads();
        if (lane == 0) sh[w] = s;
        __syncthreads();
        if (threadIdx.x == 0) A.bs[k].r[f0 + t] = sh[0] + sh[1];
    }
}

// ------------------------------------------------------------------ projection
// v = u - alpha_k sigma_k td (when td), and per item: min b_i, max b_i,
// number of y_i = +1, with b_i = y_i v_i - C [y_i > 0].
template <bool HAS_TD>
__global__ __launch_bounds__(SSN_BLOCK) void kb_proj_init(BArgs A, const double* __restrict__ u,
                                                          const double* __restrict__ td,
                                                          double* __restrict__ vout,
                                                          double* __restrict__ part) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const int nw = *A.wl_n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const BProb P = A.prob[item.x];
        const double as = A.par[item.x].alpha * A.par[item.x].sigma, C = P.C;
        double bmin = 1.0 / 0.0, bmax = -1.0 / 0.0;
        long long np = 0;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) {
            const int64_t i = P.off + r;
            double v = u[i];
            if (HAS_TD) {
                v = fma(-as, td[i], v);
                vout[i] = v;
            }
            const bool pos = P.y[r] > 0;
            const double b = pos ? v - C : -v;
            bmin = fmin(bmin, b);
            bmax = fmax(bmax, b);
            np += pos ? 1 : 0;
        }
        bmin = wave_min(bmin);
        __syncthreads();
        if (lane == 0) sh[w] = bmin;
        __syncthreads();
        double mn = sh[0];
        for (int t = 1; t < SSN_WAVES_PER_BLOCK; ++t) mn = fmin(mn, sh[t]);
        __syncthreads();
        bmax = wave_max(bmax);
        if (lane == 0) sh[w] = bmax;
        __syncthreads();
        double mx = sh[0];
        for (int t = 1; t < SSN_WAVES_PER_BLOCK; ++t) mx = fmax(mx, sh[t]);
        const long long c = block_sum_ll(np, shl);
        if (threadIdx.x == 0) {
            part[(int64_t)it * 3 + 0] = mn;
            part[(int64_t)it * 3 + 1] = mx;
            part[(int64_t)it * 3 + 2] = (double)c;
        }
    }
}

// per problem: the bracket [min b, max b + 2C], where g = -C n_+ and C n_-
__global__ void kb_proj_init_fin(BArgs A, const double* __restrict__ part, int w, int use_hint) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nprob || !A.par[k].active) return;
    const BProb Pr = A.prob[k];
    const int i0 = A.ioff[k], ni = A.icnt[k];
    double mn = 1.0 / 0.0, mx = -1.0 / 0.0;
    for (int i = 0; i < ni; ++i) {                     // min / max: order-free
        const int64_t o = (int64_t)(i0 + i) * 3;
        mn = fmin(mn, part[o]);
        mx = fmax(mx, part[o + 1]);
    }
    const double cnt = sum_items(part + (int64_t)i0 * 3 + 2, 3, ni);
    ProjState P;
    P.lo = mn;
    P.hi = mx + 2.0 * Pr.C;
    P.npos = (long long)cnt;
    P.passes = 0;
    P.approx = 0;
    P.inside = -1;
    P.mode = use_hint ? 1 : 0;
    P.pad_ = 0;
    P.hint = use_hint ? A.bs[k].ps[0].lam : 0.0;
    P.glo = -Pr.C * cnt;
    P.ghi = Pr.C * ((double)Pr.n - cnt);
    if (cnt == 0.0) {
        P.lam = mn;
        P.done = 1;
    } else {
        P.lam = 0.0;
        P.done = 0;
    }
    A.bs[k].ps[w] = P;
}

// candidate multipliers of a pass: uniform over [lo, hi], or (first pass of
// a line-search trial) hint -/+ C 4^e, e = -15..15, plus the two ends
__device__ __forceinline__ double bcand(const ProjState& P, double C, int c) {
    const double lo = P.lo, hi = P.hi;
    if (c == 0) return lo;
    if (c == BPK) return hi;
    if (P.mode == 1) {
        double v;
        if (c < 32) v = P.hint - C * ldexp(1.0, 2 * (16 - c));
        else if (c == 32) v = P.hint;
        else v = P.hint + C * ldexp(1.0, 2 * (c - 48));
        return fmin(fmax(v, lo), hi);
    }
    return lo + (hi - lo) * ((double)c / (double)BPK);
}

// one multisection pass: per item, g at the BPK+1 candidates and the
// histogram of breakpoints strictly inside every sub-interval.  Elements
// whose breakpoints b, b + C both lie outside the bracket contribute a
// constant (C or 0) or exactly (lam - lo) + (lo - b) over the whole bracket
// and are summed in closed form; the others are gathered (thread order) into
// an LDS list and evaluated at every candidate by the whole block.
// Per item: the item's partial g-values at the BPK + 1 candidates without
// the closed-form linear part, its breakpoint histogram, and the closed-form
// counts (constant part kc, linear count and sum of lo - b), combined by
// kb_proj_sel.  Elements with a breakpoint inside the bracket go to an LDS
// list (element order) and are evaluated at every candidate; candidates
// 0..BPK-1 are reduced over each wave by a reduce-scatter.
constexpr int BPU = 4;                    // elements per thread per sweep step
constexpr int BPCOL = BPNV + 1;           // doubles per item: g partials, sum of lo - b
constexpr int BPICOL = BPK + 2;           // ints per item: histogram, constant count, linear count
static_assert(BPK == SSN_WAVE, "one candidate per lane in the reduce-scatter");
__global__ __launch_bounds__(SSN_BLOCK) void kb_proj_pass(BArgs A, const double* __restrict__ v,
                                                          int w, double* __restrict__ part,
                                                          int* __restrict__ hpart) {
    __shared__ double lam_s[BPK + 1];
    __shared__ double red[SSN_WAVES_PER_BLOCK][BPCOL];
    __shared__ long long redl[SSN_WAVES_PER_BLOCK][2];
    __shared__ int hist[BPK];
    __shared__ double list[BRPI];
    __shared__ int wsum[BPU][SSN_WAVES_PER_BLOCK];
    const int nw = *A.wl_n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int k = item.x;
        const ProjState P = A.bs[k].ps[w];
        if (P.done) continue;                          // uniform over the block
        const BProb Pr = A.prob[k];
        const double C = Pr.C;
        __syncthreads();
        if (threadIdx.x <= BPK) lam_s[threadIdx.x] = bcand(P, C, threadIdx.x);
        if (threadIdx.x < BPK) hist[threadIdx.x] = 0;
        __syncthreads();
        const double blo = lam_s[0], bhi = lam_s[BPK];
        long long kc = 0, lin_n = 0;       // C times kc: exact constant part
        double lin_s = 0.0;
        int cnt = 0;
        for (int base = item.y; base < item.z; base += blockDim.x * BPU) {
            double vv[BPU];
            int yy[BPU];
#pragma unroll
            for (int u = 0; u < BPU; ++u) {            // every load of the step first
                // (a row past the item reads its last row, unused below: no load
                // sits under a branch, so all of them are in flight together)
                const int r = base + u * (int)blockDim.x + threadIdx.x;
                const int rc = r < item.z ? r : item.z - 1;
                vv[u] = v[Pr.off + rc];
                yy[u] = (int)Pr.y[rc];
            }
            bool take[BPU];
            double bb[BPU];
#pragma unroll
            for (int u = 0; u < BPU; ++u) {
                const int r = base + u * (int)blockDim.x + threadIdx.x;
                take[u] = false;
                bb[u] = 0.0;
                if (r < item.z) {
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
            cnt += block_append_multi<BPU>(take, bb, list, cnt, wsum);
        }
        __syncthreads();
        double acc[BPK];
        double acc_hi = 0.0;
#pragma unroll
        for (int c = 0; c < BPK; ++c) acc[c] = 0.0;
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            const double b = list[e];
            const double bh = b + C;
#pragma unroll
            for (int c = 0; c < BPK; ++c) acc[c] += clampd(lam_s[c] - b, 0.0, C);
            acc_hi += clampd(bhi - b, 0.0, C);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double t = h ? bh : b;
                if (t > blo && t < bhi) {
                    int lo_k = 0, hi_k = BPK;
                    while (hi_k - lo_k > 1) {
                        const int mid = (lo_k + hi_k) >> 1;
                        if (lam_s[mid] < t) lo_k = mid; else hi_k = mid;
                    }
                    if (t < lam_s[lo_k + 1]) atomicAdd(&hist[lo_k], 1);
                }
            }
        }
        double gk = 0.0, ghi = 0.0;
        if (cnt > wv * SSN_WAVE) {                 // else this wave's acc are zeros
            gk = wave_reduce_scatter64(acc);
            ghi = wave_sum(acc_hi);
        }
        const double ls = wave_sum(lin_s);
        const long long kw = wave_sum_ll(kc), lw = wave_sum_ll(lin_n);
        red[wv][lane] = gk;
        if (lane == 0) {
            red[wv][BPK] = ghi;
            red[wv][BPK + 1] = ls;
            redl[wv][0] = kw;
            redl[wv][1] = lw;
        }
        __syncthreads();
        if (threadIdx.x < BPCOL) {
            double s2 = 0.0;
#pragma unroll
            for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) s2 += red[ww][threadIdx.x];
            part[(int64_t)it * BPCOL + threadIdx.x] = s2;
        }
        if (threadIdx.x < BPK) hpart[(int64_t)it * BPICOL + threadIdx.x] = hist[threadIdx.x];
        if (threadIdx.x == 0) {
            long long k2 = 0, l2 = 0;
#pragma unroll
            for (int ww = 0; ww < SSN_WAVES_PER_BLOCK; ++ww) { k2 += redl[ww][0]; l2 += redl[ww][1]; }
            hpart[(int64_t)it * BPICOL + BPK] = (int)k2;
            hpart[(int64_t)it * BPICOL + BPK + 1] = (int)l2;
        }
    }
}

// per problem: add the item values (item order), keep the sub-interval where
// g changes sign; done when it holds no breakpoint (g affine there: linear
// interpolation), when it cannot be split further, or at the pass cap
__global__ __launch_bounds__(128) void kb_proj_sel(BArgs A, const double* __restrict__ part,
                                                   const int* __restrict__ hpart, int w) {
    __shared__ double G[BPNV];
    __shared__ int H[BPK];
    const int k = blockIdx.x;
    if (!A.par[k].active) return;
    ProjState P = A.bs[k].ps[w];
    if (P.done) return;
    const double C = A.prob[k].C;
    const int i0 = A.ioff[k], ni = A.icnt[k];
    __shared__ int K, LN;
    __shared__ double LS;
    for (int c = threadIdx.x; c < BPICOL; c += blockDim.x) {
        const int h = isum_items(hpart + (int64_t)i0 * BPICOL + c, BPICOL, ni);
        if (c < BPK) H[c] = h;
        else if (c == BPK) K = h;
        else LN = h;
    }
    if (threadIdx.x == 0) LS = sum_items(part + (int64_t)i0 * BPCOL + BPNV, BPCOL, ni);
    __syncthreads();
    const double blo = bcand(P, C, 0);
    for (int c = threadIdx.x; c < BPNV; c += blockDim.x)
        G[c] = sum_items(part + (int64_t)i0 * BPCOL + c, BPCOL, ni) + C * (double)K +
               (double)LN * (bcand(P, C, c) - blo) + LS;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int passes = P.passes + 1;
    int j = 0;
    for (int c = 0; c < BPK; ++c)
        if (G[c] < 0.0) j = c;
    const double nlo = bcand(P, C, j), nhi = bcand(P, C, j + 1);
    const double g0 = G[j], g1 = G[j + 1];
    const int ins = H[j];
    P.passes = passes;
    P.mode = 0;
    P.inside = ins;
    P.lo = nlo;
    P.hi = nhi;
    P.glo = g0;
    P.ghi = g1;
    const bool tiny = !(nlo < nhi) || !(nlo + (nhi - nlo) / (double)BPK > nlo);
    if (ins == 0 || tiny || passes >= BMAXPASS) {
        double lam;
        if (g1 == 0.0) lam = nhi;
        else if (g1 > g0) lam = nlo + (-g0) / (g1 - g0) * (nhi - nlo);
        else lam = nlo;
        P.lam = fmin(fmax(lam, nlo), nhi);
        P.approx = ins == 0 ? 0 : 1;
        P.done = 1;
    }
    A.bs[k].ps[w] = P;
}

// ------------------------------------------------------------------ finalize sums
// phi(t) = int_0^t clip(s, 0, C) ds and its increment from t to t + dt by
// the closed form of the piece when both ends lie on one piece.
__device__ __forceinline__ double bhuber_piece(double t, double C) {
    return t <= 0.0 ? 0.0 : (t < C ? 0.5 * t * t : C * (t - 0.5 * C));
}
__device__ __forceinline__ double bhuber_inc(double t, double dt, double C) {
    const double b = t + dt;
    if (t >= C && b >= C) return C * dt;
    if (t <= 0.0 && b <= 0.0) return 0.0;
    if (t > 0.0 && t < C && b > 0.0 && b < C) return dt * (t + 0.5 * dt);
    return bhuber_piece(b, C) - bhuber_piece(t, C);
}

// Line-search finalize of projection w against the base projection wb:
// x = clip(v - lam y) (v = u_base - alpha sigma td), mask = strict interior;
// item partials of the phi increments (dt_i = -alpha sigma td_i - (lam -
// lam_base) y_i), |x - x^k|^2, #free, #(x > 0).
__global__ __launch_bounds__(SSN_BLOCK) void kb_ls_fin(BArgs A, const double* __restrict__ v,
                                                       const double* __restrict__ ubase,
                                                       const double* __restrict__ td, int w, int wb,
                                                       const double* __restrict__ xk,
                                                       double* __restrict__ x,
                                                       uint8_t* __restrict__ mask,
                                                       double* __restrict__ part) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int k = item.x;
        const BProb P = A.prob[k];
        const double C = P.C, lam = A.bs[k].ps[w].lam, lamb = A.bs[k].ps[wb].lam;
        const double dl = lam - lamb, as = A.par[k].alpha * A.par[k].sigma;
        double dh = 0.0, d2 = 0.0, pc = 0.0, sv = 0.0;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) {
            const int64_t i = P.off + r;
            const double yi = (double)P.y[r];
            const double t = v[i] - lam * yi;
            const double xi = clampd(t, 0.0, C);
            const bool fr = t > 0.0 && t < C;
            x[i] = xi;
            mask[i] = fr ? 1 : 0;
            pc += fr ? 1.0 : 0.0;
            sv += xi > 0.0 ? 1.0 : 0.0;
            const double dx = xi - xk[i];
            d2 = fma(dx, dx, d2);
            const double tb = ubase[i] - lamb * yi;
            const double dt = td ? fma(-as, td[i], -dl * yi) : -dl * yi;
            dh += bhuber_inc(tb, dt, C);
        }
        const double a = block_sum(dh, sh), b = block_sum(d2, sh);
        const double c = block_sum(pc, sh), e = block_sum(sv, sh);
        if (threadIdx.x == 0) {
            part[(int64_t)it * 4 + 0] = a;
            part[(int64_t)it * 4 + 1] = b;
            part[(int64_t)it * 4 + 2] = c;
            part[(int64_t)it * 4 + 3] = e;
        }
    }
}

// KKT finalize: item partials of |x - Pi(v)|^2, |x|^2, e^T x
// item partials of |x - Pi(v)|^2, |x|^2, e^T x and the hinge sum
// sum max(0, 1 - Qx_i - y_i lam) of the C-SVC primal at the KKT bias lam
__global__ __launch_bounds__(SSN_BLOCK) void kb_kkt_fin(BArgs A, const double* __restrict__ v,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ Qx, int w,
                                                        double* __restrict__ part) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int k = item.x;
        const BProb P = A.prob[k];
        const double lam = A.bs[k].ps[w].lam, C = P.C;
        double r2 = 0.0, x2 = 0.0, sx = 0.0, hs = 0.0;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) {
            const int64_t i = P.off + r;
            const double xi = x[i];
            const double yi = (double)P.y[r];
            const double pi = clampd(v[i] - lam * yi, 0.0, C);
            const double d = xi - pi;
            r2 = fma(d, d, r2);
            x2 = fma(xi, xi, x2);
            sx += xi;
            hs += fmax(0.0, 1.0 - Qx[i] - lam * yi);
        }
        const double a = block_sum(r2, sh), b = block_sum(x2, sh), c = block_sum(sx, sh);
        const double h = block_sum(hs, sh);
        if (threadIdx.x == 0) {
            part[(int64_t)it * 4 + 0] = a;
            part[(int64_t)it * 4 + 1] = b;
            part[(int64_t)it * 4 + 2] = c;
            part[(int64_t)it * 4 + 3] = h;
        }
    }
}

// Final counts of a returned x: item partials of e^T x, #(x > 0), #(0 < x < C)
__global__ __launch_bounds__(SSN_BLOCK) void kb_count(BArgs A, const double* __restrict__ x,
                                                      double* __restrict__ part) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const BProb P = A.prob[item.x];
        double sx = 0.0, sv = 0.0, pf = 0.0;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) {
            const double xi = x[P.off + r];
            sx += xi;
            sv += xi > 0.0 ? 1.0 : 0.0;
            pf += (xi > 0.0 && xi < P.C) ? 1.0 : 0.0;
        }
        const double a = block_sum(sx, sh), b = block_sum(sv, sh), c = block_sum(pf, sh);
        if (threadIdx.x == 0) {
            part[(int64_t)it * 4 + 0] = a;
            part[(int64_t)it * 4 + 1] = b;
            part[(int64_t)it * 4 + 2] = c;
            part[(int64_t)it * 4 + 3] = 0.0;
        }
    }
}

// per problem: bs[k].r[f0 + t] = sum of the item partials t (item order), t < nf
__global__ void kb_sum4(BArgs A, const double* __restrict__ part, int f0, int nf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nprob || !A.par[k].active) return;
    const int i0 = A.ioff[k], ni = A.icnt[k];
    for (int t = 0; t < nf; ++t) A.bs[k].r[f0 + t] = sum_items(part + (int64_t)i0 * 4 + t, 4, ni);
}

// ------------------------------------------------------------------ compaction of J
__global__ __launch_bounds__(SSN_BLOCK) void kb_cmp_count(BArgs A, const uint8_t* __restrict__ mask,
                                                          int* __restrict__ cnt) {
    __shared__ long long shl[SSN_WAVES_PER_BLOCK];
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int64_t off = A.prob[item.x].off;
        long long c = 0;
        for (int r = item.y + threadIdx.x; r < item.z; r += blockDim.x) c += mask[off + r] ? 1 : 0;
        c = block_sum_ll(c, shl);
        if (threadIdx.x == 0) cnt[it] = (int)c;
    }
}
// per problem: exclusive scan of its item counts (item order), p_k
__global__ void kb_cmp_scan(BArgs A, const int* __restrict__ cnt, int* __restrict__ ofs) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nprob || !A.par[k].active) return;
    const int i0 = A.ioff[k], ni = A.icnt[k];
    long long run = 0;
    for (int i = 0; i < ni; ++i) {
        ofs[i0 + i] = (int)run;
        run += cnt[i0 + i];
    }
    A.bs[k].p = run;
}
// the J rows of every item (local row indices, ascending) at list[off + ofs]
__global__ __launch_bounds__(SSN_BLOCK) void kb_cmp_write(BArgs A, const uint8_t* __restrict__ mask,
                                                          const int* __restrict__ ofs,
                                                          int32_t* __restrict__ list) {
    __shared__ int sh[SSN_BLOCK];
    constexpr int EPT = BRPI / SSN_BLOCK;             // consecutive rows per thread
    const int nw = *A.wl_n;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 item = A.wl[it];
        const int64_t off = A.prob[item.x].off;
        const int rb = item.y + threadIdx.x * EPT;
        int c = 0;
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            if (rb + e < item.z && mask[off + rb + e]) ++c;
        __syncthreads();
        sh[threadIdx.x] = c;
        __syncthreads();
        for (int o = 1; o < SSN_BLOCK; o <<= 1) {
            const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        int pos = ofs[it] + sh[threadIdx.x] - c;
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            if (rb + e < item.z && mask[off + rb + e]) list[off + pos++] = rb + e;
    }
}

// ------------------------------------------------------------------ Newton system
// Gram work list: problem k's p_k J rows in m_k = clamp(ceil(p_k / GROWS),
// 1, GMAXI) items of equal length (0 items when p_k = 0).  m_k depends on
// p_k only.  One block.
__global__ __launch_bounds__(1024) void kb_gram_plan(BArgs A, int4* __restrict__ gwl,
                                                     int* __restrict__ gwl_n,
                                                     int* __restrict__ goff,
                                                     int* __restrict__ gcnt) {
    __shared__ int sc[1024];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int k0 = 0; k0 < A.nprob; k0 += 1024) {
        const int k = k0 + threadIdx.x;
        long long p = 0;
        int m = 0;
        if (k < A.nprob && A.par[k].active) {
            p = A.bs[k].p;
            m = p == 0 ? 0 : (int)min((p + GROWS - 1) / GROWS, (long long)GMAXI);
        }
        sc[threadIdx.x] = m;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
            __syncthreads();
            sc[threadIdx.x] += t;
            __syncthreads();
        }
        const int o = base + sc[threadIdx.x] - m;
        if (k < A.nprob) {
            goff[k] = o;
            gcnt[k] = m;
            const long long len = m > 0 ? (p + m - 1) / m : 0;
            for (int i = 0; i < m; ++i) {
                const long long c0 = i * len, c1 = min(p, c0 + len);
                gwl[o + i] = make_int4(k, (int)c0, (int)c1, 0);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) base += sc[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *gwl_n = base;
}

// G partial of one item: sum over its J rows of x x^T (q x q, fp64), 8 x 8
// outputs per thread on a 16 x 16 thread grid, rows staged through LDS.
template <typename T>
__global__ __launch_bounds__(SSN_BLOCK) void kb_gram(BArgs A, const int4* __restrict__ gwl,
                                                     const int* __restrict__ gwl_n,
                                                     const int32_t* __restrict__ list,
                                                     double* __restrict__ gpart) {
    __shared__ double Xs[GST][BQMAX + 1];
    const int nw = *gwl_n, q = A.q;
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    for (int it = blockIdx.x; it < nw; it += gridDim.x) {
        const int4 gi = gwl[it];
        const BProb P = A.prob[gi.x];
        const T* X = (const T*)P.X;
        double acc[8][8];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
        for (int rb = gi.y; rb < gi.z; rb += GST) {
            __syncthreads();
            // every load of the stage issued unconditionally (row and column
            // clamped, the value dropped), so all of them are in flight together
            static_assert(GST * BQMAX % SSN_BLOCK == 0, "whole stage per thread");
#pragma unroll
            for (int h = 0; h < GST * BQMAX / SSN_BLOCK; ++h) {
                const int e = threadIdx.x + h * SSN_BLOCK;
                const int rr = e / BQMAX, cc = e % BQMAX;
                const int r = rb + rr;
                const int rc = r < gi.z ? r : gi.z - 1, ccc = cc < q ? cc : q - 1;
                const double xv = to_f64(X[(int64_t)list[P.off + rc] * q + ccc]);
                Xs[rr][cc] = (r < gi.z && cc < q) ? xv : 0.0;
            }
            __syncthreads();
            const int nr = min(GST, gi.z - rb);
            for (int rr = 0; rr < nr; ++rr) {
                double xa[8], xb[8];
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    xa[a] = Xs[rr][ti * 8 + a];
                    xb[a] = Xs[rr][tj * 8 + a];
                }
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int b = 0; b < 8; ++b) acc[a][b] = fma(xa[a], xb[b], acc[a][b]);
            }
        }
        double* out = gpart + (int64_t)it * q * q;
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int i = ti * 8 + a, j = tj * 8 + b;
                if (i < q && j < q) out[i * q + j] = acc[a][b];
            }
    }
}

// M_k = I + sigma_k (G_k - s s^T / p_k), G_k = sum of its items (item order)
__global__ __launch_bounds__(SSN_BLOCK) void kb_gram_fin(BArgs A, const double* __restrict__ gpart,
                                                         const int* __restrict__ goff,
                                                         const int* __restrict__ gcnt,
                                                         const double* __restrict__ sv,
                                                         double* __restrict__ M) {
    const int k = blockIdx.x;
    if (!A.par[k].active) return;
    const int q = A.q, i0 = goff[k], ni = gcnt[k];
    const long long p = A.bs[k].p;
    const double sigma = A.par[k].sigma, ip = p > 0 ? 1.0 / (double)p : 0.0;
    for (int e = threadIdx.x; e < q * q; e += blockDim.x) {
        const double g = sum_items(gpart + (int64_t)i0 * q * q + e, (int64_t)q * q, ni);
        const int r = e / q, c = e % q;
        const double sr = sv[(int64_t)k * q + r], scl = sv[(int64_t)k * q + c];
        M[(int64_t)k * q * q + e] = (r == c ? 1.0 : 0.0) + sigma * (g - sr * scl * ip);
    }
}

// d_k = -M_k^{-1} g_k by Cholesky with M_k in LDS, one block per problem.  A
// non-positive pivot sets chol_fail and gives d_k = -g_k.
__global__ __launch_bounds__(1024) void kb_chol(BArgs A, const double* __restrict__ Mall,
                                                const double* __restrict__ gall,
                                                double* __restrict__ dall) {
    extern __shared__ double L[];
    __shared__ double z[BQMAX];
    __shared__ int bad;
    const int k = blockIdx.x;
    if (!A.par[k].active) return;
    const int q = A.q, tid = threadIdx.x, nt = blockDim.x;
    const double* M = Mall + (int64_t)k * q * q;
    const double* g = gall + (int64_t)k * q;
    double* d = dall + (int64_t)k * q;
    for (int e = tid; e < q * q; e += nt) L[e] = M[e];
    for (int i = tid; i < q; i += nt) z[i] = -g[i];
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int kk = 0; kk < q; ++kk) {
        const double akk = L[kk * q + kk];
        if (!(akk > 0.0)) {
            if (tid == 0) bad = 1;
            break;                                   // uniform: every thread read the same value
        }
        const double lkk = sqrt(akk);
        __syncthreads();
        for (int i = kk + 1 + tid; i < q; i += nt) L[i * q + kk] /= lkk;
        if (tid == 0) L[kk * q + kk] = lkk;
        __syncthreads();
        const int m = q - kk - 1;
        for (int e = tid; e < m * m; e += nt) {
            const int a = e / m, b = e % m;
            if (b <= a) L[(kk + 1 + a) * q + kk + 1 + b] -= L[(kk + 1 + a) * q + kk] * L[(kk + 1 + b) * q + kk];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        for (int i = tid; i < q; i += nt) d[i] = -g[i];
        if (tid == 0) A.bs[k].chol_fail = 1;
        return;
    }
    for (int j = 0; j < q; ++j) {
        if (tid == 0) z[j] /= L[j * q + j];
        __syncthreads();
        const double zj = z[j];
        for (int i = j + 1 + tid; i < q; i += nt) z[i] -= L[i * q + j] * zj;
        __syncthreads();
    }
    for (int j = q - 1; j >= 0; --j) {
        if (tid == 0) z[j] /= L[j * q + j];
        __syncthreads();
        const double zj = z[j];
        for (int i = tid; i < j; i += nt) z[i] -= L[j * q + i] * zj;
        __syncthreads();
    }
    for (int i = tid; i < q; i += nt) d[i] = z[i];
    if (tid == 0) A.bs[k].chol_fail = 0;
}

// ------------------------------------------------------------------ launchers
template <typename T, int P>
static void amul2_t(const BLaunch& L, const double* V, double* t) {
    constexpr int R = P < 8 ? P : 8;
    SSN_LAUNCH((kb_amul2<T, P, R>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, V, t);
}
template <typename T, bool VEC>
static void amul_t(const BLaunch& L, const double* V, double* t) {
    if (VEC) {
        // lanes per row: 16-byte pieces of a row, rounded up to a power of two
        const int pieces = (L.A.q * (int)sizeof(T) + 15) / 16;
        int P = 1;
        while (P < pieces) P <<= 1;
        if (P <= SSN_WAVE) {
            switch (P) {
            case 1: amul2_t<T, 1>(L, V, t); return;
            case 2: amul2_t<T, 2>(L, V, t); return;
            case 4: amul2_t<T, 4>(L, V, t); return;
            case 8: amul2_t<T, 8>(L, V, t); return;
            case 16: amul2_t<T, 16>(L, V, t); return;
            case 32: amul2_t<T, 32>(L, V, t); return;
            default: amul2_t<T, 64>(L, V, t); return;
            }
        }
    }
    if (L.unr == 1)
        SSN_LAUNCH((kb_amul<T, VEC, 1>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, V, t);
    else if (L.unr == 2)
        SSN_LAUNCH((kb_amul<T, VEC, 2>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, V, t);
    else
        SSN_LAUNCH((kb_amul<T, VEC, 4>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, V, t);
}
template <typename T, bool VEC>
static void atmul_t(const BLaunch& L, const double* z, const uint8_t* mask) {
    if (mask)
        SSN_LAUNCH((kb_atmul<T, VEC, true>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, z,
                           mask, L.part, L.part2);
    else
        SSN_LAUNCH((kb_atmul<T, VEC, false>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, z,
                           mask, L.part, L.part2);
}
#define BDISPATCH(FN, ...)                                                                  \
    do {                                                                                   \
        if (L.dtype == SSNALM_F64) {                                                       \
            if (L.vec) FN<double, true>(__VA_ARGS__); else FN<double, false>(__VA_ARGS__); \
        } else if (L.dtype == SSNALM_F32) {                                                \
            if (L.vec) FN<float, true>(__VA_ARGS__); else FN<float, false>(__VA_ARGS__);   \
        } else {                                                                           \
            if (L.vec) FN<bf16_t, true>(__VA_ARGS__); else FN<bf16_t, false>(__VA_ARGS__); \
        }                                                                                  \
    } while (0)

static inline unsigned pgrid(int n) { return (unsigned)((n + 63) / 64); }

void lb_build_wl(const BLaunch& L, const int4* items) {
    SSN_LAUNCH(kb_wl_scan, dim3(1), dim3(1024), 0, L.s, L.A);
    SSN_LAUNCH(kb_wl_copy, dim3(L.A.nprob), dim3(256), 0, L.s, L.A, items);
}
void lb_amul(const BLaunch& L, const double* V, double* t) { BDISPATCH(amul_t, L, V, t); }
void lb_atmul(const BLaunch& L, const double* z, const uint8_t* mask, const double* base,
              double sign, double* out, double* out2) {
    BDISPATCH(atmul_t, L, z, mask);
    SSN_LAUNCH(kb_atmul_fin, dim3(L.A.nprob), dim3(128), 0, L.s, L.A, L.part,
                       mask ? L.part2 : nullptr, base, sign, out, mask ? out2 : nullptr);
}
void lb_elem(const BLaunch& L, int mode, const double* a, const double* b, double* o) {
    SSN_LAUNCH(kb_elem, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, mode, a, b, o);
}
void lb_accept(const BLaunch& L, double* om, const double* d, double* aw, const double* td,
               double* u, const double* ut, double* xt, const double* xtt, uint8_t* jm,
               const uint8_t* jmt) {
    SSN_LAUNCH(kb_qvec, dim3(L.A.nprob), dim3(128), 0, L.s, L.A, 0, om, d, om);
    SSN_LAUNCH(kb_accept_n, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, aw, td, u, ut, xt,
                       xtt, jm, jmt);
}
void lb_qvec(const BLaunch& L, int mode, const double* a, const double* b, double* o) {
    SSN_LAUNCH(kb_qvec, dim3(L.A.nprob), dim3(128), 0, L.s, L.A, mode, a, b, o);
}
void lb_qdots(const BLaunch& L, int npair, const double* a0, const double* b0, const double* a1,
              const double* b1, const double* a2, const double* b2, int f0) {
    SSN_LAUNCH(kb_qdots, dim3(L.A.nprob), dim3(128), 0, L.s, L.A, npair, a0, b0, a1, b1,
                       a2, b2, f0);
}
void lb_proj_init(const BLaunch& L, const double* u, const double* td, double* vout, int w,
                  int use_hint) {
    if (td)
        SSN_LAUNCH((kb_proj_init<true>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, u, td,
                           vout, L.part);
    else
        SSN_LAUNCH((kb_proj_init<false>), dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, u, td,
                           vout, L.part);
    SSN_LAUNCH(kb_proj_init_fin, dim3(pgrid(L.A.nprob)), dim3(64), 0, L.s, L.A, L.part, w,
                       use_hint);
}
void lb_proj_passes(const BLaunch& L, const double* v, int w, int npass) {
    for (int i = 0; i < npass; ++i) {
        SSN_LAUNCH(kb_proj_pass, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, v, w, L.part,
                           L.ipart);
        SSN_LAUNCH(kb_proj_sel, dim3(L.A.nprob), dim3(128), 0, L.s, L.A, L.part, L.ipart, w);
    }
}
void lb_ls_fin(const BLaunch& L, const double* v, const double* ubase, const double* td, int w,
               int wb, const double* xk, double* x, uint8_t* mask) {
    SSN_LAUNCH(kb_ls_fin, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, v, ubase, td, w, wb,
                       xk, x, mask, L.part);
    SSN_LAUNCH(kb_sum4, dim3(pgrid(L.A.nprob)), dim3(64), 0, L.s, L.A, L.part, (int)BS_DH, 4);
}
void lb_kkt_fin(const BLaunch& L, const double* v, const double* x, const double* Qx, int w) {
    SSN_LAUNCH(kb_kkt_fin, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, v, x, Qx, w, L.part);
    SSN_LAUNCH(kb_sum4, dim3(pgrid(L.A.nprob)), dim3(64), 0, L.s, L.A, L.part, (int)BS_RES2, 4);
}
void lb_count(const BLaunch& L, const double* x) {
    SSN_LAUNCH(kb_count, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, x, L.part);
    SSN_LAUNCH(kb_sum4, dim3(pgrid(L.A.nprob)), dim3(64), 0, L.s, L.A, L.part, (int)BS_FSUMX, 3);
}
void lb_compact(const BLaunch& L, const uint8_t* mask, int32_t* list) {
    SSN_LAUNCH(kb_cmp_count, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, mask, L.ipart);
    SSN_LAUNCH(kb_cmp_scan, dim3(pgrid(L.A.nprob)), dim3(64), 0, L.s, L.A, L.ipart, L.ipart2);
    SSN_LAUNCH(kb_cmp_write, dim3(L.grid), dim3(SSN_BLOCK), 0, L.s, L.A, mask, L.ipart2, list);
}
void lb_setup_attributes() {
    static bool done = false;
    if (done) return;
    hipFuncSetAttribute((const void*)kb_chol, hipFuncAttributeMaxDynamicSharedMemorySize,
                        BQMAX * BQMAX * (int)sizeof(double));
    done = true;
}
void lb_newton(const BLaunch& L, const int32_t* list, const double* sv, const double* g, double* d,
               double* M) {
    SSN_LAUNCH(kb_gram_plan, dim3(1), dim3(1024), 0, L.s, L.A, L.gwl, L.gwl_n, L.goff, L.gcnt);
    if (L.dtype == SSNALM_F64)
        SSN_LAUNCH(kb_gram<double>, dim3(L.ggrid), dim3(SSN_BLOCK), 0, L.s, L.A, L.gwl,
                           L.gwl_n, list, L.gpart);
    else if (L.dtype == SSNALM_F32)
        SSN_LAUNCH(kb_gram<float>, dim3(L.ggrid), dim3(SSN_BLOCK), 0, L.s, L.A, L.gwl,
                           L.gwl_n, list, L.gpart);
    else
        SSN_LAUNCH(kb_gram<bf16_t>, dim3(L.ggrid), dim3(SSN_BLOCK), 0, L.s, L.A, L.gwl,
                           L.gwl_n, list, L.gpart);
    SSN_LAUNCH(kb_gram_fin, dim3(L.A.nprob), dim3(SSN_BLOCK), 0, L.s, L.A, L.gpart, L.goff,
                       L.gcnt, sv, M);
    SSN_LAUNCH(kb_chol, dim3(L.A.nprob), dim3(L.A.q <= 64 ? 256 : 1024),
                       (size_t)L.A.q * L.A.q * sizeof(double), L.s, L.A, M, g, d);
}

}  // namespace ssn
