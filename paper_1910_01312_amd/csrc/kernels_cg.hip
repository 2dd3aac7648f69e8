// Conjugate gradients for step 1 of Algorithm 3 on sparse input, solved to
// the paper's residual tolerance min(eta, |grad psi|^{1+tau}):
//     M d = -g,   M = I + sigma X_J^T (I - 1 1^T/p) X_J,
// with the Jacobi preconditioner diag(M).  Writing w = X_J v and s = X_J^T 1,
//     M v = v + sigma (X_J^T w - (s.v / p) s),
//     v.M v = |v|^2 + sigma (|w|^2 - (s.v)^2 / p),
// so one CG iteration needs X_J v, X_J^T w and a handful of q-vector sums.
//
// Cross-block sums never use atomics or fences: every kernel writes one
// partial per block, and the NEXT kernel (whose blocks all start after the
// writer finished) re-reduces those partials itself, in the same fixed order
// in every block.  All blocks therefore see bit-identical scalars.
//
// X_J^T w runs over the compact column-major copy of X_J (entries sorted by
// column) in fixed chunks of 256 entries (4 per lane, one wave per chunk).
// Runs of equal column inside a chunk are summed by a segmented scan; a run
// that reaches a chunk border is left as a carry per chunk, and the runs that
// cross borders, listed once per copy (first chunk, last chunk, column), are
// summed from their carries in chunk order by one wave each.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int KE = 4;
constexpr int KCH = KE * SSN_WAVE;     // entries per chunk

// --------------------------------------------------------------- partials
// Fixed-order sum of part[b*stride + c], b < nb, by the whole block (every
// block computes the same value).
__device__ __forceinline__ double red_col(const double* __restrict__ part, int nb, int stride,
                                          int c, double* sh) {
    double a0 = 0.0, a1 = 0.0;
    int b = threadIdx.x;
    const int T = blockDim.x;
    for (; b + T < nb; b += 2 * T) {
        a0 += part[(int64_t)b * stride + c];
        a1 += part[(int64_t)(b + T) * stride + c];
    }
    for (; b < nb; b += T) a0 += part[(int64_t)b * stride + c];
    return block_sum(a0 + a1, sh);
}

static inline unsigned qgrid(int64_t q) {
    int64_t b = (q + 511) / 512;
    if (b > 256) b = 256;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// --------------------------------------------------------------- init
// x = 0, r = -g, z = r/diag, p = z; partials: Pst = (r.z, r.r), Pdir = (p.p, s.p)
__global__ __launch_bounds__(SSN_BLOCK) void k_cg_init(const double* __restrict__ g,
                                                       const double* __restrict__ diag,
                                                       const double* __restrict__ sv, int64_t q,
                                                       double* __restrict__ x,
                                                       double* __restrict__ r,
                                                       double* __restrict__ z,
                                                       double* __restrict__ pd,
                                                       double* __restrict__ Pst,
                                                       double* __restrict__ Pdir) {
    __shared__ double sh[4 * SSN_WAVES_PER_BLOCK];
    double rz = 0.0, rr = 0.0, pp = 0.0, sp = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
        const double rj = -g[j];
        const double zj = rj / diag[j];
        x[j] = 0.0;
        r[j] = rj;
        z[j] = zj;
        pd[j] = zj;
        rz = fma(rj, zj, rz);
        rr = fma(rj, rj, rr);
        pp = fma(zj, zj, pp);
        sp = fma(sv[j], zj, sp);
    }
    double v[4] = {rz, rr, pp, sp};
    block_sum_n<4>(v, sh);
    if (threadIdx.x == 0) {
        Pst[blockIdx.x * 2] = v[0];
        Pst[blockIdx.x * 2 + 1] = v[1];
        Pdir[blockIdx.x * 2] = v[2];
        Pdir[blockIdx.x * 2 + 1] = v[3];
    }
}

// --------------------------------------------------------------- X_J v
// w[k] = (X_J v)_k for the k-th row of the ordered J list; Pw[b] = sum w^2.
// 16 lanes per row; each lane issues its loads four entries at a time, with no
// load under a per-lane branch.  Persistent workgroups keep v over the
// CGR_HEAD most frequent columns in LDS: the random gathers of v, not the
// stream of entries, are what a row product of a text-like X waits on.
constexpr int CGR_THREADS = 1024;           // 16 waves per workgroup
constexpr int CGR_WPB = CGR_THREADS / SSN_WAVE;
constexpr int CGR_HEAD = 16384;             // columns of v in LDS (128 KB)
static_assert(CGR_HEAD % CGR_THREADS == 0, "the head is copied in whole rounds");

template <typename V>
__global__ __launch_bounds__(CGR_THREADS) void k_cg_rows(const int2* __restrict__ jrow,
                                                         const int32_t* __restrict__ ci,
                                                         const V* __restrict__ val, int64_t p,
                                                         const double* __restrict__ v, int32_t H,
                                                         double* __restrict__ w,
                                                         double* __restrict__ Pw,
                                                         const Scalars* __restrict__ sc) {
    __shared__ double vh[CGR_HEAD];
    __shared__ double sh[CGR_WPB];
    if (sc->cg_done) return;                   // converged: the step passes through
    // v over the first H columns (the most frequent: columns are numbered by
    // decreasing entry count) into LDS, every load issued before any store
    {
        constexpr int PER = CGR_HEAD / CGR_THREADS;
        double t[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = (int)threadIdx.x + i * CGR_THREADS;
            t[i] = v[j < H ? j : 0];
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = (int)threadIdx.x + i * CGR_THREADS;
            if (j < H) vh[j] = t[i];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int grp = lane >> 4, sub = lane & 15;
    const int64_t wave = (int64_t)blockIdx.x * CGR_WPB + __builtin_amdgcn_readfirstlane(threadIdx.x / SSN_WAVE);
    const int64_t nwave = (int64_t)gridDim.x * CGR_WPB;
    double ww = 0.0;
    for (int64_t base = wave * 4; base < p; base += nwave * 4) {
        const int64_t k = base + grp;
        double acc = 0.0;
        if (k < p) {
            const int2 er = jrow[k];
            const int32_t e0 = er.x, e1 = er.y;
            // a lane's entries e0 + sub + 16 m, four at a time: the indices and
            // values of all four loaded at once (an entry past the row reads the
            // row's first entry and is multiplied by 0), then the four gathers,
            // each issued to LDS and to global memory (the read not needed
            // pointed at a fixed address)
            for (int32_t e = e0 + sub; e < e1; e += 64) {
                int32_t cc[4];
                double a[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int32_t em = e + 16 * m;
                    const int32_t ec = em < e1 ? em : e0;
                    cc[m] = ci[ec];
                    const double x = (double)val[ec];
                    a[m] = em < e1 ? x : 0.0;
                }
                double gl[4], gg[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    gl[m] = vh[cc[m] < H ? cc[m] : 0];
                    gg[m] = v[cc[m] < H ? 0 : cc[m]];
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) acc = fma(a[m], cc[m] < H ? gl[m] : gg[m], acc);
            }
        }
        acc += __shfl_xor(acc, 8, SSN_WAVE);
        acc += __shfl_xor(acc, 4, SSN_WAVE);
        acc += __shfl_xor(acc, 2, SSN_WAVE);
        acc += __shfl_xor(acc, 1, SSN_WAVE);
        if (k < p && sub == 0) {
            w[k] = acc;
            ww = fma(acc, acc, ww);
        }
    }
    // block sum of ww, waves in index order
    ww = wave_sum(ww);
    if (lane == 0) sh[threadIdx.x / SSN_WAVE] = ww;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < CGR_WPB; ++i) r += sh[i];
        Pw[blockIdx.x] = r;
    }
}

// one persistent workgroup per compute unit (the LDS copy of v takes 128 KB),
// fewer when J is short
unsigned cg_rows_grid(int64_t p) {
    int64_t b = (p + 4 * CGR_WPB - 1) / (4 * CGR_WPB);
    const int64_t ncu = device_cu_count();
    if (b > ncu) b = ncu;
    if (b > 1024) b = 1024;                  // the partials' buffer holds 1024
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_cg_rows(const SegPlan& F, const int2* jrow, int64_t p, int64_t q, const double* v,
                    double* w, double* Pw, const Scalars* sc, hipStream_t s) {
    const unsigned g = cg_rows_grid(p);
    const int32_t H = (int32_t)(q < CGR_HEAD ? q : CGR_HEAD);
    if (F.val_f64)
        SSN_LAUNCH((k_cg_rows<double>), dim3(g), dim3(CGR_THREADS), 0, s, jrow, F.idx,
                   (const double*)F.val, p, v, H, w, Pw, sc);
    else
        SSN_LAUNCH((k_cg_rows<float>), dim3(g), dim3(CGR_THREADS), 0, s, jrow, F.idx,
                   (const float*)F.val, p, v, H, w, Pw, sc);
}

// --------------------------------------------------------------- X_J^T w
// four consecutive values from a 16-byte aligned address
__device__ __forceinline__ void load4(const float* p, double (&a)[4]) {
    const float4 u = *reinterpret_cast<const float4*>(p);
    a[0] = u.x; a[1] = u.y; a[2] = u.z; a[3] = u.w;
}
__device__ __forceinline__ void load4(const double* p, double (&a)[4]) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 u = q[0], v = q[1];
    a[0] = u.x; a[1] = u.y; a[2] = v.x; a[3] = v.y;
}
static_assert(KE == 4, "load4 covers one lane chunk");
// out[c] = sum over compact entries of column c of coef, coef =
//   MODE 0: val * w[rank];  MODE 1: val;  MODE 2: val^2.
// Carry slots per chunk: [0] the run that ends here coming from the left,
// [1] the run that leaves to the right (possibly having come from the left).
template <typename V, int MODE>
__global__ __launch_bounds__(SSN_BLOCK) void k_keyed_tr(const int32_t* __restrict__ jr,
                                                        const int32_t* __restrict__ jc,
                                                        const V* __restrict__ jv, int64_t nnzj,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ carry,
                                                        double* __restrict__ out,
                                                        const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t ch = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    const int64_t cb = ch * KCH;
    if (cb >= nnzj) return;
    const int64_t ce = cb + KCH < nnzj ? cb + KCH : nnzj;
    const int64_t k0 = cb + (int64_t)lane * KE;
    const int64_t k1 = k0 + KE < ce ? k0 + KE : ce;
    const bool active = k0 < ce;
    const int32_t kfirst = jc[cb], klast = jc[ce - 1];
    const bool left_in = cb > 0 && jc[cb - 1] == kfirst;       // first run continues from the left
    const bool right_out = ce < nnzj && jc[ce] == klast;        // last run continues to the right
    const int32_t INF = 0x7fffffff;
    int32_t F = INF, Lt = INF;
    double fsum = 0.0, lsum = 0.0;
    if (active) {
        int32_t keys[KE];
        double cf[KE];
        if (k1 - k0 == KE) {
            // a full lane chunk (16-byte aligned: k0 is a multiple of 4)
            const int4 kc = *reinterpret_cast<const int4*>(jc + k0);
            keys[0] = kc.x; keys[1] = kc.y; keys[2] = kc.z; keys[3] = kc.w;
            double a[KE];
            load4(jv + k0, a);
            if (MODE == 0) {
                const int4 rr = *reinterpret_cast<const int4*>(jr + k0);
                cf[0] = a[0] * w[rr.x];
                cf[1] = a[1] * w[rr.y];
                cf[2] = a[2] * w[rr.z];
                cf[3] = a[3] * w[rr.w];
            } else {
#pragma unroll
                for (int e = 0; e < KE; ++e) cf[e] = MODE == 1 ? a[e] : a[e] * a[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < KE; ++e) {
                const int64_t k = k0 + e;
                if (k < k1) {
                    keys[e] = jc[k];
                    const double a = (double)jv[k];
                    if (MODE == 0) cf[e] = a * w[jr[k]];
                    else if (MODE == 1) cf[e] = a;
                    else cf[e] = a * a;
                } else {
                    keys[e] = -1;
                    cf[e] = 0.0;
                }
            }
        }
        int32_t key = keys[0];
        F = key;
        double cur = 0.0;
        bool first_closed = false;
#pragma unroll
        for (int e = 0; e < KE; ++e) {
            if (keys[e] < 0) break;
            if (keys[e] != key) {
                if (!first_closed) {
                    first_closed = true;
                    fsum = cur;
                } else {
                    out[key] = cur;                 // run strictly inside the lane: complete
                }
                key = keys[e];
                cur = 0.0;
            }
            cur += cf[e];
        }
        Lt = key;
        lsum = cur;
        if (!first_closed) F = Lt;
    }
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
    const bool has_next = lane + 1 < SSN_WAVE && (k0 + KE) < ce;
    auto emit = [&](int32_t c, double v) {
        const bool l = (c == kfirst) && left_in;
        const bool r = (c == klast) && right_out;
        if (r) carry[ch * 2 + 1] = v;
        else if (l) carry[ch * 2 + 0] = v;
        else out[c] = v;
    };
    if (active) {
        if (F < Lt) {
            double tot = fsum;
            if (lane > 0 && Lt_prev == F) tot += S_prev;
            emit(F, tot);
        }
        if (!has_next || F_next != Lt) emit(Lt, S);
    }
}

// ---- the border-crossing runs, listed once per compact copy
// flag[ch] = 1 where a border-crossing run starts: the chunk's last run
// leaves to the right without having come from the left (a chunk holding
// one column that both enters and leaves is passed through, not a start).
// The chunk count comes from the device-side entry count.
__global__ void k_fix_flags(const int32_t* __restrict__ jc, const long long* __restrict__ nnzj_dev,
                            int64_t nchmax, uint8_t* __restrict__ flag) {
    const int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= nchmax) return;
    const int64_t nnzj = *nnzj_dev;
    const int64_t cb = ch * KCH;
    uint8_t f = 0;
    if (cb < nnzj) {
        const int64_t ce = cb + KCH < nnzj ? cb + KCH : nnzj;
        const int32_t K = jc[ce - 1];
        const bool right_out = ce < nnzj && jc[ce] == K;
        const bool left_in = cb > 0 && jc[cb] == K && jc[cb - 1] == K;
        f = right_out && !left_in;
    }
    flag[ch] = f;
}
// For listed run i (starting in chunk list[i]): the chunk where it ends and
// its column.  One wave per run.
__global__ __launch_bounds__(SSN_BLOCK) void k_fix_ends(const int32_t* __restrict__ jc,
                                                        int64_t nnzj, int64_t nch,
                                                        const int32_t* __restrict__ list,
                                                        int64_t nfix, int32_t* __restrict__ fend,
                                                        int32_t* __restrict__ fcol) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t i = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (i >= nfix) return;
    const int64_t ch = list[i];
    const int64_t ce = (ch + 1) * KCH < nnzj ? (ch + 1) * KCH : nnzj;
    const int32_t K = jc[ce - 1];
    int64_t end = nch - 1;
    for (int64_t base = ch + 1; base < nch; base += SSN_WAVE) {
        const int64_t c2 = base + lane;
        bool pass = false;
        const bool valid = c2 < nch;
        if (valid) {
            const int64_t b2 = c2 * KCH;
            const int64_t e2 = b2 + KCH < nnzj ? b2 + KCH : nnzj;
            pass = jc[b2] == K && jc[e2 - 1] == K && e2 < nnzj && jc[e2] == K;
        }
        const unsigned long long stop = __ballot(valid && !pass);
        if (stop) {
            end = base + __ffsll((long long)stop) - 1;
            break;
        }
    }
    if (lane == 0) {
        fend[i] = (int32_t)end;
        fcol[i] = K;
    }
}
// out[fcol[i]] = the run's carries: slot 1 of its first chunk and of every
// chunk it passes through, slot 0 of the chunk where it ends.  One wave per
// listed run.
__global__ __launch_bounds__(SSN_BLOCK) void k_keyed_fix_list(const int32_t* __restrict__ list,
                                                              const int32_t* __restrict__ fend,
                                                              const int32_t* __restrict__ fcol,
                                                              int64_t nfix,
                                                              const double* __restrict__ carry,
                                                              double* __restrict__ out,
                                                              const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int lane = threadIdx.x & (SSN_WAVE - 1);
    const int64_t i = (int64_t)blockIdx.x * SSN_WAVES_PER_BLOCK + threadIdx.x / SSN_WAVE;
    if (i >= nfix) return;
    const int64_t c0 = list[i], c1 = fend[i];
    double v = 0.0;
    for (int64_t c = c0 + 1 + lane; c <= c1; c += SSN_WAVE) v += carry[c * 2 + (c < c1 ? 1 : 0)];
    v = wave_sum(v);
    if (lane == 0) out[fcol[i]] = carry[c0 * 2 + 1] + v;
}

int64_t keyed_chunks(int64_t nnz) { return (nnz + KCH - 1) / KCH; }

void launch_fix_flags(const int32_t* jc, const long long* nnzj_dev, int64_t nchmax, uint8_t* flag,
                      hipStream_t s) {
    if (nchmax <= 0) return;
    SSN_LAUNCH(k_fix_flags, dim3((unsigned)((nchmax + 255) / 256)), dim3(256), 0, s, jc,
                       nnzj_dev, nchmax, flag);
}

void launch_fix_ends(const int32_t* jc, int64_t nnzj, KeyedFix& fx, hipStream_t s) {
    if (fx.nfix <= 0) return;
    const unsigned nb = (unsigned)((fx.nfix + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
    SSN_LAUNCH(k_fix_ends, dim3(nb), dim3(SSN_BLOCK), 0, s, jc, nnzj, keyed_chunks(nnzj),
                       fx.list, fx.nfix, fx.fend, fx.fcol);
}

void launch_keyed_tr(int mode, const int32_t* jr, const int32_t* jc, const void* jv, int val_f64,
                     int64_t nnzj, const double* w, double* carry, double* out, int64_t q,
                     const KeyedFix& fx, hipStream_t s, bool zero_out, const int* skip) {
    if (zero_out) launch_fill(out, 0.0, q, s);
    if (nnzj <= 0) return;
    const int64_t nch = (nnzj + KCH - 1) / KCH;
    const unsigned nb = (unsigned)((nch + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
#define KT(V, M) SSN_LAUNCH((k_keyed_tr<V, M>), dim3(nb), dim3(SSN_BLOCK), 0, s, jr, jc, \
                                    (const V*)jv, nnzj, w, carry, out, skip)
    if (val_f64) {
        if (mode == 0) KT(double, 0); else if (mode == 1) KT(double, 1); else KT(double, 2);
    } else {
        if (mode == 0) KT(float, 0); else if (mode == 1) KT(float, 1); else KT(float, 2);
    }
#undef KT
    if (fx.nfix > 0) {
        const unsigned nf = (unsigned)((fx.nfix + SSN_WAVES_PER_BLOCK - 1) / SSN_WAVES_PER_BLOCK);
        SSN_LAUNCH(k_keyed_fix_list, dim3(nf), dim3(SSN_BLOCK), 0, s, fx.list, fx.fend,
                           fx.fcol, fx.nfix, carry, out, skip);
    }
}

// --------------------------------------------------------------- step
// Scalars from the partials: rz = r.z, rr = r.r (previous step), pp = p.p,
// sp = s.p (direction kernel), ww = |X_J p|^2 (row kernel).  Then
// pAp = pp + sigma (ww - sp^2/p), alpha = rz / pAp, and with
// Ap = p + sigma (t - (sp/p) s):  x += alpha p, r -= alpha Ap, z = r / diag.
// Once rr <= tol2 (or pAp <= 0) the step leaves x unchanged and passes the
// partials through, so later iterations stay put.
__global__ __launch_bounds__(SSN_BLOCK) void k_cg_step(
    double* __restrict__ x, double* __restrict__ r, const double* __restrict__ pd,
    const double* __restrict__ t, const double* __restrict__ sv, const double* __restrict__ diag,
    double* __restrict__ z, int64_t q, double sigma, double inv_p, const double* __restrict__ Pw,
    int nbw, const double* __restrict__ Pdir, const double* __restrict__ Pold,
    double* __restrict__ Pnew, double tol2, const Scalars* __restrict__ sc) {
    __shared__ double sh[5 * SSN_WAVES_PER_BLOCK];
    if (sc->cg_done) return;                   // converged in an earlier iteration
    const int nbq = gridDim.x;
    // the five partial sums, every load issued before the one block exchange
    double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nbq; b += blockDim.x) {
        red[0] += Pold[2 * b];
        red[1] += Pold[2 * b + 1];
        red[2] += Pdir[2 * b];
        red[3] += Pdir[2 * b + 1];
    }
    for (int b = threadIdx.x; b < nbw; b += blockDim.x) red[4] += Pw[b];
    block_sum_n<5>(red, sh);
    const double rz = red[0], rr = red[1], pp = red[2], sp = red[3], ww = red[4];
    const double pap = pp + sigma * (ww - sp * sp * inv_p);
    const bool done = !(rr > tol2) || !(pap > 0.0) || !(rz > 0.0);
    if (done) {
        if (threadIdx.x == 0) {
            Pnew[blockIdx.x * 2] = Pold[blockIdx.x * 2];
            Pnew[blockIdx.x * 2 + 1] = 0.0;            // sticky: rr = 0 from now on
        }
        return;
    }
    const double alpha = rz / pap, m = sp * inv_p;
    double a = 0.0, b = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
        const double pj = pd[j];
        const double apj = fma(sigma, t[j] - m * sv[j], pj);
        x[j] = fma(alpha, pj, x[j]);
        const double rj = fma(-alpha, apj, r[j]);
        r[j] = rj;
        const double zj = rj / diag[j];
        z[j] = zj;
        a = fma(rj, zj, a);
        b = fma(rj, rj, b);
    }
    double ab[2] = {a, b};
    block_sum_n<2>(ab, sh);
    if (threadIdx.x == 0) {
        Pnew[blockIdx.x * 2] = ab[0];
        Pnew[blockIdx.x * 2 + 1] = ab[1];
    }
}

// beta = rz_new / rz_old; p = z + beta p; partials (p.p, s.p).  Block 0 also
// publishes rr and the done flag for the host.
__global__ __launch_bounds__(SSN_BLOCK) void k_cg_dir(double* __restrict__ pd,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ sv, int64_t q,
                                                      const double* __restrict__ Pold,
                                                      const double* __restrict__ Pnew,
                                                      double* __restrict__ Pdir, double tol2,
                                                      Scalars* sc, double* __restrict__ tz) {
    __shared__ double sh[3 * SSN_WAVES_PER_BLOCK];
    // converged in an earlier iteration: nothing changes any more (the next
    // CG start clears tz itself)
    if (sc->cg_done) return;
    const int nbq = gridDim.x;
    double red[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nbq; b += blockDim.x) {
        red[0] += Pold[2 * b];
        red[1] += Pnew[2 * b];
        red[2] += Pnew[2 * b + 1];
    }
    block_sum_n<3>(red, sh);
    const double rz_old = red[0], rz_new = red[1], rr_new = red[2];
    const bool done = !(rr_new > tol2);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!sc->cg_done) sc->cg_count += 1;   // this iteration's step did work
        sc->cg_rr = rr_new;
        sc->cg_done = done ? 1 : 0;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (done) {                       // p unchanged; the next step passes through
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride)
            tz[j] = 0.0;
        return;
    }
    const double beta = rz_old > 0.0 ? rz_new / rz_old : 0.0;
    double pp = 0.0, sp = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < q; j += stride) {
        const double pj = fma(beta, pd[j], z[j]);
        pd[j] = pj;
        tz[j] = 0.0;                  // output of the next X_J^T w starts at zero
        pp = fma(pj, pj, pp);
        sp = fma(sv[j], pj, sp);
    }
    double ab[2] = {pp, sp};
    block_sum_n<2>(ab, sh);
    if (threadIdx.x == 0) {
        Pdir[blockIdx.x * 2] = ab[0];
        Pdir[blockIdx.x * 2 + 1] = ab[1];
    }
}

void launch_cg_init(const double* g, const double* diag, const double* sv, int64_t q, double* x,
                    double* r, double* z, double* pd, double* Pst, double* Pdir, hipStream_t s) {
    SSN_LAUNCH(k_cg_init, dim3(qgrid(q)), dim3(SSN_BLOCK), 0, s, g, diag, sv, q, x, r, z, pd,
                       Pst, Pdir);
}
void launch_cg_step(double* x, double* r, const double* pd, const double* t, const double* sv,
                    const double* diag, double* z, int64_t q, double sigma, int64_t p,
                    const double* Pw, int nbw, const double* Pdir, const double* Pold, double* Pnew,
                    double tol2, const Scalars* sc, hipStream_t s) {
    SSN_LAUNCH(k_cg_step, dim3(qgrid(q)), dim3(SSN_BLOCK), 0, s, x, r, pd, t, sv, diag, z, q,
                       sigma, p > 0 ? 1.0 / (double)p : 0.0, Pw, nbw, Pdir, Pold, Pnew, tol2, sc);
}
void launch_cg_dir(double* pd, const double* z, const double* sv, int64_t q, const double* Pold,
                   const double* Pnew, double* Pdir, double tol2, Scalars* sc, double* tz,
                   hipStream_t s) {
    SSN_LAUNCH(k_cg_dir, dim3(qgrid(q)), dim3(SSN_BLOCK), 0, s, pd, z, sv, q, Pold, Pnew,
                       Pdir, tol2, sc, tz);
}

// rr and done flag straight after init (one block)
__global__ void k_cg_publish(const double* __restrict__ Pst, int nbq, double tol2, Scalars* sc) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const double rr = red_col(Pst, nbq, 2, 1, sh);
    if (threadIdx.x == 0) {
        sc->cg_rr = rr;
        sc->cg_done = rr > tol2 ? 0 : 1;
        sc->cg_count = 0;
    }
}
void launch_cg_publish(const double* Pst, int64_t q, double tol2, Scalars* sc, hipStream_t s) {
    SSN_LAUNCH(k_cg_publish, dim3(1), dim3(SSN_BLOCK), 0, s, Pst, (int)qgrid(q), tol2, sc);
}

}  // namespace ssn
