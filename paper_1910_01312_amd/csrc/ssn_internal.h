// Internal declarations of the SSsNAL library: device state layouts shared
// between host code and kernels, and the host-side launchers of every
// kernel.  Not part of the public ABI.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ssnalm.h"

namespace ssn {

// Kernel timing (ssnalm_options.profile): while the host times a kernel
// class it installs a sink on its thread, and every launch then goes through
// hipExtLaunchKernelGGL with a start / stop event pair from the sink, which
// the runtime attaches to that dispatch: the pair measures the kernel's own
// execution, without the dispatch latency in front of it.
struct KTimeSink {
    virtual void pair(hipEvent_t* start, hipEvent_t* stop) = 0;
    virtual ~KTimeSink() = default;
};
extern thread_local KTimeSink* g_ktime;

#define SSN_LAUNCH(K, G, B, SH, ST, ...)                                                 \
    do {                                                                                \
        if (::ssn::g_ktime) {                                                           \
            hipEvent_t e0_ = nullptr, e1_ = nullptr;                                    \
            ::ssn::g_ktime->pair(&e0_, &e1_);                                           \
            hipExtLaunchKernelGGL(K, G, B, SH, ST, e0_, e1_, 0, __VA_ARGS__);           \
        } else {                                                                        \
            hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                           \
        }                                                                               \
    } while (0)

// State of one projection onto {y^T x = 0, 0 <= x <= C}: the bracket of the
// multiplier, the running flags and the result.  Lives in device memory.
struct ProjState {
    double lo, hi;        // bracket: g(lo) < 0 <= g(hi), g = -y^T clip(v - lam y)
    double glo, ghi;      // g at the bracket ends (filled by the passes)
    double lam;           // result
    int    done;          // 1 when lam is final
    int    passes;        // multisection passes run
    int    approx;        // 1 if the pass cap ended the search
    int    inside;        // breakpoints strictly inside the last bracket
    int    mode;          // 1: next pass places its points geometrically around hint
    int    pad_;
    double hint;          // multiplier of a nearby projection (warm start)
    long long npos;       // number of y_i = +1
    double gbase;         // general form: sum of the left constants K_i plus d
};

// Scalars produced by reductions, read back by the host in one copy.
struct Scalars {
    double dh;            // line search: sum of per-component phi increments
    double dist2;         // |x~ - x^k|^2
    double gnorm2;        // |g|^2
    double omega2;        // |omega|^2
    double gd, od, dd;    // g^T d, omega^T d, d^T d
    double res2, x2;      // KKT: |x - Pi(v)|^2, |x|^2
    double cg_rz, cg_pap, cg_rr, cg_alpha, cg_beta, cg_rz_new;
    double mean_w;        // PCG: mean of X_J p over J
    double sumx;          // e^T x
    double hinge;         // KKT: the primal's loss sum at the KKT bias
    double cx;            // c^T x of a returned x (problems with a linear term)
    double aja;           // general form: a_J^T a_J
    double kd0, kd1, kd2; // kernel contexts: a^T g_J, a^T r (Newton matrix), a^T v
    double kres;          // kernel contexts: (Pi r)^T Q_JJ (Pi r) of a CG residual r
    long long km;         // kernel contexts: support size of a product's input
    long long nchg;       // rows of J that changed since the stored Newton factor
    long long p;          // |J|
    long long nnzj;       // nonzeros of the rows in J (sparse input)
    long long nfix;       // chunk-crossing column runs of the compact X_J copy
    long long nsv;        // #{x_i > 0}
    int    chol_fail;     // Cholesky met a non-positive pivot
    int    cg_done;
    int    cg_count;      // CG iterations that changed x since the last start
};

// One-block sums of block-partial columns into scalars (kernels_vec.hip):
// column c goes to p[c] (skipped when null) as a double times scale[c], or
// as a long long when as_ll[c]; nothing is written when *skip is nonzero.
struct ColSumDst {
    void* p[4];
    int as_ll[4];
    double scale[4];
    const int* skip;
};
ColSumDst colsum_dst();
void launch_colsum_fin(const double* part, int nb, int stride, int ncols, const ColSumDst& d,
                       hipStream_t s);

// Dense matvecs ----------------------------------------------------------
void launch_amul_dense(int dtype, const void* X, const int8_t* y, const double* v,
                       double* t, int64_t n, int64_t q, hipStream_t s);
// part[b*q + j] = partial column sums of X^T (y .* z) over row block b
// (z may be null: no coefficient); part2 likewise for X_J^T 1 (mode 1) or
// sum_J X_ij^2 (mode 2) over the mask.  atmul_dense_nblk(n) blocks.
int  atmul_dense_nblk(int64_t n);
void launch_atmul_dense(int dtype, const void* X, const int8_t* y, const double* z,
                        const uint8_t* mask, int64_t n, int64_t q, double* part,
                        double* part2, hipStream_t s, int mask_mode = 1);
// out[j] = (base ? base[j] : 0) + sign * sum_b part[b*q + j]
void launch_reduce_cols(const double* part, int nblk, int64_t q, const double* base,
                        double sign, double* out, hipStream_t s);

// Sparse (merge-path segmented sums) -------------------------------------
struct SegPlan {               // plan of one segmented-sum operator
    int64_t nseg, nnz;         // segments (rows or columns), entries
    int32_t* ptr;              // nseg+1 offsets (device)
    int32_t* idx;              // nnz indices into the input vector (device)
    void*    val;              // nnz values (device), f32 or f64
    int      val_f64;
    int32_t* lane_seg;         // segment holding the first entry of each lane chunk
    int64_t  nlane;            // number of lane chunks
    int64_t  ntile;            // number of wave tiles
    int32_t* tile_first;       // first / last segment of each tile (device)
    int32_t* tile_last;
    double*  carry;            // 2 * ntile partial sums (device)
    int32_t* span_seg;         // segments spanning several tiles, and empty ones
    int32_t* span_t0;          // their first and last tile (t0 > t1: empty)
    int32_t* span_t1;
    int64_t  nspan;
    int64_t  nshort;           // spans [0, nshort) cover at most seg_short_tiles() tiles
};
int seg_entries_per_lane();
int seg_short_tiles();
// out[s] = scale_s * sum_{k in seg s} val[k] * coef(idx[k]); coef(i) =
// vin[i] * (yin ? yin[i] : 1) * (mask ? mask[i] : 1), or mask[i] when vin is
// null; scale_s = (yout ? yout[s] : 1) * (out_mask ? out_mask[s] : 1)
void launch_segsum(const SegPlan& P, const double* vin, const int8_t* yin,
                   const uint8_t* mask, const int8_t* yout, const uint8_t* out_mask,
                   double* out, hipStream_t s);
// row blocks of the CSC copy used by A^T z (1: the plain CSC copy)
int atmul_row_parts(int64_t n, int64_t q, int64_t nnz);
// out[s] = sum_{k in seg s} val[k] vin[idx[k]], with the tiles dealt to
// `parts` XCDs in contiguous parts (block b runs on XCD b % parts)
void launch_segsum_parts(const SegPlan& P, int parts, const double* vin, double* out,
                         hipStream_t s);
// out[s] = sum_{k in seg s} val[k]^2 mask(idx[k])

// Projection ---------------------------------------------------------------
// v_out = (td ? u - alpha_sigma * td : u); initialise the bracket in st.
void launch_proj_init(const double* u, const double* td, double alpha_sigma, double* v_out,
                      const int8_t* y, int64_t n, double C, ProjState* st, double* part,
                      unsigned* counter, hipStream_t s, const ProjState* hint = nullptr);
void launch_proj_pass(const double* v, const int8_t* y, int64_t n, double C, ProjState* st,
                      double* part, unsigned* counter, hipStream_t s);
int  proj_max_passes();
// x = clip(v - lam y), mask = free set; counts p, nsv into sc.
void launch_proj_apply(const double* v, const int8_t* y, int64_t n, double C,
                       const ProjState* st, double* x, uint8_t* mask, Scalars* sc,
                       double* part, unsigned* counter, hipStream_t s);
// line-search finalize: as proj_apply on v = u_base - as*td, plus dh = sum of
// phi increments relative to (u_base, lam_base) and dist2 = |x - xk|^2.
void launch_ls_finalize(const double* v, const double* u_base, const double* td, double as,
                        const int8_t* y, int64_t n, double C, const ProjState* st,
                        const ProjState* st_base, const double* xk, double* x,
                        uint8_t* mask, Scalars* sc, double* part, unsigned* counter,
                        hipStream_t s);
// KKT: v = x - Qx + 1; after projecting v: res2 = |x - Pi(v)|^2, x2 = |x|^2, sumx
void launch_kkt_prepare(const double* x, const double* Qx, double* v, int64_t n, hipStream_t s,
                        const double* lin = nullptr);
// |x - Pi(v)|^2, |x|^2, e^T x (c^T x when lin is given) and the primal's
// loss sum into sc (res2, x2, sumx, hinge); eps-SVR when lin is given
// (svr_n rows of X, tube width eps)
void launch_kkt_finalize(const double* v, const double* x, const double* Qx, const int8_t* y,
                         int64_t n, double C, const ProjState* st, Scalars* sc, double* part,
                         unsigned* counter, hipStream_t s, const double* lin = nullptr,
                         int64_t svr_n = 0, double eps = 0.0);
// ordered compaction of mask into list; total written to *count
int  compact_blocks(int64_t n);
void launch_compact(const uint8_t* mask, int64_t n, int32_t* list, long long* count,
                    int* blk, unsigned* counter, hipStream_t s);

// Vector ops ------------------------------------------------------------------
void launch_dots(int npair, const double* a0, const double* b0, double* r0,
                 const double* a1, const double* b1, double* r1,
                 const double* a2, const double* b2, double* r2,
                 int64_t len, double* part, unsigned* counter, hipStream_t s);
void launch_axpy(double* y, const double* x, double a, int64_t len, hipStream_t s);
void launch_scale_copy(double* y, const double* x, double a, int64_t len, hipStream_t s);
void launch_u_from(const double* xk, const double* aw, double sigma, double* u, int64_t n,
                   hipStream_t s, const double* lin = nullptr);
void launch_sub(const double* a, const double* b, double* out, int64_t len, hipStream_t s);
void launch_mul_y(const double* z, const int8_t* y, double* out, int64_t n, hipStream_t s);
// perm[j] = internal index of original column j; to_internal: dst[perm[j]] =
// src[j], else dst[j] = src[perm[j]]
void launch_permute(const double* src, const int32_t* perm, double* dst, int64_t q, bool to_internal,
                    hipStream_t s);
void launch_fill(double* p, double v, int64_t len, hipStream_t s);
void launch_count_x(const double* x, int64_t n, double C, Scalars* sc, double* part,
                    unsigned* counter, hipStream_t s);

// Newton system --------------------------------------------------------------
// G (q x q, full) = X_J^T X_J over the listed rows; fp64 accumulation
int64_t syrk_part_size(int64_t q, int64_t p);
void launch_syrk_gather(int dtype, const void* X, int64_t q, const int32_t* list,
                        int64_t p, double* G, double* part, int64_t part_cap,
                        hipStream_t s);
// bf16 MFMA variant (fp32 accumulation) for the mixed-precision mode
bool syrk_mfma_supported(int dtype, int64_t q);
int64_t syrk_mfma_part_size(int64_t q, int64_t p);
void launch_syrk_mfma(const void* X, int dtype, int64_t q, const int32_t* list, int64_t p,
                      double* G, float* part, int64_t part_cap, hipStream_t s);
// mixed-precision refinement pieces (kernels_mfma.hip)
unsigned dense_rows_grid(int64_t p);
void launch_dense_rows(int dtype, const void* X, int64_t q, const int32_t* list, int64_t p,
                       const double* v, double* w, double* Pw, hipStream_t s);
void launch_scatter_centered(const int32_t* list, int64_t p, const double* w, const double* Pw,
                             int nbw, const int8_t* y, double* z, hipStream_t s);
void launch_refine_res(const double* g, const double* d, const double* t, double sigma, double* rn,
                       int64_t q, hipStream_t s);
// M = I + sigma (G - s s^T / p)
void launch_form_M(const double* G, const double* sv, double sigma, int64_t p, double* M,
                   int64_t q, hipStream_t s);
// d = -M^{-1} g by Cholesky in one workgroup (q <= chol_small_max())
int  chol_small_max();
void launch_chol_solve_small(const double* M, const double* g, double* d, int64_t q,
                             Scalars* sc, hipStream_t s);
// Blocked Cholesky for larger q (kernels_chol.hip): the factor in place on M
// (lower triangle and its upper mirror), the inverses of the 64 x 64 diagonal
// factors in inv (chol_inv_size(q) doubles); then d = -M^{-1} g from both
int     chol_blocked_max();
int64_t chol_inv_size(int64_t q);
void launch_chol_factor_blocked(double* M, int64_t q, double* inv, Scalars* sc, hipStream_t s);
// D[:, c] = -M^{-1} G[:, c] for k right-hand sides (columns of q doubles), q <= chol_blocked_max()
void launch_chol_solve_factored_multi(const double* M, const double* inv, const double* G, double* D,
                                      int64_t q, int64_t k, hipStream_t s);
// Low-rank (Woodbury) update of the dense Newton step (kernels_lowrank.hip)
int  lowrank_max();
void launch_mask_diff(const uint8_t* a, const uint8_t* b, int64_t n, uint8_t* out, hipStream_t s);
void launch_lr_build(int dtype, const void* X, int64_t q, const int32_t* chg, int nchg, const uint8_t* mask,
                     double sigma, const double* s0, int64_t p0, const double* s1, int64_t p1, double* U,
                     double* wgt, int k, hipStream_t s);
// T = S^{-1} - U^T Zn, then T = P^T L D L^T P in place (perm: P's order)
void launch_lr_factor(const double* U, const double* Zn, int64_t q, int k, const double* wgt, double* Tm,
                      int32_t* perm, Scalars* sc, hipStream_t s);
void launch_lr_apply(const double* U, const double* Zn, int64_t q, int k, const double* LD, const int32_t* perm,
                     const double* d0, double* out, hipStream_t s);
// d = -M^{-1} g from the blocked factor for any q (multi-workgroup solves;
// w: q doubles of scratch for the forward solution)
void launch_chol_solve_blocked(const double* M, const double* inv, const double* g, double* d, int64_t q,
                               double* w, hipStream_t s);
void launch_chol_solve_factored(const double* M, const double* inv, const double* g, double* d,
                                int64_t q, hipStream_t s);

// Sparse products restricted to J (kernels_jcsr.hip) --------------------------
void launch_rank_from_list(const int32_t* list, const long long* pdev, int64_t n, int32_t* rank,
                           const int32_t* rp, int2* jrow, hipStream_t s);
// column-major copy of X_J filtered from the full one (entries: rank, column, value)
// the J mask is turned into bits (jcsc_bits_words(n) words of scratch in
// bits), staged in LDS when it fits (jcsc_bits_fit: n <= 1310720 rows)
int  jcsc_bits_words(int64_t n);
bool jcsc_bits_fit(int64_t n);
// tcv: the (column, value) of every entry of T, ColValF or ColValD by T's
// value type
struct alignas(8) ColValF { int32_t col; float v; };
struct alignas(16) ColValD { int32_t col; int32_t pad; double v; };
// Sliced-ELL copy of the CSR rows (fp32 values) for the forward product:
// rows sorted by decreasing length inside windows of SELL_WINDOW rows, 64
// sorted rows per slice, slice s column-major from cv + ptr[s] (entry k of
// its row l at ptr[s] + 64 k + l), len[s] its padded length (a multiple of
// SELL_PAD), perm[64 s + l] the row's original index (-1 past n).
constexpr int SELL_SLICE = 64;      // rows per slice: one wave, one lane per row
constexpr int SELL_WINDOW = 1024;
constexpr int SELL_PAD = 4;
constexpr int SELL_MAX_LEN = 1024;   // longest row the copy is built for
struct SellPlan {
    int64_t  nslice;           // 0: no copy (the merge-path plan serves A v)
    int64_t* ptr;              // nslice entry offsets (device)
    int32_t* len;              // nslice padded lengths (device)
    int32_t* perm;             // 64 * nslice original row indices (device)
    ColValF* cv;               // padded entries (device)
};
// out[i] = y[i] * sum_k X_ik v[k] over the sliced-ELL copy
void launch_sell_amul(const SellPlan& P, const double* v, int64_t q, const int8_t* y, double* out,
                      hipStream_t s);
void launch_jcsc_build(const SegPlan& T, const void* tcv, const uint8_t* mask, int64_t n,
                       uint32_t* bits,
                       const int32_t* rank, int* tcount, int* toff, long long* total, int32_t* jr,
                       int32_t* jc, void* jv, hipStream_t s);

// Fence-free CG on the compact X_J (kernels_cg.hip) ----------------------------
unsigned cg_rows_grid(int64_t p);
// compute units of the current device (read once per device)
int device_cu_count();
void launch_cg_init(const double* g, const double* diag, const double* sv, int64_t q, double* x,
                    double* r, double* z, double* pd, double* Pst, double* Pdir, hipStream_t s);
void launch_cg_publish(const double* Pst, int64_t q, double tol2, Scalars* sc, hipStream_t s);
// w[k] = (X_J v)_k for the k-th row of J (entry range jrow[k]); Pw: block sums of w^2
// returns at once when sc->cg_done is set (the CG has converged)
void launch_cg_rows(const SegPlan& F, const int2* jrow, int64_t p, int64_t q, const double* v,
                    double* w, double* Pw, const Scalars* sc, hipStream_t s);
// The runs of equal column that cross chunk borders of a compact copy:
// their first chunks (ascending), last chunks and columns; nfix on the host.
struct KeyedFix {
    int32_t* list;
    int32_t* fend;
    int32_t* fcol;
    int64_t nfix;
};
int64_t keyed_chunks(int64_t nnz);
// flag[ch] = 1 where a crossing run starts (chunks of the copy with
// *nnzj_dev entries; nchmax >= its chunk count); compact the flags into
// KeyedFix::list, then launch_fix_ends fills fend/fcol.
void launch_fix_flags(const int32_t* jc, const long long* nnzj_dev, int64_t nchmax, uint8_t* flag,
                      hipStream_t s);
void launch_fix_ends(const int32_t* jc, int64_t nnzj, KeyedFix& fx, hipStream_t s);
// out = X_J^T coef over the compact copy (mode 0: coef = w[rank], 1: values,
// 2: squared values); the crossing runs fx are summed by a second kernel
void launch_keyed_tr(int mode, const int32_t* jr, const int32_t* jc, const void* jv, int val_f64,
                     int64_t nnzj, const double* w, double* carry, double* out, int64_t q,
                     const KeyedFix& fx, hipStream_t s, bool zero_out = true,
                     const int* skip = nullptr);   // skip: no work while *skip is nonzero
void launch_cg_step(double* x, double* r, const double* pd, const double* t, const double* sv,
                    const double* diag, double* z, int64_t q, double sigma, int64_t p,
                    const double* Pw, int nbw, const double* Pdir, const double* Pold, double* Pnew,
                    double tol2, const Scalars* sc, hipStream_t s);
void launch_cg_dir(double* pd, const double* z, const double* sv, int64_t q, const double* Pold,
                   const double* Pnew, double* Pdir, double tol2, Scalars* sc, double* tz,
                   hipStream_t s);

// PCG pieces -------------------------------------------------------------------
void launch_jacobi_diag(const double* sq, const double* sv, double sigma, int64_t p,
                        double* diag, int64_t q, hipStream_t s);
void launch_pcg_init(const double* g, const double* diag, double* x, double* r, double* z, double* pd,
                     int64_t q, double tol2, Scalars* sc, double* part, unsigned* counter,
                     hipStream_t s);
void launch_pcg_pap(const double* pd, const double* Ap, int64_t q, Scalars* sc, double* part,
                    unsigned* counter, hipStream_t s);
void launch_pcg_step(double* x, double* r, double* pd, const double* Ap, const double* diag,
                     double* z, int64_t q, Scalars* sc, double tol2, double* part,
                     unsigned* counter, hipStream_t s);
void launch_pcg_dir(double* pd, const double* z, int64_t q, Scalars* sc, hipStream_t s);
void launch_masked_mean(const double* t, const int8_t* y, const uint8_t* mask, int64_t n,
                        int64_t p, double* mean_out, double* part, unsigned* counter,
                        hipStream_t s);
void launch_masked_center_t(double* t, const int8_t* y, const uint8_t* mask, int64_t n,
                            const double* mean, double* z, hipStream_t s);
void launch_mop_finish(const double* pd, const double* z, double sigma, const double* unused1,
                       const double* unused2, int64_t unused3, double* Ap, int64_t q,
                       hipStream_t s);

// Batched solve (kernels_batch.hip) ------------------------------------------------
constexpr int BRPI = 4096;     // rows per work item
constexpr int BQMAX = 128;     // largest q of a batched solve
int batch_rows_per_item();
int batch_qmax();
int batch_gram_items_max(int64_t n);   // Gram items of a problem with n rows (upper bound)
int batch_proj_max_passes();

struct BProb {                 // static description of problem k (device)
    const void*   X;           // n x q row-major
    const int8_t* y;           // n labels
    int64_t n;
    int64_t off;               // first row of problem k in the concatenated n-vectors
    double  C;
    int     item0, nitem;      // its items in the static item list
};
struct BPar {                  // per-phase parameters of problem k (uploaded by the host)
    int    active;             // 1: problem k takes part in the launches
    int    pad_;
    double sigma, alpha;
};
enum {                         // per-problem scalar slots (BState::r)
    BS_GN2 = 0, BS_OM2, BS_GD, BS_OD, BS_DD,
    BS_DH, BS_DIST2, BS_PF, BS_NSV,
    BS_RES2, BS_X2, BS_SUMX, BS_HINGE,
    BS_FSUMX, BS_FNSV, BS_FP, BS_W2,
    BS_NR
};
struct BState {                // per-problem device results, read back by the host
    ProjState ps[3];           // 0: line-search base, 1: trial, 2: KKT
    double    r[BS_NR];
    long long p;               // |J| of the last compaction
    int       chol_fail, pad_;
};
struct BArgs {                 // what every batched kernel receives
    const BProb* prob;
    const BPar*  par;
    BState*      bs;
    int4*        wl;           // active work list: (problem, first row, end row, 0)
    int*         wl_n;
    int*         ioff;         // per problem: first item in wl, item count
    int*         icnt;
    int          q, nprob;
};
struct BLaunch {
    BArgs  A;
    int    dtype, vec, unr, grid, ggrid;
    double *part, *part2;      // item partials (max(q, 65) doubles per item)
    int    *ipart, *ipart2;    // item partials (66 ints per item), item offsets
    int4*  gwl;                // Gram work list and its per-problem offsets / counts
    int*   gwl_n;
    int    *goff, *gcnt;
    double* gpart;             // q*q doubles per Gram item
    hipStream_t s;
};
void lb_setup_attributes();
void lb_build_wl(const BLaunch& L, const int4* items);
void lb_amul(const BLaunch& L, const double* V, double* t);
void lb_atmul(const BLaunch& L, const double* z, const uint8_t* mask, const double* base,
              double sign, double* out, double* out2);
void lb_elem(const BLaunch& L, int mode, const double* a, const double* b, double* o);
void lb_accept(const BLaunch& L, double* om, const double* d, double* aw, const double* td,
               double* u, const double* ut, double* xt, const double* xtt, uint8_t* jm,
               const uint8_t* jmt);
void lb_qvec(const BLaunch& L, int mode, const double* a, const double* b, double* o);
void lb_qdots(const BLaunch& L, int npair, const double* a0, const double* b0, const double* a1,
              const double* b1, const double* a2, const double* b2, int f0);
void lb_proj_init(const BLaunch& L, const double* u, const double* td, double* vout, int w,
                  int use_hint);
void lb_proj_passes(const BLaunch& L, const double* v, int w, int npass);
void lb_ls_fin(const BLaunch& L, const double* v, const double* ubase, const double* td, int w,
               int wb, const double* xk, double* x, uint8_t* mask);
void lb_kkt_fin(const BLaunch& L, const double* v, const double* x, const double* Qx, int w);
void lb_count(const BLaunch& L, const double* x);
void lb_compact(const BLaunch& L, const uint8_t* mask, int32_t* list);
void lb_newton(const BLaunch& L, const int32_t* list, const double* sv, const double* g, double* d,
               double* M);

// Warm-start network (kernels_mlp.hip) -------------------------------------------
constexpr int MLP_IN = 66, MLP_HID = 256, MLP_OUT = 4;
int  mlp_splits(int64_t n);
void launch_mlp_forward(const float* th, const float* Z, int64_t n, float* work, float* O,
                        float* out, hipStream_t s);
void launch_mlp_backward(const float* th, const float* Z, int64_t n, const float* work,
                         const float* out, const int32_t* st, const float* tg, float w,
                         float* grad, float* loss, float* scratch, hipStream_t s);
void launch_adam(float* th, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                 float b2, float eps, int step, hipStream_t s);
void launch_class_sums(const double* aw, const int8_t* y, int64_t n, double* part, int nb,
                       hipStream_t s);
void launch_ws_features(int dtype, const void* X, const int8_t* y, int64_t n, int64_t q,
                        const float* R, const double* aw, double b1, float lognc, float* Z,
                        hipStream_t s);
void launch_ws_x0(const float* out, int64_t n, double C, double* x0, hipStream_t s);
void launch_ws_labels(const double* x, int64_t n, double C, int32_t* status, float* target,
                      hipStream_t s);
void launch_gather_rows(int dtype, const void* X, const int8_t* y, const int32_t* list, int64_t m,
                        int64_t q, void* Xk, int8_t* yk, hipStream_t s);
void launch_scatter(const int32_t* list, int64_t m, const double* xk, double* x, hipStream_t s);
int  p0_hist_bins();
void launch_p0_hist(const float* out, int64_t n, unsigned* hist, hipStream_t s);
void launch_ws_keep_bin(const float* out, int64_t n, int cut, uint8_t* keep, hipStream_t s);
void launch_gather_vec(const double* x, const int32_t* list, int64_t m, double* xk, hipStream_t s);
void launch_ws_violators(const double* aw, const int8_t* y, int64_t n, double b, uint8_t* keep,
                         hipStream_t s);

// error reporting shared by the host files
ssnalm_status set_error(ssnalm_status st, const char* fmt, ...);

// RBF feature maps (kernels_features.hip) ----------------------------------
// Z (n x 2N) = cos / sin pairs of X W^T, scaled by 1/sqrt(N); z_f64: Z is
// fp64, else fp32.
void launch_rff(int dtype, const void* X, int64_t n, int64_t q, const double* W, int64_t N, void* Z,
                int z_f64, hipStream_t s);
// out[i] = |row rows[i] (or i) of X|^2
void launch_row_norms(int dtype, const void* X, const int32_t* rows, int64_t n, int64_t q,
                      double* out, hipStream_t s);
// K (na x r) of the RBF kernel between rows arows (or all) and the landmarks,
// + shift on the diagonal when arows is given (the landmark block)
// Q_ij = y_i y_j k(x_i, x_j) (rbf: exp(-|x_i - x_j|^2 / (2 alpha)); else
// x_i^T x_j), n x n with row stride ld (a multiple of 32, zero padding).
void launch_kernel_q(int dtype, const void* X, int64_t n, int64_t q, const double* norms,
                     const int8_t* y, int rbf, double alpha, double* Q, int64_t ld, hipStream_t s);
// Kernel-context products (kernels_kernel.hip)
constexpr int kQcolsMaxChunks = 256;
void launch_nz_mask(const double* v, int64_t n, uint8_t* mask, hipStream_t s);
int  qcols_chunks(int64_t n, int64_t m);
// part[c * n + j] (c < nchunk) = partial sums of coef_k Q[list_k][j] over the m listed rows
void launch_qcols(const double* Q, int64_t n, int64_t ld, const int32_t* list, int64_t m, const double* v,
                  int by_row, double* part, int nchunk, hipStream_t s);
void launch_qjj_mv(const double* Q, int64_t ld, const int32_t* J, int64_t p, const double* v, double* out,
                   hipStream_t s);
void launch_qjj_form(const double* Q, int64_t ld, const int32_t* J, int64_t p, const double* aJ,
                     const double* r, const double* rho, double sigma, double* M, hipStream_t s);
void launch_qjj_diag(const double* Q, int64_t ld, const int32_t* J, int64_t p, const double* aJ,
                     const double* r, const double* rho, double sigma, double* diag, hipStream_t s);
void launch_kgather(const int32_t* J, int64_t p, const int8_t* y, const double* g, double* aJ, double* gJ,
                    hipStream_t s);
void launch_kcenter(const double* u, const double* aJ, const double* dot, int64_t p, double scale,
                    const double* base, double* out, hipStream_t s);
void launch_scatter_add(const int32_t* J, int64_t p, const double* z, double* d, hipStream_t s);
void launch_rbf_block(int dtype, const void* X, int64_t q, const int32_t* arows, int64_t na,
                      const double* anorm, const int32_t* lm, int64_t r, const double* lnorm,
                      double alpha, double shift, double* K, hipStream_t s);
// Zw (n x r, fp64) = K L^{-T} with the blocked Cholesky factor of the
// landmark block (lower triangle of F, diagonal-block inverses in inv)
void launch_nys_solve(const double* K, int64_t n, int64_t r, const double* F, const double* inv,
                      double* Zw, hipStream_t s);
void launch_copy_z(const double* Zw, int64_t count, void* Z, int z_f64, hipStream_t s);

// General form (P): projection onto {l <= x <= u, a^T x = d} and the
// general problem's n-vector steps (kernels_gproj.hip)
struct GBox {
    const double* a;
    const double* l;
    const double* u;
    double d;
};
void launch_gproj_init(const double* u0, const double* td, double as, double* vout, const GBox& box,
                       int64_t n, ProjState* st, double* part, hipStream_t s);
void launch_gproj_pass(const double* v, const GBox& box, int64_t n, ProjState* st, double* part,
                       hipStream_t s);
int  gproj_max_passes();
// x = clip(v - lam a, l, u), J mask, |x - xk|^2 (xk), psi increment (u_base), |J|, #(x > l)
void launch_gfinalize(const double* v, const double* u_base, const double* td, double as,
                      const GBox& box, int64_t n, const ProjState* st, const ProjState* st_base,
                      const double* xk, double* x, uint8_t* mask, Scalars* sc, double* part,
                      hipStream_t s);
void launch_gkkt_finalize(const double* v, const double* x, const double* c, const GBox& box,
                          int64_t n, const ProjState* st, Scalars* sc, double* part, hipStream_t s);
void launch_gcoef(const double* a, const uint8_t* mask, int64_t n, double* zc, Scalars* sc,
                  double* part, hipStream_t s);
void launch_gcount(const double* x, const GBox& box, int64_t n, Scalars* sc, double* part,
                   hipStream_t s);
void launch_form_M_inv(const double* G, const double* sv, double sigma, double inv_den, double* M,
                       int64_t q, hipStream_t s);

// eps-SVR as an instance of (P) (kernels_vec.hip): labels a = [e; -e] and
// c = [eps + y; eps - y] from the targets; B v from X v; the folds giving
// B^T z and B_J^T a_J as products with X; free-list rows mapped into X
void launch_svr_setup(const double* yr, int64_t n, double eps, int8_t* a, double* lin, hipStream_t s);
void launch_svr_expand(double* t, int64_t n, hipStream_t s);
void launch_svr_fold(const double* z, const uint8_t* mask, int64_t n, double* zc, uint8_t* mc,
                     hipStream_t s);
void launch_list_mod(int32_t* list, int64_t p, int64_t n, hipStream_t s);
// NaN / Inf scan of `count` elements of X (device) on the host
ssnalm_status scan_finite(const void* X, int dtype, int64_t count);

}  // namespace ssn
