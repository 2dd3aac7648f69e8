// Host side of the SSsNAL solver and the C ABI (include/ssnalm.h).
//
// Algorithm 1 (outer augmented Lagrangian loop on the restricted dual (D))
// and Algorithm 3 (semismooth Newton on psi, eq. Def_psi) run here; every
// vector operation is a kernel on the context's stream.  The host only
// takes the scalar decisions (inner/outer stopping tests, Armijo verdict),
// reading a small block of device scalars after each Newton step and each
// line-search trial.
//
// State is kept in omega-space, omega = A^T w: Q w = A omega and
// <w, Q w> = |omega|^2 (Section 3.2.4 with L = A), so
//   u     = x^k + sigma (e - A omega)
//   g     = grad psi = omega - A^T Pi(u)
//   M     = I + sigma (X_J^T X_J - s s^T / p),  s = X_J^T 1,  p = |J|
//   x^{k+1} = Pi(u(omega^{k+1}))                     (eq. Def_new_update_xkplus)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ssn_internal.h"


using namespace ssn;

namespace ssn {
thread_local KTimeSink* g_ktime = nullptr;
}

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

static ssnalm_status fail(ssnalm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

namespace ssn {
ssnalm_status set_error(ssnalm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
}  // namespace ssn

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(SSNALM_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                \
    } while (0)

#define STCHK(expr)                          \
    do {                                     \
        ssnalm_status s_ = (expr);           \
        if (s_ < 0) return s_;               \
    } while (0)

// ---------------------------------------------------------------- context
struct DevState {
    ProjState ps[4];    // 0/1: base and trial of the line search (swapped), 2: KKT, 3: ops
    Scalars sc;
};

struct ssnalm_ctx {
    // problem
    int kind = 0, dtype = 0;
    int64_t n = 0, q = 0, nnz = 0;
    const void* X = nullptr;
    const int8_t* y = nullptr;
    double C = 1.0, tol = 1e-6;
    ssnalm_options opt{};
    hipStream_t st = nullptr;        // the context's own stream (default priority)
    hipStream_t ust = nullptr;       // the caller's stream: work is ordered after / before it
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int device = 0;
    // sparse operator plans (forward on CSR rows, transpose on CSC columns)
    SegPlan fwd{}, tr{};
    SellPlan sell{};                 // sliced-ELL rows for A v (fp32 values; nslice 0: none)
    int32_t* qperm = nullptr;        // CSR: internal index of each original column (null: identity)
    double *qin = nullptr, *qout = nullptr;   // q-vectors crossing the boundary, relabelled
    SegPlan trb{};                   // CSC cut into row blocks (segment = block * q + column)
    int trb_parts = 1;               // row blocks of trb (1: trb unused)
    double* qparts = nullptr;        // trb_parts * q per-block column sums
    std::vector<void*> owned;
    // n-vectors
    double *xk = nullptr, *aw = nullptr, *u = nullptr, *ut = nullptr, *td = nullptr;
    double *xt = nullptr, *xtt = nullptr, *nv = nullptr, *nv2 = nullptr;
    uint8_t *jm = nullptr, *jmt = nullptr;
    int32_t* jlist = nullptr;
    // compact column-major copy of X_J (sparse PCG), rebuilt per Newton step
    int32_t *jrank = nullptr, *jr = nullptr, *jc = nullptr;
    int2* jrow = nullptr;            // entry range of each row of J (sparse input)
    uint32_t* jbits = nullptr;       // the J mask as bits (sparse input)
    void* tcv = nullptr;             // (column, value) of every entry of the CSC copy (sparse input)
    void* jv = nullptr;
    int *tcount = nullptr, *toff = nullptr;
    double *wJ = nullptr, *kcarry = nullptr, *cgpart = nullptr;
    int64_t nchmax = 0;              // chunks of the largest compact X_J copy
    uint8_t* fixflag = nullptr;      // per chunk: a crossing run starts here
    int* fixblk = nullptr;           // compaction scratch for fixflag
    KeyedFix fix{};                  // the crossing runs of the current copy
    double* zJ = nullptr;            // n-vector, nonzero on J only (mixed refinement)
    double* yz = nullptr;            // n-vector y .* z for the sparse A^T z
    bool mixed = false;              // bf16 SYRK + refinement
    // eps-SVR (ssnalm_create_svr): n = 2 nphys variables [x; z] over the
    // nphys rows of X, B = [X; -X] = diag(a) [X; X] with a = y (the labels
    // array), linear term c = lin (null: the C-SVC's c = -e)
    bool svr = false;
    int64_t nphys = 0;
    double svr_eps = 0.0;
    const double* lin = nullptr;
    int8_t* yphys = nullptr;         // nphys ones: plain products with X
    double* zc = nullptr;            // z_top - z_bot (nphys)
    uint8_t* mc = nullptr;           // mask_top + mask_bot (nphys)
    // general form (ssnalm_create_general): a, l, u, d of the constraints,
    // c = lin; the rows of X are B's rows (y holds ones)
    bool gen = false;
    GBox gbox{};
    bool zero_feasible = true;       // x = 0 satisfies the constraints
    double* gzc = nullptr;           // a_i [i in J], the coefficients of s = B_J^T a_J
    // kernel C-SVC (ssnalm_create_kernel): the resident Q (n x n, row stride
    // kld), the w-space n-vectors and the p-space Newton buffers
    bool kern = false;
    double* Qk = nullptr;
    int64_t kld = 0;
    double *kw = nullptr, *ks = nullptr, *kqs = nullptr, *kd = nullptr;
    uint8_t* knz = nullptr;          // nonzero mask of a product's input
    int32_t* klist = nullptr;        // its support, compacted
    double *kaJ = nullptr, *kgJ = nullptr, *kr = nullptr, *krhs = nullptr, *kv = nullptr,
           *kz = nullptr;
    double *kcx = nullptr, *kcr = nullptr, *kcz = nullptr, *kcp = nullptr, *kcap = nullptr,
           *kdiag = nullptr, *kt1 = nullptr, *kt2 = nullptr;
    double* kpart = nullptr;         // kQcolsMaxChunks x n partial rows
    int64_t kchol = 0;               // largest p solved by Cholesky
    int refine_total = 0;
    // low-rank updates of the dense Newton factor (kernels_lowrank.hip): the
    // factor in M / linv is that of (lr_sigma, the J mask jm0, s0v, lr_p0)
    bool lr_valid = false;
    double lr_sigma = 0.0;
    int64_t lr_p0 = 0;
    int lr_k = 0;                    // rank of the update in force for this step (0: fresh factor)
    int lowrank_steps = 0;
    uint8_t *jm0 = nullptr, *chg_mask = nullptr;
    int32_t *chg_list = nullptr, *lr_perm = nullptr;
    double *s0v = nullptr, *lrU = nullptr, *lrZ = nullptr, *lrW = nullptr, *lrT = nullptr;
    // q-vectors
    double *om = nullptr, *g = nullptr, *sv = nullptr, *sq = nullptr, *d = nullptr;
    double *qv = nullptr, *qv2 = nullptr;
    double *cg_x = nullptr, *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_ap = nullptr,
           *diag = nullptr;
    // q x q
    double *G = nullptr, *M = nullptr;
    double* linv = nullptr;          // inverses of the diagonal factors (blocked Cholesky)
    // reduction scratch
    double *part = nullptr, *part2 = nullptr;
    int64_t part_cap = 0;
    double* spart = nullptr;         // small partials (<= 4 * 1024 doubles)
    float* mpart = nullptr;          // MFMA SYRK partials
    int64_t mpart_cap = 0;
    int* blk = nullptr;
    unsigned* counters = nullptr;    // one per reduction site
    DevState* ds = nullptr;          // device scalars
    DevState* hs = nullptr;          // pinned host mirror
    int base = 0;                    // index of the accepted projection state (0/1)
    int chol_max = 0;
    bool use_chol = true;
    // statistics of the current solve
    int proj_passes = 0;
    int proj_capped = 0;             // projections that ended at the pass cap
    long long last_nsv = -1;         // support rows of the current x~ (for byte counts)
    // kernel profiling (opt.profile): HIP event pairs around the hot launches
    // one timed kernel: its event pair; `first` marks the first kernel of a
    // class launch, which carries the launch's bytes and flops
    struct Pending { int cls; hipEvent_t a, b; double bytes, flops; int cg_iter; bool first; };
    int cg_iter = -1;                // CG iteration being launched (-1: outside a CG solve)
    struct Sink : KTimeSink {
        ssnalm_ctx* c = nullptr;
        int cls = 0;
        size_t group = 0;            // index in pend of the class launch's first kernel
        void pair(hipEvent_t* start, hipEvent_t* stop) override;
    } sink;
    std::vector<hipEvent_t> ev_free;
    std::vector<Pending> pend;
    ssnalm_kstat kst[SSNALM_K_COUNT] = {};
};

// Orders the context's stream after the caller's stream on entry to an ABI
// call and the caller's stream after the context's stream on exit.
struct StreamScope {
    ssnalm_ctx* c;
    explicit StreamScope(ssnalm_ctx* c_) : c(c_) {
        if (c->ev_in) {
            (void)hipEventRecord(c->ev_in, c->ust);
            (void)hipStreamWaitEvent(c->st, c->ev_in, 0);
        }
    }
    ~StreamScope() {
        if (c->ev_out) {
            (void)hipEventRecord(c->ev_out, c->st);
            (void)hipStreamWaitEvent(c->ust, c->ev_out, 0);
        }
    }
};

enum { CNT_PROJ_INIT = 0, CNT_PROJ_PASS, CNT_APPLY, CNT_LS, CNT_KKT, CNT_CMP, CNT_DOTS, CNT_DOTS2,
       CNT_MEAN, CNT_PCG, CNT_PCG2, CNT_PCG3, CNT_N };

template <typename T>
static ssnalm_status dalloc(ssnalm_ctx* c, T** p, int64_t count) {
    void* q = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(SSNALM_E_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    c->owned.push_back(q);
    *p = (T*)q;
    return SSNALM_OK;
}

static ssnalm_status sync_state(ssnalm_ctx* c) {
    HIPCHK(hipMemcpyAsync(c->hs, c->ds, sizeof(DevState), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    c->last_nsv = c->hs->sc.nsv;
    return SSNALM_OK;
}

// ---------------------------------------------------------------- profiling
static hipEvent_t ev_get(ssnalm_ctx* c) {
    if (c->ev_free.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
}
// After a CG solve whose first `worked` iterations changed x: launches of
// its later iterations passed through (the kernels saw the converged flag)
// and are dropped from the statistics, so a class's bytes and time cover
// only launches that did the work counted in their bytes.
static void prof_drop_idle_cg(ssnalm_ctx* c, int worked) {
    std::vector<ssnalm_ctx::Pending> keep;
    keep.reserve(c->pend.size());
    for (auto& p : c->pend) {
        if (p.cg_iter >= worked) {
            if (p.a) c->ev_free.push_back(p.a);
            if (p.b) c->ev_free.push_back(p.b);
        } else {
            p.cg_iter = -1;
            keep.push_back(p);
        }
    }
    c->pend.swap(keep);
}
// A class launch's time is the sum of its kernels' execution times (each
// kernel bracketed by its own dispatch-attached event pair); gaps between
// the kernels are not counted.
static void prof_harvest(ssnalm_ctx* c) {
    for (auto& p : c->pend) {
        float ms = 0.f;
        if (p.a && p.b && hipEventSynchronize(p.b) == hipSuccess &&
            hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ssnalm_kstat& k = c->kst[p.cls];
            if (p.first) k.launches += 1;
            k.seconds += 1e-3 * (double)ms;
            k.bytes += p.bytes;
            k.flops += p.flops;
        }
        if (p.a) c->ev_free.push_back(p.a);
        if (p.b) c->ev_free.push_back(p.b);
    }
    c->pend.clear();
}
void ssnalm_ctx::Sink::pair(hipEvent_t* start, hipEvent_t* stop) {
    *start = ev_get(c);
    *stop = ev_get(c);
    c->pend.push_back({cls, *start, *stop, 0.0, 0.0, c->cg_iter, c->pend.size() == group});
}
// opt.profile: 1 times every class; a value > 1 is a mask, bit (k + 1) for class k.
// The CG's classes are sampled, one iteration in eight (iterations 3, 11,
// ...): an event pair costs a few microseconds on a ~15 us kernel, and
// timing all ~1700 launches per solve would slow the solve by ~15%.
static bool prof_on(const ssnalm_ctx* c, int cls) {
    const int p = c->opt.profile;
    const bool on = p == 1 || (p > 1 && ((p >> (cls + 1)) & 1));
    if (on && c->cg_iter >= 0 && (cls == SSNALM_K_AMUL_J || cls == SSNALM_K_ATMUL_J))
        return (c->cg_iter & 7) == 3;
    return on;
}
static void prof_begin(ssnalm_ctx* c, int cls) {
    if (!prof_on(c, cls)) return;
    c->sink.c = c;
    c->sink.cls = cls;
    c->sink.group = c->pend.size();
    g_ktime = &c->sink;
}
static void prof_end(ssnalm_ctx* c, int cls, double bytes, double flops) {
    if (!prof_on(c, cls) || g_ktime != &c->sink) return;
    g_ktime = nullptr;
    if (c->pend.size() > c->sink.group) {
        c->pend[c->sink.group].bytes += bytes;
        c->pend[c->sink.group].flops += flops;
    }
    if (c->pend.size() >= 8192 && c->cg_iter < 0) prof_harvest(c);
}
static double elem_bytes(int dtype) { return dtype == SSNALM_F64 ? 8.0 : (dtype == SSNALM_F32 ? 4.0 : 2.0); }
// algorithmic bytes of A v over all rows and of A^T z over `rows` rows
static double bytes_amul(const ssnalm_ctx* c) {
    if (c->svr)      // one pass over X, the n-vector written twice
        return (double)c->nphys * c->q * elem_bytes(c->dtype) + 17.0 * c->nphys + 8.0 * c->q;
    if (c->kind == SSNALM_DENSE)
        return (double)c->n * c->q * elem_bytes(c->dtype) + 9.0 * c->n + 8.0 * c->q;
    return (double)c->nnz * (elem_bytes(c->dtype) + 4.0) + 4.0 * (c->n + 1) + 9.0 * c->n + 8.0 * c->q;
}
static double bytes_atmul(const ssnalm_ctx* c, long long rows) {
    if (c->svr)      // the 2n-vector folded, then every row of X with its coefficient
        return (double)c->nphys * c->q * elem_bytes(c->dtype) + 25.0 * c->nphys + 8.0 * c->q;
    if (c->kind == SSNALM_DENSE) {
        const double r = rows >= 0 ? (double)rows : (double)c->n;
        return r * c->q * elem_bytes(c->dtype) + 9.0 * c->n + 8.0 * c->q;
    }
    return (double)c->nnz * (elem_bytes(c->dtype) + 4.0) + 4.0 * (c->q + 1) + 9.0 * c->n + 8.0 * c->q;
}

static ProjState* dps(ssnalm_ctx* c, int k) { return &c->ds->ps[k]; }
static Scalars* dsc(ssnalm_ctx* c) { return &c->ds->sc; }
static unsigned* cnt(ssnalm_ctx* c, int k) { return c->counters + k; }

// ---------------------------------------------------------------- operators
// t = A v over all rows
static void op_amul(ssnalm_ctx* c, const double* v, double* t) {
    prof_begin(c, SSNALM_K_AMUL);
    if (c->svr) {
        launch_amul_dense(c->dtype, c->X, c->yphys, v, t, c->nphys, c->q, c->st);
        launch_svr_expand(t, c->nphys, c->st);
    } else if (c->kind == SSNALM_DENSE)
        launch_amul_dense(c->dtype, c->X, c->y, v, t, c->n, c->q, c->st);
    else if (c->sell.nslice)
        launch_sell_amul(c->sell, v, c->q, c->y, t, c->st);
    else
        launch_segsum(c->fwd, v, nullptr, nullptr, c->y, nullptr, t, c->st);
    prof_end(c, SSNALM_K_AMUL, bytes_amul(c), 2.0 * (c->kind == SSNALM_DENSE ? (double)c->n * c->q : (double)c->nnz));
}

// r = base + sign * A^T z  (z an n-vector; base may be null); when mask is
// given, also s_out = X_J^T 1.
static void op_atmul(ssnalm_ctx* c, const double* z, const uint8_t* mask, const double* base,
                     double sign, double* r, double* s_out, int cls = SSNALM_K_ATMUL) {
    prof_begin(c, cls);
    if (c->svr) {
        // B^T z = X^T (z_top - z_bot), B_J^T a_J = X^T (mask_top + mask_bot)
        const int nb = atmul_dense_nblk(c->nphys);
        launch_svr_fold(z, mask, c->nphys, c->zc, mask ? c->mc : nullptr, c->st);
        launch_atmul_dense(c->dtype, c->X, c->yphys, c->zc, mask ? c->mc : nullptr, c->nphys, c->q,
                           c->part, c->part2, c->st);
        launch_reduce_cols(c->part, nb, c->q, base, sign, r, c->st);
        if (mask) launch_reduce_cols(c->part2, nb, c->q, nullptr, 1.0, s_out, c->st);
    } else if (c->kind == SSNALM_DENSE) {
        const int nb = atmul_dense_nblk(c->n);
        launch_atmul_dense(c->dtype, c->X, c->y, z, mask, c->n, c->q, c->part, c->part2, c->st);
        launch_reduce_cols(c->part, nb, c->q, base, sign, r, c->st);
        if (mask) launch_reduce_cols(c->part2, nb, c->q, nullptr, 1.0, s_out, c->st);
    } else {
        // one gathered coefficient per entry: y .* z, formed once
        launch_mul_y(z, c->y, c->yz, c->n, c->st);
        if (c->trb_parts > 1) {
            // per-row-block column sums, then r = base + sign * (their sum in
            // block order); sign is always -1 with a base
            launch_segsum_parts(c->trb, c->trb_parts, c->yz, c->qparts, c->st);
            launch_reduce_cols(c->qparts, c->trb_parts, c->q, base, base ? -1.0 : sign, r, c->st);
        } else {
            launch_segsum(c->tr, c->yz, nullptr, nullptr, nullptr, nullptr, c->qv2, c->st);
            if (base)
                launch_sub(base, c->qv2, r, c->q, c->st);
            else
                launch_scale_copy(r, c->qv2, sign, c->q, c->st);
        }
        if (mask) launch_segsum(c->tr, nullptr, nullptr, mask, nullptr, nullptr, s_out, c->st);
    }
    if (cls == SSNALM_K_ATMUL)
        prof_end(c, cls, bytes_atmul(c, c->last_nsv) * (mask && c->kind == SSNALM_CSR ? 2.0 : 1.0),
                 2.0 * (c->kind == SSNALM_DENSE ? (double)c->n * c->q : (double)c->nnz));
    else
        prof_end(c, cls, 0.0, 0.0);
}

// A user q-vector in the internal column order (CSR contexts relabel their
// columns; the vector is copied into qin), and an internal one written back
// in the user's order (nothing to do without relabelling: the internal
// result was already written to dst).
static const double* q_in(ssnalm_ctx* c, const double* v) {
    if (!c->qperm) return v;
    launch_permute(v, c->qperm, c->qin, c->q, true, c->st);
    return c->qin;
}
static void q_out(ssnalm_ctx* c, const double* src, double* dst) {
    if (c->qperm) launch_permute(src, c->qperm, dst, c->q, false, c->st);
}

// ---------------------------------------------------------------- projection
static const int kPassBatch = 5;

// Projection of v (or of u - as*td, materialised into vout) into state k.
static ssnalm_status project_into(ssnalm_ctx* c, const double* u, const double* td, double as,
                                  double* vout, int k, const ProjState* hint = nullptr) {
    if (c->gen) {
        launch_gproj_init(u, td, as, vout, c->gbox, c->n, dps(c, k), c->spart, c->st);
        const double* v = td ? vout : u;
        for (int i = 0; i < kPassBatch; ++i) {
            prof_begin(c, SSNALM_K_PROJ);
            launch_gproj_pass(v, c->gbox, c->n, dps(c, k), c->spart, c->st);
            prof_end(c, SSNALM_K_PROJ, 32.0 * c->n, 0.0);
        }
        return SSNALM_OK;
    }
    launch_proj_init(u, td, as, vout, c->y, c->n, c->C, dps(c, k), c->spart,
                     cnt(c, CNT_PROJ_INIT), c->st, hint);
    const double* v = td ? vout : u;
    for (int i = 0; i < kPassBatch; ++i) {
        prof_begin(c, SSNALM_K_PROJ);
        launch_proj_pass(v, c->y, c->n, c->C, dps(c, k), c->spart, cnt(c, CNT_PROJ_PASS), c->st);
        prof_end(c, SSNALM_K_PROJ, 9.0 * c->n, 0.0);
    }
    return SSNALM_OK;
}

// Make sure state k is final (after a sync showed done == 0, run more passes).
static ssnalm_status project_finish(ssnalm_ctx* c, const double* v, int k, bool* more) {
    *more = false;
    if (c->hs->ps[k].done) return SSNALM_OK;
    *more = true;
    if (c->gen) {
        for (int i = 0; i < gproj_max_passes(); ++i)
            launch_gproj_pass(v, c->gbox, c->n, dps(c, k), c->spart, c->st);
        return SSNALM_OK;
    }
    for (int i = 0; i < proj_max_passes(); ++i)
        launch_proj_pass(v, c->y, c->n, c->C, dps(c, k), c->spart, cnt(c, CNT_PROJ_PASS), c->st);
    return SSNALM_OK;
}

// x = Pi(v) from the final state k, with the free mask (when given), |J|
// and the support count into the scalars.
static void proj_apply(ssnalm_ctx* c, const double* v, int k, double* x, uint8_t* mask) {
    if (c->gen)
        launch_gfinalize(v, nullptr, nullptr, 0.0, c->gbox, c->n, dps(c, k), dps(c, k), nullptr, x,
                         mask, dsc(c), c->spart, c->st);
    else
        launch_proj_apply(v, c->y, c->n, c->C, dps(c, k), x, mask, dsc(c), c->spart,
                          cnt(c, CNT_APPLY), c->st);
}

// The line-search trial's n-side: x~ = Pi(v) from state k, its free mask,
// |x~ - xk|^2 and the psi increment against the base state kb (at u_base).
static void ls_fin(ssnalm_ctx* c, const double* v, const double* u_base, const double* td, double as,
                   int k, int kb, const double* xk, double* x, uint8_t* mask) {
    if (c->gen)
        launch_gfinalize(v, u_base, td, as, c->gbox, c->n, dps(c, k), dps(c, kb), xk, x, mask, dsc(c),
                         c->spart, c->st);
    else
        launch_ls_finalize(v, u_base, td, as, c->y, c->n, c->C, dps(c, k), dps(c, kb), xk, x, mask,
                           dsc(c), c->spart, cnt(c, CNT_LS), c->st);
}

// ---------------------------------------------------------------- Newton
// d = -M^{-1} g for the free set in c->jm (count p).
static ssnalm_status newton_dir(ssnalm_ctx* c, const uint8_t* mask, int64_t p, const double* g,
                                const double* sv, double sigma, double cg_tol, double* d,
                                int* cg_iters) {
    *cg_iters = 0;
    if (p == 0) {
        launch_scale_copy(d, g, -1.0, c->q, c->st);
        return SSNALM_OK;
    }
    if (c->use_chol) {
        long long* pcount = &dsc(c)->p;
        launch_compact(mask, c->n, c->jlist, pcount, c->blk, cnt(c, CNT_CMP), c->st);
        if (c->svr) launch_list_mod(c->jlist, p, c->nphys, c->st);   // rows of X (repeats allowed)
        // A step at the sigma of the stored factor whose J differs from the
        // factor's in few rows updates that factor (Woodbury) instead of
        // forming and factoring M again.
        const bool lr_ok = c->lrU && !c->gen && !c->svr && (c->mixed ? c->opt.lowrank >= 1 : c->opt.lowrank >= 2);
        c->lr_k = 0;
        bool took_lr = false;
        if (lr_ok && c->lr_valid && sigma == c->lr_sigma) {
            launch_mask_diff(mask, c->jm0, c->n, c->chg_mask, c->st);
            launch_compact(c->chg_mask, c->n, c->chg_list, &dsc(c)->nchg, c->blk, cnt(c, CNT_CMP), c->st);
            STCHK(sync_state(c));
            const int64_t nchg = c->hs->sc.nchg;
            const int64_t k = nchg + (c->lr_p0 > 0 ? 1 : 0) + (p > 0 ? 1 : 0);
            if (c->opt.verbose >= 2)
                fprintf(stderr, "[ssnalm]   newton step: sigma=%.3g p=%lld rows changed since the factor=%lld\n",
                        sigma, (long long)p, (long long)nchg);
            if (k <= lowrank_max()) {
                HIPCHK(hipMemsetAsync(&dsc(c)->chol_fail, 0, sizeof(int), c->st));
                prof_begin(c, SSNALM_K_CHOL);
                if (k > 0) {
                    launch_lr_build(c->dtype, c->X, c->q, c->chg_list, (int)nchg, mask, sigma, c->s0v, c->lr_p0,
                                    sv, p, c->lrU, c->lrW, (int)k, c->st);
                    launch_chol_solve_factored_multi(c->M, c->linv, c->lrU, c->lrZ, c->q, k, c->st);
                    launch_lr_factor(c->lrU, c->lrZ, c->q, (int)k, c->lrW, c->lrT, c->lr_perm, dsc(c), c->st);
                }
                launch_chol_solve_factored(c->M, c->linv, g, d, c->q, c->st);
                if (k > 0) launch_lr_apply(c->lrU, c->lrZ, c->q, (int)k, c->lrT, c->lr_perm, d, d, c->st);
                prof_end(c, SSNALM_K_CHOL, 8.0 * c->q * c->q + 16.0 * c->q * k,
                         2.0 * (k + 1) * (double)c->q * c->q + 4.0 * (double)k * k * c->q);
                c->lr_k = (int)k;
                ++c->lowrank_steps;
                took_lr = true;
            }
        }
        if (!took_lr) {
            prof_begin(c, SSNALM_K_SYRK);
            if (c->mixed)
                launch_syrk_mfma(c->X, c->dtype, c->q, c->jlist, p, c->G, c->mpart, c->mpart_cap, c->st);
            else
                launch_syrk_gather(c->dtype, c->X, c->q, c->jlist, p, c->G, c->part, c->part_cap, c->st);
            prof_end(c, SSNALM_K_SYRK, (double)p * c->q * elem_bytes(c->dtype) + 4.0 * p + 8.0 * c->q * c->q,
                     (double)p * c->q * (c->q + 1));
            if (c->gen) {
                const double den = c->hs->sc.aja;            // a_J^T a_J (0: no rank-one term)
                launch_form_M_inv(c->G, sv, sigma, den > 0.0 ? 1.0 / den : 0.0, c->M, c->q, c->st);
            } else {
                launch_form_M(c->G, sv, sigma, p, c->M, c->q, c->st);
            }
            prof_begin(c, SSNALM_K_CHOL);
            if (!c->mixed && c->q <= chol_small_max()) {
                launch_chol_solve_small(c->M, g, d, c->q, dsc(c), c->st);
            } else {
                launch_chol_factor_blocked(c->M, c->q, c->linv, dsc(c), c->st);
                launch_chol_solve_factored(c->M, c->linv, g, d, c->q, c->st);
            }
            prof_end(c, SSNALM_K_CHOL, 8.0 * c->q * c->q, (double)c->q * c->q * c->q / 3.0 + 2.0 * c->q * c->q);
            if (lr_ok) {
                // the new factor's (sigma, J, s, p), for later steps' updates
                HIPCHK(hipMemcpyAsync(c->jm0, mask, c->n, hipMemcpyDeviceToDevice, c->st));
                HIPCHK(hipMemcpyAsync(c->s0v, sv, sizeof(double) * c->q, hipMemcpyDeviceToDevice, c->st));
                c->lr_p0 = p;
                c->lr_sigma = sigma;
                c->lr_valid = true;
            }
        }
        if (c->mixed) {
            // iterative refinement with the exact operator
            //   M v = v + sigma X_J^T (X_J v - mean(X_J v) 1)
            // in fp64, preconditioned by the factor of the bf16 Gram matrix
            const double tol2 = cg_tol * cg_tol;
            const int nbw = (int)dense_rows_grid(p);
            launch_fill(c->zJ, 0.0, c->n, c->st);
            for (int it = 0; it < 10; ++it) {
                launch_dense_rows(c->dtype, c->X, c->q, c->jlist, p, d, c->wJ, c->cgpart, c->st);
                launch_scatter_centered(c->jlist, p, c->wJ, c->cgpart, nbw, c->y, c->zJ, c->st);
                op_atmul(c, c->zJ, nullptr, nullptr, 1.0, c->qv, nullptr, SSNALM_K_ATMUL_J);
                launch_refine_res(g, d, c->qv, sigma, c->qv2, c->q, c->st);
                launch_dots(1, c->qv2, c->qv2, &dsc(c)->cg_rr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, c->q, c->spart, cnt(c, CNT_DOTS), c->st);
                STCHK(sync_state(c));
                ++*cg_iters;
                if (!(c->hs->sc.cg_rr > tol2)) break;
                launch_chol_solve_factored(c->M, c->linv, c->qv2, c->qv, c->q, c->st);
                if (c->lr_k > 0)
                    launch_lr_apply(c->lrU, c->lrZ, c->q, c->lr_k, c->lrT, c->lr_perm, c->qv, c->qv, c->st);
                launch_axpy(d, c->qv, 1.0, c->q, c->st);
            }
        }
        return SSNALM_OK;
    }
    if (c->kind == SSNALM_CSR) {
        // compact X_J for this Newton step, then fence-free PCG on it
        launch_compact(mask, c->n, c->jlist, &dsc(c)->p, c->blk, cnt(c, CNT_CMP), c->st);
        launch_rank_from_list(c->jlist, &dsc(c)->p, c->n, c->jrank, c->fwd.ptr, c->jrow, c->st);
        launch_jcsc_build(c->tr, c->tcv, mask, c->n, c->jbits, c->jrank, c->tcount, c->toff,
                          &dsc(c)->nnzj, c->jr, c->jc, c->jv, c->st);
        launch_fix_flags(c->jc, &dsc(c)->nnzj, c->nchmax, c->fixflag, c->st);
        launch_compact(c->fixflag, c->nchmax, c->fix.list, &dsc(c)->nfix, c->fixblk,
                       cnt(c, CNT_CMP), c->st);
        STCHK(sync_state(c));
        const int64_t nnzj = c->hs->sc.nnzj;
        c->fix.nfix = c->hs->sc.nfix;
        launch_fix_ends(c->jc, nnzj, c->fix, c->st);
        const int vf64 = c->dtype == SSNALM_F64;
        launch_keyed_tr(1, c->jr, c->jc, c->jv, vf64, nnzj, nullptr, c->kcarry, c->sv, c->q, c->fix,
                        c->st);
        launch_keyed_tr(2, c->jr, c->jc, c->jv, vf64, nnzj, nullptr, c->kcarry, c->sq, c->q, c->fix,
                        c->st);
        launch_jacobi_diag(c->sq, c->sv, sigma, p, c->diag, c->q, c->st);
        const double tol2 = cg_tol * cg_tol;
        double* Pw = c->cgpart;
        double* Pdir = c->cgpart + 1024;
        double* Pst[2] = {c->cgpart + 1024 + 512, c->cgpart + 1024 + 1024};
        launch_cg_init(g, c->diag, c->sv, c->q, c->cg_x, c->cg_r, c->cg_z, c->cg_p, Pst[0], Pdir,
                       c->st);
        launch_cg_publish(Pst[0], c->q, tol2, dsc(c), c->st);
        launch_fill(c->qv, 0.0, c->q, c->st);      // later zeroed by the direction kernel
        // no host check before the first batch: when the start already meets the
        // tolerance the batch's kernels see the done flag and pass through
        const int nbw = (int)cg_rows_grid(p);
        const double vb = elem_bytes(c->dtype);
        int it = 0;
        // One CG iteration: X_J p, X_J^T w, the step and the direction (no host
        // decision inside; the kernels stop changing x once the tolerance is met).
        auto cg_iteration = [&](int par) {
            prof_begin(c, SSNALM_K_AMUL_J);
            launch_cg_rows(c->fwd, c->jrow, p, c->q, c->cg_p, c->wJ, Pw, dsc(c), c->st);
            prof_end(c, SSNALM_K_AMUL_J, (double)nnzj * (vb + 4.0) + 20.0 * p + 8.0 * c->q,
                     2.0 * (double)nnzj);
            prof_begin(c, SSNALM_K_ATMUL_J);
            launch_keyed_tr(0, c->jr, c->jc, c->jv, vf64, nnzj, c->wJ, c->kcarry, c->qv, c->q,
                            c->fix, c->st, false, &dsc(c)->cg_done);
            prof_end(c, SSNALM_K_ATMUL_J, (double)nnzj * (8.0 + vb) + 8.0 * p + 8.0 * c->q,
                     2.0 * (double)nnzj);
            launch_cg_step(c->cg_x, c->cg_r, c->cg_p, c->qv, c->sv, c->diag, c->cg_z, c->q,
                           sigma, p, Pw, nbw, Pdir, Pst[par], Pst[1 - par], tol2, dsc(c), c->st);
            launch_cg_dir(c->cg_p, c->cg_z, c->sv, c->q, Pst[par], Pst[1 - par], Pdir, tol2,
                          dsc(c), c->qv, c->st);
        };
        // Batches of kCgBatch iterations between host checks, launched directly:
        // a HIP graph of a batch would have to be captured again every Newton
        // step (grid sizes follow |J| and nnz_J), which costs more host time
        // than the 40 launches it replaces (measured: a solve 4.5% slower).
        constexpr int kCgBatch = 8;
        bool first = true;
        while (it < c->opt.max_cg && (first || !c->hs->sc.cg_done)) {
            first = false;
            const int batch = std::min(kCgBatch, c->opt.max_cg - it);
            for (int b = 0; b < batch; ++b) {
                c->cg_iter = it + b;
                cg_iteration(b & 1);
            }
            it += batch;
            c->cg_iter = -1;
            STCHK(sync_state(c));
        }
        if (first) STCHK(sync_state(c));   // no batch ran (max_cg = 0)
        *cg_iters = c->hs->sc.cg_count;     // iterations that did work (a batch may end early)
        prof_drop_idle_cg(c, *cg_iters);
        HIPCHK(hipMemcpyAsync(d, c->cg_x, sizeof(double) * c->q, hipMemcpyDeviceToDevice, c->st));
        return SSNALM_OK;
    }
    // Dense X: PCG on M (matrix-free), Jacobi preconditioner diag(M), with
    // sq_j = sum_J X_ij^2
    launch_atmul_dense(c->dtype, c->X, c->y, nullptr, mask, c->n, c->q, c->part, c->part2,
                       c->st, 2);
    launch_reduce_cols(c->part2, atmul_dense_nblk(c->n), c->q, nullptr, 1.0, c->sq, c->st);
    launch_jacobi_diag(c->sq, sv, sigma, p, c->diag, c->q, c->st);
    const double tol2 = cg_tol * cg_tol;
    launch_pcg_init(g, c->diag, c->cg_x, c->cg_r, c->cg_z, c->cg_p, c->q, tol2, dsc(c), c->spart,
                    cnt(c, CNT_PCG), c->st);
    STCHK(sync_state(c));
    int it = 0;
    while (it < c->opt.max_cg && !c->hs->sc.cg_done) {
        const int batch = std::min(8, c->opt.max_cg - it);
        for (int b = 0; b < batch; ++b) {
            // Ap = p + sigma (X_J^T (X_J p - mean) )  with mean over J
            op_amul(c, c->cg_p, c->nv);   // nv = y .* X p (rows outside J masked below)
            launch_masked_mean(c->nv, c->y, mask, c->n, p, &dsc(c)->mean_w, c->spart,
                               cnt(c, CNT_MEAN), c->st);
            launch_masked_center_t(c->nv, c->y, mask, c->n, &dsc(c)->mean_w, c->nv2, c->st);
            op_atmul(c, c->nv2, nullptr, nullptr, 1.0, c->qv, nullptr, SSNALM_K_ATMUL_J);  // qv = X_J^T (w - mean)
            launch_mop_finish(c->cg_p, c->qv, sigma, nullptr, nullptr, p, c->cg_ap, c->q, c->st);
            launch_pcg_pap(c->cg_p, c->cg_ap, c->q, dsc(c), c->spart, cnt(c, CNT_PCG2), c->st);
            launch_pcg_step(c->cg_x, c->cg_r, c->cg_p, c->cg_ap, c->diag, c->cg_z, c->q, dsc(c),
                            tol2, c->spart, cnt(c, CNT_PCG3), c->st);
            launch_pcg_dir(c->cg_p, c->cg_z, c->q, dsc(c), c->st);
        }
        it += batch;
        STCHK(sync_state(c));
    }
    *cg_iters = c->hs->sc.cg_count;     // iterations that changed x (a batch may end early)
    HIPCHK(hipMemcpyAsync(d, c->cg_x, sizeof(double) * c->q, hipMemcpyDeviceToDevice, c->st));
    return SSNALM_OK;
}

// ---------------------------------------------------------------- gradient
// g = omega - A^T xt, s = X_J^T 1 (mask), and |g|^2, |omega|^2 into the scalars.
static void gradient(ssnalm_ctx* c, const double* xt, const uint8_t* mask) {
    if (c->gen) {
        // g = omega - B^T x~; s = B_J^T a_J and a_J^T a_J (the rank-one term
        // of Theorem 3.1's HS-Jacobian) from the coefficients a_i [i in J]
        op_atmul(c, xt, nullptr, c->om, -1.0, c->g, nullptr);
        launch_gcoef(c->gbox.a, mask, c->n, c->gzc, dsc(c), c->spart, c->st);
        op_atmul(c, c->gzc, nullptr, nullptr, 1.0, c->sv, nullptr);
        launch_dots(2, c->g, c->g, &dsc(c)->gnorm2, c->om, c->om, &dsc(c)->omega2, nullptr, nullptr,
                    nullptr, c->q, c->spart, cnt(c, CNT_DOTS), c->st);
        return;
    }
    // s = X_J^T 1 rides along the dense transposed product; the sparse path
    // computes it from the compact copy of X_J in the Newton step
    op_atmul(c, xt, c->kind == SSNALM_DENSE ? mask : nullptr, c->om, -1.0, c->g, c->sv);
    launch_dots(2, c->g, c->g, &dsc(c)->gnorm2, c->om, c->om, &dsc(c)->omega2, nullptr, nullptr,
                nullptr, c->q, c->spart, cnt(c, CNT_DOTS), c->st);
}

// ---------------------------------------------------------------- KKT
// R_KKT(x) of eq. Def_Rkkt with Qx = A w, w = A^T x given (q-vector).
// kkt_nv: the same with Q x already in c->nv.
static ssnalm_status kkt_nv(ssnalm_ctx* c, const double* x, double* R, double* b, double* sumx,
                            double* hinge = nullptr);
static ssnalm_status kkt(ssnalm_ctx* c, const double* x, const double* w, double* R, double* b,
                         double* sumx, double* hinge = nullptr) {
    op_amul(c, w, c->nv);                                       // Qx
    return kkt_nv(c, x, R, b, sumx, hinge);
}
static ssnalm_status kkt_nv(ssnalm_ctx* c, const double* x, double* R, double* b, double* sumx,
                            double* hinge) {
    launch_kkt_prepare(x, c->nv, c->nv2, c->n, c->st, c->lin);  // v = x - Qx - c
    STCHK(project_into(c, c->nv2, nullptr, 0.0, nullptr, 2));
    STCHK(sync_state(c));
    bool more = false;
    STCHK(project_finish(c, c->nv2, 2, &more));
    if (c->gen)
        launch_gkkt_finalize(c->nv2, x, c->lin, c->gbox, c->n, dps(c, 2), dsc(c), c->spart, c->st);
    else
        launch_kkt_finalize(c->nv2, x, c->nv, c->y, c->n, c->C, dps(c, 2), dsc(c), c->spart,
                            cnt(c, CNT_KKT), c->st, c->lin, c->svr ? c->nphys : 0, c->svr_eps);
    STCHK(sync_state(c));
    c->proj_passes += c->hs->ps[2].passes;
    c->proj_capped += c->hs->ps[2].approx;
    *R = std::sqrt(c->hs->sc.res2) / (1.0 + std::sqrt(c->hs->sc.x2));
    *b = c->hs->ps[2].lam;
    if (sumx) *sumx = c->hs->sc.sumx;
    if (hinge) *hinge = c->gen ? NAN : c->hs->sc.hinge;   // no primal loss for the general form
    return SSNALM_OK;
}

// ---------------------------------------------------------------- kernel C-SVC
// Largest free set whose p x p Newton matrix is factored (8.6 GB at the cap);
// larger ones are solved by CG.
static constexpr int64_t kKernelCholMax = 32768;
// Products with the resident Q of a kernel context (rows of Q at the listed
// indices; coefficients v[list_k] when by_row, else v[k]):
//   out = (base ? base : 0) + sign * sum_k coef_k Q[list_k][:].
static void qlist_prod(ssnalm_ctx* c, const int32_t* list, int64_t m, const double* v, int by_row,
                       double* out, const double* base = nullptr, double sign = 1.0) {
    const int64_t n = c->n;
    const int nch = qcols_chunks(n, m);
    prof_begin(c, SSNALM_K_QCOLS);
    launch_qcols(c->Qk, n, c->kld, list, m, v, by_row, c->kpart, nch, c->st);
    launch_reduce_cols(c->kpart, nch, n, base, sign, out, c->st);
    prof_end(c, SSNALM_K_QCOLS, 8.0 * (double)m * n + 12.0 * m + (base ? 16.0 : 8.0) * n,
             2.0 * (double)m * n);
}

// out = Q v over the support of v (one host round trip for its size).
static ssnalm_status qprod(ssnalm_ctx* c, const double* v, double* out) {
    launch_nz_mask(v, c->n, c->knz, c->st);
    launch_compact(c->knz, c->n, c->klist, &dsc(c)->km, c->blk, cnt(c, CNT_CMP), c->st);
    STCHK(sync_state(c));
    qlist_prod(c, c->klist, c->hs->sc.km, v, 1, out);
    return SSNALM_OK;
}

// The w-space gradient: s = w - x~, Q s, and the Q-norms |s|_Q^2 (gnorm2),
// |w|_Q^2 (omega2) into the scalars.
static ssnalm_status kernel_gradient(ssnalm_ctx* c, const double* xt) {
    launch_sub(c->kw, xt, c->ks, c->n, c->st);
    STCHK(qprod(c, c->ks, c->kqs));
    launch_dots(2, c->ks, c->kqs, &dsc(c)->gnorm2, c->kw, c->aw, &dsc(c)->omega2, nullptr, nullptr,
                nullptr, c->n, c->spart, cnt(c, CNT_DOTS), c->st);
    return SSNALM_OK;
}

// Newton step of Algorithm 3 by Proposition 5 (p x p system on the free set
// J of mask, p = |J|), for s and g = Q s:
//   (I_p + sigma Pi Q_JJ Pi) v = Pi g_J,  Pi = I - a a^T / p,  a = y_J,
//   z = sigma Pi v,  d = -s + z on J,  t = Q d = -g + sum_b z_b Q[J_b][:].
// Cholesky when p <= kchol (and opt.newton is not PCG), else Jacobi PCG on
// the same matrix to |M v - Pi g_J| <= cg_tol.
static ssnalm_status kernel_newton(ssnalm_ctx* c, const uint8_t* mask, int64_t p, const double* s,
                                   const double* g, double sigma, double cg_tol, double* d, double* t,
                                   int* cg_iters, bool* direct_out) {
    *cg_iters = 0;
    *direct_out = false;
    const int64_t n = c->n;
    if (p == 0) {
        launch_scale_copy(d, s, -1.0, n, c->st);
        launch_scale_copy(t, g, -1.0, n, c->st);
        return SSNALM_OK;
    }
    Scalars* ds = dsc(c);
    launch_compact(mask, n, c->jlist, &ds->p, c->blk, cnt(c, CNT_CMP), c->st);
    launch_kgather(c->jlist, p, c->y, g, c->kaJ, c->kgJ, c->st);
    launch_dots(1, c->kaJ, c->kgJ, &ds->kd0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, p,
                c->spart, cnt(c, CNT_DOTS), c->st);
    launch_kcenter(c->kgJ, c->kaJ, &ds->kd0, p, 1.0, nullptr, c->krhs, c->st);          // Pi g_J
    const bool direct = c->opt.newton != SSNALM_NEWTON_PCG && p <= c->kchol;
    prof_begin(c, SSNALM_K_QJJ);
    launch_qjj_mv(c->Qk, c->kld, c->jlist, p, c->kaJ, c->kr, c->st);                   // r = Q_JJ a
    launch_dots(1, c->kaJ, c->kr, &ds->kd1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, p,
                c->spart, cnt(c, CNT_DOTS), c->st);                                   // rho = a^T r
    if (direct)
        launch_qjj_form(c->Qk, c->kld, c->jlist, p, c->kaJ, c->kr, &ds->kd1, sigma, c->M, c->st);
    else
        launch_qjj_diag(c->Qk, c->kld, c->jlist, p, c->kaJ, c->kr, &ds->kd1, sigma, c->kdiag, c->st);
    prof_end(c, SSNALM_K_QJJ, 8.0 * (double)p * p * (direct ? 3.0 : 1.0) + 24.0 * p,
             (direct ? 8.0 : 2.0) * (double)p * p);
    const double* vneg;                               // -M^{-1} Pi g_J
    if (direct) {
        *direct_out = true;
        prof_begin(c, SSNALM_K_CHOL);
        if (p <= chol_small_max()) {
            launch_chol_solve_small(c->M, c->krhs, c->kv, p, ds, c->st);
        } else {
            launch_chol_factor_blocked(c->M, p, c->linv, ds, c->st);
            if (p <= chol_blocked_max())
                launch_chol_solve_factored(c->M, c->linv, c->krhs, c->kv, p, c->st);
            else
                launch_chol_solve_blocked(c->M, c->linv, c->krhs, c->kv, p, c->kt1, c->st);
        }
        prof_end(c, SSNALM_K_CHOL, 8.0 * (double)p * p, (double)p * p * p / 3.0 + 2.0 * (double)p * p);
        vneg = c->kv;
    } else {
        // CG on M v = Pi g_J.  Its residual r maps to the residual of the
        // omega-space system (I + sigma B^T P B) d = -g as sigma L_J^T Pi r,
        // of norm sigma ((Pi r)^T Q_JJ (Pi r))^(1/2): the test of Algorithm 3
        // (|residual| <= cg_tol) is taken on that norm, every 8 iterations.
        launch_pcg_init(c->krhs, c->kdiag, c->kcx, c->kcr, c->kcz, c->kcp, p, 0.0, ds, c->spart,
                        cnt(c, CNT_PCG), c->st);
        int it = 0;
        for (;;) {
            launch_dots(1, c->kaJ, c->kcr, &ds->kd2, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                        p, c->spart, cnt(c, CNT_DOTS), c->st);
            launch_kcenter(c->kcr, c->kaJ, &ds->kd2, p, 1.0, nullptr, c->kt1, c->st);
            launch_qjj_mv(c->Qk, c->kld, c->jlist, p, c->kt1, c->kt2, c->st);
            launch_dots(1, c->kt1, c->kt2, &ds->kres, nullptr, nullptr, nullptr, nullptr, nullptr,
                        nullptr, p, c->spart, cnt(c, CNT_DOTS), c->st);
            STCHK(sync_state(c));
            const double res = sigma * std::sqrt(std::max(c->hs->sc.kres, 0.0));
            if (res <= cg_tol || c->hs->sc.cg_done || it >= c->opt.max_cg) break;
            const int batch = std::min(8, c->opt.max_cg - it);
            for (int b = 0; b < batch; ++b) {
                // Ap = p + sigma Pi Q_JJ Pi p
                launch_dots(1, c->kaJ, c->kcp, &ds->kd2, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, p, c->spart, cnt(c, CNT_DOTS), c->st);
                launch_kcenter(c->kcp, c->kaJ, &ds->kd2, p, 1.0, nullptr, c->kt1, c->st);
                prof_begin(c, SSNALM_K_QJJ);
                launch_qjj_mv(c->Qk, c->kld, c->jlist, p, c->kt1, c->kt2, c->st);
                prof_end(c, SSNALM_K_QJJ, 8.0 * (double)p * p + 20.0 * p, 2.0 * (double)p * p);
                launch_dots(1, c->kaJ, c->kt2, &ds->kd2, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, p, c->spart, cnt(c, CNT_DOTS), c->st);
                launch_kcenter(c->kt2, c->kaJ, &ds->kd2, p, sigma, c->kcp, c->kcap, c->st);
                launch_pcg_pap(c->kcp, c->kcap, p, ds, c->spart, cnt(c, CNT_PCG2), c->st);
                launch_pcg_step(c->kcx, c->kcr, c->kcp, c->kcap, c->kdiag, c->kcz, p, ds, 0.0, c->spart,
                                cnt(c, CNT_PCG3), c->st);
                launch_pcg_dir(c->kcp, c->kcz, p, ds, c->st);
            }
            it += batch;
        }
        *cg_iters = c->hs->sc.cg_count;
        vneg = c->kcx;
    }
    // z = sigma Pi v = -sigma Pi vneg
    launch_dots(1, c->kaJ, vneg, &ds->kd2, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, p,
                c->spart, cnt(c, CNT_DOTS), c->st);
    launch_kcenter(vneg, c->kaJ, &ds->kd2, p, -sigma, nullptr, c->kz, c->st);
    launch_scale_copy(d, s, -1.0, n, c->st);
    launch_scatter_add(c->jlist, p, c->kz, d, c->st);
    qlist_prod(c, c->jlist, p, c->kz, 0, t);
    launch_axpy(t, g, -1.0, n, c->st);
    return SSNALM_OK;
}

// ---------------------------------------------------------------- C ABI
extern "C" {

void ssnalm_default_options(ssnalm_options* o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->sigma0 = 1.0;
    o->rho = 2.0;
    o->sigma_max = 1e6;
    o->mu = 1e-4;
    o->ls_delta = 0.5;
    o->tau = 0.5;
    o->eta = 0.1;
    o->eps_decay = 0.5;
    o->floor_rel = 1e-14;
    o->max_outer = 200;
    o->max_inner = 50;
    o->max_backtracks = 40;
    o->newton = SSNALM_NEWTON_AUTO;
    o->precision = SSNALM_PREC_FP64;
    o->max_cg = 500;
    o->verbose = 0;
    o->check_finite = 0;
    o->profile = 0;
    o->batch_graphs = 1;
    o->autotune = 1;
    o->lowrank = 1;
}

const char* ssnalm_last_error(void) { return g_err.c_str(); }

void ssnalm_destroy(ssnalm_ctx* c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    for (auto& p : c->pend) { c->ev_free.push_back(p.a); c->ev_free.push_back(p.b); }
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    for (void* p : c->owned) (void)hipFree(p);
    if (c->hs) (void)hipHostFree(c->hs);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->st) (void)hipStreamDestroy(c->st);
    delete c;
}

}  // extern "C"

// Build the merge-path plan of a CSR-like structure on the host.
static ssnalm_status build_plan(ssnalm_ctx* c, SegPlan* P, int64_t nseg, int64_t nnz,
                                const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx,
                                const void* val_host, int val_f64) {
    const int E = seg_entries_per_lane();
    const int64_t TILE = (int64_t)E * 64;
    P->nseg = nseg;
    P->nnz = nnz;
    P->val_f64 = val_f64;
    P->nlane = (nnz + E - 1) / E;
    P->ntile = (nnz + TILE - 1) / TILE;
    std::vector<int32_t> lane_seg(std::max<int64_t>(P->ntile * 64, 1), 0);
    // segment containing entry k: last s with ptr[s] <= k (ptr[s+1] > k)
    {
        int64_t s = 0;
        for (int64_t cidx = 0; cidx < P->ntile * 64; ++cidx) {
            const int64_t k = cidx * E;
            if (k >= nnz) { lane_seg[cidx] = (int32_t)std::max<int64_t>(nseg - 1, 0); continue; }
            while (ptr[s + 1] <= k) ++s;
            lane_seg[cidx] = (int32_t)s;
        }
    }
    std::vector<int32_t> tfirst(std::max<int64_t>(P->ntile, 1)), tlast(std::max<int64_t>(P->ntile, 1));
    for (int64_t t = 0; t < P->ntile; ++t) tfirst[t] = lane_seg[t * 64];
    {
        int64_t s = 0;
        for (int64_t t = 0; t < P->ntile; ++t) {
            const int64_t k = std::min<int64_t>((t + 1) * TILE, nnz) - 1;
            while (ptr[s + 1] <= k) ++s;
            tlast[t] = (int32_t)s;
        }
    }
    // spans: short ones (empty, or at most seg_short_tiles() tiles) first
    std::vector<int32_t> sseg, st0, st1, lseg, lt0, lt1;
    const int64_t SHORT = seg_short_tiles();
    for (int64_t s = 0; s < nseg; ++s) {
        const int64_t a = ptr[s], b = ptr[s + 1];
        if (a == b) {                                  // empty: written as 0 by the fix-up
            sseg.push_back((int32_t)s); st0.push_back(1); st1.push_back(0);
            continue;
        }
        const int64_t t0 = a / TILE, t1 = (b - 1) / TILE;
        if (t0 == t1) continue;
        if (t1 - t0 < SHORT) { sseg.push_back((int32_t)s); st0.push_back((int32_t)t0); st1.push_back((int32_t)t1); }
        else { lseg.push_back((int32_t)s); lt0.push_back((int32_t)t0); lt1.push_back((int32_t)t1); }
    }
    P->nshort = (int64_t)sseg.size();
    sseg.insert(sseg.end(), lseg.begin(), lseg.end());
    st0.insert(st0.end(), lt0.begin(), lt0.end());
    st1.insert(st1.end(), lt1.begin(), lt1.end());
    P->nspan = (int64_t)sseg.size();
    STCHK(dalloc(c, &P->ptr, nseg + 1));
    STCHK(dalloc(c, &P->idx, nnz));
    STCHK(dalloc(c, &P->lane_seg, (int64_t)lane_seg.size()));
    STCHK(dalloc(c, &P->tile_first, (int64_t)tfirst.size()));
    STCHK(dalloc(c, &P->tile_last, (int64_t)tlast.size()));
    STCHK(dalloc(c, &P->carry, 2 * std::max<int64_t>(P->ntile, 1)));
    STCHK(dalloc(c, &P->span_seg, std::max<int64_t>(P->nspan, 1)));
    STCHK(dalloc(c, &P->span_t0, std::max<int64_t>(P->nspan, 1)));
    STCHK(dalloc(c, &P->span_t1, std::max<int64_t>(P->nspan, 1)));
    const size_t vb = val_f64 ? sizeof(double) : sizeof(float);
    void* vd = nullptr;
    if (val_f64) { double* t; STCHK(dalloc(c, &t, nnz)); vd = t; }
    else { float* t; STCHK(dalloc(c, &t, nnz)); vd = t; }
    P->val = vd;
    HIPCHK(hipMemcpy(P->ptr, ptr.data(), sizeof(int32_t) * (nseg + 1), hipMemcpyHostToDevice));
    if (nnz) {
        HIPCHK(hipMemcpy(P->idx, idx.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(P->val, val_host, vb * nnz, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(P->lane_seg, lane_seg.data(), sizeof(int32_t) * lane_seg.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(P->tile_first, tfirst.data(), sizeof(int32_t) * tfirst.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(P->tile_last, tlast.data(), sizeof(int32_t) * tlast.size(), hipMemcpyHostToDevice));
    if (P->nspan) {
        HIPCHK(hipMemcpy(P->span_seg, sseg.data(), sizeof(int32_t) * P->nspan, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(P->span_t0, st0.data(), sizeof(int32_t) * P->nspan, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(P->span_t1, st1.data(), sizeof(int32_t) * P->nspan, hipMemcpyHostToDevice));
    }
    return SSNALM_OK;
}

// The sliced-ELL copy of the rows (fp32 values) for the forward product.  It
// is built only when the padding stays within a quarter of the entries and no
// row is longer than SELL_MAX_LEN (a wave walks its slice's longest row
// alone); otherwise the merge-path plan serves A v.
static ssnalm_status build_sell(ssnalm_ctx* c, int64_t n, const std::vector<int64_t>& rp,
                                const std::vector<int32_t>& ci, const float* vals) {
    const int64_t W = SELL_SLICE;
    const int64_t nslice = (n + W - 1) / W;
    const int64_t nnz = rp[n];
    std::vector<int32_t> perm(nslice * W, -1);
    for (int64_t w0 = 0; w0 < n; w0 += SELL_WINDOW) {
        const int64_t w1 = std::min<int64_t>(n, w0 + SELL_WINDOW);
        for (int64_t i = w0; i < w1; ++i) perm[i] = (int32_t)i;
        std::stable_sort(perm.begin() + w0, perm.begin() + w1, [&](int32_t a, int32_t b) {
            return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
        });
    }
    std::vector<int32_t> len(std::max<int64_t>(nslice, 1), 0);
    std::vector<int64_t> ptr(std::max<int64_t>(nslice, 1), 0);
    int64_t tot = 0;
    for (int64_t s = 0; s < nslice; ++s) {
        // windows are whole slices, sorted: the slice's first row is its longest
        const int32_t r = perm[s * W];
        const int64_t L = (rp[r + 1] - rp[r] + SELL_PAD - 1) / SELL_PAD * SELL_PAD;
        if (L > SELL_MAX_LEN) return SSNALM_OK;
        len[s] = (int32_t)L;
        ptr[s] = tot;
        tot += W * L;
    }
    if (tot > nnz + nnz / 4 + W * SELL_PAD * nslice) return SSNALM_OK;
    std::vector<ColValF> cv(std::max<int64_t>(tot, 1), ColValF{0, 0.0f});
    for (int64_t s = 0; s < nslice; ++s)
        for (int64_t l = 0; l < W; ++l) {
            const int32_t r = perm[s * W + l];
            if (r < 0) continue;
            for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
                cv[ptr[s] + (k - rp[r]) * W + l] = ColValF{ci[k], vals[k]};
        }
    SellPlan P{};
    STCHK(dalloc(c, &P.ptr, std::max<int64_t>(nslice, 1)));
    STCHK(dalloc(c, &P.len, std::max<int64_t>(nslice, 1)));
    STCHK(dalloc(c, &P.perm, std::max<int64_t>(nslice * W, 1)));
    STCHK(dalloc(c, &P.cv, std::max<int64_t>(tot, 1)));
    HIPCHK(hipMemcpy(P.ptr, ptr.data(), sizeof(int64_t) * ptr.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(P.len, len.data(), sizeof(int32_t) * len.size(), hipMemcpyHostToDevice));
    if (nslice) HIPCHK(hipMemcpy(P.perm, perm.data(), sizeof(int32_t) * perm.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(P.cv, cv.data(), sizeof(ColValF) * cv.size(), hipMemcpyHostToDevice));
    P.nslice = nslice;
    c->sell = P;
    return SSNALM_OK;
}

// CSR input: validate, build the internal int32 CSR (rows) and the CSC copy
// (columns, rows ascending inside each column: a stable counting sort).
static ssnalm_status setup_csr(ssnalm_ctx* c, const ssnalm_problem* pr) {
    const int64_t n = c->n, q = c->q, nnz = pr->nnz;
    if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail(SSNALM_E_BADARG, "nnz out of range");
    if (!pr->row_ptr || (!pr->col_idx && nnz > 0) || (!pr->X && nnz > 0))
        return fail(SSNALM_E_BADARG, "CSR arrays missing");
    if (c->dtype == SSNALM_BF16) return fail(SSNALM_E_BADARG, "CSR values must be F64 or F32");
    std::vector<int64_t> rp(n + 1);
    HIPCHK(hipMemcpy(rp.data(), pr->row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    if (rp[0] != 0 || rp[n] != nnz) return fail(SSNALM_E_BADARG, "row_ptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(SSNALM_E_BADARG, "row_ptr not monotone at row %lld", (long long)i);
    std::vector<int32_t> ci(nnz);
    if (nnz) HIPCHK(hipMemcpy(ci.data(), pr->col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < nnz; ++k)
        if (ci[k] < 0 || ci[k] >= q) return fail(SSNALM_E_BADARG, "col_idx out of range at %lld", (long long)k);
    const size_t vb = c->dtype == SSNALM_F64 ? 8 : 4;
    std::vector<char> vals(vb * std::max<int64_t>(nnz, 1));
    if (nnz) HIPCHK(hipMemcpy(vals.data(), pr->X, vb * nnz, hipMemcpyDeviceToHost));
    if (c->opt.check_finite) {
        for (int64_t k = 0; k < nnz; ++k) {
            const double v = vb == 8 ? ((double*)vals.data())[k] : ((float*)vals.data())[k];
            if (!std::isfinite(v)) return fail(SSNALM_E_NONFINITE, "non-finite value at entry %lld", (long long)k);
        }
    }
    // Columns relabelled by decreasing entry count (ties by index), so that
    // the gathers of a q-vector in X v concentrate on a few cache lines for
    // the frequent columns; q-vectors are relabelled where they cross the API.
    {
        std::vector<int64_t> cnt(q, 0);
        for (int64_t k = 0; k < nnz; ++k) cnt[ci[k]]++;
        std::vector<int32_t> order(q);
        for (int64_t j = 0; j < q; ++j) order[j] = (int32_t)j;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cnt[a] > cnt[b]; });
        std::vector<int32_t> perm(q);
        bool ident = true;
        for (int64_t r = 0; r < q; ++r) {
            perm[order[r]] = (int32_t)r;
            ident = ident && order[r] == r;
        }
        if (!ident) {
            for (int64_t k = 0; k < nnz; ++k) ci[k] = perm[ci[k]];
            STCHK(dalloc(c, &c->qperm, q));
            STCHK(dalloc(c, &c->qin, q));
            STCHK(dalloc(c, &c->qout, q));
            HIPCHK(hipMemcpy(c->qperm, perm.data(), sizeof(int32_t) * q, hipMemcpyHostToDevice));
        }
    }
    std::vector<int32_t> rp32(n + 1);
    for (int64_t i = 0; i <= n; ++i) rp32[i] = (int32_t)rp[i];
    STCHK(build_plan(c, &c->fwd, n, nnz, rp32, ci, vals.data(), vb == 8));
    if (vb == 4) STCHK(build_sell(c, n, rp, ci, (const float*)vals.data()));
    // CSC by a stable counting sort over rows
    std::vector<int32_t> cp(q + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) cp[ci[k] + 1]++;
    for (int64_t j = 0; j < q; ++j) cp[j + 1] += cp[j];
    std::vector<int32_t> pos(cp.begin(), cp.end() - 1), ri(nnz);
    std::vector<char> cv(vb * std::max<int64_t>(nnz, 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = ci[k];
            const int32_t d = pos[j]++;
            ri[d] = (int32_t)i;
            memcpy(cv.data() + vb * d, vals.data() + vb * k, vb);
        }
    STCHK(build_plan(c, &c->tr, q, nnz, cp, ri, cv.data(), vb == 8));
    // The CSC cut into row blocks of about equal entry counts, one per XCD,
    // for A^T z once the gathered n-vector outgrows an XCD's L2
    const int parts = atmul_row_parts(n, q, nnz);
    if (parts > 1) {
        std::vector<int32_t> rb(parts + 1, 0);
        for (int r = 1; r < parts; ++r)
            rb[r] = (int32_t)(std::lower_bound(rp.begin(), rp.end(), (int64_t)(nnz * (double)r / parts)) - rp.begin());
        rb[parts] = (int32_t)n;
        std::vector<int32_t> bp((size_t)parts * q + 1, 0), ri2(std::max<int64_t>(nnz, 1));
        std::vector<char> cv2(vb * std::max<int64_t>(nnz, 1));
        for (int r = 0; r < parts; ++r)
            for (int64_t k = rp[rb[r]]; k < rp[rb[r + 1]]; ++k) bp[(size_t)r * q + ci[k] + 1]++;
        for (size_t s = 0; s < (size_t)parts * q; ++s) bp[s + 1] += bp[s];
        std::vector<int32_t> at(bp.begin(), bp.end() - 1);
        for (int r = 0; r < parts; ++r)
            for (int64_t i = rb[r]; i < rb[r + 1]; ++i)
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                    const int32_t d = at[(size_t)r * q + ci[k]]++;
                    ri2[d] = (int32_t)i;
                    memcpy(cv2.data() + vb * d, vals.data() + vb * k, vb);
                }
        STCHK(build_plan(c, &c->trb, (int64_t)parts * q, nnz, bp, ri2, cv2.data(), vb == 8));
        STCHK(dalloc(c, &c->qparts, (int64_t)parts * q));
        c->trb_parts = parts;
    }
    // the column and value of every CSC entry side by side: the J filter
    // copies both per kept entry with one load
    {
        const int64_t m = std::max<int64_t>(nnz, 1);
        hipError_t e;
        if (vb == 4) {
            std::vector<ColValF> t(m, ColValF{0, 0.0f});
            for (int64_t j = 0; j < q; ++j)
                for (int32_t k = cp[j]; k < cp[j + 1]; ++k) {
                    t[k].col = (int32_t)j;
                    memcpy(&t[k].v, cv.data() + 4 * (size_t)k, 4);
                }
            ColValF* d = nullptr;
            STCHK(dalloc(c, &d, m));
            c->tcv = d;
            e = hipMemcpy(d, t.data(), sizeof(ColValF) * m, hipMemcpyHostToDevice);
        } else {
            std::vector<ColValD> t(m, ColValD{0, 0, 0.0});
            for (int64_t j = 0; j < q; ++j)
                for (int32_t k = cp[j]; k < cp[j + 1]; ++k) {
                    t[k].col = (int32_t)j;
                    memcpy(&t[k].v, cv.data() + 8 * (size_t)k, 8);
                }
            ColValD* d = nullptr;
            STCHK(dalloc(c, &d, m));
            c->tcv = d;
            e = hipMemcpy(d, t.data(), sizeof(ColValD) * m, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) return fail(SSNALM_E_HIP, "upload of the CSC columns failed");
    }
    return SSNALM_OK;
}

namespace ssn {
// Scan `count` elements of X (device, dtype) for NaN / Inf on the host, in
// blocks of 4M elements.
ssnalm_status scan_finite(const void* X, int dtype, int64_t total) {
    const size_t eb = dtype == SSNALM_F64 ? 8 : (dtype == SSNALM_F32 ? 4 : 2);
    const int64_t blkn = 1 << 22;
    std::vector<char> buf(eb * blkn);
    for (int64_t off = 0; off < total; off += blkn) {
        const int64_t m = std::min(blkn, total - off);
        if (hipMemcpy(buf.data(), (const char*)X + eb * off, eb * m, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(SSNALM_E_HIP, "reading X failed");
        for (int64_t k = 0; k < m; ++k) {
            double v;
            if (eb == 8) v = ((double*)buf.data())[k];
            else if (eb == 4) v = ((float*)buf.data())[k];
            else { uint32_t b = ((uint32_t)((uint16_t*)buf.data())[k]) << 16; float f; memcpy(&f, &b, 4); v = f; }
            if (!std::isfinite(v)) return fail(SSNALM_E_NONFINITE, "non-finite X entry %lld", (long long)(off + k));
        }
    }
    return SSNALM_OK;
}
}  // namespace ssn

// x_rows: rows of the X array (n, or n / 2 for the eps-SVR's two copies).
static ssnalm_status create_impl(ssnalm_ctx** out, const ssnalm_problem* pr,
                                 const ssnalm_options* opt, void* stream, int64_t x_rows);

extern "C" ssnalm_status ssnalm_create(ssnalm_ctx** out, const ssnalm_problem* pr,
                                       const ssnalm_options* opt, void* stream) {
    if (!out || !pr) return fail(SSNALM_E_BADARG, "null argument");
    return create_impl(out, pr, opt, stream, pr->n);
}

extern "C" ssnalm_status ssnalm_create_svr(ssnalm_ctx** out, const ssnalm_svr_problem* pr,
                                           const ssnalm_options* opt, void* stream) {
    if (!out || !pr) return fail(SSNALM_E_BADARG, "null argument");
    *out = nullptr;
    if (pr->kind != SSNALM_DENSE) return fail(SSNALM_E_BADARG, "eps-SVR needs dense X");
    if (pr->n < 1 || pr->q < 1 || 2 * pr->n >= INT32_MAX || pr->q >= INT32_MAX)
        return fail(SSNALM_E_BADARG, "n must be in [1, 2^30) and q in [1, 2^31)");
    if (!pr->X || !pr->y) return fail(SSNALM_E_BADARG, "X and y are required");
    if (!(pr->eps >= 0.0) || !std::isfinite(pr->eps)) return fail(SSNALM_E_BADARG, "eps must be finite and >= 0");
    ssnalm_options o;
    if (opt) o = *opt; else ssnalm_default_options(&o);
    if (o.precision != SSNALM_PREC_FP64) return fail(SSNALM_E_BADARG, "eps-SVR runs in fp64 precision");
    if (o.newton == SSNALM_NEWTON_PCG) return fail(SSNALM_E_BADARG, "eps-SVR uses the Cholesky Newton step");
    if (pr->q > std::max(chol_small_max(), chol_blocked_max()))
        return fail(SSNALM_E_BADARG, "eps-SVR needs q <= %d", std::max(chol_small_max(), chol_blocked_max()));
    o.newton = SSNALM_NEWTON_CHOL;
    const int64_t n = pr->n;
    // the targets are read by a kernel on the caller's stream: the labels a
    // and the linear term c of the 2n-variable problem
    int8_t* a = nullptr;
    double* lin = nullptr;
    if (hipMalloc(&a, 2 * n) != hipSuccess) return fail(SSNALM_E_OOM, "allocation of the labels failed");
    if (hipMalloc(&lin, sizeof(double) * 2 * n) != hipSuccess) {
        (void)hipFree(a);
        return fail(SSNALM_E_OOM, "allocation of the linear term failed");
    }
    launch_svr_setup(pr->y, n, pr->eps, a, lin, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
        (void)hipFree(a);
        (void)hipFree(lin);
        return fail(SSNALM_E_HIP, "building the eps-SVR problem failed");
    }
    ssnalm_problem p2;
    memset(&p2, 0, sizeof p2);
    p2.kind = SSNALM_DENSE;
    p2.dtype = pr->dtype;
    p2.n = 2 * n;
    p2.q = pr->q;
    p2.X = pr->X;
    p2.y = a;
    p2.C = pr->C;
    p2.tol = pr->tol;
    ssnalm_ctx* c = nullptr;
    ssnalm_status s = create_impl(&c, &p2, &o, stream, n);
    if (s < 0) {
        (void)hipFree(a);
        (void)hipFree(lin);
        return s;
    }
    c->owned.push_back(a);
    c->owned.push_back(lin);
    c->svr = true;
    c->nphys = n;
    c->svr_eps = pr->eps;
    c->lin = lin;
    if ((s = dalloc(c, &c->yphys, n)) < 0 || (s = dalloc(c, &c->zc, n)) < 0 ||
        (s = dalloc(c, &c->mc, n)) < 0) {
        ssnalm_destroy(c);
        return s;
    }
    if (hipMemsetAsync(c->yphys, 1, n, c->st) != hipSuccess || hipStreamSynchronize(c->st) != hipSuccess) {
        ssnalm_destroy(c);
        return fail(SSNALM_E_HIP, "setting up the eps-SVR context failed");
    }
    *out = c;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_create_general(ssnalm_ctx** out, const ssnalm_general_problem* pr,
                                               const ssnalm_options* opt, void* stream) {
    if (!out || !pr) return fail(SSNALM_E_BADARG, "null argument");
    *out = nullptr;
    if (pr->kind != SSNALM_DENSE) return fail(SSNALM_E_BADARG, "the general form needs dense B");
    if (pr->n < 1 || pr->q < 1 || pr->n >= INT32_MAX || pr->q >= INT32_MAX)
        return fail(SSNALM_E_BADARG, "n and q must be in [1, 2^31)");
    if (!pr->B || !pr->c || !pr->a || !pr->l || !pr->u)
        return fail(SSNALM_E_BADARG, "B, c, a, l and u are required");
    if (!std::isfinite(pr->d)) return fail(SSNALM_E_BADARG, "d must be finite");
    ssnalm_options o;
    if (opt) o = *opt; else ssnalm_default_options(&o);
    if (o.precision != SSNALM_PREC_FP64) return fail(SSNALM_E_BADARG, "the general form runs in fp64 precision");
    if (o.newton == SSNALM_NEWTON_PCG) return fail(SSNALM_E_BADARG, "the general form uses the Cholesky Newton step");
    if (pr->q > std::max(chol_small_max(), chol_blocked_max()))
        return fail(SSNALM_E_BADARG, "the general form needs q <= %d", std::max(chol_small_max(), chol_blocked_max()));
    o.newton = SSNALM_NEWTON_CHOL;
    const int64_t n = pr->n;
    // a, l, u are checked on the host once the caller's stream has written them
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(SSNALM_E_HIP, "waiting for the caller's stream failed");
    bool zero_ok = pr->d == 0.0;
    {
        std::vector<double> ah(n), lh(n), uh(n);
        if (hipMemcpy(ah.data(), pr->a, 8 * n, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(lh.data(), pr->l, 8 * n, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(uh.data(), pr->u, 8 * n, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(SSNALM_E_HIP, "reading a, l, u failed");
        double lo = 0.0, hi = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!std::isfinite(ah[i]) || !std::isfinite(lh[i]) || !std::isfinite(uh[i]))
                return fail(SSNALM_E_BADARG, "a, l, u must be finite (entry %lld)", (long long)i);
            if (!(lh[i] < uh[i])) return fail(SSNALM_E_BADARG, "l_%lld >= u_%lld", (long long)i, (long long)i);
            lo += std::min(ah[i] * lh[i], ah[i] * uh[i]);
            hi += std::max(ah[i] * lh[i], ah[i] * uh[i]);
            zero_ok = zero_ok && lh[i] <= 0.0 && uh[i] >= 0.0;
        }
        const double slack = 1e-12 * (std::fabs(lo) + std::fabs(hi) + 1.0);
        if (pr->d < lo - slack || pr->d > hi + slack)
            return fail(SSNALM_E_BADARG, "no x in [l, u] has a^T x = d");
    }
    int8_t* ones = nullptr;
    if (hipMalloc(&ones, n) != hipSuccess) return fail(SSNALM_E_OOM, "allocation failed");
    if (hipMemset(ones, 1, n) != hipSuccess) {
        (void)hipFree(ones);
        return fail(SSNALM_E_HIP, "memset failed");
    }
    ssnalm_problem p2;
    memset(&p2, 0, sizeof p2);
    p2.kind = SSNALM_DENSE;
    p2.dtype = pr->dtype;
    p2.n = n;
    p2.q = pr->q;
    p2.X = pr->B;
    p2.y = ones;
    p2.C = 1.0;                           // unused: the box is [l, u]
    p2.tol = pr->tol;
    ssnalm_ctx* c = nullptr;
    ssnalm_status s = create_impl(&c, &p2, &o, stream, n);
    if (s < 0) {
        (void)hipFree(ones);
        return s;
    }
    c->owned.push_back(ones);
    c->gen = true;
    c->gbox = GBox{pr->a, pr->l, pr->u, pr->d};
    c->lin = pr->c;
    c->zero_feasible = zero_ok;
    if ((s = dalloc(c, &c->gzc, n)) < 0) {
        ssnalm_destroy(c);
        return s;
    }
    *out = c;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_create_kernel(ssnalm_ctx** out, const ssnalm_kernel_problem* pr,
                                              const ssnalm_options* opt, void* stream) {
    if (!out || !pr) return fail(SSNALM_E_BADARG, "null argument");
    *out = nullptr;
    if (pr->kernel != SSNALM_KERNEL_RBF && pr->kernel != SSNALM_KERNEL_LINEAR)
        return fail(SSNALM_E_BADARG, "unknown kernel %d", (int)pr->kernel);
    if (pr->kernel == SSNALM_KERNEL_RBF && !(pr->alpha > 0.0 && std::isfinite(pr->alpha)))
        return fail(SSNALM_E_BADARG, "alpha must be finite and > 0");
    if (!pr->X) return fail(SSNALM_E_BADARG, "X missing");
    ssnalm_options o;
    if (opt) o = *opt; else ssnalm_default_options(&o);
    if (o.precision != SSNALM_PREC_FP64) return fail(SSNALM_E_BADARG, "kernel problems run in fp64 precision");
    // the base context needs no q x q Newton buffers: built in PCG mode, the
    // requested mode restored afterwards
    ssnalm_options o2 = o;
    o2.newton = SSNALM_NEWTON_PCG;
    ssnalm_problem p2;
    memset(&p2, 0, sizeof p2);
    p2.kind = SSNALM_DENSE;
    p2.dtype = pr->dtype;
    p2.n = pr->n;
    p2.q = pr->q;
    p2.X = pr->X;
    p2.y = pr->y;
    p2.C = pr->C;
    p2.tol = pr->tol;
    ssnalm_ctx* c = nullptr;
    ssnalm_status s = create_impl(&c, &p2, &o2, stream, pr->n);
    if (s < 0) return s;
    c->opt.newton = o.newton;
    c->kern = true;
    const int64_t n = c->n;
    auto bail = [&](ssnalm_status st) { ssnalm_destroy(c); return st; };
    c->kld = (n + 31) / 32 * 32;
    {
        void* q = nullptr;
        const size_t bytes = (size_t)n * (size_t)c->kld * sizeof(double);
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(SSNALM_E_OOM, "Q (%lld x %lld doubles, %zu bytes) does not fit in device memory",
                             (long long)n, (long long)n, bytes));
        }
        c->owned.push_back(q);
        c->Qk = (double*)q;
    }
#define KALLOC(ptr, cnt_)                                         \
    do {                                                          \
        if ((s = dalloc(c, &(ptr), (cnt_))) < 0) return bail(s);  \
    } while (0)
    c->kchol = std::min<int64_t>(n, kKernelCholMax);
    KALLOC(c->kw, n); KALLOC(c->ks, n); KALLOC(c->kqs, n); KALLOC(c->kd, n);
    KALLOC(c->knz, n); KALLOC(c->klist, n);
    KALLOC(c->kaJ, n); KALLOC(c->kgJ, n); KALLOC(c->kr, n); KALLOC(c->krhs, n); KALLOC(c->kv, n);
    KALLOC(c->kz, n);
    KALLOC(c->kcx, n); KALLOC(c->kcr, n); KALLOC(c->kcz, n); KALLOC(c->kcp, n); KALLOC(c->kcap, n);
    KALLOC(c->kdiag, n); KALLOC(c->kt1, n); KALLOC(c->kt2, n);
    KALLOC(c->kpart, (int64_t)kQcolsMaxChunks * n);
    KALLOC(c->M, c->kchol * c->kchol);
    KALLOC(c->linv, chol_inv_size(c->kchol));
    double* norms = nullptr;
    KALLOC(norms, n);
#undef KALLOC
    const int rbf = pr->kernel == SSNALM_KERNEL_RBF;
    if (rbf) launch_row_norms(pr->dtype, pr->X, nullptr, n, pr->q, norms, c->st);
    launch_kernel_q(pr->dtype, pr->X, n, pr->q, norms, pr->y, rbf, pr->alpha, c->Qk, c->kld, c->st);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->st) != hipSuccess)
        return bail(fail(SSNALM_E_HIP, "forming Q failed"));
    // X is not read after this call
    c->X = nullptr;
    *out = c;
    return SSNALM_OK;
}

static ssnalm_status create_impl(ssnalm_ctx** out, const ssnalm_problem* pr,
                                 const ssnalm_options* opt, void* stream, int64_t x_rows) {
    if (!out || !pr) return fail(SSNALM_E_BADARG, "null argument");
    *out = nullptr;
    if (pr->n < 1 || pr->q < 1 || pr->n >= INT32_MAX || pr->q >= INT32_MAX)
        return fail(SSNALM_E_BADARG, "n and q must be in [1, 2^31)");
    if (!(pr->C > 0.0) || !std::isfinite(pr->C)) return fail(SSNALM_E_BADARG, "C must be finite and > 0");
    if (!(pr->tol > 0.0)) return fail(SSNALM_E_BADARG, "tol must be > 0");
    if (pr->kind != SSNALM_DENSE && pr->kind != SSNALM_CSR) return fail(SSNALM_E_BADARG, "unknown kind");
    if (pr->dtype < SSNALM_F64 || pr->dtype > SSNALM_BF16) return fail(SSNALM_E_BADARG, "unknown dtype");
    if (!pr->y) return fail(SSNALM_E_BADARG, "y missing");
    if (pr->kind == SSNALM_DENSE && !pr->X) return fail(SSNALM_E_BADARG, "X missing");
    ssnalm_ctx* c = new ssnalm_ctx();
    if (opt) c->opt = *opt; else ssnalm_default_options(&c->opt);
    c->kind = pr->kind;
    c->dtype = pr->dtype;
    c->n = pr->n;
    c->q = pr->q;
    c->nnz = pr->nnz;
    c->X = pr->X;
    c->y = pr->y;
    c->C = pr->C;
    c->tol = pr->tol;
    c->ust = (hipStream_t)stream;
    auto bail = [&](ssnalm_status s) { ssnalm_destroy(c); return s; };
    if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
        return bail(fail(SSNALM_E_HIP, "stream or event creation failed"));
    // The checks below read the caller's arrays from the host: wait until the
    // work already queued on the caller's stream (which may be a non-blocking
    // stream that the null stream does not order against) has written them.
    if (hipEventRecord(c->ev_in, c->ust) != hipSuccess || hipEventSynchronize(c->ev_in) != hipSuccess)
        return bail(fail(SSNALM_E_HIP, "waiting for the caller's stream failed"));
    (void)hipStreamWaitEvent(c->st, c->ev_in, 0);
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(SSNALM_E_HIP, "no HIP device"));
    const int64_t n = c->n, q = c->q;
    // labels must be exactly +-1
    {
        std::vector<int8_t> yh(n);
        if (hipMemcpy(yh.data(), pr->y, n, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(SSNALM_E_HIP, "reading y failed"));
        for (int64_t i = 0; i < n; ++i)
            if (yh[i] != 1 && yh[i] != -1) return bail(fail(SSNALM_E_BADARG, "label %lld is %d, not +-1", (long long)i, (int)yh[i]));
    }
    ssnalm_status s;
#define ALLOC(ptr, cnt_)                                   \
    do {                                                   \
        if ((s = dalloc(c, &(ptr), (cnt_))) < 0) return bail(s); \
    } while (0)
    ALLOC(c->xk, n); ALLOC(c->aw, n); ALLOC(c->u, n); ALLOC(c->ut, n); ALLOC(c->td, n);
    ALLOC(c->xt, n); ALLOC(c->xtt, n); ALLOC(c->nv, n); ALLOC(c->nv2, n);
    ALLOC(c->jm, n); ALLOC(c->jmt, n); ALLOC(c->jlist, n);
    ALLOC(c->om, q); ALLOC(c->g, q); ALLOC(c->sv, q); ALLOC(c->sq, q); ALLOC(c->d, q);
    ALLOC(c->qv, q); ALLOC(c->qv2, q);
    ALLOC(c->cg_x, q); ALLOC(c->cg_r, q); ALLOC(c->cg_z, q); ALLOC(c->cg_p, q); ALLOC(c->cg_ap, q);
    ALLOC(c->diag, q);
    ALLOC(c->spart, 8 * 4096);
    ALLOC(c->blk, compact_blocks(n) + 1);
    ALLOC(c->counters, CNT_N);
    ALLOC(c->ds, 1);
    if (hipHostMalloc((void**)&c->hs, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
        return bail(fail(SSNALM_E_OOM, "pinned allocation failed"));
    memset(c->hs, 0, sizeof(DevState));
    if (hipMemset(c->counters, 0, sizeof(unsigned) * CNT_N) != hipSuccess ||
        hipMemset(c->ds, 0, sizeof(DevState)) != hipSuccess)
        return bail(fail(SSNALM_E_HIP, "memset failed"));
    // Newton mode: Cholesky on the q x q system when q is small enough
    c->chol_max = std::max(chol_small_max(), chol_blocked_max());
    if (c->opt.newton == SSNALM_NEWTON_CHOL)
        c->use_chol = true;
    else if (c->opt.newton == SSNALM_NEWTON_PCG)
        c->use_chol = false;
    else
        c->use_chol = (pr->kind == SSNALM_DENSE) && q <= c->chol_max;
    if (c->use_chol && (pr->kind != SSNALM_DENSE || q > c->chol_max))
        return bail(fail(SSNALM_E_BADARG, "Cholesky Newton mode needs dense X and q <= %d", c->chol_max));
    if (c->use_chol) {
        ALLOC(c->G, q * q);
        ALLOC(c->M, q * q);
        c->mixed = c->opt.precision == SSNALM_PREC_MIXED && syrk_mfma_supported(c->dtype, q);
        if (c->mixed || q > chol_small_max()) {
            ALLOC(c->linv, chol_inv_size(q));
            const int lr = lowrank_max();
            ALLOC(c->jm0, n); ALLOC(c->chg_mask, n); ALLOC(c->chg_list, n);
            ALLOC(c->s0v, q); ALLOC(c->lrU, q * lr); ALLOC(c->lrZ, q * lr); ALLOC(c->lrW, lr);
            ALLOC(c->lrT, lr * lr); ALLOC(c->lr_perm, lr);
        }
        if (c->mixed) {
            ALLOC(c->zJ, n); ALLOC(c->wJ, n); ALLOC(c->cgpart, 1024 + 512 + 1024);
        }
    }
    // reduction scratch for the dense transpose (nblk x q, twice) and SYRK partials
    int64_t pc = (int64_t)atmul_dense_nblk(n) * q;
    if (c->use_chol) pc = std::max<int64_t>(pc, syrk_part_size(q, n));
    if (c->use_chol) pc = std::max<int64_t>(pc, q * q + 4 * q);
    c->part_cap = pc;
    ALLOC(c->part, pc);
    ALLOC(c->part2, (int64_t)atmul_dense_nblk(n) * q);
    if (c->mixed) {
        c->mpart_cap = syrk_mfma_part_size(q, n);
        ALLOC(c->mpart, c->mpart_cap);
    }
    if (pr->kind == SSNALM_CSR) {
        if ((s = setup_csr(c, pr)) < 0) return bail(s);
        ALLOC(c->yz, n);
        if (!c->use_chol) {
            const int64_t nz = std::max<int64_t>(pr->nnz, 1);
            ALLOC(c->jrank, n); ALLOC(c->jr, nz); ALLOC(c->jc, nz); ALLOC(c->wJ, n);
            ALLOC(c->jrow, n); ALLOC(c->jbits, jcsc_bits_words(n));
            ALLOC(c->tcount, c->tr.ntile + 1); ALLOC(c->toff, c->tr.ntile + 2);
            ALLOC(c->kcarry, 2 * (nz / 128 + 2)); ALLOC(c->cgpart, 1024 + 512 + 1024);
            c->nchmax = keyed_chunks(nz);
            ALLOC(c->fixflag, c->nchmax); ALLOC(c->fixblk, compact_blocks(c->nchmax) + 1);
            ALLOC(c->fix.list, c->nchmax); ALLOC(c->fix.fend, c->nchmax); ALLOC(c->fix.fcol, c->nchmax);
            if (c->dtype == SSNALM_F64) { double* t; ALLOC(t, nz); c->jv = t; }
            else { float* t; ALLOC(t, nz); c->jv = t; }
        }
    } else if (c->opt.check_finite) {
        if ((s = scan_finite(pr->X, pr->dtype, x_rows * q)) < 0) return bail(s);
    }
#undef ALLOC
    if (hipStreamSynchronize(c->st) != hipSuccess) return bail(fail(SSNALM_E_HIP, "stream sync failed"));
    *out = c;
    return SSNALM_OK;
}

// ---------------------------------------------------------------- solve
// Algorithm 1 with Algorithm 3 for a kernel context, in w-space: the state
// is w (kw) with Q w (aw); the gradient is Q s with s = w - Pi(u(w)) (ks,
// kqs); the Newton step gives d (kd) and Q d (td).  The scalars of the
// omega-space loop are Q-inner products: |omega|^2 = w^T Q w, |g|^2 =
// s^T Q s, g^T d = d^T Q s, omega^T d = w^T Q d, d^T d = d^T Q d.
static ssnalm_status solve_kernel(ssnalm_ctx* c, const double* x0, double* x_out, double* b_out,
                                  ssnalm_info* info) {
    const auto t_begin = std::chrono::steady_clock::now();
    const ssnalm_options& o = c->opt;
    const int64_t n = c->n;
    c->proj_passes = 0;
    c->proj_capped = 0;
    ssnalm_info inf;
    memset(&inf, 0, sizeof inf);
    int inner_total = 0, cg_total = 0, ls_fail = 0, outer = 0, ls_trials = 0, grad_steps = 0;
    ssnalm_status status = SSNALM_MAXITER;
    // x^0: zero or the projection of the warm start; w^0 = x^0
    if (x0) {
        STCHK(project_into(c, x0, nullptr, 0.0, nullptr, 3));
        STCHK(sync_state(c));
        bool more;
        STCHK(project_finish(c, x0, 3, &more));
        proj_apply(c, x0, 3, c->xk, nullptr);
    } else {
        launch_fill(c->xk, 0.0, n, c->st);
    }
    HIPCHK(hipMemcpyAsync(c->kw, c->xk, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    double sigma = o.sigma0;
    double R = INFINITY, b = NAN, best_R = INFINITY, best_b = NAN, hinge = NAN, best_hinge = NAN;
    bool have_best = false;
    for (int k = 0; k < o.max_outer; ++k) {
        outer = k + 1;
        const double eps_k = std::pow(o.eps_decay, (double)k);
        STCHK(qprod(c, c->kw, c->aw));                       // fresh Q w
        launch_u_from(c->xk, c->aw, sigma, c->u, n, c->st);
        c->base = 0;
        STCHK(project_into(c, c->u, nullptr, 0.0, nullptr, c->base));
        STCHK(sync_state(c));
        bool more;
        STCHK(project_finish(c, c->u, c->base, &more));
        ls_fin(c, c->u, c->u, nullptr, 0.0, c->base, c->base, c->xk, c->xt, c->jm);
        STCHK(kernel_gradient(c, c->xt));
        STCHK(sync_state(c));
        c->proj_passes += c->hs->ps[c->base].passes;
        c->proj_capped += c->hs->ps[c->base].approx;
        for (int j = 0; j < o.max_inner; ++j) {
            const Scalars& hsc = c->hs->sc;
            const double gn = std::sqrt(std::max(hsc.gnorm2, 0.0));
            const double dist = std::sqrt(hsc.dist2);
            const double crit = std::min(eps_k, eps_k * dist) / std::sqrt(sigma);
            const double flo = o.floor_rel * (1.0 + std::sqrt(std::max(hsc.omega2, 0.0)));
            if (!std::isfinite(gn)) return fail(SSNALM_E_NONFINITE, "non-finite gradient");
            if (gn <= std::max(crit, flo)) break;
            const int64_t p = hsc.p;
            int cgi = 0;
            bool direct = false;
            const double cg_tol = std::min(o.eta, std::pow(gn, 1.0 + o.tau));
            STCHK(kernel_newton(c, c->jm, p, c->ks, c->kqs, sigma, cg_tol, c->kd, c->td, &cgi, &direct));
            cg_total += cgi;
            ++inner_total;
            launch_dots(3, c->kd, c->kqs, &dsc(c)->gd, c->kw, c->td, &dsc(c)->od, c->kd, c->td,
                        &dsc(c)->dd, n, c->spart, cnt(c, CNT_DOTS2), c->st);
            double alpha = 1.0;
            bool accepted = false, fell_back = false;
            const int trial = 1 - c->base;
            for (int m = 0; m <= o.max_backtracks; ++m) {
                ++ls_trials;
                STCHK(project_into(c, c->u, c->td, alpha * sigma, c->ut, trial, dps(c, c->base)));
                ls_fin(c, c->ut, c->u, c->td, alpha * sigma, trial, c->base, c->xk, c->xtt, c->jmt);
                STCHK(sync_state(c));
                STCHK(project_finish(c, c->ut, trial, &more));
                if (more) {
                    ls_fin(c, c->ut, c->u, c->td, alpha * sigma, trial, c->base, c->xk, c->xtt, c->jmt);
                    STCHK(sync_state(c));
                }
                c->proj_passes += c->hs->ps[trial].passes;
                c->proj_capped += c->hs->ps[trial].approx;
                const Scalars& s2 = c->hs->sc;
                if (m == 0 && !fell_back && gn > 0.0 && (!(s2.gd < 0.0) || (direct && s2.chol_fail))) {
                    // not a descent direction (an inexact CG solve): take -grad,
                    // d = -s with Q d = -Q s, and search again from alpha = 1
                    fell_back = true;
                    ++grad_steps;
                    launch_scale_copy(c->kd, c->ks, -1.0, n, c->st);
                    launch_scale_copy(c->td, c->kqs, -1.0, n, c->st);
                    launch_dots(3, c->kd, c->kqs, &dsc(c)->gd, c->kw, c->td, &dsc(c)->od, c->kd, c->td,
                                &dsc(c)->dd, n, c->spart, cnt(c, CNT_DOTS2), c->st);
                    m = -1;
                    continue;
                }
                const double dpsi = alpha * s2.od + 0.5 * alpha * alpha * s2.dd + s2.dh / sigma;
                if (!std::isfinite(dpsi)) return fail(SSNALM_E_NONFINITE, "non-finite line search value");
                if (dpsi <= o.mu * alpha * s2.gd) { accepted = true; break; }
                alpha *= o.ls_delta;
            }
            if (!accepted) { ++ls_fail; break; }
            launch_axpy(c->kw, c->kd, alpha, n, c->st);
            launch_axpy(c->aw, c->td, alpha, n, c->st);
            std::swap(c->u, c->ut);
            std::swap(c->xt, c->xtt);
            std::swap(c->jm, c->jmt);
            c->base = trial;
            STCHK(kernel_gradient(c, c->xt));
            STCHK(sync_state(c));
        }
        // x^{k+1} = x~, and Q x^{k+1} = Q w - Q s
        std::swap(c->xk, c->xt);
        launch_sub(c->aw, c->kqs, c->nv, n, c->st);
        double sumx = 0.0;
        STCHK(kkt_nv(c, c->xk, &R, &b, &sumx, &hinge));
        if (o.verbose)
            fprintf(stderr, "[ssnalm] k=%d sigma=%.3g R_KKT=%.3e newton=%d cg=%d p=%lld passes=%d\n", k,
                    sigma, R, inner_total, cg_total, (long long)c->hs->sc.p, c->proj_passes);
        if (!std::isfinite(R)) return fail(SSNALM_E_NONFINITE, "non-finite KKT residual");
        if (R <= c->tol) { status = SSNALM_OK; break; }
        if (R < best_R) {
            best_R = R;
            best_b = b;
            best_hinge = hinge;
            HIPCHK(hipMemcpyAsync(x_out, c->xk, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
            have_best = true;
        }
        sigma = std::min(o.rho * sigma, o.sigma_max);
    }
    if (status == SSNALM_OK || !have_best || R <= best_R) {
        HIPCHK(hipMemcpyAsync(x_out, c->xk, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        R = best_R;
        b = best_b;
        hinge = best_hinge;
    }
    if (status != SSNALM_OK && ls_fail > 0 && ls_fail >= outer) status = SSNALM_LINESEARCH_FAIL;
    // x^T Q x of the returned x and the paper's columns
    STCHK(qprod(c, x_out, c->nv));
    launch_dots(1, x_out, c->nv, &dsc(c)->dd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, n,
                c->spart, cnt(c, CNT_DOTS), c->st);
    launch_count_x(x_out, n, c->C, dsc(c), c->spart, cnt(c, CNT_APPLY), c->st);
    HIPCHK(hipGetLastError());
    STCHK(sync_state(c));
    const double sumx = c->hs->sc.sumx;
    prof_harvest(c);
    const double xqx = c->hs->sc.dd;
    const auto t_end = std::chrono::steady_clock::now();
    inf.rkkt = R;
    inf.obj = 0.5 * xqx - sumx;
    inf.b = b;
    {
        const double P = 0.5 * xqx + c->C * hinge;
        inf.gap = std::isfinite(P) ? (P + inf.obj) / (1.0 + std::fabs(P) + std::fabs(inf.obj)) : NAN;
    }
    if (b_out) *b_out = b;
    inf.sigma = sigma;
    inf.time_s = std::chrono::duration<double>(t_end - t_begin).count();
    inf.iters_outer = outer;
    inf.iters_inner = inner_total;
    inf.cg_iters = cg_total;
    inf.proj_passes = c->proj_passes;
    inf.p = (int32_t)c->hs->sc.p;
    inf.n_sv = (int32_t)c->hs->sc.nsv;
    inf.ls_fail = ls_fail;
    inf.ls_trials = ls_trials;
    inf.grad_steps = grad_steps;
    inf.proj_capped = c->proj_capped;
    inf.status = status;
    inf.lowrank_steps = c->lowrank_steps;
    if (info) *info = inf;
    return status;
}

extern "C" ssnalm_status ssnalm_solve(ssnalm_ctx* c, const double* x0, double* x_out, double* w_out,
                                      double* b_out, ssnalm_info* info) {
    if (c && c->kern) {
        if (!x_out) return fail(SSNALM_E_BADARG, "null argument");
        if (w_out) return fail(SSNALM_E_BADARG, "kernel contexts have no primal weights: pass w_out = NULL");
        StreamScope scope_(c);
        return solve_kernel(c, x0, x_out, b_out, info);
    }
    if (!c || !x_out) return fail(SSNALM_E_BADARG, "null argument");
    StreamScope scope_(c);
    const auto t_begin = std::chrono::steady_clock::now();
    const ssnalm_options& o = c->opt;
    const int64_t n = c->n, q = c->q;
    c->proj_passes = 0;
    c->proj_capped = 0;
    c->lr_valid = false;             // repeated solves take identical steps
    c->lowrank_steps = 0;
    ssnalm_info inf;
    memset(&inf, 0, sizeof inf);
    int inner_total = 0, cg_total = 0, ls_fail = 0, outer = 0, ls_trials = 0, grad_steps = 0;
    ssnalm_status status = SSNALM_MAXITER;

    // x^0: zero or the projection of the warm start; omega^0 = A^T x^0
    if (x0) {
        STCHK(project_into(c, x0, nullptr, 0.0, nullptr, 3));
        STCHK(sync_state(c));
        bool more;
        STCHK(project_finish(c, x0, 3, &more));
        proj_apply(c, x0, 3, c->xk, nullptr);
        op_atmul(c, c->xk, nullptr, nullptr, 1.0, c->om, nullptr);
    } else if (!c->zero_feasible) {
        // x^0 = Pi(0) when 0 violates the constraints (general form)
        launch_fill(c->nv, 0.0, n, c->st);
        STCHK(project_into(c, c->nv, nullptr, 0.0, nullptr, 3));
        STCHK(sync_state(c));
        bool more;
        STCHK(project_finish(c, c->nv, 3, &more));
        proj_apply(c, c->nv, 3, c->xk, nullptr);
        op_atmul(c, c->xk, nullptr, nullptr, 1.0, c->om, nullptr);
    } else {
        launch_fill(c->xk, 0.0, n, c->st);
        launch_fill(c->om, 0.0, q, c->st);
    }
    double sigma = o.sigma0;
    double R = INFINITY, b = NAN, best_R = INFINITY, best_b = NAN, hinge = NAN, best_hinge = NAN;
    bool have_best = false;      // x_out holds the best x seen when the cap is hit

    for (int k = 0; k < o.max_outer; ++k) {
        outer = k + 1;
        const double eps_k = std::pow(o.eps_decay, (double)k);
        // fresh A omega and u for this outer iteration
        op_amul(c, c->om, c->aw);
        launch_u_from(c->xk, c->aw, sigma, c->u, n, c->st, c->lin);
        c->base = 0;
        STCHK(project_into(c, c->u, nullptr, 0.0, nullptr, c->base));
        STCHK(sync_state(c));
        bool more;
        STCHK(project_finish(c, c->u, c->base, &more));
        // x~, J and distance to x^k: reuse the line-search finalize with alpha = 0
        ls_fin(c, c->u, c->u, nullptr, 0.0, c->base, c->base, c->xk, c->xt, c->jm);
        gradient(c, c->xt, c->jm);
        STCHK(sync_state(c));
        c->proj_passes += c->hs->ps[c->base].passes;
        c->proj_capped += c->hs->ps[c->base].approx;
        for (int j = 0; j < o.max_inner; ++j) {
            const Scalars& hsc = c->hs->sc;
            const double gn = std::sqrt(hsc.gnorm2);
            const double dist = std::sqrt(hsc.dist2);
            const double crit = std::min(eps_k, eps_k * dist) / std::sqrt(sigma);
            const double flo = o.floor_rel * (1.0 + std::sqrt(hsc.omega2));
            if (!std::isfinite(gn)) return fail(SSNALM_E_NONFINITE, "non-finite gradient");
            if (gn <= std::max(crit, flo)) break;
            const int64_t p = hsc.p;
            // Step 1: Newton direction
            int cgi = 0;
            const double cg_tol = std::min(o.eta, std::pow(gn, 1.0 + o.tau));
            STCHK(newton_dir(c, c->jm, p, c->g, c->sv, sigma, cg_tol, c->d, &cgi));
            cg_total += cgi;
            ++inner_total;
            // t = A d and the q-side scalars of the line search
            op_amul(c, c->d, c->td);
            launch_dots(3, c->g, c->d, &dsc(c)->gd, c->om, c->d, &dsc(c)->od, c->d, c->d,
                        &dsc(c)->dd, q, c->spart, cnt(c, CNT_DOTS2), c->st);
            // Step 2: Armijo line search on psi
            double alpha = 1.0;
            bool accepted = false, fell_back = false;
            const int trial = 1 - c->base;
            for (int m = 0; m <= o.max_backtracks; ++m) {
                ++ls_trials;
                STCHK(project_into(c, c->u, c->td, alpha * sigma, c->ut, trial, dps(c, c->base)));
                // the trial's sums are launched before the host knows whether the
                // first passes finished the projection (they nearly always do):
                // one host round trip per trial; otherwise more passes and the
                // sums again
                ls_fin(c, c->ut, c->u, c->td, alpha * sigma, trial, c->base, c->xk, c->xtt, c->jmt);
                STCHK(sync_state(c));
                STCHK(project_finish(c, c->ut, trial, &more));
                if (more) {
                    ls_fin(c, c->ut, c->u, c->td, alpha * sigma, trial, c->base, c->xk, c->xtt, c->jmt);
                    STCHK(sync_state(c));
                }
                c->proj_passes += c->hs->ps[trial].passes;
                c->proj_capped += c->hs->ps[trial].approx;
                const Scalars& s2 = c->hs->sc;
                if (m == 0 && !fell_back && gn > 0.0 &&
                    (!(s2.gd < 0.0) || (c->use_chol && s2.chol_fail))) {
                    // The direction is not one of descent (an inexact solve
                    // stopped early, or the factorisation met a non-positive
                    // pivot): psi is convex, so no step along it can pass the
                    // Armijo test.  Take the steepest-descent direction -g
                    // instead and start the search again at alpha = 1.
                    fell_back = true;
                    ++grad_steps;
                    c->lr_valid = false;     // the next step factors afresh
                    launch_scale_copy(c->d, c->g, -1.0, q, c->st);
                    op_amul(c, c->d, c->td);
                    launch_dots(3, c->g, c->d, &dsc(c)->gd, c->om, c->d, &dsc(c)->od, c->d, c->d,
                                &dsc(c)->dd, q, c->spart, cnt(c, CNT_DOTS2), c->st);
                    m = -1;
                    continue;
                }
                const double dpsi = alpha * s2.od + 0.5 * alpha * alpha * s2.dd + s2.dh / sigma;
                if (!std::isfinite(dpsi)) return fail(SSNALM_E_NONFINITE, "non-finite line search value");
                if (dpsi <= o.mu * alpha * s2.gd) { accepted = true; break; }
                alpha *= o.ls_delta;
            }
            if (!accepted) { ++ls_fail; break; }
            // Step 3: accept
            launch_axpy(c->om, c->d, alpha, q, c->st);
            launch_axpy(c->aw, c->td, alpha, n, c->st);
            std::swap(c->u, c->ut);
            std::swap(c->xt, c->xtt);
            std::swap(c->jm, c->jmt);
            c->base = trial;
            gradient(c, c->xt, c->jm);
            STCHK(sync_state(c));
        }
        // Step 2 of Algorithm 1: x^{k+1} = Pi(u(omega^{k+1})) = xt
        std::swap(c->xk, c->xt);
        // A^T x^{k+1} = omega - g
        launch_sub(c->om, c->g, c->qv, q, c->st);
        double sumx = 0.0;
        STCHK(kkt(c, c->xk, c->qv, &R, &b, &sumx, &hinge));
        if (o.verbose)
            fprintf(stderr, "[ssnalm] k=%d sigma=%.3g R_KKT=%.3e newton=%d cg=%d p=%lld passes=%d\n",
                    k, sigma, R, inner_total, cg_total, (long long)c->hs->sc.p, c->proj_passes);
        if (!std::isfinite(R)) return fail(SSNALM_E_NONFINITE, "non-finite KKT residual");
        if (R <= c->tol) { status = SSNALM_OK; break; }
        if (R < best_R) {
            best_R = R;
            best_b = b;
            best_hinge = hinge;
            HIPCHK(hipMemcpyAsync(x_out, c->xk, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
            have_best = true;
        }
        sigma = std::min(o.rho * sigma, o.sigma_max);
    }
    if (status == SSNALM_OK || !have_best || R <= best_R) {
        HIPCHK(hipMemcpyAsync(x_out, c->xk, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        R = best_R;
        b = best_b;
        hinge = best_hinge;
    }
    if (status != SSNALM_OK && ls_fail > 0 && ls_fail >= outer) status = SSNALM_LINESEARCH_FAIL;
    // w = A^T x, objective and the paper's columns
    op_atmul(c, x_out, nullptr, nullptr, 1.0, c->qv, nullptr);
    launch_dots(1, c->qv, c->qv, &dsc(c)->dd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                q, c->spart, cnt(c, CNT_DOTS), c->st);
    if (c->gen) launch_gcount(x_out, c->gbox, n, dsc(c), c->spart, c->st);
    else launch_count_x(x_out, n, c->C, dsc(c), c->spart, cnt(c, CNT_APPLY), c->st);
    if (c->lin)
        launch_dots(1, c->lin, x_out, &dsc(c)->cx, nullptr, nullptr, nullptr, nullptr, nullptr,
                    nullptr, n, c->spart, cnt(c, CNT_DOTS2), c->st);
    if (w_out) {
        if (c->svr) launch_scale_copy(w_out, c->qv, -1.0, q, c->st);   // w = X^T (z - x)
        else if (c->qperm) q_out(c, c->qv, w_out);
        else HIPCHK(hipMemcpyAsync(w_out, c->qv, sizeof(double) * q, hipMemcpyDeviceToDevice, c->st));
    }
    HIPCHK(hipGetLastError());
    STCHK(sync_state(c));
    const double sumx = c->hs->sc.sumx;
    prof_harvest(c);
    const double w2 = c->hs->sc.dd;
    const auto t_end = std::chrono::steady_clock::now();
    inf.rkkt = R;
    inf.obj = 0.5 * w2 + (c->lin ? c->hs->sc.cx : -sumx);
    if (c->svr) b = -b;          // the regression bias (the tube's center is w^T x + b)
    inf.b = b;
    {
        // relative duality gap of the C-SVC primal at (w, b) and the dual
        // objective: P(w, b) + f(x) >= 0 for every feasible x and every b
        const double P = 0.5 * w2 + c->C * hinge;
        inf.gap = std::isfinite(P) ? (P + inf.obj) / (1.0 + std::fabs(P) + std::fabs(inf.obj)) : NAN;
    }
    if (b_out) *b_out = b;
    inf.sigma = sigma;
    inf.time_s = std::chrono::duration<double>(t_end - t_begin).count();
    inf.iters_outer = outer;
    inf.iters_inner = inner_total;
    inf.cg_iters = cg_total;
    inf.proj_passes = c->proj_passes;
    inf.p = (int32_t)c->hs->sc.p;
    inf.n_sv = (int32_t)c->hs->sc.nsv;
    inf.ls_fail = ls_fail;
    inf.ls_trials = ls_trials;
    inf.grad_steps = grad_steps;
    inf.proj_capped = c->proj_capped;
    inf.status = status;
    inf.lowrank_steps = c->lowrank_steps;
    if (info) *info = inf;
    return status;
}


// ---------------------------------------------------------------- step ops
extern "C" ssnalm_status ssnalm_op_amul(ssnalm_ctx* c, const double* v, double* t) {
    if (!c || !v || !t) return fail(SSNALM_E_BADARG, "null argument");
    StreamScope scope_(c);
    if (c->kern) STCHK(qprod(c, v, t));                 // t = Q v
    else op_amul(c, q_in(c, v), t);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_atmul(ssnalm_ctx* c, const double* z, double* r) {
    if (!c || !z || !r) return fail(SSNALM_E_BADARG, "null argument");
    if (c->kern) return fail(SSNALM_E_BADARG, "op_atmul needs the samples: not for kernel contexts");
    StreamScope scope_(c);
    op_atmul(c, z, nullptr, nullptr, 1.0, c->qperm ? c->qout : r, nullptr);
    q_out(c, c->qout, r);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_project(ssnalm_ctx* c, const double* v, double* x,
                                           uint8_t* free_mask, double* lam, int64_t* p,
                                           int32_t* passes) {
    if (!c || !v || !x) return fail(SSNALM_E_BADARG, "null argument");
    StreamScope scope_(c);
    STCHK(project_into(c, v, nullptr, 0.0, nullptr, 3));
    STCHK(sync_state(c));
    bool more;
    STCHK(project_finish(c, v, 3, &more));
    proj_apply(c, v, 3, x, free_mask);
    HIPCHK(hipGetLastError());
    STCHK(sync_state(c));
    if (lam) *lam = c->hs->ps[3].lam;
    if (p) *p = c->hs->sc.p;
    if (passes) *passes = c->hs->ps[3].passes;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_newton(ssnalm_ctx* c, const uint8_t* free_mask, const double* g,
                                          double sigma, double cg_tol, double* d, int32_t* cg_iters) {
    if (!c || !free_mask || !g || !d) return fail(SSNALM_E_BADARG, "null argument");
    if (c->svr || c->gen || c->kern) return fail(SSNALM_E_BADARG, "op_newton is for linear C-SVC contexts");
    StreamScope scope_(c);
    if (!(sigma > 0.0)) return fail(SSNALM_E_BADARG, "sigma must be > 0");
    // s = X_J^T 1 and p
    launch_compact(free_mask, c->n, c->jlist, &dsc(c)->p, c->blk, cnt(c, CNT_CMP), c->st);
    if (c->kind == SSNALM_DENSE) {
        const int nb = atmul_dense_nblk(c->n);
        launch_fill(c->nv, 0.0, c->n, c->st);
        launch_atmul_dense(c->dtype, c->X, c->y, c->nv, free_mask, c->n, c->q, c->part, c->part2, c->st);
        launch_reduce_cols(c->part2, nb, c->q, nullptr, 1.0, c->sv, c->st);
    } else {
        launch_segsum(c->tr, nullptr, nullptr, free_mask, nullptr, nullptr, c->sv, c->st);
    }
    STCHK(sync_state(c));
    int cgi = 0;
    STCHK(newton_dir(c, free_mask, c->hs->sc.p, q_in(c, g), c->sv, sigma, cg_tol,
                     c->qperm ? c->qout : d, &cgi));
    q_out(c, c->qout, d);
    HIPCHK(hipGetLastError());
    STCHK(sync_state(c));
    if (c->use_chol && c->hs->sc.chol_fail) return fail(SSNALM_E_NONFINITE, "Cholesky met a non-positive pivot");
    if (cg_iters) *cg_iters = cgi;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_gram(ssnalm_ctx* c, const uint8_t* free_mask, double* G) {
    if (!c || !free_mask || !G) return fail(SSNALM_E_BADARG, "null argument");
    if (c->svr || c->gen || c->kern) return fail(SSNALM_E_BADARG, "op_gram is for linear C-SVC contexts");
    StreamScope scope_(c);
    if (c->kind != SSNALM_DENSE || !c->use_chol) return fail(SSNALM_E_BADARG, "Gram matrix needs a dense Cholesky context");
    launch_compact(free_mask, c->n, c->jlist, &dsc(c)->p, c->blk, cnt(c, CNT_CMP), c->st);
    STCHK(sync_state(c));
    const int64_t p = c->hs->sc.p;
    if (p == 0) {
        launch_fill(G, 0.0, c->q * c->q, c->st);
    } else if (c->mixed) {
        launch_syrk_mfma(c->X, c->dtype, c->q, c->jlist, p, G, c->mpart, c->mpart_cap, c->st);
    } else {
        launch_syrk_gather(c->dtype, c->X, c->q, c->jlist, p, G, c->part, c->part_cap, c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_kernel_newton(ssnalm_ctx* c, const uint8_t* free_mask,
                                                  const double* sv, double sigma, double cg_tol,
                                                  double* d, double* Qd, double* dQd, int32_t* cg_iters) {
    if (!c || !free_mask || !sv || !d || !Qd) return fail(SSNALM_E_BADARG, "null argument");
    if (!c->kern) return fail(SSNALM_E_BADARG, "op_kernel_newton is for kernel contexts");
    if (!(sigma > 0.0)) return fail(SSNALM_E_BADARG, "sigma must be > 0");
    StreamScope scope_(c);
    launch_compact(free_mask, c->n, c->jlist, &dsc(c)->p, c->blk, cnt(c, CNT_CMP), c->st);
    HIPCHK(hipMemcpyAsync(c->ks, sv, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->st));
    STCHK(qprod(c, c->ks, c->kqs));
    int cgi = 0;
    bool direct = false;
    STCHK(kernel_newton(c, free_mask, c->hs->sc.p, c->ks, c->kqs, sigma, cg_tol, d, Qd, &cgi, &direct));
    launch_dots(1, d, Qd, &dsc(c)->dd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c->n,
                c->spart, cnt(c, CNT_DOTS), c->st);
    HIPCHK(hipGetLastError());
    STCHK(sync_state(c));
    if (direct && c->hs->sc.chol_fail) return fail(SSNALM_E_NONFINITE, "Cholesky met a non-positive pivot");
    if (dQd) *dQd = c->hs->sc.dd;
    if (cg_iters) *cg_iters = cgi;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_linesearch_trial(ssnalm_ctx* c, const double* u, const double* t,
                                                    double lam, double alpha, double sigma,
                                                    double* lam_a, double* dh) {
    if (!c || !u || !t) return fail(SSNALM_E_BADARG, "null argument");
    StreamScope scope_(c);
    // base state: the given lam
    c->hs->ps[0] = ProjState{};
    c->hs->ps[0].lam = lam;
    c->hs->ps[0].done = 1;
    HIPCHK(hipMemcpyAsync(&c->ds->ps[0], &c->hs->ps[0], sizeof(ProjState), hipMemcpyHostToDevice, c->st));
    launch_fill(c->nv2, 0.0, c->n, c->st);
    STCHK(project_into(c, u, t, alpha * sigma, c->ut, 1));
    STCHK(sync_state(c));
    bool more;
    STCHK(project_finish(c, c->ut, 1, &more));
    ls_fin(c, c->ut, u, t, alpha * sigma, 1, 0, c->nv2, c->xtt, c->jmt);
    HIPCHK(hipGetLastError());
    STCHK(sync_state(c));
    if (lam_a) *lam_a = c->hs->ps[1].lam;
    if (dh) *dh = c->hs->sc.dh;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_kernel_stats(ssnalm_ctx* c, int32_t which, ssnalm_kstat* out,
                                             int32_t reset) {
    if (!c || which < 0 || which >= SSNALM_K_COUNT) return fail(SSNALM_E_BADARG, "bad kernel class");
    prof_harvest(c);
    if (out) *out = c->kst[which];
    if (reset) memset(c->kst, 0, sizeof c->kst);
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_set_profile(ssnalm_ctx* c, int32_t profile) {
    if (!c) return fail(SSNALM_E_BADARG, "null argument");
    c->opt.profile = profile;
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_op_rkkt(ssnalm_ctx* c, const double* x, double* rkkt, double* b) {
    if (!c || !x) return fail(SSNALM_E_BADARG, "null argument");
    StreamScope scope_(c);
    double R, bb;
    if (c->kern) {
        STCHK(qprod(c, x, c->nv));
        STCHK(kkt_nv(c, x, &R, &bb, nullptr));
    } else {
        op_atmul(c, x, nullptr, nullptr, 1.0, c->qv, nullptr);
        STCHK(kkt(c, x, c->qv, &R, &bb, nullptr));
    }
    HIPCHK(hipGetLastError());
    if (rkkt) *rkkt = R;
    if (b) *b = bb;
    return SSNALM_OK;
}

// ---------------------------------------------------------------- warm start
// Features of the learned warm start (definition in include/ssnalm.h):
// p = Pi(C e), w1 = t* A^T p with the exact step t*, b1 from the class
// means of x_i^T w1, margins m_i, and the projection X R.
extern "C" ssnalm_status ssnalm_ws_features(ssnalm_ctx* c, const float* R, float* Z) {
    if (!c || !R || !Z) return fail(SSNALM_E_BADARG, "null argument");
    if (c->svr || c->gen || c->kern) return fail(SSNALM_E_BADARG, "ws_features is for linear C-SVC contexts");
    StreamScope scope_(c);
    if (c->kind != SSNALM_DENSE) return fail(SSNALM_E_BADARG, "warm-start features need dense X");
    const int64_t n = c->n, q = c->q;
    const double C = c->C;
    launch_fill(c->nv, C, n, c->st);
    STCHK(project_into(c, c->nv, nullptr, 0.0, nullptr, 3));
    STCHK(sync_state(c));
    bool more;
    STCHK(project_finish(c, c->nv, 3, &more));
    launch_proj_apply(c->nv, c->y, n, C, dps(c, 3), c->xt, nullptr, dsc(c), c->spart,
                      cnt(c, CNT_APPLY), c->st);
    op_atmul(c, c->xt, nullptr, nullptr, 1.0, c->qv, nullptr);              // A^T p
    launch_dots(1, c->qv, c->qv, &dsc(c)->dd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                q, c->spart, cnt(c, CNT_DOTS), c->st);
    launch_count_x(c->xt, n, C, dsc(c), c->spart, cnt(c, CNT_APPLY), c->st);   // e^T p
    STCHK(sync_state(c));
    const double den = c->hs->sc.dd, sum = c->hs->sc.sumx;
    const double t = den > 0.0 ? std::min(std::max(sum / den, 0.0), 1.0) : 0.0;
    launch_scale_copy(c->qv2, c->qv, t, q, c->st);                            // w1
    op_amul(c, c->qv2, c->aw);                                                // A w1
    constexpr int nb = 256;
    launch_class_sums(c->aw, c->y, n, c->spart, nb, c->st);
    std::vector<double> cs(4 * nb);
    HIPCHK(hipMemcpyAsync(cs.data(), c->spart, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double sp = 0.0, cp = 0.0, sn = 0.0, cn = 0.0;
    for (int b = 0; b < nb; ++b) {
        sp += cs[4 * b];
        cp += cs[4 * b + 1];
        sn += cs[4 * b + 2];
        cn += cs[4 * b + 3];
    }
    const double b1 = (cp > 0.0 && cn > 0.0) ? -0.5 * (sp / cp + sn / cn) : -(sp + sn) / (cp + cn);
    launch_ws_features(c->dtype, c->X, c->y, n, q, R, c->aw, b1, (float)std::log10((double)n * C), Z,
                       c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_ws_x0(ssnalm_ctx* c, const float* out, double* x0) {
    if (!c || !out || !x0) return fail(SSNALM_E_BADARG, "null argument");
    if (c->svr || c->gen) return fail(SSNALM_E_BADARG, "ws_x0 is for C-SVC contexts");
    StreamScope scope_(c);
    launch_ws_x0(out, c->n, c->C, x0, c->st);
    HIPCHK(hipGetLastError());
    return SSNALM_OK;
}

extern "C" ssnalm_status ssnalm_ws_labels(ssnalm_ctx* c, const double* x, int32_t* status,
                                          float* target) {
    if (!c || !x || !status || !target) return fail(SSNALM_E_BADARG, "null argument");
    if (c->svr || c->gen) return fail(SSNALM_E_BADARG, "ws_labels is for C-SVC contexts");
    StreamScope scope_(c);
    launch_ws_labels(x, c->n, c->C, status, target, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return SSNALM_OK;
}

// Screening solve from the network's status prediction (include/ssnalm.h).
extern "C" ssnalm_status ssnalm_ws_solve(ssnalm_ctx* c, const float* out, double keep_frac,
                                         int32_t max_rounds, double* x_out, double* w_out,
                                         ssnalm_info* info, ssnalm_ws_stats* stats) {
    if (!c || !out || !x_out) return fail(SSNALM_E_BADARG, "null argument");
    if (c->svr || c->gen || c->kern) return fail(SSNALM_E_BADARG, "ws_solve is for linear C-SVC contexts");
    StreamScope scope_(c);
    if (c->kind != SSNALM_DENSE) return fail(SSNALM_E_BADARG, "screening needs dense X");
    if (!(keep_frac > 0.0) || keep_frac > 1.0) return fail(SSNALM_E_BADARG, "keep_frac must be in (0, 1]");
    const auto t_begin = std::chrono::steady_clock::now();
    const int64_t n = c->n, q = c->q;
    const size_t esz = c->dtype == SSNALM_F64 ? 8 : (c->dtype == SSNALM_F32 ? 4 : 2);
    ssnalm_ws_stats st;
    memset(&st, 0, sizeof st);
    ssnalm_info agg;
    memset(&agg, 0, sizeof agg);
    // per-call buffers: keep mask, row list, reduced X / y / x / w
    struct Bufs {
        std::vector<void*> v;
        ~Bufs() { for (void* p : v) hipFree(p); }
    } bufs;
    auto dal = [&](void** p, size_t bytes) -> ssnalm_status {
        if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            hipGetLastError();
            return fail(SSNALM_E_OOM, "screening buffers: allocation of %zu bytes failed", bytes);
        }
        bufs.v.push_back(*p);
        return SSNALM_OK;
    };
    uint8_t* keep = nullptr;
    int32_t* list = nullptr;
    void* Xk = nullptr;
    int8_t* yk = nullptr;
    double* xk = nullptr;
    double* x0k = nullptr;
    STCHK(dal((void**)&x0k, 8 * n));
    STCHK(dal((void**)&keep, n));
    STCHK(dal((void**)&list, 4 * n));
    STCHK(dal(&Xk, esz * (size_t)n * q));
    STCHK(dal((void**)&yk, n));
    STCHK(dal((void**)&xk, 8 * n));
    // rows ranked by P(x_i* = 0): keep the keep_frac n rows least surely at 0
    // (cut at a histogram bin of -log10(1 - P0); ties in the cut bin are kept)
    {
        const int nb = p0_hist_bins();
        unsigned* hist = nullptr;
        STCHK(dal((void**)&hist, sizeof(unsigned) * nb));
        launch_p0_hist(out, n, hist, c->st);
        std::vector<unsigned> hh(nb);
        HIPCHK(hipMemcpyAsync(hh.data(), hist, sizeof(unsigned) * nb, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        const double want = keep_frac * (double)n;
        double acc = 0.0;
        int cut = nb;
        for (int b = 0; b < nb; ++b) {
            acc += hh[b];
            if (acc >= want) { cut = b + 1; break; }
        }
        launch_ws_keep_bin(out, n, cut, keep, c->st);
    }
    double t_red = 0.0;
    bool done = false;
    long long prev_m = -1;
    // The reduced problem is solved at the full problem's tol: with the left-out
    // rows at 0 and outside the margin their residual terms vanish, so the
    // full-problem R_KKT is the reduced one.  When it is not (no new margin
    // violators, R_KKT still above tol), the same rows are solved again from
    // that solution at half the previous tolerance.
    double tol_k = c->tol;
    for (int round = 0; round < max_rounds && !done; ++round) {
        launch_compact(keep, n, list, &dsc(c)->p, c->blk, cnt(c, CNT_CMP), c->st);
        STCHK(sync_state(c));
        const long long m = c->hs->sc.p;
        if (m < 2 || 2 * m > n) break;                      // not worth it
        if (m == prev_m) tol_k *= 0.5;                      // nothing new: tighten instead
        prev_m = m;
        launch_gather_rows(c->dtype, c->X, c->y, list, m, q, Xk, yk, c->st);
        HIPCHK(hipStreamSynchronize(c->st));
        const auto t0 = std::chrono::steady_clock::now();
        ssnalm_problem pk;
        memset(&pk, 0, sizeof pk);
        pk.kind = SSNALM_DENSE;
        pk.dtype = c->dtype;
        pk.n = m;
        pk.q = q;
        pk.X = Xk;
        pk.y = yk;
        pk.C = c->C;
        pk.tol = tol_k;
        ssnalm_options ok = c->opt;
        ok.profile = 0;
        ssnalm_ctx* sub = nullptr;
        ssnalm_status s1 = ssnalm_create(&sub, &pk, &ok, c->st);
        if (s1 < 0) return s1;
        ssnalm_info ik;
        // later rounds start from the previous round's solution (0 on the added rows)
        if (round > 0) launch_gather_vec(x_out, list, m, x0k, c->st);
        s1 = ssnalm_solve(sub, round > 0 ? x0k : nullptr, xk, c->qv2, nullptr, &ik);
        ssnalm_destroy(sub);
        if (s1 < 0) return s1;
        t_red += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        st.rounds = round + 1;
        st.kept = (int32_t)m;
        agg.iters_outer += ik.iters_outer;
        agg.iters_inner += ik.iters_inner;
        agg.proj_passes += ik.proj_passes;
        agg.proj_capped += ik.proj_capped;
        agg.grad_steps += ik.grad_steps;
        agg.ls_trials += ik.ls_trials;
        agg.ls_fail += ik.ls_fail;
        // x on all rows, judged on the full problem; w = A_K^T x_K
        launch_fill(x_out, 0.0, n, c->st);
        launch_scatter(list, m, xk, x_out, c->st);
        double R, b, sumx, hinge;
        STCHK(kkt(c, x_out, c->qv2, &R, &b, &sumx, &hinge));
        if (s1 == SSNALM_OK && R <= c->tol) {
            done = true;
            st.rkkt_full = R;
            agg.rkkt = R;
            agg.b = b;
            agg.gap = hinge;          // turned into the gap once |w|^2 is known
            break;
        }
        // add the rows whose margin under (w, b) is below 1 (x_out keeps the
        // reduced solution for the next round's start)
        op_amul(c, c->qv2, c->aw);
        launch_ws_violators(c->aw, c->y, n, b, keep, c->st);
    }
    st.t_reduced = t_red;
    if (!done) {
        // the prediction did not lead to a solution: the plain cold solve of
        // the full problem decides, and an OK result is reported as
        // WARMSTART_REJECTED
        st.fallback = 1;
        ssnalm_info ic;
        const ssnalm_status s2 = ssnalm_solve(c, nullptr, x_out, w_out, nullptr, &ic);
        st.rkkt_full = ic.rkkt;
        if (stats) *stats = st;
        if (s2 == SSNALM_OK) ic.status = SSNALM_WARMSTART_REJECTED;
        if (info) *info = ic;
        return s2 == SSNALM_OK ? SSNALM_WARMSTART_REJECTED : s2;
    }
    // w, objective and counts of the returned x
    op_atmul(c, x_out, nullptr, nullptr, 1.0, c->qv, nullptr);
    launch_dots(1, c->qv, c->qv, &dsc(c)->dd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                q, c->spart, cnt(c, CNT_DOTS), c->st);
    launch_count_x(x_out, n, c->C, dsc(c), c->spart, cnt(c, CNT_APPLY), c->st);
    if (w_out) HIPCHK(hipMemcpyAsync(w_out, c->qv, sizeof(double) * q, hipMemcpyDeviceToDevice, c->st));
    STCHK(sync_state(c));
    if (info) {
        agg.obj = 0.5 * c->hs->sc.dd - c->hs->sc.sumx;
        const double P = 0.5 * c->hs->sc.dd + c->C * agg.gap;
        agg.gap = (P + agg.obj) / (1.0 + std::fabs(P) + std::fabs(agg.obj));
        agg.sigma = NAN;
        agg.p = (int32_t)c->hs->sc.p;
        agg.n_sv = (int32_t)c->hs->sc.nsv;
        agg.status = SSNALM_OK;
        agg.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
        *info = agg;
    }
    if (stats) *stats = st;
    return SSNALM_OK;
}
