// Host side of the batched solve (ssnalm_solve_batch, include/ssnalm.h).
//
// Every problem runs Algorithm 1 (augmented Lagrangian on the restricted
// dual) with Algorithm 3 (semismooth Newton on psi, Cholesky step) exactly as
// ssnalm_solve does; what changes is the schedule.  The host keeps one small
// state machine per problem (start of an ALM iteration -> Newton steps ->
// KKT test) and advances all of them in lockstep sweeps.  Each phase of a
// sweep uploads the per-problem parameters (active flag, sigma, step
// length), issues one launch per kernel for all problems taking part, and
// reads back one array of per-problem scalars: the stopping tests and the
// Armijo verdicts are taken on the host for all problems at once.  The
// Newton-direction sequence and the line-search-trial sequence have no host
// decision inside, so they are captured once into HIP graphs and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "ssn_internal.h"

using namespace ssn;

#define BCHK(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_error(SSNALM_E_HIP, "%s failed: %s (%s:%d)", #expr,                   \
                             hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)
#define BST(expr)                            \
    do {                                     \
        ssnalm_status s_ = (expr);           \
        if (s_ < 0) return s_;               \
    } while (0)

namespace {

enum Phase { PH_OUTER, PH_INNER, PH_KKT, PH_DONE };

struct HP {                        // host state of one problem
    Phase  phase = PH_OUTER;
    int    outer = 0, inner = 0;   // ALM iterations started; Newton steps in this one
    double sigma = 1.0, eps = 1.0, tol = 1e-6;
    double R = INFINITY, b = NAN, best_R = INFINITY, best_b = NAN;
    double hinge = NAN, best_hinge = NAN;   // hinge sum of the C-SVC primal at (A^T x, b)
    bool   have_best = false;
    int    inner_total = 0, ls_fail = 0, ls_trials = 0, passes = 0;
    double alpha = 1.0;
    int    status = SSNALM_MAXITER;
};

struct Shape { int grid, unr; };
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, Shape> g_tune;   // (dtype, q, vec, log2 items)

thread_local ssnalm_kstat g_bks[SSNALM_K_COUNT];

constexpr int kRing = 16;          // pinned parameter slots between two syncs
constexpr int kPassBatch = 5;      // multisection passes issued before the first check

struct Batch {
    int nprob = 0, q = 0, dtype = 0, vec = 1, nitems = 0, gcap = 0;
    int64_t ntot = 0;
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<void*> owned;
    std::vector<BProb> hprob;
    BPar* par_h = nullptr;         // pinned: kRing slots of nprob entries
    int ring = 0;
    BState* bs_h = nullptr;        // pinned mirror of bs_d
    BLaunch L{};
    int4* items = nullptr;
    BProb* prob_d = nullptr;
    BPar* par_d = nullptr;
    BState* bs_d = nullptr;
    double *xk = nullptr, *aw = nullptr, *u = nullptr, *ut = nullptr, *td = nullptr;
    double *xt = nullptr, *xtt = nullptr, *nv = nullptr, *nv2 = nullptr, *xbest = nullptr;
    uint8_t *jm = nullptr, *jmt = nullptr;
    int32_t* list = nullptr;
    double *om = nullptr, *g = nullptr, *sv = nullptr, *d = nullptr, *qv = nullptr, *M = nullptr;
    hipGraphExec_t gx_newton = nullptr, gx_trial = nullptr;
    std::vector<char> built;       // active set of the current work list (empty: none)
    // HIP-event timing of the full-pass A v launches (profile = 1)
    bool prof = false;
    struct Pend { hipEvent_t a, b; double bytes; int first; };
    std::vector<Pend> pend;
    std::vector<hipEvent_t> evpool;
    ~Batch() {
        if (s) hipStreamSynchronize(s);
        for (auto& p : pend) { evpool.push_back(p.a); evpool.push_back(p.b); }
        for (hipEvent_t e : evpool) hipEventDestroy(e);
        if (gx_newton) hipGraphExecDestroy(gx_newton);
        if (gx_trial) hipGraphExecDestroy(gx_trial);
        for (void* p : owned) hipFree(p);
        if (par_h) hipHostFree(par_h);
        if (bs_h) hipHostFree(bs_h);
        if (ev) hipEventDestroy(ev);
        if (s) hipStreamDestroy(s);
    }
};

template <typename T>
ssnalm_status balloc(Batch& B, T** p, int64_t count) {
    void* q = nullptr;
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (hipMalloc(&q, bytes) != hipSuccess) {
        hipGetLastError();
        return set_error(SSNALM_E_OOM, "device allocation of %zu bytes failed", bytes);
    }
    B.owned.push_back(q);
    *p = (T*)q;
    return SSNALM_OK;
}

// Upload the per-problem parameters with the given active set.
ssnalm_status upload(Batch& B, const std::vector<HP>& hp, const std::vector<char>& act) {
    if (B.ring == kRing) {
        BCHK(hipStreamSynchronize(B.s));
        B.ring = 0;
    }
    BPar* slot = B.par_h + (size_t)B.ring * B.nprob;
    ++B.ring;
    for (int k = 0; k < B.nprob; ++k) {
        slot[k].active = act[k] ? 1 : 0;
        slot[k].pad_ = 0;
        slot[k].sigma = hp[k].sigma;
        slot[k].alpha = hp[k].alpha;
    }
    BCHK(hipMemcpyAsync(B.par_d, slot, sizeof(BPar) * B.nprob, hipMemcpyHostToDevice, B.s));
    return SSNALM_OK;
}

// Upload, then rebuild the work list when the active set changed.
ssnalm_status activate(Batch& B, const std::vector<HP>& hp, const std::vector<char>& act) {
    BST(upload(B, hp, act));
    if (B.built != act) {
        lb_build_wl(B.L, B.items);
        B.built = act;
    }
    return SSNALM_OK;
}

ssnalm_status readback(Batch& B) {
    BCHK(hipGetLastError());
    BCHK(hipMemcpyAsync(B.bs_h, B.bs_d, sizeof(BState) * B.nprob, hipMemcpyDeviceToHost, B.s));
    BCHK(hipStreamSynchronize(B.s));
    B.ring = 0;
    for (auto& p : B.pend) {              // every event pair has completed
        float ms = 0.f;
        hipEventElapsedTime(&ms, p.a, p.b);
        ssnalm_kstat& k = g_bks[SSNALM_K_AMUL];
        k.launches += p.first;
        k.seconds += 1e-3 * ms;
        k.bytes += p.bytes;
        B.evpool.push_back(p.a);
        B.evpool.push_back(p.b);
    }
    B.pend.clear();
    return SSNALM_OK;
}

hipEvent_t ev_get(Batch& B) {
    if (!B.evpool.empty()) {
        hipEvent_t e = B.evpool.back();
        B.evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
}

// A v over the rows of the active problems, timed when profiling.  Bytes:
// X rows, labels, the n-vector written, the q-vectors read.
void timed_amul(Batch& B, const std::vector<char>& act, const double* V, double* t) {
    if (!B.prof) {
        lb_amul(B.L, V, t);
        return;
    }
    const double esz = B.dtype == SSNALM_F64 ? 8.0 : (B.dtype == SSNALM_F32 ? 4.0 : 2.0);
    double bytes = 0.0;
    for (int k = 0; k < B.nprob; ++k)
        if (act[k]) bytes += (double)B.hprob[k].n * (B.q * esz + 1.0 + 8.0) + 8.0 * B.q;
    // each kernel of the launch gets a dispatch-attached event pair (its own
    // execution time); the launch's bytes ride on the first pair
    struct S : KTimeSink {
        Batch* B;
        double bytes;
        int first = 1;
        void pair(hipEvent_t* a, hipEvent_t* b) override {
            *a = ev_get(*B);
            *b = ev_get(*B);
            B->pend.push_back(Batch::Pend{*a, *b, bytes, first});
            bytes = 0.0;
            first = 0;
        }
    } sink;
    sink.B = &B;
    sink.bytes = bytes;
    g_ktime = &sink;
    lb_amul(B.L, V, t);
    g_ktime = nullptr;
}

// Newton direction for the active problems: J compaction, Gram, M,
// Cholesky solve, t = A d and g^T d, omega^T d, d^T d.
void seq_newton(Batch& B) {
    lb_compact(B.L, B.jm, B.list);
    lb_newton(B.L, B.list, B.sv, B.g, B.d, B.M);
    lb_amul(B.L, B.d, B.td);
    lb_qdots(B.L, 3, B.g, B.d, B.om, B.d, B.d, B.d, BS_GD);
}

// One line-search trial at each active problem's alpha: project
// u - alpha sigma t (first pass placed around the accepted multiplier), then
// the increments of psi and |x - x^k|.
void seq_trial(Batch& B) {
    lb_proj_init(B.L, B.u, B.td, B.ut, 1, 1);
    lb_proj_passes(B.L, B.ut, 1, kPassBatch);
    lb_ls_fin(B.L, B.ut, B.u, B.td, 1, 0, B.xk, B.xtt, B.jmt);
}

ssnalm_status run_seq(Batch& B, hipGraphExec_t* gx, void (*fn)(Batch&), bool graphs) {
    if (!graphs) {
        fn(B);
        BCHK(hipGetLastError());
        return SSNALM_OK;
    }
    if (!*gx) {
        hipGraph_t gr = nullptr;
        BCHK(hipStreamBeginCapture(B.s, hipStreamCaptureModeRelaxed));
        fn(B);
        const hipError_t e = hipStreamEndCapture(B.s, &gr);
        if (e != hipSuccess) return set_error(SSNALM_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(gx, gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        if (e2 != hipSuccess) {
            *gx = nullptr;
            return set_error(SSNALM_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e2));
        }
    }
    BCHK(hipGraphLaunch(*gx, B.s));
    return SSNALM_OK;
}

// Autotuner: time the dominant streaming kernel (A v over every row of the
// batch) for each candidate (persistent grid, rows in flight per lane
// group) and keep the fastest.  Both change only the schedule, not the
// arithmetic, so the choice never changes results.  Cached per shape class.
ssnalm_status choose_shape(Batch& B, const std::vector<HP>& hp, bool tune) {
    int lg = 0;
    while ((1 << lg) < B.nitems) ++lg;
    const auto key = std::make_tuple(B.dtype, B.q, B.vec, lg);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            B.L.grid = it->second.grid;
            B.L.unr = it->second.unr;
            return SSNALM_OK;
        }
    }
    B.L.grid = std::min(B.nitems, 1024);
    B.L.unr = 2;
    if (!tune) return SSNALM_OK;
    std::vector<char> all(B.nprob, 1);
    BST(activate(B, hp, all));
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    float best = INFINITY;
    Shape bs{B.L.grid, B.L.unr};
    const int grids[] = {256, 512, 1024, 2048, 4096};
    const int unrs[] = {1, 2, 4};
    for (int gcand : grids) {
        if (gcand > 2 * B.nitems && gcand != 256) continue;
        for (int ucand : unrs) {
            B.L.grid = gcand;
            B.L.unr = ucand;
            lb_amul(B.L, B.om, B.nv);                     // warm-up
            float tmin = INFINITY;
            for (int rep = 0; rep < 2; ++rep) {
                hipEventRecord(e0, B.s);
                lb_amul(B.L, B.om, B.nv);
                hipEventRecord(e1, B.s);
                hipEventSynchronize(e1);
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                tmin = std::min(tmin, ms);
            }
            if (tmin < best) {
                best = tmin;
                bs = Shape{gcand, ucand};
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    BCHK(hipGetLastError());
    B.L.grid = bs.grid;
    B.L.unr = bs.unr;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = bs;
    return SSNALM_OK;
}

ssnalm_status validate(int32_t count, const ssnalm_problem* probs, const ssnalm_options& o,
                       double* const* x_out) {
    if (count < 1 || !probs || !x_out) return set_error(SSNALM_E_BADARG, "count >= 1, probs and x_out are required");
    if (o.newton != SSNALM_NEWTON_AUTO && o.newton != SSNALM_NEWTON_CHOL)
        return set_error(SSNALM_E_BADARG, "the batched solve uses the Cholesky Newton step");
    if (o.precision != SSNALM_PREC_FP64) return set_error(SSNALM_E_BADARG, "the batched solve runs in fp64");
    const ssnalm_problem& p0 = probs[0];
    for (int32_t k = 0; k < count; ++k) {
        const ssnalm_problem& p = probs[k];
        if (p.kind != SSNALM_DENSE) return set_error(SSNALM_E_BADARG, "problem %d: batched problems must be dense", k);
        if (p.dtype < SSNALM_F64 || p.dtype > SSNALM_BF16) return set_error(SSNALM_E_BADARG, "problem %d: unknown dtype", k);
        if (p.dtype != p0.dtype || p.q != p0.q) return set_error(SSNALM_E_BADARG, "problem %d: dtype and q must match problem 0", k);
        if (p.q < 1 || p.q > batch_qmax()) return set_error(SSNALM_E_BADARG, "problem %d: q must be in [1, %d]", k, batch_qmax());
        if (p.n < 1 || p.n >= INT32_MAX) return set_error(SSNALM_E_BADARG, "problem %d: n must be in [1, 2^31)", k);
        if (!(p.C > 0.0) || !std::isfinite(p.C)) return set_error(SSNALM_E_BADARG, "problem %d: C must be finite and > 0", k);
        if (!(p.tol > 0.0)) return set_error(SSNALM_E_BADARG, "problem %d: tol must be > 0", k);
        if (!p.X || !p.y) return set_error(SSNALM_E_BADARG, "problem %d: X and y are required", k);
        if (!x_out[k]) return set_error(SSNALM_E_BADARG, "problem %d: x_out is null", k);
    }
    return SSNALM_OK;
}

ssnalm_status setup(Batch& B, int32_t count, const ssnalm_problem* probs, const ssnalm_options& o) {
    B.nprob = count;
    B.q = (int)probs[0].q;
    B.dtype = probs[0].dtype;
    const int esz = B.dtype == SSNALM_F64 ? 8 : (B.dtype == SSNALM_F32 ? 4 : 2);
    const int V = 16 / esz;
    B.vec = (B.q % V == 0) ? 1 : 0;
    // labels exactly +-1, finite X when asked, alignment for the vector loads
    std::vector<int8_t> yh;
    for (int k = 0; k < count; ++k) {
        const ssnalm_problem& p = probs[k];
        if (((uintptr_t)p.X) % 16 != 0) B.vec = 0;
        yh.resize(p.n);
        BCHK(hipMemcpy(yh.data(), p.y, p.n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < p.n; ++i)
            if (yh[i] != 1 && yh[i] != -1)
                return set_error(SSNALM_E_BADARG, "problem %d: label %lld is %d, not +-1", k, (long long)i, (int)yh[i]);
        if (o.check_finite) BST(scan_finite(p.X, p.dtype, p.n * p.q));
    }
    // static items and problem descriptors
    std::vector<int4> items;
    B.hprob.resize(count);
    int64_t off = 0;
    int gcap = 0;
    for (int k = 0; k < count; ++k) {
        const ssnalm_problem& p = probs[k];
        BProb& P = B.hprob[k];
        P.X = p.X;
        P.y = p.y;
        P.n = p.n;
        P.off = off;
        P.C = p.C;
        P.item0 = (int)items.size();
        for (int64_t r = 0; r < p.n; r += BRPI)
            items.push_back(make_int4(k, (int)r, (int)std::min<int64_t>(p.n, r + BRPI), 0));
        P.nitem = (int)items.size() - P.item0;
        off += p.n;
        gcap += batch_gram_items_max(p.n);
    }
    B.ntot = off;
    B.nitems = (int)items.size();
    B.gcap = gcap;
    const int64_t n = B.ntot, q = B.q, np = B.nprob, ni = B.nitems;
    BCHK(hipStreamCreateWithFlags(&B.s, hipStreamNonBlocking));
    BCHK(hipEventCreateWithFlags(&B.ev, hipEventDisableTiming));
#define BA(ptr, cnt_) BST(balloc(B, &(ptr), (cnt_)))
    BA(B.xk, n); BA(B.aw, n); BA(B.u, n); BA(B.ut, n); BA(B.td, n); BA(B.xt, n); BA(B.xtt, n);
    BA(B.nv, n); BA(B.nv2, n); BA(B.xbest, n); BA(B.jm, n); BA(B.jmt, n); BA(B.list, n);
    BA(B.om, np * q); BA(B.g, np * q); BA(B.sv, np * q); BA(B.d, np * q); BA(B.qv, np * q);
    BA(B.M, np * q * q);
    BA(B.items, ni); BA(B.prob_d, np); BA(B.par_d, np); BA(B.bs_d, np);
    BLaunch& L = B.L;
    BA(L.A.wl, ni); BA(L.A.wl_n, 1); BA(L.A.ioff, np); BA(L.A.icnt, np);
    BA(L.part, ni * std::max<int64_t>(q, 66)); BA(L.part2, ni * q);
    BA(L.ipart, ni * 66); BA(L.ipart2, ni);
    BA(L.gwl, gcap); BA(L.gwl_n, 1); BA(L.goff, np); BA(L.gcnt, np);
    BA(L.gpart, (int64_t)gcap * q * q);
#undef BA
    if (hipHostMalloc((void**)&B.par_h, sizeof(BPar) * kRing * np, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&B.bs_h, sizeof(BState) * np, hipHostMallocDefault) != hipSuccess)
        return set_error(SSNALM_E_OOM, "pinned allocation failed");
    memset(B.bs_h, 0, sizeof(BState) * np);
    BCHK(hipMemcpyAsync(B.items, items.data(), sizeof(int4) * ni, hipMemcpyHostToDevice, B.s));
    BCHK(hipMemcpyAsync(B.prob_d, B.hprob.data(), sizeof(BProb) * np, hipMemcpyHostToDevice, B.s));
    BCHK(hipMemsetAsync(B.bs_d, 0, sizeof(BState) * np, B.s));
    BCHK(hipMemsetAsync(B.xk, 0, sizeof(double) * n, B.s));
    BCHK(hipMemsetAsync(B.om, 0, sizeof(double) * np * q, B.s));
    L.A.prob = B.prob_d;
    L.A.par = B.par_d;
    L.A.bs = B.bs_d;
    L.A.q = B.q;
    L.A.nprob = B.nprob;
    L.dtype = B.dtype;
    L.vec = B.vec;
    L.ggrid = std::max(1, std::min(gcap, 1024));
    L.s = B.s;
    lb_setup_attributes();
    BCHK(hipStreamSynchronize(B.s));
    return SSNALM_OK;
}

// Finish the projections of state w that the first passes left open, then
// re-run `fin` for those problems.
template <typename F>
ssnalm_status finish_open(Batch& B, const std::vector<HP>& hp, const std::vector<int>& set, int w,
                          const double* v, F fin) {
    std::vector<char> open(B.nprob, 0);
    bool any = false;
    for (int k : set)
        if (!B.bs_h[k].ps[w].done) open[k] = 1, any = true;
    if (!any) return SSNALM_OK;
    BST(activate(B, hp, open));
    lb_proj_passes(B.L, v, w, batch_proj_max_passes() - kPassBatch);
    fin();
    BST(readback(B));
    return SSNALM_OK;
}

}  // namespace

extern "C" ssnalm_status ssnalm_solve_batch(int32_t count, const ssnalm_problem* probs,
                                            const ssnalm_options* opt, void* stream,
                                            double* const* x_out, double* const* w_out,
                                            ssnalm_info* infos) {
    const auto t_begin = std::chrono::steady_clock::now();
    ssnalm_options o;
    if (opt) o = *opt; else ssnalm_default_options(&o);
    BST(validate(count, probs, o, x_out));
    // The setup reads the labels from the host: wait until the work already
    // queued on the caller's stream (possibly a non-blocking stream that the
    // null stream does not order against) has written the problem arrays.
    {
        hipEvent_t ev = nullptr;
        BCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        const hipError_t e1 = hipEventRecord(ev, (hipStream_t)stream);
        const hipError_t e2 = e1 == hipSuccess ? hipEventSynchronize(ev) : e1;
        (void)hipEventDestroy(ev);
        BCHK(e2);
    }
    Batch B;
    BST(setup(B, count, probs, o));
    B.prof = o.profile != 0;
    if (B.prof) memset(g_bks, 0, sizeof g_bks);
    // order after the caller's stream
    BCHK(hipEventRecord(B.ev, (hipStream_t)stream));
    BCHK(hipStreamWaitEvent(B.s, B.ev, 0));

    const int np = B.nprob;
    std::vector<HP> hp(np);
    for (int k = 0; k < np; ++k) {
        hp[k].sigma = o.sigma0;
        hp[k].tol = probs[k].tol;
    }
    BST(choose_shape(B, hp, o.autotune != 0));
    const bool graphs = o.batch_graphs != 0;
    std::vector<char> act(np);
    auto set_of = [&](Phase ph) {
        std::vector<int> v;
        for (int k = 0; k < np; ++k)
            if (hp[k].phase == ph) v.push_back(k);
        return v;
    };
    auto flags = [&](const std::vector<int>& v) {
        std::fill(act.begin(), act.end(), 0);
        for (int k : v) act[k] = 1;
        return act;
    };
    int sweeps = 0;
    for (;;) {
        // ---- start of an ALM iteration: A omega, u, x~ = Pi(u), J, g, s
        std::vector<int> S1 = set_of(PH_OUTER);
        if (!S1.empty()) {
            BST(activate(B, hp, flags(S1)));
            timed_amul(B, act, B.om, B.aw);
            lb_elem(B.L, 0, B.xk, B.aw, B.u);
            lb_proj_init(B.L, B.u, nullptr, nullptr, 0, 0);
            lb_proj_passes(B.L, B.u, 0, kPassBatch);
            BST(readback(B));
            BST(finish_open(B, hp, S1, 0, B.u, [] {}));
            BST(activate(B, hp, flags(S1)));
            lb_ls_fin(B.L, B.u, B.u, nullptr, 0, 0, B.xk, B.xt, B.jm);
            lb_atmul(B.L, B.xt, B.jm, B.om, -1.0, B.g, B.sv);
            lb_qdots(B.L, 2, B.g, B.g, B.om, B.om, nullptr, nullptr, BS_GN2);
            BST(readback(B));
            for (int k : S1) {
                HP& h = hp[k];
                h.passes += B.bs_h[k].ps[0].passes;
                h.eps = std::pow(o.eps_decay, (double)h.outer);
                h.outer += 1;
                h.inner = 0;
                h.phase = PH_INNER;
            }
        }
        // ---- inner stopping tests (A') / (B') and the Newton steps
        std::vector<int> S2;
        for (int k = 0; k < np; ++k) {
            HP& h = hp[k];
            if (h.phase != PH_INNER) continue;
            const double* r = B.bs_h[k].r;
            const double gn = std::sqrt(r[BS_GN2]);
            if (!std::isfinite(gn)) {
                h.status = SSNALM_E_NONFINITE;
                h.phase = PH_DONE;
                continue;
            }
            const double crit = std::min(h.eps, h.eps * std::sqrt(r[BS_DIST2])) / std::sqrt(h.sigma);
            const double flo = o.floor_rel * (1.0 + std::sqrt(r[BS_OM2]));
            if (h.inner >= o.max_inner || gn <= std::max(crit, flo)) {
                h.phase = PH_KKT;
                continue;
            }
            S2.push_back(k);
        }
        if (!S2.empty()) {
            for (int k : S2) {
                hp[k].alpha = 1.0;
                hp[k].inner += 1;
                hp[k].inner_total += 1;
            }
            BST(activate(B, hp, flags(S2)));
            BST(run_seq(B, &B.gx_newton, seq_newton, graphs));
            // Armijo line search on psi, all problems in step
            std::vector<int> Lset = S2, accepted;
            for (int m = 0; !Lset.empty(); ++m) {
                if (m > 0) BST(activate(B, hp, flags(Lset)));
                BST(run_seq(B, &B.gx_trial, seq_trial, graphs));
                BST(readback(B));
                BST(finish_open(B, hp, Lset, 1, B.ut, [&] {
                    lb_ls_fin(B.L, B.ut, B.u, B.td, 1, 0, B.xk, B.xtt, B.jmt);
                }));
                std::vector<int> next;
                for (int k : Lset) {
                    HP& h = hp[k];
                    const double* r = B.bs_h[k].r;
                    h.ls_trials += 1;
                    h.passes += B.bs_h[k].ps[1].passes;
                    const double a = h.alpha;
                    const double dpsi = a * r[BS_OD] + 0.5 * a * a * r[BS_DD] + r[BS_DH] / h.sigma;
                    if (!std::isfinite(dpsi)) {
                        h.status = SSNALM_E_NONFINITE;
                        h.phase = PH_DONE;
                    } else if (dpsi <= o.mu * a * r[BS_GD]) {
                        accepted.push_back(k);
                    } else if (m >= o.max_backtracks) {
                        h.ls_fail += 1;
                        h.phase = PH_KKT;
                    } else {
                        h.alpha *= o.ls_delta;
                        next.push_back(k);
                    }
                }
                Lset.swap(next);
            }
            if (!accepted.empty()) {
                BST(activate(B, hp, flags(accepted)));
                lb_accept(B.L, B.om, B.d, B.aw, B.td, B.u, B.ut, B.xt, B.xtt, B.jm, B.jmt);
                lb_atmul(B.L, B.xt, B.jm, B.om, -1.0, B.g, B.sv);
                lb_qdots(B.L, 2, B.g, B.g, B.om, B.om, nullptr, nullptr, BS_GN2);
                BST(readback(B));
            }
        }
        // ---- end of an ALM iteration: x^{k+1} = x~, R_KKT, sigma update
        std::vector<int> S3 = set_of(PH_KKT);
        if (!S3.empty()) {
            BST(activate(B, hp, flags(S3)));
            lb_elem(B.L, 2, B.xt, nullptr, B.xk);
            lb_qvec(B.L, 1, B.om, B.g, B.qv);                 // A^T x^{k+1} = omega - g
            timed_amul(B, act, B.qv, B.nv);                   // Q x
            lb_elem(B.L, 1, B.xk, B.nv, B.nv2);               // x - Qx + e
            lb_proj_init(B.L, B.nv2, nullptr, nullptr, 2, 0);
            lb_proj_passes(B.L, B.nv2, 2, kPassBatch);
            lb_kkt_fin(B.L, B.nv2, B.xk, B.nv, 2);
            BST(readback(B));
            BST(finish_open(B, hp, S3, 2, B.nv2, [&] { lb_kkt_fin(B.L, B.nv2, B.xk, B.nv, 2); }));
            std::vector<int> improved;
            for (int k : S3) {
                HP& h = hp[k];
                const double* r = B.bs_h[k].r;
                h.passes += B.bs_h[k].ps[2].passes;
                h.R = std::sqrt(r[BS_RES2]) / (1.0 + std::sqrt(r[BS_X2]));
                h.b = B.bs_h[k].ps[2].lam;
                h.hinge = r[BS_HINGE];
                if (!std::isfinite(h.R)) {
                    h.status = SSNALM_E_NONFINITE;
                    h.phase = PH_DONE;
                    continue;
                }
                if (o.verbose)
                    fprintf(stderr, "[ssnalm batch] problem %d k=%d sigma=%.3g R_KKT=%.3e newton=%d\n", k,
                            h.outer - 1, h.sigma, h.R, h.inner_total);
                if (h.R <= h.tol) {
                    h.status = SSNALM_OK;
                    h.phase = PH_DONE;
                    continue;
                }
                if (h.R < h.best_R) {
                    h.best_R = h.R;
                    h.best_b = h.b;
                    h.best_hinge = h.hinge;
                    h.have_best = true;
                    improved.push_back(k);
                }
                h.sigma = std::min(o.rho * h.sigma, o.sigma_max);
                h.phase = h.outer >= o.max_outer ? PH_DONE : PH_OUTER;
            }
            if (!improved.empty()) {
                BST(activate(B, hp, flags(improved)));
                lb_elem(B.L, 2, B.xk, nullptr, B.xbest);
            }
        }
        ++sweeps;
        bool all_done = true;
        for (int k = 0; k < np; ++k) all_done = all_done && hp[k].phase == PH_DONE;
        if (all_done) break;
    }
    // ---- results: the best x where the cap was hit, w = A^T x, counts
    std::vector<int> from_best;
    for (int k = 0; k < np; ++k) {
        HP& h = hp[k];
        if (h.status != SSNALM_OK && h.status >= 0 && h.have_best && h.R > h.best_R) {
            h.R = h.best_R;
            h.b = h.best_b;
            h.hinge = h.best_hinge;
            from_best.push_back(k);
        }
        if (h.status == SSNALM_MAXITER && h.ls_fail > 0 && h.ls_fail >= h.outer)
            h.status = SSNALM_LINESEARCH_FAIL;
    }
    if (!from_best.empty()) {
        BST(activate(B, hp, flags(from_best)));
        lb_elem(B.L, 2, B.xbest, nullptr, B.xk);
    }
    std::vector<int> everyone(np);
    for (int k = 0; k < np; ++k) everyone[k] = k;
    BST(activate(B, hp, flags(everyone)));
    lb_count(B.L, B.xk);
    lb_atmul(B.L, B.xk, nullptr, nullptr, 1.0, B.qv, nullptr);
    lb_qdots(B.L, 1, B.qv, B.qv, nullptr, nullptr, nullptr, nullptr, BS_W2);
    for (int k = 0; k < np; ++k) {
        BCHK(hipMemcpyAsync(x_out[k], B.xk + B.hprob[k].off, sizeof(double) * B.hprob[k].n,
                            hipMemcpyDeviceToDevice, B.s));
        if (w_out && w_out[k])
            BCHK(hipMemcpyAsync(w_out[k], B.qv + (int64_t)k * B.q, sizeof(double) * B.q,
                                hipMemcpyDeviceToDevice, B.s));
    }
    BST(readback(B));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
    ssnalm_status ret = SSNALM_OK;
    for (int k = 0; k < np; ++k) {
        const HP& h = hp[k];
        if (ret == SSNALM_OK && h.status != SSNALM_OK) ret = (ssnalm_status)h.status;
        if (!infos) continue;
        ssnalm_info& in = infos[k];
        memset(&in, 0, sizeof in);
        const double* r = B.bs_h[k].r;
        in.rkkt = h.R;
        in.obj = 0.5 * r[BS_W2] - r[BS_FSUMX];
        in.b = h.b;
        {
            const double P = 0.5 * r[BS_W2] + B.hprob[k].C * h.hinge;
            in.gap = std::isfinite(P) ? (P + in.obj) / (1.0 + std::fabs(P) + std::fabs(in.obj)) : NAN;
        }
        in.sigma = h.sigma;
        in.time_s = secs;
        in.iters_outer = h.outer;
        in.iters_inner = h.inner_total;
        in.cg_iters = 0;
        in.proj_passes = h.passes;
        in.p = (int32_t)r[BS_FP];
        in.n_sv = (int32_t)r[BS_FNSV];
        in.ls_fail = h.ls_fail;
        in.ls_trials = h.ls_trials;
        in.status = h.status;
    }
    (void)sweeps;
    return ret;
}

extern "C" ssnalm_status ssnalm_batch_kernel_stats(int32_t which, ssnalm_kstat* out) {
    if (!out || which < 0 || which >= SSNALM_K_COUNT) return set_error(SSNALM_E_BADARG, "bad class or null pointer");
    *out = g_bks[which];
    return SSNALM_OK;
}
