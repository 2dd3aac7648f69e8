/*
 * ssnalm.h - C ABI of the MI355X (gfx950) SSsNAL solver for the linear C-SVC
 * dual quadratic program
 *
 *     min_x 1/2 x^T Q x - e^T x   s.t.  y^T x = 0,  0 <= x_i <= C,
 *     Q = A A^T,  A = diag(y) X   (Q is never formed),
 *
 * of arXiv 1910.01312, Section 1 (eq. Def_Dual_of_C_SVM_Problem), solved by
 * the sparse semismooth Newton augmented Lagrangian method of Section 3
 * (Algorithm 1 for the outer loop, Algorithm 3 for the inner loop, the
 * breakpoint projection of Section 3.2.1 and the reduced Newton system of
 * Proposition 5), stopped on the relative KKT residual of eq. Def_Rkkt.
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer (memory of the GPU the context
 *    lives on), unless the parameter says "host".
 *  - The library never frees caller memory.  ssnalm_create BORROWS the
 *    problem arrays (X, row_ptr, col_idx, y): they must stay valid and
 *    unchanged until ssnalm_destroy.  The library allocates and owns its
 *    own workspace (n-vectors, index lists, q x q blocks, the internal row
 *    and column copies of a CSR matrix, with fp32 values also a sliced-ELL
 *    row copy for A v: up to about 40 bytes per nonzero in all) and frees it in
 *    ssnalm_destroy.
 *  - All GPU work is enqueued on the stream given to ssnalm_create (NULL =
 *    the null stream).  Every entry point returns after that stream has
 *    finished the work it enqueued, so outputs are ready on return.
 *  - Negative status codes are errors; ssnalm_last_error() then returns a
 *    message (thread-local, valid until the next call on the same thread).
 *  - Limits: 1 <= n, q < 2^31; nnz < 2^31 for CSR input.
 *  - Reductions are performed in a fixed order: repeated calls on the same
 *    inputs give bitwise identical results.
 */
#ifndef SSNALM_H
#define SSNALM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssnalm_ctx ssnalm_ctx;            /* opaque */

typedef enum {
    SSNALM_OK = 0,                 /* R_KKT <= tol reached                         */
    SSNALM_MAXITER = 1,            /* iteration cap hit; best feasible x returned  */
    SSNALM_LINESEARCH_FAIL = 2,    /* Armijo search exhausted repeatedly            */
    SSNALM_WARMSTART_REJECTED = 3, /* the warm start was set aside and the plain    */
                                   /* cold solve reached tol (ssnalm_ws_solve)      */
    SSNALM_E_BADARG = -1,          /* invalid argument (message says which)         */
    SSNALM_E_NONFINITE = -2,       /* NaN/Inf in the data or in an iterate          */
    SSNALM_E_OOM = -3,             /* device allocation failed                      */
    SSNALM_E_HIP = -4              /* a HIP runtime call failed                     */
} ssnalm_status;

enum { SSNALM_DENSE = 0, SSNALM_CSR = 1 };                  /* ssnalm_problem.kind  */
enum { SSNALM_F64 = 0, SSNALM_F32 = 1, SSNALM_BF16 = 2 };   /* ssnalm_problem.dtype */
enum { SSNALM_NEWTON_AUTO = 0, SSNALM_NEWTON_CHOL = 1, SSNALM_NEWTON_PCG = 2 };
enum { SSNALM_PREC_FP64 = 0, SSNALM_PREC_MIXED = 1 };

/*
 * The problem (Section 1).  X holds the n samples x~_i in R^q as rows:
 *  kind = SSNALM_DENSE: X is n*q elements, row-major (row i = sample i),
 *    dtype F64, F32 or BF16 (raw bfloat16 bit patterns, uint16).
 *  kind = SSNALM_CSR: X is the nnz values (dtype F64 or F32), row_ptr the
 *    n+1 row offsets (int64, row_ptr[0] = 0, nondecreasing, row_ptr[n] =
 *    nnz) and col_idx the nnz column indices (int32, in [0, q); column
 *    indices within a row need not be sorted; duplicates are summed).
 * y holds n labels, each exactly +1 or -1 (int8).  C > 0 is the box bound,
 * tol > 0 the target relative KKT residual of eq. Def_Rkkt.
 */
typedef struct {
    int32_t kind;
    int32_t dtype;
    int64_t n, q, nnz;
    const void*    X;
    const int64_t* row_ptr;
    const int32_t* col_idx;
    const int8_t*  y;
    double C;
    double tol;
} ssnalm_problem;

/*
 * Solver options.  The paper fixes none of these constants except the
 * iteration cap of 200 outer iterations and x^0 = 0 (Section 4.1); the
 * defaults set by ssnalm_default_options are this library's readings of the
 * open constants: sigma0 = 1, sigma_{k+1} = min(rho sigma_k, sigma_max) with
 * rho = 2 and sigma_max = 1e6; eps_k = delta_k = eps_decay^k (0.5^k) in the
 * inner stopping tests (A') and (B'); mu = 1e-4, line-search factor 0.5,
 * tau = 0.5, eta = 0.1 in Algorithm 3; 50 inner iterations, 40 backtracks.
 */
typedef struct {
    double  sigma0, rho, sigma_max;
    double  mu, ls_delta, tau, eta, eps_decay;
    double  floor_rel;          /* inner stop floor: |g| <= floor_rel (1+|omega|)        */
    int32_t max_outer, max_inner, max_backtracks;
    int32_t newton;             /* SSNALM_NEWTON_*                                        */
    int32_t precision;          /* SSNALM_PREC_*                                          */
    int32_t max_cg;             /* PCG iteration cap per Newton step                      */
    int32_t verbose;            /* 1: one line per outer iteration on stderr, 2: also one */
                                /* per Newton step at the stored factor's sigma           */
    int32_t check_finite;       /* 1: ssnalm_create scans X for NaN/Inf                   */
    int32_t profile;            /* HIP-event timing of the hot kernel classes: 0 off, 1    */
                                /* all classes, > 1 a mask with bit (k + 1) for class k    */
                                /* (SSNALM_K_*).  Classes timed one by one are launched    */
                                /* eagerly instead of from a captured graph                */
    int32_t batch_graphs;       /* batched solve: 1 replays captured HIP graphs of the    */
                                /* Newton-direction and line-search-trial launches, 0     */
                                /* issues the same launches one by one (same results)     */
    int32_t autotune;           /* batched solve: 1 times candidate launch shapes once    */
                                /* per shape class and keeps the fastest (same results)   */
    int32_t lowrank;            /* dense Cholesky Newton steps at the sigma of the stored  */
                                /* factor: 1 (default) updates that factor by the Woodbury */
                                /* identity when at most 94 rows of J changed (mixed       */
                                /* precision, whose refinement then uses the updated       */
                                /* operator), 2 also in fp64, 0 always refactors           */
} ssnalm_options;

/* What the paper reports per solve (Section 4, Table 2 columns) plus timing. */
typedef struct {
    double  rkkt;               /* R_KKT(x) of eq. Def_Rkkt at the returned x             */
    double  obj;                /* 1/2 |A^T x|^2 - e^T x                                  */
    double  b;                  /* bias: lam_hat of the final KKT projection              */
    double  gap;                /* relative duality gap (P + obj) / (1 + |P| + |obj|),    */
                                /* P = 1/2 |w|^2 + C sum_i max(0, 1 - y_i (x~_i^T w + b)) */
                                /* the C-SVC primal (Section 1) at w = A^T x and this b;  */
                                /* P + obj >= 0 for every feasible x and every b          */
    double  sigma;              /* final penalty parameter                                */
    double  time_s;             /* wall time of ssnalm_solve                              */
    double  t_matvec, t_proj, t_newton, t_other;   /* seconds per phase (host clock)      */
    int32_t iters_outer;        /* ALM iterations                                         */
    int32_t iters_inner;        /* Newton steps, summed                                   */
    int32_t cg_iters;           /* PCG iterations, summed                                 */
    int32_t proj_passes;        /* multisection passes, summed                            */
    int32_t p;                  /* #unbounded SVs, 0 < x_i < C ("suppvec")                */
    int32_t n_sv;               /* #SVs, x_i > 0                                          */
    int32_t ls_fail;            /* line searches that exhausted their backtracks          */
    int32_t ls_trials;          /* line-search trials (projections of u - alpha sigma t)  */
    int32_t grad_steps;         /* Newton directions replaced by -grad psi because they   */
                                /* were not descent directions (g^T d >= 0, a non-        */
                                /* positive Cholesky pivot, or in a low-rank step a pivot */
                                /* of the capacitance matrix with the wrong sign)         */
    int32_t proj_capped;        /* projections that hit the multisection pass cap (their  */
                                /* multiplier is the interpolation of the last bracket)   */
    int32_t status;             /* same as the return value                               */
    int32_t lowrank_steps;      /* Newton steps taken by a low-rank update of the stored  */
                                /* Cholesky factor instead of a new factorisation         */
} ssnalm_info;

/* Fill *opt with the defaults.  opt: host pointer. */
void ssnalm_default_options(ssnalm_options* opt);

/*
 * Create a solver context for one problem.  Validates the arguments (see
 * E_BADARG cases below), allocates the workspace and, for CSR input, builds
 * the column-major copy used by the A^T r products.
 *   out    : host pointer that receives the context.
 *   prob   : host pointer to the problem; its arrays are device pointers.
 *   opt    : host pointer or NULL for the defaults.
 *   stream : a hipStream_t, or NULL for the null stream.  The context works on
 *            its own stream (default priority); every call is ordered after
 *            the work already queued on `stream`, and work queued on `stream`
 *            after a call returns is ordered after that call's work.
 * E_BADARG: n < 1, q < 1, C <= 0 or non-finite, tol <= 0, unknown kind or
 * dtype, CSR with BF16 values, row_ptr not monotone / not ending at nnz,
 * col_idx out of range, a label not in {+1,-1}.  E_NONFINITE: NaN/Inf in X
 * (only when opt->check_finite).  E_OOM / E_HIP: allocation / runtime error.
 */
ssnalm_status ssnalm_create(ssnalm_ctx** out, const ssnalm_problem* prob,
                            const ssnalm_options* opt, void* stream);

/*
 * The eps-SVR dual (Section 1, eq. Def_Dual_of_SVR_Problem) as an instance
 * of the unified problem (P): variables [x; z] in R^{2n},
 *   min 1/2 |X^T (x - z)|^2 + eps e^T (x + z) + y^T (x - z)
 *   s.t. e^T x - e^T z = 0,  0 <= x, z <= C,
 * i.e. Q = B B^T with B = [X; -X], c = [eps e + y; eps e - y], a = [e; -e],
 * d = 0, l = 0, u = C e.  B is never formed: products with B are products
 * with X (two signed copies of its rows).
 *   kind  : SSNALM_DENSE (CSR is not accepted), dtype F64, F32 or BF16.
 *   X     : n x q row-major (device), borrowed like ssnalm_create's.
 *   y     : n regression targets (doubles, device), read during the call.
 * The context then solves with ssnalm_solve: x_out holds 2n doubles [x; z],
 * w_out the primal weights w = X^T (z - x) of the regression function
 * w^T x~ + b, b_out (and info->b) its bias b, info->obj the dual objective
 * above and info->gap the relative gap to the eps-insensitive primal
 * 1/2 |w|^2 + C sum_i max(0, |y_i - w^T x~_i - b| - eps).  Newton steps
 * use the Cholesky factorisation (q <= 2048), fp64 precision.
 * E_BADARG: as ssnalm_create, plus eps < 0 or non-finite, CSR input,
 * PCG or mixed precision requested, q > 2048.
 */
typedef struct {
    int32_t kind;
    int32_t dtype;
    int64_t n, q;
    const void*   X;
    const double* y;
    double C;
    double eps;
    double tol;
} ssnalm_svr_problem;

ssnalm_status ssnalm_create_svr(ssnalm_ctx** out, const ssnalm_svr_problem* prob,
                                const ssnalm_options* opt, void* stream);

/*
 * The unified problem (P) of Section 1 (eq. Problem_P1_classical1) with a
 * linear kernel:
 *   min 1/2 x^T B B^T x + c^T x   s.t.  a^T x = d,  l <= x <= u,
 * for a general B (n x q, dense, rows as given), c, a, l < u (n doubles
 * each) and d.  The same Algorithms 1 and 3 run in omega = B^T w space; the
 * projection onto {a^T x = d, l <= x <= u} (Section 3.2.1) finds the
 * smallest zero of -a^T clip(v - lam a, l, u) + d by multisection over the
 * breakpoints (v_i - u_i)/a_i, (v_i - l_i)/a_i (a_i = 0 components are
 * clipped alone); the Newton matrix is I + sigma (B_J^T B_J - s s^T /
 * (a_J^T a_J)), s = B_J^T a_J (Theorem 3.1; no rank-one term when a_J = 0).
 * x^0 = 0 when it is feasible, else its projection.  After solving,
 * info->obj is 1/2 |B^T x|^2 + c^T x, info->b (and b_out) the multiplier
 * lam of the constraint a^T x = d in the projection of R_KKT, info->gap is
 * NaN (no primal is defined), w_out = B^T x.
 *   B: n x q row-major (dtype F64, F32 or BF16), borrowed; c, a, l, u:
 *   device doubles, borrowed (valid and unchanged until ssnalm_destroy).
 * E_BADARG: null pointer, kind not dense, n, q out of range, a non-finite
 * a_i, l_i or u_i, l_i >= u_i, no x in [l, u] with a^T x = d, PCG or mixed
 * precision requested, q > 2048.
 */
typedef struct {
    int32_t kind;
    int32_t dtype;
    int64_t n, q;
    const void*   B;
    const double* c;
    const double* a;
    const double* l;
    const double* u;
    double d;
    double tol;
} ssnalm_general_problem;

ssnalm_status ssnalm_create_general(ssnalm_ctx** out, const ssnalm_general_problem* prob,
                                    const ssnalm_options* opt, void* stream);

/*
 * The C-SVC dual with a nonlinear kernel (Section 1, eq.
 * Def_Dual_of_C_SVM_Problem with Q_ij = y_i y_j k(x~_i, x~_j); the problem
 * of Table 3):
 *   SSNALM_KERNEL_RBF    : k(x, z) = exp(-|x - z|^2 / (2 alpha)), alpha > 0
 *                          (the Gaussian kernel of Section 4);
 *   SSNALM_KERNEL_LINEAR : k(x, z) = x^T z (alpha unused), the linear C-SVC
 *                          through the same kernel path.
 * The method runs in the paper's w-space (w in R^n): Q is formed once, in
 * fp64, from the samples by a tiled kernel-evaluation pass and kept in
 * device memory (n^2 doubles: n = 20000 takes 3.2 GB, n = 100000 80 GB);
 * the products Q v read only the rows of Q at the nonzeros of v, and the
 * Newton step of Algorithm 3 is the p x p system of Proposition 5 on the
 * free set J (p = |J|), written with the projector
 * Pi = I - y_J y_J^T / p inside the matrix:
 *   (I_p + sigma Pi Q_JJ Pi) v = Pi (Q s)_J,   s = w - Pi(u(w)),
 *   z = sigma Pi v,   d = -s + z on J,   Q d = -Q s + Q_{:,J} z,
 * solved by Cholesky (p <= 32768; the p x p matrix takes p^2 doubles of
 * device memory, allocated for min(n, 32768)) or by Jacobi-preconditioned CG
 * on the same matrix to |residual| <= min(eta, |grad|^(1+tau)) (p > 32768,
 * or always with opt.newton = SSNALM_NEWTON_PCG).  Norms of the stopping tests are
 * Q-norms (|omega| = (w^T Q w)^(1/2), |grad| = (s^T Q s)^(1/2)), the
 * omega-space norms of the linear path.
 *   dtype : F64, F32 or BF16 samples (values used in fp64).
 *   X     : n x q row-major (device), read during ssnalm_create_kernel only.
 *   y     : n labels +-1 (int8, device), borrowed (valid until destroy).
 * ssnalm_solve then returns x_out (n), b_out / info->b (the bias of the
 * decision function sum_i x_i y_i k(x~_i, .) + b, the lam_hat of R_KKT's
 * projection), info->obj = 1/2 x^T Q x - e^T x and info->gap, the relative
 * gap to the primal 1/2 x^T Q x + C sum_i max(0, 1 - (Q x)_i - y_i b);
 * w_out must be NULL (the primal weights live in the kernel's feature
 * space).  ssnalm_op_amul on such a context computes t = Q v (v, t: n
 * doubles), ssnalm_op_rkkt, ssnalm_op_project, ssnalm_op_linesearch_trial,
 * ssnalm_ws_labels and ssnalm_ws_x0 work as for ssnalm_create;
 * ssnalm_op_kernel_newton takes the Newton step; ssnalm_op_atmul,
 * ssnalm_op_newton, ssnalm_op_gram, ssnalm_ws_features, ssnalm_ws_solve and
 * opt.precision = MIXED are rejected.
 * E_BADARG: null pointer, unknown kernel, n out of [1, 2^31), q < 1,
 * alpha not finite and > 0 (RBF), labels not +-1, C or tol invalid.
 * E_OOM: Q does not fit in device memory.
 */
enum { SSNALM_KERNEL_RBF = 0, SSNALM_KERNEL_LINEAR = 1 };
typedef struct {
    int32_t kernel;
    int32_t dtype;
    int64_t n, q;
    const void*   X;
    const int8_t* y;
    double C;
    double alpha;
    double tol;
} ssnalm_kernel_problem;

ssnalm_status ssnalm_create_kernel(ssnalm_ctx** out, const ssnalm_kernel_problem* prob,
                                   const ssnalm_options* opt, void* stream);

/*
 * Solve (Algorithm 1 with Algorithm 3 as its inner solver).
 *   x0    : optional warm start, n doubles (device) or NULL for x^0 = 0.
 *           It is projected onto {y^T x = 0, 0 <= x <= C} first and omega^0
 *           is set to A^T x^0.
 *   x_out : n doubles (device), the dual solution x.
 *   w_out : q doubles (device) or NULL, the primal weights w = A^T x.
 *   b_out : one double (HOST) or NULL, the bias b of the decision function
 *           sign(w^T x~ + b): the multiplier lam_hat of the projection in
 *           R_KKT at the returned x (eq. Def_Rkkt), as info->b.
 *   info  : host pointer or NULL.
 * An inexact Newton direction that is not a descent direction is replaced
 * by -grad psi for that step (counted in info->grad_steps).
 * Returns OK, MAXITER (cap hit; the x with the smallest R_KKT seen is
 * returned) or LINESEARCH_FAIL, or a negative error.  If y has one class
 * only, x = 0 is the only feasible point: OK with x = 0 and b = NaN.
 */
ssnalm_status ssnalm_solve(ssnalm_ctx* ctx, const double* x0, double* x_out,
                           double* w_out, double* b_out, ssnalm_info* info);

/*
 * Solve `count` independent problems with one launch per phase for all of
 * them: the C-grid / one-vs-rest / cross-validation use of the method
 * (Section 4 solves one QP per C value and per fold).  Each problem runs
 * Algorithm 1 with Algorithm 3 as in ssnalm_solve (x^0 = 0, the Cholesky
 * Newton step, the same options); the kernels sum in a different order than
 * the single-problem ones, so iterates agree with ssnalm_solve to rounding.
 * A problem that meets its own tol (or its caps) leaves the later launches.
 *   count  : number of problems, >= 1.
 *   probs  : host array of `count` problems; all SSNALM_DENSE with the same
 *            dtype and the same q <= 128; n, C, tol, X and y per problem
 *            (device pointers, X row-major as in ssnalm_create).
 *   opt    : host pointer or NULL for the defaults (newton must be AUTO or
 *            CHOL, precision FP64).
 *   stream : hipStream_t or NULL; the call runs on a private stream ordered
 *            after the work already on `stream` and returns when done.
 *   x_out  : host array of `count` device pointers, n_k doubles each.
 *   w_out  : host array of `count` device pointers (q doubles) or NULL;
 *            a NULL entry skips that problem's w.
 *   infos  : host array of `count` infos or NULL; time_s is the batch's
 *            wall time, the per-phase times are 0.
 * Returns OK when every problem reached its tol, otherwise the first
 * non-OK status in problem order (infos[k].status has each one).
 * E_BADARG: count < 1, a null pointer, a problem that is not dense, mixed
 * dtypes or q, q > 128, or any ssnalm_create argument error; E_OOM / E_HIP.
 */
ssnalm_status ssnalm_solve_batch(int32_t count, const ssnalm_problem* probs,
                                 const ssnalm_options* opt, void* stream,
                                 double* const* x_out, double* const* w_out,
                                 ssnalm_info* infos);

/* Release the context and everything the library allocated for it. */
void ssnalm_destroy(ssnalm_ctx* ctx);

/* Message of the last error on this thread ("" if none). */
const char* ssnalm_last_error(void);

/* ------------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the hot path on the data
 * of an existing context, so that every step can be checked on its own.
 * ---------------------------------------------------------------------- */

/* t = A v = y .* (X v)  (the product Q w = A omega of eq. Def_psi).
 * v: q doubles, t: n doubles (device). */
ssnalm_status ssnalm_op_amul(ssnalm_ctx* ctx, const double* v, double* t);

/* r = A^T z = X^T (y .* z)  (the product inside grad psi,
 * eq. Def_differential_of_psi).  z: n doubles, r: q doubles (device). */
ssnalm_status ssnalm_op_atmul(ssnalm_ctx* ctx, const double* z, double* r);

/* Projection onto K ∩ L = {y^T x = 0, 0 <= x <= C} (Section 3.2.1):
 * x = clip(v - lam y, 0, C) with lam the smallest zero of
 * lam -> -y^T clip(v - lam y, 0, C) (the value Algorithm 2 returns).
 *   v: n doubles, x: n doubles, free_mask: n bytes or NULL (1 where
 *   0 < v_i - lam y_i < C: the index set J of Proposition 5),
 *   lam: host double, p: host int64 (|J|), passes: host int32 or NULL. */
ssnalm_status ssnalm_op_project(ssnalm_ctx* ctx, const double* v, double* x,
                                uint8_t* free_mask, double* lam, int64_t* p,
                                int32_t* passes);

/* The projection of ssnalm_op_project without a context and without any
 * device allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Its
 * scratch (search state, block partials, counts; ssnalm_noalloc_scratch_bytes()
 * bytes, about 260 KB) is a device array inside the library that each GPU
 * holds until the process ends.  Calls that overlap on one GPU share that
 * array and race: the caller must order them.
 *   v: n doubles, y: n labels (+1 / -1), x: n doubles, free_mask: n bytes or
 *   NULL (as ssnalm_op_project), all device; lam (the multiplier), p (|J|):
 *   host or NULL; stream: hipStream_t or NULL.  Returns after the stream
 *   has finished the call's work.
 * E_BADARG: null v, y or x; n < 1 or n > ssnalm_noalloc_max_n(); C <= 0 or
 * non-finite.  Labels are not checked (they must be exactly +1 or -1). */
ssnalm_status ssnalm_project_noalloc(const double* v, const int8_t* y, int64_t n, double C,
                                     double* x, uint8_t* free_mask, double* lam, int64_t* p,
                                     void* stream);
int64_t ssnalm_noalloc_max_n(void);
int64_t ssnalm_noalloc_scratch_bytes(void);

/* Newton direction of Algorithm 3, step 1, in omega-space:
 * d = -(I + sigma (X_J^T X_J - s s^T / p))^{-1} g,  s = X_J^T 1,  p = |J|
 * (Proposition 5 with L = A; d = -g when p = 0).  free_mask: n bytes
 * (device, 1 = in J); g, d: q doubles (device); cg_iters: host or NULL.
 * Uses the context's Newton mode (Cholesky or PCG to the tolerance
 * cg_tol) and precision. */
ssnalm_status ssnalm_op_newton(ssnalm_ctx* ctx, const uint8_t* free_mask,
                               const double* g, double sigma, double cg_tol,
                               double* d, int32_t* cg_iters);

/* Kernel contexts (ssnalm_create_kernel): the Newton step of Algorithm 3
 * by Proposition 5's p x p system, as ssnalm_solve takes it.  free_mask: n
 * bytes (device, 1 = in J); s = w - Pi(u(w)): n doubles (device); d, Qd:
 * n doubles (device) receive the representative d = -s + z on J and Q d;
 * dQd: host double (d^T Q d); cg_iters: host or NULL (0 for Cholesky).
 * cg_tol: the CG tolerance when the step is solved by CG. */
ssnalm_status ssnalm_op_kernel_newton(ssnalm_ctx* ctx, const uint8_t* free_mask,
                                      const double* s, double sigma, double cg_tol,
                                      double* d, double* Qd, double* dQd, int32_t* cg_iters);

/* Gram matrix of the free rows, G = X_J^T X_J (q x q, row-major, full),
 * the product inside A^T P A of Proposition 5 (labels cancel).  Uses the
 * context's SYRK: bf16 operands on the matrix cores with fp32 accumulation
 * when the context is mixed precision with bf16 X, fp64 otherwise.
 * free_mask: n bytes (device, 1 = in J); G: q*q doubles (device).  Dense
 * contexts only. */
ssnalm_status ssnalm_op_gram(ssnalm_ctx* ctx, const uint8_t* free_mask, double* G);

/* One trial of the Armijo line search of Algorithm 3, step 2, on the n-side
 * terms of psi (eq. Def_psi): with u_a = u - alpha sigma t it projects u_a
 * and returns
 *   dh = sum_i [phi(u_a,i - lam_a y_i) - phi(u_i - lam y_i)],
 *   phi(t) = int_0^t clip(s, 0, C) ds,
 * which equals 1/2(|u_a|^2 - |u_a - Pi(u_a)|^2) - 1/2(|u|^2 - |u - Pi(u)|^2);
 * each term is formed from its own increment so that no two large numbers
 * are subtracted.  u, t: n doubles (device); lam: the multiplier of Pi(u);
 * lam_a, dh: host doubles. */
ssnalm_status ssnalm_op_linesearch_trial(ssnalm_ctx* ctx, const double* u,
                                         const double* t, double lam,
                                         double alpha, double sigma,
                                         double* lam_a, double* dh);

/* Kernel classes timed when ssnalm_options.profile = 1. */
enum {
    SSNALM_K_AMUL = 0,        /* A v over all rows (line-search direction, KKT)      */
    SSNALM_K_ATMUL = 1,       /* A^T z over the support rows (gradient of psi)       */
    SSNALM_K_AMUL_J = 2,      /* X_J v inside the matrix-free Newton operator        */
    SSNALM_K_ATMUL_J = 3,     /* X_J^T w inside the matrix-free Newton operator      */
    SSNALM_K_PROJ = 4,        /* one multisection pass of the projection             */
    SSNALM_K_SYRK = 5,        /* X_J^T X_J                                           */
    SSNALM_K_CHOL = 6,        /* Cholesky factor + solves                            */
    SSNALM_K_QCOLS = 7,       /* kernel contexts: Q v over the rows of Q at the      */
                              /* nonzeros of v (gradient, Newton step, KKT)          */
    SSNALM_K_QJJ = 8,         /* kernel contexts: the p x p Newton matrix from Q_JJ   */
    SSNALM_K_COUNT = 9
};
typedef struct {
    int64_t launches;         /* timed launches since the last reset                 */
    double  seconds;          /* summed device time between the event pairs          */
    double  bytes;            /* summed algorithmic HBM bytes (what the step must    */
                              /* read and write at least once)                       */
    double  flops;            /* summed algorithmic flops                            */
} ssnalm_kstat;

/* Per-class kernel statistics accumulated by ssnalm_solve while
 * opt.profile = 1.  A launch's time is the sum of its kernels' execution
 * times, each taken by an event pair attached to the kernel's dispatch.  The
 * sparse CG's classes (SSNALM_K_AMUL_J, SSNALM_K_ATMUL_J) are sampled: one
 * CG iteration in eight is timed, and launches after the CG met its
 * tolerance (which pass through) are not counted.  which: SSNALM_K_*; out:
 * host pointer.  reset != 0 clears all classes after reading. */
ssnalm_status ssnalm_kernel_stats(ssnalm_ctx* ctx, int32_t which, ssnalm_kstat* out,
                                  int32_t reset);

/* Change opt.profile of an existing context (same meaning). */
ssnalm_status ssnalm_set_profile(ssnalm_ctx* ctx, int32_t profile);

/* The same statistics for the last ssnalm_solve_batch call made on this
 * thread with opt.profile = 1 (launches timed outside the captured graphs:
 * SSNALM_K_AMUL covers the A omega and Q x passes over all active
 * problems; other classes read 0).  which: SSNALM_K_*; out: host pointer. */
ssnalm_status ssnalm_batch_kernel_stats(int32_t which, ssnalm_kstat* out);

/* Relative KKT residual of eq. Def_Rkkt at x (n doubles, device), with
 * the bias lam of its projection.  rkkt, b: host doubles. */
ssnalm_status ssnalm_op_rkkt(ssnalm_ctx* ctx, const double* x, double* rkkt,
                             double* b);

/* ------------------------------------------------------------------------
 * RBF kernels through explicit features (Section 4, the approximations of
 * Tables 3_1 and 3_2).  With k(x, z) = exp(-|x - z|^2 / (2 alpha)) the
 * C-SVC dual has Q = diag(y) K diag(y); a feature matrix Z with Z Z^T ~ K
 * makes it the linear problem of this library with X = Z: pass Z (dense,
 * fp64 or fp32) to ssnalm_create.  X: n x q row-major (dtype F64, F32 or
 * BF16), Z: output, row-major, z_dtype F64 or F32; all device pointers.
 * Both calls run on `stream` (hipStream_t or NULL) and return when done.
 * ---------------------------------------------------------------------- */

/* Random Fourier features: W holds N frequencies (N x q doubles, device),
 * drawn by the caller from the Gaussian with covariance I / alpha (the
 * spectral density of k).  Z is n x 2N with Z[i][2k] = cos(w_k^T x_i) /
 * sqrt(N) and Z[i][2k+1] = sin(w_k^T x_i) / sqrt(N), so that Z Z^T is the
 * average of the N sampled kernels.  Products and cos / sin in fp64.
 * E_BADARG: null pointer, n, q < 1, N outside [1, 4194240], bad dtype. */
ssnalm_status ssnalm_rff_features(const void* X, int32_t dtype, int64_t n, int64_t q,
                                  const double* W, int64_t N, void* Z, int32_t z_dtype,
                                  void* stream);

/* Nystroem features: landmarks holds r row indices of X (int32, device; the
 * paper picks them by k-means, any choice is accepted).  Z is n x r with
 * Z = K_nr L^{-T}, K_nr[i][j] = k(x_i, x_{l_j}), K_rr + shift I = L L^T
 * (the paper's shift is 1e-3), so Z Z^T = K_nr (K_rr + shift I)^{-1}
 * K_nr^T.  fp64 throughout (blocked Cholesky, blocked triangular solve).
 * Allocates its workspace (about 8 (n + r) r bytes) per call.
 * E_BADARG: null pointer, r outside [1, 2048], alpha <= 0, shift < 0, a
 * landmark outside [0, n), K_rr + shift I not positive definite. */
ssnalm_status ssnalm_nystroem_features(const void* X, int32_t dtype, int64_t n, int64_t q,
                                       const int32_t* landmarks, int64_t r, double alpha,
                                       double shift, void* Z, int32_t z_dtype, void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start.  The paper starts its exact-kernel solves from a
 * cheaper approximate solution (Section 4, RBF experiments) and stresses
 * the value of a good initial point (Remark 2); here a small network
 * predicts x^0 for ssnalm_solve.  Nothing in the paper fixes the network, so
 * its definition is this library's:
 *   features  z_i = [x_i^T R (64), m_i, log10(n C)]  (66 floats, row-major),
 *             R: q x 64 (caller's, float32, device);
 *             p = Pi(C e) onto {y^T x = 0, 0 <= x <= C}; t* = clip(e^T p /
 *             |A^T p|^2, 0, 1) (exact line search of the dual objective
 *             along x = t p: one projected-gradient step from x = 0);
 *             w1 = t* A^T p, s_i = x_i^T w1, b1 = -(mean of s over y = +1 +
 *             mean of s over y = -1) / 2, m_i = y_i (s_i + b1).
 *   network   A1 = Z W1 + b1, H1 = gelu(A1), A2 = H1 W2 + b2, H2 = gelu(A2),
 *             O = H2 W3 + b3 (66 -> 256 -> 256 -> 4), gelu(a) = a Phi(a).
 *   output    (P0, P1, P2, mult) = (softmax(O[0:3]), sigmoid(O[3])): the
 *             probabilities of x_i* = 0, 0 < x_i* < C, x_i* = C, and x_i* / C.
 *   loss      mean_i [-log P_{s_i}] + w_mse mean_i [s_i = 1] (mult_i - t_i)^2
 *             with status s_i in {0, 1, 2} and target t_i = x_i* / C.
 *   x0        by the most probable status (ties to the lower index):
 *             x0_i = 0, C mult or C.
 * Parameters live in one flat float32 vector: W1 (66 x 256, row-major), b1
 * (256), W2 (256 x 256), b2 (256), W3 (256 x 4), b3 (4).  All pointers of
 * the mlp_ calls are device pointers; every call is asynchronous on
 * `stream` (hipStream_t or NULL).  Results are deterministic.
 * ---------------------------------------------------------------------- */
#define SSNALM_MLP_IN   66
#define SSNALM_MLP_HID  256
#define SSNALM_MLP_OUT  4
#define SSNALM_MLP_NPROJ 64

/* Number of parameters (floats) of the flat vector. */
int64_t ssnalm_mlp_param_count(void);
/* Floats of the forward workspace for n rows (activations kept for the
 * backward pass) and of the backward scratch. */
int64_t ssnalm_mlp_work_floats(int64_t n);
int64_t ssnalm_mlp_scratch_floats(int64_t n);

/* Forward pass: Z (n x 66) -> out (n x 4) = (P0, P1, P2, mult).  work:
 * ssnalm_mlp_work_floats(n) floats.  E_BADARG: null pointer or n < 1 or
 * n > 4194304. */
ssnalm_status ssnalm_mlp_forward(const float* theta, const float* Z, int64_t n, float* out,
                                 float* work, void* stream);

/* Loss and gradient of the mean loss over the n rows of the last forward
 * call on (theta, Z, work, out).  status: n int32 in {0, 1, 2}; target: n
 * floats (read where status = 1); grad: param_count floats (overwritten);
 * loss: 1 float; scratch: ssnalm_mlp_scratch_floats(n) floats. */
ssnalm_status ssnalm_mlp_backward(const float* theta, const float* Z, int64_t n,
                                  const float* work, const float* out, const int32_t* status,
                                  const float* target, float w_mse, float* grad, float* loss,
                                  float* scratch, void* stream);

/* One Adam update (Kingma and Ba, bias-corrected) of count parameters at
 * step >= 1; m and v are the moment vectors (zero before step 1). */
ssnalm_status ssnalm_mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t count,
                              float lr, float beta1, float beta2, float eps, int32_t step,
                              void* stream);

/* Features z (n x 66 floats, device) of the context's problem (dense only)
 * with projection R (q x 64 floats, device).  Runs on the context's stream
 * and returns when done.  E_BADARG: null pointer, CSR problem. */
ssnalm_status ssnalm_ws_features(ssnalm_ctx* ctx, const float* R, float* Z);

/* What ssnalm_ws_solve did. */
typedef struct {
    int32_t rounds;           /* reduced solves run (0: went straight to the cold solve) */
    int32_t kept;             /* rows of the last reduced problem                       */
    int32_t fallback;         /* 1: the plain cold solve of the full problem was used   */
    int32_t pad_;
    double  rkkt_full;        /* R_KKT of the returned x on the full problem            */
    double  t_reduced;        /* seconds spent in the reduced solves                   */
} ssnalm_ws_stats;

/*
 * Solve the context's problem using the network's bound-status prediction
 * (out: n x 4 floats, device, from ssnalm_mlp_forward on the features):
 * the rows are ranked by P(x_i* = 0) and about keep_frac n of them, those
 * least surely at 0, are kept (cut on a 4096-bin histogram of
 * -log10(1 - P(x_i* = 0)) over [0, 8), ties in the cut bin kept); the kept
 * rows are solved by ssnalm_solve at tol, the result (zero on the left-out
 * rows) is judged by R_KKT of the FULL problem (eq. Def_Rkkt); rows whose
 * margin y_i (w^T x_i + b) is below 1 are added and the reduced solve
 * repeated from the previous round's solution (at half the previous
 * tolerance when no row was added), at most max_rounds times; otherwise (or
 * when more than half of the rows are kept) the plain cold solve of the full
 * problem runs.  The returned x
 * always satisfies R_KKT <= tol on the full problem when status is OK.
 * x_out: n doubles (device); w_out: q doubles (device) or NULL; info,
 * stats: host pointers or NULL.  Allocates the reduced copies per call.
 * E_BADARG: null pointer, CSR problem, keep_frac outside (0, 1].
 */
ssnalm_status ssnalm_ws_solve(ssnalm_ctx* ctx, const float* out, double keep_frac,
                              int32_t max_rounds, double* x_out, double* w_out,
                              ssnalm_info* info, ssnalm_ws_stats* stats);

/* Training labels of the network from a solution x of the context's problem
 * (n doubles, device): status[i] = 0 if x_i <= 1e-8 C, 2 if x_i >= (1 - 1e-8)
 * C, else 1 (n int32, device); target[i] = x_i / C (n floats, device).
 * Returns when done.  E_BADARG: null pointer. */
ssnalm_status ssnalm_ws_labels(ssnalm_ctx* ctx, const double* x, int32_t* status, float* target);

/* x0 (n doubles, device) from the network output (n x 4 floats, device):
 * 0, C mult or C by the most probable status, for ssnalm_solve(ctx, x0). */
ssnalm_status ssnalm_ws_x0(ssnalm_ctx* ctx, const float* out, double* x0);

#ifdef __cplusplus
}
#endif
#endif /* SSNALM_H */
