"""The C-SVC dual with a nonlinear kernel on the GPU (ssnalm_create_kernel:
Q_ij = y_i y_j k(x_i, x_j), the problem of Table 3) against the w-space
kernel oracle (oracle/kernel.py) (GPU only).

  * Q v for dense, sparse and zero v against the oracle's explicit Q, over
    several 256-column tiles with ragged tails, for fp64 and fp32 samples;
  * the Newton step of Proposition 5 (d, Q d, d^T Q d) against the oracle's
    p x p step: the single-workgroup Cholesky, the blocked factorisation with
    the single-workgroup and the multi-workgroup triangular solves, and the
    CG solve of the same matrix;
  * full solves: equal iteration counts, x and the objective against the
    oracle's w-space solve at the same tolerance, R_KKT recomputed by the
    oracle, the bias and the duality gap;
  * a solve whose first free sets take the multi-workgroup solves (equal
    counts), the same solve with CG steps against the oracle's optimum, the
    linear kernel against the linear C-SVC path, a
    warm start, the iteration cap, one-class labels, n = 1 and the rejected
    arguments.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import features, general, kernel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _svc(X, y, C_, alpha, tol=1e-6, **kw):
    from paper_1910_01312_amd.solver import KernelSVC
    return KernelSVC(X, y, C_, alpha, tol=tol, **kw)


def _Q(X, y, alpha, kind="rbf"):
    K = features.rbf_kernel(X, X, alpha) if kind == "rbf" else X @ X.T
    return kernel.kernel_q(K, y)


@pytest.mark.parametrize("n,q,dtype", [(1, 3, "f64"), (37, 5, "f64"), (300, 20, "f64"),
                                       (1000, 50, "f32"), (2051, 17, "f64")])
def test_q_products(n, q, dtype):
    X, y = synth.rbf_problem(n, q, seed=n)
    if n == 1:
        y[:] = 1
    if dtype == "f32":
        X = X.astype(np.float32)
    alpha = q / 20.0
    Q = _Q(X.astype(np.float64), y, alpha)
    rng = np.random.default_rng(n)
    v_dense = rng.standard_normal(n)
    v_sparse = np.where(rng.random(n) < 0.1, rng.standard_normal(n), 0.0)
    with _svc(X, y, 1.0, alpha) as s:
        for v in (v_dense, v_sparse, np.zeros(n)):
            t = s.amul(v).cpu().numpy()
            ref = Q @ v
            np.testing.assert_allclose(t, ref, atol=1e-12 * (1.0 + np.abs(v).sum()))


def _state(n, q, seed, sigma, C_, alpha, free_frac_high=False):
    """A w-space state (w, x^k, sigma) and the quantities of one Newton step."""
    X, y = synth.rbf_problem(n, q, seed=seed)
    Q = _Q(X, y, alpha)
    rng = np.random.default_rng(seed)
    xk = rng.uniform(0.0, C_, n)
    w = (0.01 if free_frac_high else 0.3) * rng.standard_normal(n)
    u = xk - sigma * (Q @ w - 1.0)
    xt, lam, free = general.projection(kernel.box_problem(y, C_), u)
    return X, y, Q, w, xt, free


@pytest.mark.parametrize("n,sigma,high", [(200, 2.0, False), (900, 0.01, True), (2600, 0.3, False),
                                           (2600, 0.001, True), (3600, 0.001, True)])
def test_newton_step_cholesky(n, sigma, high):
    """p = 35 (one workgroup), 891 and 1359 (blocked factor, ragged last
    block, one-workgroup solves), 2201 (multi-workgroup solves) and 3169
    (the trailing updates right of the first two groups of eight block
    columns, 2657 and 2145 rows, in 128 x 128 tiles; the later ones in
    64 x 64 tiles)."""
    C_, alpha = 1.0, 1.0
    X, y, Q, w, xt, free = _state(n, 20, 40 + n, sigma, C_, alpha, high)
    s = w - xt
    p = int(free.sum())
    d_ref, Qd_ref, dQd_ref = kernel.newton_pspace(Q, y.astype(np.float64), free, s, sigma)
    with _svc(X, y, C_, alpha) as sv:
        d, Qd, dQd, it = sv.newton_step(free.astype(np.uint8), s, sigma)
    assert it == 0 and 0 < p
    scale = 1.0 + np.abs(Qd_ref).max()
    np.testing.assert_allclose(Qd.cpu().numpy(), Qd_ref, atol=1e-9 * scale)
    np.testing.assert_allclose(d.cpu().numpy(), d_ref, atol=1e-9 * (1.0 + np.abs(d_ref).max()))
    assert dQd == pytest.approx(dQd_ref, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("n,sigma,seed", [(1500, 0.05, 7), (2600, 0.001, 2640)])
def test_newton_step_pcg(n, sigma, seed):
    """The same matrix solved by CG (forced) to a tight tolerance."""
    C_, alpha, mode = 1.0, 1.0, "pcg"
    X, y, Q, w, xt, free = _state(n, 20, seed, sigma, C_, alpha, True)
    s = w - xt
    d_ref, Qd_ref, dQd_ref = kernel.newton_pspace(Q, y.astype(np.float64), free, s, sigma)
    with _svc(X, y, C_, alpha, newton=mode, max_cg=2000) as sv:
        d, Qd, dQd, it = sv.newton_step(free.astype(np.uint8), s, sigma, cg_tol=1e-11)
    assert it > 0
    scale = 1.0 + np.abs(Qd_ref).max()
    np.testing.assert_allclose(Qd.cpu().numpy(), Qd_ref, atol=1e-8 * scale)
    assert dQd == pytest.approx(dQd_ref, rel=1e-8)


def test_newton_step_empty_free_set():
    n, C_, alpha = 100, 1.0, 1.0
    X, y, Q, w, xt, _ = _state(n, 10, 3, 1.0, C_, alpha)
    s = w - xt
    with _svc(X, y, C_, alpha) as sv:
        d, Qd, dQd, _ = sv.newton_step(np.zeros(n, np.uint8), s, 1.0)
    np.testing.assert_array_equal(d.cpu().numpy(), -s)
    np.testing.assert_allclose(Qd.cpu().numpy(), -(Q @ s), atol=1e-12 * (1 + np.abs(s).sum()))
    assert dQd == pytest.approx(float(s @ Q @ s), rel=1e-10)


@pytest.mark.parametrize("n,q,C_", [(400, 20, 0.5), (400, 20, 10.0), (1200, 40, 1.0)])
def test_solve_vs_oracle(n, q, C_):
    X, y = synth.rbf_problem(n, q, seed=5 + n)
    alpha = q / 20.0
    K = features.rbf_kernel(X, X, alpha)
    Q = kernel.kernel_q(K, y)
    tol = 1e-7
    ref = kernel.solve_p5(K, y, C_, tol=tol)
    assert ref.status == "OK"
    with _svc(X, y, C_, alpha, tol=tol) as s:
        x, w, info = s.solve()
    assert w is None
    x = x.cpu().numpy()
    assert info["status_name"] == "OK"
    assert (info["iters_outer"], info["iters_inner"]) == (ref.outer, ref.inner)
    np.testing.assert_allclose(x, ref.x, atol=1e-7 * C_)
    f = kernel.objective_q(Q, x)
    assert f == pytest.approx(ref.obj, rel=1e-8)
    assert info["obj"] == pytest.approx(f, rel=1e-10)
    R, lam = kernel.rkkt_q(Q, y, C_, x)
    assert R <= tol
    # R_KKT, the bias and the gap are small differences of O(1) terms: the
    # GPU's Q x (accumulated over the Newton steps) and the oracle's differ
    # by rounding, which these bounds allow
    assert info["rkkt"] == pytest.approx(R, rel=1e-3, abs=1e-12)
    assert info["b"] == pytest.approx(lam, abs=1e-8) and info["b_out"] == info["b"]
    gap = kernel.duality_gap_at_q(Q, y, C_, x, lam)[0]
    assert abs(info["gap"] - gap) <= 1e-10
    assert np.all(x >= 0.0) and np.all(x <= C_)
    assert abs(float(y.astype(np.float64) @ x)) <= 1e-9 * (1.0 + np.abs(x).sum())


def test_solve_large_free_sets():
    """n = 3000 with every sample free in the first step (p > 2048: the
    multi-workgroup triangular solves): the oracle's iteration counts and
    optimum; then the same problem with every step solved by CG, against the
    oracle's optimum."""
    n, q, C_ = 3000, 50, 10.0
    X, y = synth.rbf_problem(n, q, seed=5)
    alpha = 2.5
    K = features.rbf_kernel(X, X, alpha)
    Q = kernel.kernel_q(K, y)
    ref = kernel.solve_p5(K, y, C_, tol=1e-8)
    assert ref.status == "OK"
    with _svc(X, y, C_, alpha, tol=1e-8) as s:
        x, _, info = s.solve()
    x = x.cpu().numpy()
    assert info["status_name"] == "OK" and info["cg_iters"] == 0
    assert (info["iters_outer"], info["iters_inner"]) == (ref.outer, ref.inner)
    np.testing.assert_allclose(x, ref.x, atol=1e-7 * C_)
    assert kernel.rkkt_q(Q, y, C_, x)[0] <= 1e-8
    assert kernel.objective_q(Q, x) == pytest.approx(ref.obj, rel=1e-9)
    with _svc(X, y, C_, alpha, tol=1e-8, newton="pcg", max_cg=2000) as s:
        x, _, info = s.solve()
    x = x.cpu().numpy()
    assert info["status_name"] == "OK" and info["cg_iters"] > 0
    assert kernel.rkkt_q(Q, y, C_, x)[0] <= 1e-8
    assert kernel.objective_q(Q, x) == pytest.approx(ref.obj, rel=1e-8)


def test_linear_kernel_matches_linear_path():
    from paper_1910_01312_amd.solver import Solver
    X, y = synth.dense_two_gaussians(n=600, q=12, seed=4)
    C_ = 0.8
    with Solver(X, y, C_, tol=1e-8) as s:
        x_lin, _, info_lin = s.solve()
    with _svc(X, y, C_, 1.0, tol=1e-8, kernel="linear") as s:
        x_k, _, info_k = s.solve()
    assert info_lin["status_name"] == info_k["status_name"] == "OK"
    assert info_k["obj"] == pytest.approx(info_lin["obj"], rel=1e-8)
    assert (info_k["iters_outer"], info_k["iters_inner"]) == (info_lin["iters_outer"], info_lin["iters_inner"])
    np.testing.assert_allclose(x_k.cpu().numpy(), x_lin.cpu().numpy(), atol=1e-6 * C_)


def test_warm_start_and_iteration_cap():
    n, q, C_ = 500, 20, 2.0
    X, y = synth.rbf_problem(n, q, seed=9)
    alpha = 1.0
    Q = _Q(X, y, alpha)
    with _svc(X, y, C_, alpha, tol=1e-7) as s:
        x, _, info = s.solve()
        x_ws, _, info_ws = s.solve(x0=x)
    assert info["status_name"] == info_ws["status_name"] == "OK"
    assert info_ws["iters_inner"] < info["iters_inner"]
    assert kernel.rkkt_q(Q, y, C_, x_ws.cpu().numpy())[0] <= 1e-7
    with _svc(X, y, C_, alpha, tol=1e-12, max_outer=2) as s:
        x2, _, info2 = s.solve()
    assert info2["status_name"] == "MAXITER" and info2["iters_outer"] == 2
    assert kernel.rkkt_q(Q, y, C_, x2.cpu().numpy())[0] == pytest.approx(info2["rkkt"], rel=1e-3)


def test_one_class_and_single_sample():
    X, y = synth.rbf_problem(50, 4, seed=1)
    y[:] = -1
    with _svc(X, y, 1.0, 1.0) as s:
        x, _, info = s.solve()
    assert info["status_name"] == "OK"
    assert np.all(x.cpu().numpy() == 0.0)
    with _svc(X[:1], np.array([1], np.int8), 1.0, 1.0) as s:
        x, _, info = s.solve()
    assert info["status_name"] == "OK" and x.cpu().numpy()[0] == 0.0


def test_rejections():
    from paper_1910_01312_amd import _lib as L
    X, y = synth.rbf_problem(40, 4, seed=2)
    with pytest.raises(L.SsnalmError):
        _svc(X, y, 1.0, 0.0)                              # alpha must be > 0
    with pytest.raises(L.SsnalmError):
        _svc(X, y, 1.0, 1.0, precision="mixed")
    bad = y.copy()
    bad[3] = 0
    with pytest.raises(L.SsnalmError):
        _svc(X, bad, 1.0, 1.0)
    with pytest.raises(KeyError):
        _svc(X, y, 1.0, 1.0, kernel="poly")
    with _svc(X, y, 1.0, 1.0) as s:
        with pytest.raises(L.SsnalmError):
            s.atmul(np.ones(40))
        with pytest.raises(L.SsnalmError):
            s.newton(np.ones(40, np.uint8), np.ones(40), 1.0)
        # w_out must be NULL for a kernel context
        x = torch.empty(40, dtype=torch.float64, device="cuda")
        w = torch.empty(40, dtype=torch.float64, device="cuda")
        st = s._lib.ssnalm_solve(s._ctx, None, C.c_void_p(x.data_ptr()), C.c_void_p(w.data_ptr()),
                                 None, None)
        assert st == L.E_BADARG
