"""Pins of the nonlinear-kernel C-SVC oracle (Table 3's problem): the XOR
closed form under the RBF kernel, 3^n enumeration with the explicit Q, and
the linear kernel against the linear C-SVC oracle."""
import numpy as np
import pytest

import synth
from oracle import bruteforce, features, kernel, ssnal


@pytest.mark.parametrize("alpha,C", [(1.0, 100.0), (0.5, 100.0), (1.0, 0.5)])
def test_xor_closed_form(alpha, C):
    """Corners (+-1, +-1) with y = x1 x2.  Each point has two neighbours of the
    other class at squared distance 4 and one point of its own class at 8,
    so with x_i = t for all i (symmetry; y^T x = 0 holds) (Q x)_i =
    t (1 - exp(-2/alpha))^2 =: t kappa and f = 2 kappa t^2 - 4 t, minimised
    at t = min(1/kappa, C)."""
    X = np.array([[1.0, 1.0], [-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
    y = np.array([1, 1, -1, -1], np.int8)
    K = features.rbf_kernel(X, X, alpha)
    kappa = (1.0 - np.exp(-2.0 / alpha)) ** 2
    t = min(1.0 / kappa, C)
    r = kernel.solve(K, y, C, tol=1e-10)
    assert r.status == "OK"
    np.testing.assert_allclose(r.x, t, rtol=1e-8)
    assert r.obj == pytest.approx(2 * kappa * t * t - 4 * t, rel=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_rbf_matches_enumeration(seed):
    rng = np.random.default_rng(700 + seed)
    X = rng.standard_normal((7, 2))
    y = np.where(X[:, 0] * X[:, 1] > 0, 1, -1).astype(np.int8)
    if np.all(y == y[0]):
        y[0] = -y[0]
    K = features.rbf_kernel(X, X, 0.8)
    Q = kernel.kernel_q(K, y)
    C = 2.0
    f_star, x_star = bruteforce.general_qp_by_enumeration(
        Q, -np.ones(7), y.astype(np.float64), 0.0, np.zeros(7), np.full(7, C))
    r = kernel.solve(K, y, C, tol=1e-10)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
    np.testing.assert_allclose(r.x, x_star, atol=1e-6)       # RBF Q is positive definite


def test_linear_kernel_matches_linear_oracle():
    X, y = synth.tiny_problem(30, 4, 9)
    C = 1.0
    r_lin = ssnal.solve(X, y, C, tol=1e-10)
    r_ker = kernel.solve(X @ X.T, y, C, tol=1e-10)
    assert r_ker.status == "OK"
    assert r_ker.obj == pytest.approx(r_lin.obj, abs=1e-8 * (1 + abs(r_lin.obj)))


# ---------------------------------------------------------------- w-space (Proposition 5)

def _rbf_state(n, seed, sigma, C=1.0):
    from oracle import general
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 3))
    y = np.where(rng.standard_normal(n) > 0, 1, -1).astype(np.int8)
    K = features.rbf_kernel(X, X, 0.7)
    prob = kernel.kernel_problem(K, y, C)
    Q = kernel.kernel_q(K, y)
    w = 0.3 * rng.standard_normal(n)
    xk = np.clip(rng.standard_normal(n), 0.0, C)
    u = xk - sigma * (Q @ w - 1.0)
    xt, _, free = general.projection(prob, u)
    return prob, Q, w, xt, free


@pytest.mark.parametrize("seed,sigma", [(1, 3.0), (2, 0.1), (3, 50.0), (4, 1e4)])
def test_newton_pspace_matches_omega_space(seed, sigma):
    """The p x p step reproduces the omega-space Newton direction of the
    factored Q: Q d = B d_omega, d^T Q d = |d_omega|^2, B^T d = d_omega."""
    from oracle import general
    prob, Q, w, xt, free = _rbf_state(60, seed, sigma)
    s = w - xt
    d, Qd, dQd = kernel.newton_pspace(Q, prob.a, free, s, sigma)
    g = prob.B.T @ w - prob.B.T @ xt
    dom = general.newton_direction(prob, free, g, sigma)
    scale = 1.0 + np.abs(Qd).max()
    np.testing.assert_allclose(Qd, prob.B @ dom, atol=1e-10 * scale)
    np.testing.assert_allclose(prob.B.T @ d, dom, atol=1e-10 * scale)
    assert dQd == pytest.approx(float(dom @ dom), rel=1e-9, abs=1e-12)


def test_newton_pspace_empty_free_set():
    """J empty: P = 0 (Theorem 3.1), the step is -s with Q d = -Q s."""
    prob, Q, w, xt, _ = _rbf_state(20, 5, 1.0)
    s = w - xt
    d, Qd, dQd = kernel.newton_pspace(Q, prob.a, np.zeros(20, bool), s, 1.0)
    np.testing.assert_array_equal(d, -s)
    np.testing.assert_allclose(Qd, -(Q @ s), atol=1e-13)
    assert dQd == pytest.approx(float(s @ Q @ s), rel=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_newton_pspace_matches_prop5_as_printed(seed):
    """Against Proposition 5 (a) evaluated literally (eq. Def_small_linear_eq,
    Def_Qd_start1, Def_dQd) on a linear-kernel Q."""
    from oracle import literal
    X, y = synth.tiny_problem(25, 4, 40 + seed)
    rng = np.random.default_rng(seed)
    w = 0.2 * rng.standard_normal(25)
    xk = np.clip(rng.standard_normal(25), 0.0, 1.0)
    sigma = 2.0
    Q, u, xt, free, grad = literal.state_nspace(X, y, w, xk, sigma, 1.0)
    Qd_ref, dQd_ref, case = literal.prop5_paper(X, y, w, xk, sigma, 1.0)
    assert case == "a"
    _, Qd, dQd = kernel.newton_pspace(Q, np.asarray(y, np.float64), free, w - xt, sigma)
    np.testing.assert_allclose(Qd, Qd_ref, atol=1e-9 * (1 + np.abs(Qd_ref).max()))
    assert dQd == pytest.approx(dQd_ref, rel=1e-8)


@pytest.mark.parametrize("C", [0.5, 10.0])
def test_solve_p5_matches_omega_space(C):
    """Same decisions in both formulations: equal iteration counts, x and
    objective to rounding."""
    X, y = synth.mixture_problem(150, q=5, seed=11)
    K = features.rbf_kernel(X, X, 2.0)
    r = kernel.solve(K, y, C, tol=1e-8)
    r5 = kernel.solve_p5(K, y, C, tol=1e-8)
    assert r.status == r5.status == "OK"
    assert (r5.outer, r5.inner) == (r.outer, r.inner)
    np.testing.assert_allclose(r5.x, r.x, atol=1e-8 * C)
    assert r5.obj == pytest.approx(r.obj, rel=1e-11)


@pytest.mark.parametrize("seed", range(3))
def test_solve_p5_matches_enumeration(seed):
    rng = np.random.default_rng(900 + seed)
    X = rng.standard_normal((7, 2))
    y = np.where(X[:, 0] > 0, 1, -1).astype(np.int8)
    if np.all(y == y[0]):
        y[0] = -y[0]
    K = features.rbf_kernel(X, X, 1.3)
    Q = kernel.kernel_q(K, y)
    f_star, x_star = bruteforce.general_qp_by_enumeration(
        Q, -np.ones(7), y.astype(np.float64), 0.0, np.zeros(7), np.full(7, 3.0))
    r = kernel.solve_p5(K, y, 3.0, tol=1e-10)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
    np.testing.assert_allclose(r.x, x_star, atol=1e-6)


def test_solve_p5_xor_closed_form():
    X = np.array([[1.0, 1.0], [-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
    y = np.array([1, 1, -1, -1], np.int8)
    K = features.rbf_kernel(X, X, 1.0)
    kappa = (1.0 - np.exp(-2.0)) ** 2
    r = kernel.solve_p5(K, y, 100.0, tol=1e-10)
    assert r.status == "OK"
    np.testing.assert_allclose(r.x, 1.0 / kappa, rtol=1e-8)


def test_kernel_gap_and_rkkt_reduce_to_linear():
    """With k(x, z) = x^T z the kernel residual and gap are the linear
    oracle's, at any x and b."""
    X, y = synth.tiny_problem(40, 5, 3)
    C = 0.7
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, C, 40)
    Q = kernel.kernel_q(X @ X.T, y)
    R, lam = kernel.rkkt_q(Q, y, C, x)
    R_lin, b_lin = ssnal.rkkt(X, y, C, x)
    assert R == pytest.approx(R_lin, rel=1e-12)
    assert lam == pytest.approx(b_lin, rel=1e-12, abs=1e-14)
    for b in (-0.3, 0.0, 0.8):
        assert kernel.duality_gap_at_q(Q, y, C, x, b)[0] == pytest.approx(
            ssnal.duality_gap_at(X, y, C, x, b)[0], rel=1e-12)
