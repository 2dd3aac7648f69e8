"""Pins of the oracle's SSsNAL solver (Algorithms 1 and 3 in omega-space)
against brute-force enumeration, hand-derived closed forms, the paper's own
n-space Newton system and Proposition 5, finite differences and the KKT /
duality-gap invariants."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import bruteforce, literal, ssnal
from oracle.projection import project_svm


def _state(X, y, C, sigma, seed):
    """A random ALM state (omega = A^T w in Ran(A^T), x^k feasible)."""
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    yf = y.astype(np.float64)
    A = yf[:, None] * X
    w = rng.normal(size=n) * 0.3
    xk, _, _ = project_svm(rng.random(n) * C * 2, y, C)
    omega = A.T @ w
    u = xk + sigma * (1.0 - A @ omega)
    xt, lam, free = project_svm(u, y, C)
    g = omega - A.T @ xt
    return A, w, xk, omega, u, xt, lam, free, g


# ---------------------------------------------------------------- whole QP

def test_golden_qp(golden):
    for case in golden["qp_cases"]:
        X = np.array(case["X"], dtype=np.float64)
        y = np.array(case["y"], dtype=np.int8)
        r = ssnal.solve(X, y, case["C"], tol=1e-12)
        assert r.obj == pytest.approx(case["f_star"], abs=1e-9), case["name"]
        np.testing.assert_allclose(r.w, case["w_star"], atol=1e-8)
        if case["b_star"] is not None:
            assert r.b == pytest.approx(case["b_star"], abs=1e-7), case["name"]


@pytest.mark.parametrize("seed", range(12))
def test_qp_vs_enumeration(seed):
    n = 6 + seed % 3
    q = 2 + seed % 3
    X, y = synth.tiny_problem(n, q, seed, integer=(seed % 2 == 0))
    C = [0.1, 1.0, 10.0][seed % 3]
    f_star, x_star, _ = bruteforce.qp_by_enumeration(X, y, C)
    r = ssnal.solve(X, y, C, tol=1e-11)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, rel=1e-9, abs=1e-10)
    yf = y.astype(np.float64)
    w_star = (yf[:, None] * X).T @ x_star
    np.testing.assert_allclose(r.w, w_star, atol=1e-6 * (1 + np.abs(w_star).max()))


def test_closed_form_two_points():
    rng = np.random.default_rng(11)
    for _ in range(10):
        X = rng.normal(size=(2, 4))
        y = np.array([1, -1], np.int8)
        C = float(rng.uniform(0.05, 5))
        D = X[0] - X[1]
        t = min(C, 2.0 / float(D @ D))
        f = 0.5 * t * t * float(D @ D) - 2 * t
        r = ssnal.solve(X, y, C, tol=1e-12)
        assert r.obj == pytest.approx(f, rel=1e-10, abs=1e-12)
        if t < C:
            b = (float(X[1] @ X[1]) - float(X[0] @ X[0])) / float(D @ D)
            assert r.b == pytest.approx(b, abs=1e-7)


def test_duality_gap_capped_two_points():
    """Two points with the box active (t* = C < 2/|D|^2, D = x~_1 - x~_2):
    x* = (C, C), w* = C D, f* = C^2|D|^2/2 - 2C, and the C-SVC primal at w*
    with the best bias is C^2|D|^2/2 + C (2 - C|D|^2) = 2C - C^2|D|^2/2
    (both hinge terms active between the two kinks), so P* + f* = 0.  A C
    missing from the hinge term of the primal breaks this for C != 1."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        X = rng.normal(size=(2, 3))
        y = np.array([1, -1], np.int8)
        D = X[0] - X[1]
        dd = float(D @ D)
        C = float(rng.uniform(0.05, 0.9)) * 2.0 / dd       # strictly capped, C != 1
        x = np.array([C, C])
        gap, P, f = ssnal.duality_gap(X, y, C, x)
        assert f == pytest.approx(0.5 * C * C * dd - 2 * C, rel=1e-12)
        assert P == pytest.approx(2 * C - 0.5 * C * C * dd, rel=1e-12)
        assert abs(gap) <= 1e-13
        # any bias between the kinks gives the same primal value; outside, more
        gb, Pb, _ = ssnal.duality_gap_at(X, y, C, x, b=1e3)
        assert Pb > P and gb > gap
        # planted: the hinge sum without its C factor misses P* unless C = 1
        w = C * D
        b = ssnal.best_bias(X, y, C, w)
        m = X @ w + b
        P_planted = 0.5 * float(w @ w) + float(np.sum(np.maximum(0.0, 1.0 - y * m)))
        assert abs(P_planted - P) > 1e-6


def test_single_class_gives_zero():
    X = np.random.default_rng(0).normal(size=(20, 3))
    y = np.ones(20, np.int8)
    r = ssnal.solve(X, y, 1.0)
    assert np.all(r.x == 0.0)


# ---------------------------------------------------------------- dense C1

@pytest.fixture(scope="module")
def c1():
    X, y = synth.dense_two_gaussians()
    return X, y, ssnal.solve(X, y, 1.0, tol=1e-6), ssnal.solve(X, y, 1.0, tol=1e-10)


def test_c1_optimality(c1):
    X, y, r, rref = c1
    assert r.status == "OK" and r.rkkt <= 1e-6
    R, _ = ssnal.rkkt(X, y, 1.0, r.x)
    assert R == pytest.approx(r.rkkt)
    yf = y.astype(np.float64)
    # the last projection acts on u = x + sigma (e - A omega): its rounding
    # scale is |u|_inf, not C
    u_scale = 1.0 + r.sigma * (1.0 + np.abs(yf * (X @ r.omega)).max())
    assert abs(float(yf @ r.x)) <= 4 * X.shape[0] * np.finfo(float).eps * u_scale
    assert np.all(r.x >= 0) and np.all(r.x <= 1.0)
    assert rref.status == "OK"
    gap, P, f = ssnal.duality_gap(X, y, 1.0, rref.x)
    assert gap >= -1e-12 and gap <= 1e-9
    assert abs(r.obj - rref.obj) / abs(rref.obj) <= 1e-7


@pytest.mark.parametrize("sigma0,rho", [(0.1, 2.0), (10.0, 10.0), (1.0, 3.0)])
def test_schedule_independence(c1, sigma0, rho):
    X, y, _, rref = c1
    r = ssnal.solve(X, y, 1.0, tol=1e-10, sigma0=sigma0, rho=rho)
    assert r.obj == pytest.approx(rref.obj, rel=1e-10)
    np.testing.assert_allclose(r.w, rref.w, atol=1e-6)


@pytest.mark.parametrize("mode", ["pspace", "pcg"])
def test_newton_modes_same_solution(c1, mode):
    X, y, _, rref = c1
    r = ssnal.solve(X, y, 1.0, tol=1e-10, newton=mode)
    assert r.obj == pytest.approx(rref.obj, rel=1e-10)


def test_sparse_input_same_solution():
    X, y = synth.dense_two_gaussians(n=400, q=20)
    X[np.abs(X) < 0.8] = 0.0
    rd = ssnal.solve(X, y, 0.5, tol=1e-10)
    rs = ssnal.solve(sp.csr_matrix(X), y, 0.5, tol=1e-10, newton="pcg")
    assert rs.obj == pytest.approx(rd.obj, rel=1e-10)


# ---------------------------------------------------------------- pieces

@pytest.mark.parametrize("seed", range(6))
def test_newton_four_ways(seed):
    X, y = synth.tiny_problem(9, 3, 40 + seed)
    C, sigma = 1.0, [0.3, 1.0, 4.0][seed % 3]
    A, w, xk, omega, u, xt, lam, free, g = _state(X, y, C, sigma, seed)
    dq = ssnal.newton_qspace(X, free, g, sigma)
    dp = ssnal.newton_pspace_centered(X, free, g, sigma)
    dc, _ = ssnal.newton_pcg(X, free, g, sigma, 1e-14, 200)
    dn, Q = literal.newton_nspace(X, y, w, xk, sigma, C)
    Qd, dQd, _ = literal.prop5_paper(X, y, w, xk, sigma, C)
    scale = 1 + np.linalg.norm(dq)
    np.testing.assert_allclose(dp, dq, atol=1e-11 * scale)
    np.testing.assert_allclose(dc, dq, atol=1e-9 * scale)
    np.testing.assert_allclose(A.T @ dn, dq, atol=1e-10 * scale)
    np.testing.assert_allclose(A @ dq, Qd, atol=1e-10 * scale)
    assert float(dq @ dq) == pytest.approx(dQd, rel=1e-9, abs=1e-12)
    assert float(g @ dq) < 0 or np.linalg.norm(g) == 0


def test_planted_centering_drop_is_caught():
    """Dropping the -s s^T/p term of A^T P A (a plausible slip) makes the
    omega-space direction disagree with the paper's n-space system."""
    X, y = synth.tiny_problem(9, 3, 77)
    C, sigma = 1.0, 2.0
    A, w, xk, omega, u, xt, lam, free, g = _state(X, y, C, sigma, 3)
    idx = np.flatnonzero(free)
    assert idx.size > 1
    XJ = X[idx]
    M_bad = np.eye(3) + sigma * XJ.T @ XJ
    d_bad = -np.linalg.solve(M_bad, g)
    dn, _ = literal.newton_nspace(X, y, w, xk, sigma, C)
    assert np.linalg.norm(A.T @ dn - d_bad) > 1e-6


@pytest.mark.parametrize("seed", range(5))
def test_gradient_by_finite_differences(seed):
    X, y = synth.tiny_problem(30, 4, 90 + seed)
    C, sigma = 1.0, 1.5
    A, w, xk, omega, u, xt, lam, free, g = _state(X, y, C, sigma, seed)
    rng = np.random.default_rng(seed)
    h = rng.normal(size=omega.size)
    eps = 1e-6

    def psi_at(om):
        uu = xk + sigma * (1.0 - A @ om)
        return ssnal.psi_literal(om, uu, xk, sigma, y, C)

    fd = (psi_at(omega + eps * h) - psi_at(omega - eps * h)) / (2 * eps)
    assert fd == pytest.approx(float(g @ h), rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("seed", range(5))
def test_psi_increment_equals_literal_difference(seed):
    X, y = synth.tiny_problem(40, 5, 120 + seed)
    C, sigma = 0.7, 2.0
    A, w, xk, omega, u, xt, lam, free, g = _state(X, y, C, sigma, seed)
    d = ssnal.newton_qspace(X, free, g, sigma)
    for alpha in (1.0, 0.5, 0.125):
        om2 = omega + alpha * d
        u2 = xk + sigma * (1.0 - A @ om2)
        _, lam2, _ = project_svm(u2, y, C)
        inc = ssnal.psi_increment(omega, d, alpha, u, lam, u2, lam2, sigma, y, C)
        lit = (ssnal.psi_literal(om2, u2, xk, sigma, y, C)
               - ssnal.psi_literal(omega, u, xk, sigma, y, C))
        assert inc == pytest.approx(lit, rel=1e-9, abs=1e-11)


def test_x_update_identity():
    """x^{k+1} = x^k - sigma (Q w + z + c) with z from eq. Def bar_w and bar_v2
    equals Pi(u(w)) (eq. Def_new_update_xkplus)."""
    X, y = synth.tiny_problem(25, 4, 5)
    C, sigma = 2.0, 3.0
    A, w, xk, omega, u, xt, lam, free, g = _state(X, y, C, sigma, 1)
    z = (u - xt) / sigma
    x_next = xk - sigma * (A @ omega + z - 1.0)
    np.testing.assert_allclose(x_next, xt, atol=1e-12)


def test_armijo_and_monotone_psi():
    X, y = synth.dense_two_gaussians(n=300, q=8)
    r = ssnal.solve(X, y, 1.0, tol=1e-9, record=True)
    assert r.status == "OK"
    assert r.ls_fail == 0
    rk = [h["rkkt"] for h in r.history]
    assert rk[-1] <= 1e-9


def test_newton_lowrank_matches_cholesky():
    """The Woodbury correction of an earlier step's factor (same sigma) gives
    the direction of the fresh Cholesky solve, for J changes of a few rows and
    of many rows, including an empty previous J."""
    import scipy.linalg as sla
    X, y = synth.dense_two_gaussians(n=400, q=12, seed=3)
    rng = np.random.default_rng(0)
    sigma = 7.0
    g = rng.standard_normal(12)
    base = rng.random(400) < 0.3
    for flips in (0, 1, 5, 60, 400):
        free = base.copy()
        free[rng.choice(400, flips, replace=False)] ^= True
        for prev in (base, np.zeros(400, bool)):
            idx0 = np.flatnonzero(prev)
            M0 = np.eye(12)
            if idx0.size:
                XJ = X[idx0]
                s0 = XJ.sum(0)
                M0 = M0 + sigma * (XJ.T @ XJ - np.outer(s0, s0) / idx0.size)
            d = ssnal.newton_lowrank(X, free, g, sigma, prev, sla.cho_factor(M0, lower=True))
            d_ref = ssnal.newton_qspace(X, free, g, sigma)
            assert np.linalg.norm(d - d_ref) <= 1e-9 * np.linalg.norm(d_ref)
