"""Pins of the oracle's SSsNAL on the unified problem (P) (Section 1,
eq. Problem_P1_classical1) with Q = B B^T: brute-force enumeration of the
3^n active sets, the C-SVC instance against the C-SVC brute force, the
eps-SVR instance (eq. Def_Dual_of_SVR_Problem) against its primal through
the duality gap, a closed form (eps above every |y_i| gives x = z = 0),
finite differences of psi and the dense HS-Jacobian of Theorem 3.1."""
import numpy as np
import pytest

import synth
from oracle import bruteforce, general
from oracle.projection import hs_jacobian


def _prob(n, q, seed, zero_a=0):
    B, c, a, d, l, u = synth.tiny_general(n, q, seed, zero_a)
    return general.Problem(B=B, c=c, a=a, d=d, l=l, u=u)


@pytest.mark.parametrize("seed", range(8))
def test_general_matches_enumeration(seed):
    n = 5 + seed % 3
    prob = _prob(n, n + 2, 100 + seed, zero_a=1 if seed % 4 == 3 else 0)
    Q = prob.B @ prob.B.T
    f_star, x_star = bruteforce.general_qp_by_enumeration(Q, prob.c, prob.a, prob.d, prob.l, prob.u)
    r = general.solve(prob, tol=1e-10)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
    np.testing.assert_allclose(r.x, x_star, atol=1e-7)       # Q positive definite: unique
    assert abs(float(prob.a @ r.x) - prob.d) <= 1e-10 * (1 + abs(prob.d))
    assert np.all(r.x >= prob.l) and np.all(r.x <= prob.u)
    # eq. Def_Rkkt vanishes at the enumerated optimum and not at a feasible non-optimal point
    assert general.rkkt(prob, x_star) <= 1e-10
    x_mid = general.projection(prob, 0.5 * (prob.l + prob.u))[0]
    if general.objective(prob, x_mid) > f_star + 1e-6:
        assert general.rkkt(prob, x_mid) > 1e-6


@pytest.mark.parametrize("seed", range(4))
def test_csvc_instance_matches_csvc_enumeration(seed):
    X, y = synth.tiny_problem(7, 3, 200 + seed)
    C = 1.5
    f_star, _, _ = bruteforce.qp_by_enumeration(X, y, C)
    r = general.solve(general.csvc_problem(X, y, C), tol=1e-10)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))


@pytest.mark.parametrize("n,q,C,eps", [(6, 2, 1.0, 0.1), (20, 3, 0.5, 0.2), (40, 5, 2.0, 0.05)])
def test_svr_duality_gap(n, q, C, eps):
    X, yr = synth.tiny_regression(n, q, seed=n)
    prob = general.svr_problem(X, yr, C, eps)
    r = general.solve(prob, tol=1e-10)
    assert r.status == "OK"
    x, z = r.x[:n], r.x[n:]
    assert abs(float(x.sum() - z.sum())) <= 1e-10
    assert np.all(r.x >= 0.0) and np.all(r.x <= C)
    # eps > 0: no sample uses both of its multipliers
    assert np.max(np.minimum(x, z)) <= 1e-8
    w = general.svr_weights(X, x, z)
    b = general.svr_best_bias(X, yr, C, eps, w)
    P = general.svr_primal(X, yr, C, eps, w, b)
    gap = P + r.obj                      # >= 0 by weak duality, 0 at the optimum
    assert gap >= -1e-10 * (1 + abs(P))
    assert gap <= 1e-7 * (1 + abs(P) + abs(r.obj))


def test_svr_eps_above_targets_gives_zero():
    X, yr = synth.tiny_regression(12, 3, seed=5)
    eps = float(np.max(np.abs(yr))) + 0.1
    r = general.solve(general.svr_problem(X, yr, 1.0, eps), tol=1e-12)
    assert r.status == "OK" and r.outer == 1
    assert np.all(r.x == 0.0) and r.rkkt == 0.0


def _state(prob, sigma, seed):
    rng = np.random.default_rng(seed)
    n, q = prob.B.shape
    xk = general.projection(prob, rng.uniform(prob.l, prob.u))[0]
    omega = prob.B.T @ (0.3 * rng.standard_normal(n))
    return xk, omega


@pytest.mark.parametrize("seed", range(4))
def test_general_gradient_by_finite_differences(seed):
    prob = _prob(9, 4, 300 + seed)
    sigma = 2.0
    xk, omega = _state(prob, sigma, seed)
    u = xk - sigma * (prob.B @ omega + prob.c)
    xt, _, _ = general.projection(prob, u)
    g = omega - prob.B.T @ xt
    h = 1e-6
    fd = np.array([(general.psi_literal(prob, omega + h * e, xk, sigma)
                    - general.psi_literal(prob, omega - h * e, xk, sigma)) / (2 * h)
                   for e in np.eye(omega.size)])
    np.testing.assert_allclose(fd, g, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_general_psi_increment_matches_literal(seed):
    prob = _prob(10, 4, 400 + seed)
    sigma = 1.5
    xk, omega = _state(prob, sigma, seed)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(omega.size)
    u = xk - sigma * (prob.B @ omega + prob.c)
    _, lam, _ = general.projection(prob, u)
    for alpha in (1.0, 0.25, 1e-3):
        u_a = u - alpha * sigma * (prob.B @ d)
        _, lam_a, _ = general.projection(prob, u_a)
        inc = general.psi_increment(prob, omega, d, alpha, u, lam, u_a, lam_a, sigma)
        lit = (general.psi_literal(prob, omega + alpha * d, xk, sigma)
               - general.psi_literal(prob, omega, xk, sigma))
        assert inc == pytest.approx(lit, rel=1e-8, abs=1e-10)


def test_h_increment_pieces():
    rng = np.random.default_rng(7)
    for l, u in ((0.0, 1.0), (0.4, 2.0), (-3.0, -1.0), (-1.0, 0.5)):
        t = rng.uniform(-4, 4, 2000)
        dt = rng.uniform(-3, 3, 2000) * (rng.random(2000) < 0.5) + rng.uniform(-1e-3, 1e-3, 2000)
        ref = general.h_piece(t + dt, l, u) - general.h_piece(t, l, u)
        np.testing.assert_allclose(general.h_increment(t, dt, l, u), ref, rtol=1e-9, atol=1e-12)
        # h' = clip(t): a midpoint-rule check of the slope
        e = 1e-6
        slope = (general.h_piece(t + e, l, u) - general.h_piece(t - e, l, u)) / (2 * e)
        np.testing.assert_allclose(slope, np.clip(t, l, u), atol=1e-6)


@pytest.mark.parametrize("zero_a", [0, 3])
def test_general_newton_matches_dense_hs_jacobian(zero_a):
    prob = _prob(12, 5, 500 + zero_a, zero_a=zero_a)
    sigma = 3.0
    xk, omega = _state(prob, sigma, zero_a)
    u = xk - sigma * (prob.B @ omega + prob.c)
    xt, _, free = general.projection(prob, u)
    g = omega - prob.B.T @ xt
    P = hs_jacobian(free, prob.a)
    M = np.eye(omega.size) + sigma * prob.B.T @ P @ prob.B
    d_ref = -np.linalg.solve(M, g)
    d = general.newton_direction(prob, free, g, sigma)
    np.testing.assert_allclose(d, d_ref, rtol=1e-10, atol=1e-12)


def test_planted_mistake_svr_sign_is_caught():
    """A plausible mistake (eps - y and eps + y swapped in c) solves a
    different QP; the duality-gap pin against the SVR primal rejects it."""
    n, q, C, eps = 20, 3, 0.5, 0.2
    X, yr = synth.tiny_regression(n, q, seed=n)
    good = general.svr_problem(X, yr, C, eps)
    bad = general.Problem(B=good.B, c=np.concatenate([good.c[n:], good.c[:n]]), a=good.a,
                          d=good.d, l=good.l, u=good.u)
    r = general.solve(bad, tol=1e-10)
    x, z = r.x[:n], r.x[n:]
    w = general.svr_weights(X, x, z)
    b = general.svr_best_bias(X, yr, C, eps, w)
    P = general.svr_primal(X, yr, C, eps, w, b)
    f_true = general.objective(good, r.x)
    assert P + f_true > 1e-3 * (1 + abs(P) + abs(f_true))


def test_svr_on_csr_rows():
    """The eps-SVR instance built from CSR data (B = [X; -X] kept sparse)
    gives the dense-data solution and a vanishing duality gap."""
    import scipy.sparse as sp
    rng = np.random.default_rng(11)
    n, q = 60, 8
    Xd = rng.standard_normal((n, q)) * (rng.random((n, q)) < 0.4)
    yr = Xd @ rng.standard_normal(q) + 0.05 * rng.standard_normal(n)
    C, eps = 1.0, 0.1
    r_s = general.solve(general.svr_problem(sp.csr_matrix(Xd), yr, C, eps), tol=1e-10)
    r_d = general.solve(general.svr_problem(Xd, yr, C, eps), tol=1e-10)
    assert r_s.status == "OK" and r_d.status == "OK"
    assert r_s.obj == pytest.approx(r_d.obj, abs=1e-9 * (1 + abs(r_d.obj)))
    x, z = r_s.x[:n], r_s.x[n:]
    w = general.svr_weights(Xd, x, z)
    b = general.svr_best_bias(Xd, yr, C, eps, w)
    gap = general.svr_primal(Xd, yr, C, eps, w, b) + r_s.obj
    assert -1e-9 <= gap <= 1e-7 * (1 + abs(r_s.obj))


@pytest.mark.parametrize("zero_a", [0, 3])
def test_general_pcg_matches_cholesky_direction(zero_a):
    prob = _prob(40, 6, 800 + zero_a, zero_a=zero_a)
    sigma = 5.0
    xk, omega = _state(prob, sigma, zero_a)
    u = xk - sigma * (prob.B @ omega + prob.c)
    xt, _, free = general.projection(prob, u)
    g = omega - prob.B.T @ xt
    d_ref = general.newton_direction(prob, free, g, sigma)
    d, it = general.newton_pcg(prob, free, g, sigma, tol=1e-13 * np.linalg.norm(g))
    assert it <= 12                  # q = 6: q steps in exact arithmetic, a few more in fp64
    np.testing.assert_allclose(d, d_ref, rtol=1e-9, atol=1e-12)


def test_svr_pcg_solve_matches_cholesky_solve():
    import scipy.sparse as sp
    X, yr = synth.tiny_regression(80, 6, seed=4)
    prob = general.svr_problem(sp.csr_matrix(X), yr, 1.0, 0.1)
    r_c = general.solve(prob, tol=1e-9)
    r_p = general.solve(prob, tol=1e-9, newton="pcg")
    assert r_c.status == "OK" and r_p.status == "OK" and r_p.cg_iters > 0
    assert r_p.obj == pytest.approx(r_c.obj, abs=1e-8 * (1 + abs(r_c.obj)))
