"""Pins of the oracle's projection onto K ∩ L (Section 3.2.1, Algorithm 2)
and of the HS-Jacobian (Theorem 3.1) against brute force, hand-derived cases,
a textbook special case and invariants."""
import numpy as np
import pytest

from oracle import bruteforce
from oracle.projection import (breakpoint_search, clip_box, hs_jacobian,
                               project, project_svm)

pytestmark = pytest.mark.filterwarnings("ignore")


def _rand_case(rng, n):
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    if np.all(y == y[0]):
        y[0] = -y[0]
    v = rng.normal(0.0, 2.0, size=n)
    C = float(rng.uniform(0.3, 3.0))
    return v, y, C


def test_golden_projection(golden):
    for case in golden["projection_cases"]:
        x, lam, free = project_svm(np.array(case["v"]), np.array(case["y"]), case["C"])
        assert lam == pytest.approx(case["lam"], abs=1e-14), case["name"]
        np.testing.assert_allclose(x, case["x"], atol=1e-14)
        assert list(free) == case["free"], case["name"]


@pytest.mark.parametrize("seed", range(25))
def test_projection_vs_enumeration(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    v, y, C = _rand_case(rng, n)
    x, lam, _ = project_svm(v, y, C)
    xb, _ = bruteforce.projection_by_enumeration(v, y, C)
    np.testing.assert_allclose(x, xb, atol=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_projection_invariants(seed):
    rng = np.random.default_rng(100 + seed)
    n = 500
    v, y, C = _rand_case(rng, n)
    v *= 10
    x, lam, _ = project_svm(v, y, C)
    yf = y.astype(np.float64)
    assert abs(float(yf @ x)) <= 4 * n * np.finfo(float).eps * C * 10
    assert np.all(x >= 0.0) and np.all(x <= C)
    x2, _, _ = project_svm(x, y, C)
    np.testing.assert_allclose(x2, x, atol=1e-12)
    # variational inequality (v - Pi)^T (z - Pi) <= 0 for feasible z
    for _ in range(5):
        z, _, _ = project_svm(rng.normal(0, 5, size=n), y, C)
        assert float((v - x) @ (z - x)) <= 1e-9 * (1 + np.abs(v).sum())


def _simplex_sort(v):
    """Textbook sort-based projection onto the probability simplex
    {x >= 0, sum x = 1} (threshold rule of Held, Wolfe & Crowder)."""
    u = np.sort(v)[::-1]
    css = np.cumsum(u)
    k = np.arange(1, v.size + 1)
    rho = np.nonzero(u - (css - 1.0) / k > 0)[0][-1]
    theta = (css[rho] - 1.0) / (rho + 1)
    return np.maximum(v - theta, 0.0)


@pytest.mark.parametrize("seed", range(10))
def test_simplex_special_case(seed):
    # a = e, d = 1, l = 0, u = +large: K ∩ L is the probability simplex
    rng = np.random.default_rng(200 + seed)
    v = rng.normal(size=50) * 3
    x, _ = project(v, np.ones(50), 0.0, 1e6, 1.0)
    np.testing.assert_allclose(x, _simplex_sort(v), atol=1e-12)


def test_breakpoint_search_matches_bisection():
    rng = np.random.default_rng(7)
    v, y, C = _rand_case(rng, 2000)
    yf = y.astype(np.float64)
    lam = breakpoint_search(v, yf, 0.0, C, 0.0)
    # independent bisection on h(lam) = y^T clip(v - lam y)
    lo, hi = -100.0, 100.0
    h = lambda t: float(yf @ clip_box(v - t * yf, 0.0, C))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if h(mid) > 0:
            lo = mid
        else:
            hi = mid
    assert lam == pytest.approx(0.5 * (lo + hi), abs=1e-9)


@pytest.mark.parametrize("seed", range(8))
def test_hs_jacobian_properties(seed):
    rng = np.random.default_rng(300 + seed)
    n = 12
    v, y, C = _rand_case(rng, n)
    x, lam, free = project_svm(v, y, C)
    yf = y.astype(np.float64)
    P = hs_jacobian(free, yf)
    np.testing.assert_allclose(P, P.T, atol=1e-14)
    np.testing.assert_allclose(P @ P, P, atol=1e-13)
    np.testing.assert_allclose(P @ yf, 0.0, atol=1e-13)
    # directional derivative by finite differences away from breakpoints
    t = v - lam * yf
    gap = np.min(np.minimum(np.abs(t), np.abs(t - C)))
    if gap < 1e-6:
        # lam sits on a breakpoint (e.g. no free component): Pi is not
        # differentiable there, so only the algebraic properties apply
        return
    eps = min(1e-7, 0.1 * gap)
    h = rng.normal(size=n)
    xe, _, _ = project_svm(v + eps * h, y, C)
    np.testing.assert_allclose((xe - x) / eps, P @ h, atol=1e-6)


def test_planted_sign_error_is_caught():
    """A plausible slip (clipping v + lam*y instead of v - lam*y) breaks the
    brute-force pin: the pins are sensitive to it."""
    rng = np.random.default_rng(5)
    bad_hits = 0
    for _ in range(10):
        v, y, C = _rand_case(rng, 6)
        x, lam, _ = project_svm(v, y, C)
        bad = clip_box(v + lam * y.astype(np.float64), 0.0, C)
        xb, _ = bruteforce.projection_by_enumeration(v, y, C)
        if not np.allclose(bad, xb, atol=1e-9):
            bad_hits += 1
    assert bad_hits >= 8
