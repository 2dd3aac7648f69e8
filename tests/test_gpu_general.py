"""The unified problem (P) of Section 1 with general c, a, d, l, u and a
linear kernel Q = B B^T on the GPU (ssnalm_create_general) against the
general-form oracle (oracle/general.py) (GPU only).

  * tiny instances with Q positive definite: the optimum by 3^n enumeration
    of the active sets (unique x), including a_i = 0 components, boxes that
    exclude 0 (x^0 = Pi(0)) and d != 0;
  * the projection onto {a^T x = d, l <= x <= u} (mixed-sign and zero a):
    the multiplier, x and the free set against the oracle's breakpoint
    search, element by element, across several 1024-element blocks;
  * one line-search trial: the psi increment against the oracle's;
  * a medium instance: R_KKT <= 1e-6 recomputed by the oracle and the 1e-8
    objective bar against the oracle's reference on one solution;
  * the C-SVC written as (P) gives the C-SVC path's optimum.
"""
import numpy as np
import pytest

import synth
from oracle import bruteforce, general, ssnal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _prob(n, q, seed, zero_a=0):
    B, c, a, d, l, u = synth.tiny_general(n, q, seed, zero_a)
    return general.Problem(B=B, c=c, a=a, d=d, l=l, u=u)


def _ctx(prob, tol, **kw):
    from paper_1910_01312_amd.solver import General
    return General(prob.B, prob.c, prob.a, prob.l, prob.u, prob.d, tol=tol, **kw)


@pytest.mark.parametrize("seed", range(6))
def test_general_tiny_vs_enumeration(seed):
    n = 5 + seed % 3
    prob = _prob(n, n + 2, 100 + seed, zero_a=1 if seed % 3 == 2 else 0)
    Q = prob.B @ prob.B.T
    f_star, x_star = bruteforce.general_qp_by_enumeration(Q, prob.c, prob.a, prob.d, prob.l, prob.u)
    with _ctx(prob, 1e-10) as s:
        x, w, info = s.solve()
    x = x.cpu().numpy()
    assert info["status_name"] == "OK"
    assert general.objective(prob, x) == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
    np.testing.assert_allclose(x, x_star, atol=1e-7)
    assert abs(float(prob.a @ x) - prob.d) <= 1e-9 * (1 + abs(prob.d))
    assert np.all(x >= prob.l) and np.all(x <= prob.u)
    assert info["obj"] == pytest.approx(general.objective(prob, x), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("n,zero_a", [(3000, 0), (2500, 40), (1, 0), (777, 0)])
def test_general_projection_vs_oracle(n, zero_a):
    prob = _prob(n, 4, 7 + n, zero_a=zero_a)
    rng = np.random.default_rng(n)
    with _ctx(prob, 1e-6) as s:
        for scale in (0.1, 1.0, 30.0):
            v = rng.standard_normal(n) * scale + 0.5 * (prob.l + prob.u)
            x, m, lam, p, _ = s.project(v)
            x, m = x.cpu().numpy(), m.cpu().numpy().astype(bool)
            x_ref, lam_ref, free_ref = general.projection(prob, v)
            sc = 1.0 + np.abs(v).max()
            assert lam == pytest.approx(lam_ref, rel=1e-10, abs=1e-12 * sc)
            np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-11 * sc)
            # the free set agrees except where t_i sits within rounding of a bound
            t = v - lam_ref * prob.a
            near = (np.abs(t - prob.l) <= 1e-10 * sc) | (np.abs(t - prob.u) <= 1e-10 * sc)
            assert np.all((m == free_ref) | near)
            assert p == int(m.sum())
            assert abs(float(prob.a @ x) - prob.d) <= 1e-9 * sc * (1 + np.abs(prob.a).sum())


def test_general_linesearch_trial_vs_oracle():
    n = 2000
    prob = _prob(n, 6, 55)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(n) + 0.5 * (prob.l + prob.u)
    t = rng.standard_normal(n)
    _, lam, _ = general.projection(prob, u)
    alpha, sigma = 0.5, 2.0
    with _ctx(prob, 1e-6) as s:
        lam_a, dh = s.linesearch_trial(u, t, lam, alpha, sigma)
    u_a = u - alpha * sigma * t
    _, lam_a_ref, _ = general.projection(prob, u_a)
    assert lam_a == pytest.approx(lam_a_ref, rel=1e-10, abs=1e-12)
    tt = u - lam * prob.a
    dt = (u_a - u) - (lam_a_ref - lam) * prob.a
    dh_ref = float(np.sum(general.h_increment(tt, dt, prob.l, prob.u))) + (lam_a_ref - lam) * prob.d
    assert dh == pytest.approx(dh_ref, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("n,q,seed,zero_a", [(4000, 30, 1, 0), (3001, 12, 2, 25), (1500, 200, 3, 0)])
def test_general_vs_oracle(n, q, seed, zero_a):
    prob = _prob(n, q, 900 + seed, zero_a=zero_a)
    ref = general.solve(prob, tol=1e-8)
    assert ref.status == "OK", (ref.status, ref.rkkt)
    with _ctx(prob, 1e-6) as s:
        x, w, info = s.solve()
    x = x.cpu().numpy()
    assert info["status_name"] == "OK"
    R = general.rkkt(prob, x)
    assert R <= 1e-6 * 1.0001
    assert abs(info["rkkt"] - R) <= 1e-3 * R + 1e-12
    np.testing.assert_allclose(w.cpu().numpy(), general.btmul(prob.B, x), rtol=0,
                               atol=1e-10 * (1 + np.abs(x).max() * np.abs(prob.B).sum(0).max()))
    f = general.objective(prob, x)
    rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
    print(f"n={n} q={q}: tol 1e-6 R_KKT {R:.2e}, relative objective error {rel:.2e}")
    if rel > 1e-8:
        with _ctx(prob, 1e-8) as s:
            x, w, info = s.solve()
        x = x.cpu().numpy()
        assert general.rkkt(prob, x) <= 1e-8 * 1.0001
        f = general.objective(prob, x)
        rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
    assert rel <= 1e-8
    assert np.isnan(info["gap"])


def test_csvc_written_as_general():
    X, y = synth.dense_two_gaussians(n=1500, q=10, shift=0.3, seed=12)
    C = 0.7
    prob = general.csvc_problem(X, y, C)
    from paper_1910_01312_amd.solver import Solver
    with _ctx(prob, 1e-8) as s:
        xg, _, ig = s.solve()
    with Solver(X, y, C, tol=1e-8) as s:
        xc, _, ic = s.solve()
    fg = ssnal.dual_objective(X, y, xg.cpu().numpy())
    fc = ssnal.dual_objective(X, y, xc.cpu().numpy())
    assert ig["status_name"] == "OK" and ic["status_name"] == "OK"
    assert abs(fg - fc) <= 1e-8 * max(1.0, abs(fc))
    # the same steps: the multiplier of a^T x = 0 is the C-SVC bias
    assert ig["b"] == pytest.approx(ic["b"], rel=1e-6, abs=1e-8)
