"""The eps-SVR dual (Section 1, eq. Def_Dual_of_SVR_Problem), an instance of
the unified problem (P) with B = [X; -X], c = [eps e + y; eps e - y],
a = [e; -e], solved on the GPU (ssnalm_create_svr) against the general-form
oracle (oracle/general.py) (GPU only).

  * tiny instances: the 2n-variable QP by 3^(2n) enumeration of its active
    sets (Q = B B^T explicit);
  * the bars of the C-SVC tests on the same problem: R_KKT <= 1e-6 as the
    oracle computes it from the returned [x; z], and the objective within
    1e-8 of the oracle's reference (solved to 1e-8) on one solution;
  * the primal side: w = X^T (z - x), the returned bias, and the reported
    duality gap equal to the oracle's eps-insensitive primal at that (w, b);
    x_i z_i = 0 at the solution (eps > 0);
  * eps above every |y_i| gives x = z = 0.
Sizes cover one partial row group up to several hundred 64-row groups.
"""
import numpy as np
import pytest

import synth
from oracle import bruteforce, general

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _svr(X, yr, C, eps, tol, **kw):
    from paper_1910_01312_amd.solver import SVR
    with SVR(X, yr, C, eps, tol, **kw) as s:
        xz, w, info = s.solve()
    return xz.cpu().numpy(), w.cpu().numpy(), info


@pytest.mark.parametrize("seed", range(3))
def test_svr_tiny_vs_enumeration(seed):
    n, q = 4, 2 + seed % 2
    X, yr = synth.tiny_regression(n, q, seed=300 + seed)
    C, eps = [0.5, 1.0, 3.0][seed], 0.1
    prob = general.svr_problem(X, yr, C, eps)
    Q = prob.B @ prob.B.T
    f_star, _ = bruteforce.general_qp_by_enumeration(Q, prob.c, prob.a, prob.d, prob.l, prob.u)
    xz, w, info = _svr(X, yr, C, eps, 1e-10)
    assert info["status_name"] == "OK"
    f = general.objective(prob, xz)
    assert f == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
    assert info["obj"] == pytest.approx(f, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("n,q,C,eps,dtype", [(5000, 20, 1.0, 0.1, np.float64),
                                             (3001, 8, 10.0, 0.05, np.float64),
                                             (4177, 8, 0.5, 0.2, np.float32),
                                             (2000, 160, 1.0, 0.1, np.float64)])
def test_svr_vs_oracle(n, q, C, eps, dtype):
    X, yr = synth.tiny_regression(n, q, seed=n + q)
    Xs = X.astype(dtype)
    Xr = Xs.astype(np.float64)
    prob = general.svr_problem(Xr, yr, C, eps)
    ref = general.solve(prob, tol=1e-8)
    assert ref.status == "OK", (ref.status, ref.rkkt)
    xz, w, info = _svr(Xs, yr, C, eps, 1e-6)
    assert info["status_name"] == "OK"
    assert xz.shape == (2 * n,)
    assert np.all(xz >= 0.0) and np.all(xz <= C)
    x, z = xz[:n], xz[n:]
    R = general.rkkt(prob, xz)
    assert R <= 1e-6 * 1.0001
    assert abs(info["rkkt"] - R) <= 1e-3 * R + 1e-12
    w_ref = general.svr_weights(Xr, x, z)
    np.testing.assert_allclose(w, w_ref, rtol=0, atol=1e-10 * (1 + np.abs(w_ref).max()))
    # the reported gap is the oracle's primal at the reported (w, b)
    P = general.svr_primal(Xr, yr, C, eps, w_ref, info["b"])
    f = general.objective(prob, xz)
    assert info["obj"] == pytest.approx(f, rel=1e-9, abs=1e-9)
    gap = (P + f) / (1 + abs(P) + abs(f))
    assert info["gap"] == pytest.approx(gap, rel=1e-6, abs=1e-12)
    assert -1e-12 <= gap <= 1e-5
    rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
    print(f"n={n} q={q}: tol 1e-6 R_KKT {R:.2e}, relative objective error {rel:.2e}")
    if rel > 1e-8:
        xz, w, info = _svr(Xs, yr, C, eps, 1e-8)
        R = general.rkkt(prob, xz)
        assert R <= 1e-8 * 1.0001
        f = general.objective(prob, xz)
        rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
        x, z = xz[:n], xz[n:]
    assert rel <= 1e-8
    assert np.max(np.minimum(x, z)) <= 1e-6 * C


def test_svr_eps_above_targets_gives_zero():
    X, yr = synth.tiny_regression(300, 3, seed=5)
    eps = float(np.max(np.abs(yr))) + 0.1
    xz, w, info = _svr(X, yr, 1.0, eps, 1e-12)
    assert info["status_name"] == "OK" and info["iters_outer"] == 1
    assert np.all(xz == 0.0)


def test_svr_rejects_unsupported():
    from paper_1910_01312_amd._lib import SsnalmError
    X, yr = synth.tiny_regression(50, 3, seed=6)
    with pytest.raises(SsnalmError):
        _svr(X, yr, 1.0, -0.1, 1e-6)
    with pytest.raises(SsnalmError):
        _svr(X, yr, 1.0, 0.1, 1e-6, newton="pcg")
