"""The low-rank (Woodbury) update of the dense Newton step (GPU only): a step
at the sigma of the stored Cholesky factor whose free set J differs from the
factor's in at most 94 rows is solved from that factor, M = M0 + U S U^T
(U: the changed rows and the two centring vectors).  Checked against the
oracle's fresh Cholesky step (`ssnal.newton_qspace`) and its low-rank step
(`ssnal.newton_lowrank`) for 0 to 94 changed rows and past the rank cap, in
fp64 and in mixed precision (where the refinement then uses the updated
operator), and through full solves against the oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import ssnal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(X, y, C, **kw):
    from paper_1910_01312_amd.solver import Solver
    return Solver(X, y, C, **kw)


def _masks(n, nchg, seed):
    rng = np.random.default_rng(seed)
    f0 = rng.random(n) < 0.4
    f1 = f0.copy()
    idx = rng.choice(n, size=nchg, replace=False)
    f1[idx] = ~f1[idx]
    return f0, f1


def _m0_factor(X, free, sigma):
    XJ = X[np.flatnonzero(free)]
    s = XJ.sum(axis=0)
    M0 = np.eye(X.shape[1]) + sigma * (XJ.T @ XJ - np.outer(s, s) / free.sum())
    return sla.cho_factor(M0, lower=True)


@pytest.mark.parametrize("q,nchg", [(160, 0), (160, 5), (512, 60), (200, 62), (200, 63), (200, 94),
                                    (200, 95)])
def test_lowrank_step_fp64(q, nchg):
    """Second op_newton call at the same sigma: the update of the first
    call's factor (nchg <= 94) or a new factorisation (95: past the cap),
    either way the oracle's direction.  62 and 63 changed rows give a
    capacitance matrix of order 64 and 65, where its factorisation and
    solves start using a second entry per lane."""
    X, y = synth.dense_two_gaussians(n=3000, q=q, seed=12)
    sigma = 7.0
    f0, f1 = _masks(X.shape[0], nchg, 3 + q)
    rng = np.random.default_rng(q)
    g0, g1 = rng.standard_normal(q), rng.standard_normal(q)
    d_ref = ssnal.newton_qspace(X, f1, g1, sigma)
    d_lr = ssnal.newton_lowrank(X, f1, g1, sigma, f0, _m0_factor(X, f0, sigma))
    assert np.linalg.norm(d_lr - d_ref) <= 1e-9 * (1 + np.linalg.norm(d_ref))
    with _solver(X, y, 1.0, newton="chol", lowrank=2) as s:
        s.newton(f0.astype(np.uint8), g0, sigma)
        d, _ = s.newton(f1.astype(np.uint8), g1, sigma)
    d = d.cpu().numpy()
    assert np.linalg.norm(d - d_ref) <= 1e-9 * (1 + np.linalg.norm(d_ref))
    assert np.linalg.norm(d - d_lr) <= 1e-9 * (1 + np.linalg.norm(d_ref))


def test_lowrank_step_mixed():
    """bf16 Gram factor of the first step, updated for the second; the
    refinement with the exact operator reaches the fp64 direction."""
    bits, y = synth.dense_bf16_directions(n=6000, q=256, seed=31)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    sigma = 40.0
    f0, f1 = _masks(6000, 20, 9)
    rng = np.random.default_rng(5)
    g0, g1 = rng.standard_normal(256), rng.standard_normal(256)
    d_ref = ssnal.newton_qspace(Xr, f1, g1, sigma)
    tol = 1e-10 * np.linalg.norm(g1)
    with _solver(bits, y, 1.0, bf16=True, newton="chol", precision="mixed") as s:
        s.newton(f0.astype(np.uint8), g0, sigma, cg_tol=tol)
        d, its = s.newton(f1.astype(np.uint8), g1, sigma, cg_tol=tol)
    d = d.cpu().numpy()
    assert its <= 6
    assert np.linalg.norm(d - d_ref) <= 1e-8 * (1 + np.linalg.norm(d_ref))


def _check(X, y, C, x, info, ref, tol):
    assert info["status_name"] == "OK"
    R, _ = ssnal.rkkt(X, y, C, x)
    assert R <= tol * 1.0001
    f = ssnal.dual_objective(X, y, x)
    assert abs(f - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))


def test_lowrank_solve_fp64():
    """fp64 dense q = 200 with the updates on and off: the oracle's counts and
    optimum either way, and most same-sigma steps taken by the update."""
    X, y = synth.dense_two_gaussians(n=8000, q=200, seed=21)
    C, tol = 1.0, 1e-8
    ref = ssnal.solve(X, y, C, tol=tol)
    assert ref.status == "OK"
    out = {}
    for lr in (0, 2):
        with _solver(X, y, C, tol=tol, lowrank=lr) as s:
            x, _, info = s.solve()
        x = x.cpu().numpy()
        _check(X, y, C, x, info, ref, tol)
        assert (info["iters_outer"], info["iters_inner"]) == (ref.outer, ref.inner)
        out[lr] = info
    assert out[0]["lowrank_steps"] == 0
    assert out[2]["lowrank_steps"] > 0


@pytest.mark.parametrize("C", [0.1, 1.0])
def test_lowrank_solve_mixed(C):
    """Mixed precision (the default enables the updates): the fp64 oracle's
    optimum on the same bf16 data, with updates taken."""
    bits, y = synth.dense_bf16_directions(n=8000, q=256, seed=41)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    tol = 1e-8
    ref = ssnal.solve(Xr, y, C, tol=tol)
    assert ref.status == "OK"
    with _solver(bits, y, C, tol=tol, bf16=True, precision="mixed") as s:
        x, _, info = s.solve()
    _check(Xr, y, C, x.cpu().numpy(), info, ref, tol)
    assert info["lowrank_steps"] > 0
