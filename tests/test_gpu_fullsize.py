"""The workloads at their full sizes, in the launch configurations the
benchmark times (GPU only):
  * sparse text-like CSR, n = 500,000, q = 100,000, ~60 nonzeros per row,
    Zipf(1.1) columns (A^T z over the row-blocked CSC copy, one row block per
    XCD);
  * dense bf16, n = 1,000,000, q = 512, mixed precision, C in {0.1, 1};
  * a batch whose largest problem (n = 120,000, C = 10) has |J| = n in its
    first Newton step, past the batched Gram product's per-problem cap.

Checked against the oracle's definitions (FP64 products on the host, a
library primitive) and against oracle reference solves stored by
tests/golden/make_refs.py (inputs regenerated here and matched by checksum):
  * every element of A v and A^T z within 1e-12 relative to |X||v|, |X|^T|z|;
  * R_KKT <= 1e-6 (eq. Def_Rkkt) as the oracle computes it from the returned
    x, agreeing with the library's own R_KKT, feasibility, w = A^T x, the
    duality gap at the returned bias;
  * where a reference is stored (the dense C = 0.1 one is not yet: its oracle
    solve runs for many hours), |f - f*| / max(1, |f*|) <= 1e-8 with f* the
    oracle's, on the same
    solution as the R_KKT bar: the tol-1e-6 solve when it meets 1e-8, else
    a tol-1e-8 solve (the tol-1e-6 error is printed).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import ssnal

REFS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_refs.json")


def _refs():
    with open(REFS) as f:
        return json.load(f)


def _objective_bar(f6, f_star, rerun):
    """Both bars on one solution; rerun() -> (f, R) of a tol-1e-8 solve."""
    rel = abs(f6 - f_star) / max(1.0, abs(f_star))
    print(f"tol 1e-06: relative objective error {rel:.2e}")
    if rel > 1e-8:
        f8, R8 = rerun()
        assert R8 <= 1e-8 * 1.0001, R8
        rel = abs(f8 - f_star) / max(1.0, abs(f_star))
        print(f"tol 1e-08: R_KKT {R8:.2e}, relative objective error {rel:.2e}")
    assert rel <= 1e-8, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, Q = 500_000, 100_000


@pytest.fixture(scope="module")
def workload():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01312_amd import _lib
    _lib.load()
    vals, ci, rp, y = synth.sparse_text()
    assert rp.size - 1 == N
    X = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(N, Q))
    return vals, ci, rp, y, X


@pytest.fixture(scope="module")
def solver(workload):
    from paper_1910_01312_amd.solver import Solver
    vals, ci, rp, y, _ = workload
    s = Solver(csr=(vals, ci, rp, N, Q), y=y, C_=1.0, tol=1e-6)
    yield s
    s.close()


def test_fullsize_sparse_matvecs(workload, solver):
    _, _, _, y, X = workload
    rng = np.random.default_rng(123)
    v = rng.standard_normal(Q)
    z = rng.standard_normal(N)
    t = solver.amul(v).cpu().numpy()
    r = solver.atmul(z).cpu().numpy()
    absX = abs(X)
    assert np.all(np.abs(t - ssnal.amul(X, y, v)) <= 1e-12 * (absX @ np.abs(v)) + 1e-300)
    assert np.all(np.abs(r - ssnal.atmul(X, y, z)) <= 1e-12 * (absX.T @ np.abs(z)) + 1e-300)


def test_fullsize_sparse_solve(workload, solver):
    vals, ci, rp, y, X = workload
    ref = _refs()["sparse_text_full"]
    assert ref["status"] == "OK"
    assert float(np.sum(vals, dtype=np.float64)) == ref["inputs"]["sum_x"]
    assert int(np.sum(ci, dtype=np.int64)) == ref["inputs"]["sum_col"]
    x, w, info = solver.solve()
    assert info["status_name"] == "OK"
    xh = x.cpu().numpy()
    R, _ = ssnal.rkkt(X, y, 1.0, xh)
    assert R <= 1e-6
    assert abs(R - info["rkkt"]) <= 1e-3 * R + 1e-12
    assert np.all(xh >= 0.0) and np.all(xh <= 1.0)
    w_ref = ssnal.atmul(X, y, xh)
    absX = abs(X)
    assert np.all(np.abs(w.cpu().numpy() - w_ref) <= 1e-12 * (absX.T @ np.abs(xh)) + 1e-300)
    g_at, _, _ = ssnal.duality_gap_at(X, y, 1.0, xh, info["b"])
    assert info["gap"] == pytest.approx(g_at, rel=1e-6, abs=1e-12)

    def rerun():
        from paper_1910_01312_amd.solver import Solver
        with Solver(csr=(vals, ci, rp, N, Q), y=y, C_=1.0, tol=1e-8) as s8:
            x8, _, i8 = s8.solve()
        assert i8["status_name"] == "OK"
        x8 = x8.cpu().numpy()
        return ssnal.dual_objective(X, y, x8), ssnal.rkkt(X, y, 1.0, x8)[0]

    _objective_bar(ssnal.dual_objective(X, y, xh), ref["f_star"], rerun)


# ---------------------------------------------------------------- dense bf16

@pytest.fixture(scope="module")
def dense_bf16():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bits, y = synth.dense_bf16_directions()
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    return bits, y, Xr


def _bf16_solve(dense_bf16, C, tol):
    from paper_1910_01312_amd.solver import Solver
    bits, y, _ = dense_bf16
    bd = torch.from_numpy(bits.view(np.int16)).cuda()
    with Solver(bd, y, C, tol=tol, bf16=True, precision="mixed") as s:
        x, w, info = s.solve()
    assert info["status_name"] == "OK"
    return x.cpu().numpy(), w.cpu().numpy(), info


@pytest.mark.parametrize("C", [0.1, 1.0])
def test_fullsize_dense_bf16_mixed_kkt(dense_bf16, C):
    """The checks that need no stored reference: R_KKT as the oracle computes
    it from the returned x (and agreeing with the library's), feasibility,
    w = A^T x element by element, and the library's duality gap against the
    oracle's at the returned bias."""
    _, y, Xr = dense_bf16
    xh, w, info = _bf16_solve(dense_bf16, C, 1e-6)
    assert np.all(xh >= 0.0) and np.all(xh <= C)
    R, _ = ssnal.rkkt(Xr, y, C, xh)
    assert R <= 1e-6 * 1.0001
    assert abs(R - info["rkkt"]) <= 1e-3 * R + 1e-12
    w_ref = ssnal.atmul(Xr, y, xh)
    assert np.all(np.abs(w - w_ref) <= 1e-12 * (np.abs(Xr).T @ xh) + 1e-300)
    g_at, _, _ = ssnal.duality_gap_at(Xr, y, C, xh, info["b"])
    assert info["gap"] == pytest.approx(g_at, rel=1e-6, abs=1e-12)


@pytest.mark.parametrize("C", [0.1, 1.0])
def test_fullsize_dense_bf16_mixed_objective(dense_bf16, C):
    """The objective against the oracle's f* (tol-1e-8 oracle solve stored by
    tests/golden/make_refs.py)."""
    _, y, Xr = dense_bf16
    name = "dense_bf16_full_C" + ("0.1" if C == 0.1 else "1")
    refs = _refs()
    if name not in refs:
        # the oracle's tol-1e-8 solve of n = 10^6, q = 512 runs for hours on
        # the CPU; the reference is added by tests/golden/make_refs.py
        pytest.skip(f"oracle reference {name} not computed yet (tests/golden/make_refs.py {name})")
    ref = refs[name]
    assert ref["status"] == "OK" and ref["C"] == C
    assert float(np.sum(Xr, dtype=np.float64)) == ref["inputs"]["sum_x"]
    xh, _, _ = _bf16_solve(dense_bf16, C, 1e-6)

    def rerun():
        x8, _, _ = _bf16_solve(dense_bf16, C, 1e-8)
        return ssnal.dual_objective(Xr, y, x8), ssnal.rkkt(Xr, y, C, x8)[0]

    _objective_bar(ssnal.dual_objective(Xr, y, xh), ref["f_star"], rerun)


# ---------------------------------------------------------------- batched

def test_fullsize_batch_gram_cap():
    """A batch mixing n = 120,000 (C = 10: |J| = n at the first Newton step,
    so its Gram product runs capped at 32 work items) with n = 1000 and
    n = 5003: every problem against its stored oracle reference."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01312_amd.solver import solve_batch
    refs = _refs()["batch_gram_cap"]
    probs = []
    for r in refs:
        X, y = synth.mixture_problem(r["n"], q=128, seed=r["seed"])
        assert float(np.sum(X, dtype=np.float64)) == r["inputs"]["sum_x"]
        probs.append((X, y, r["C"]))
    res6 = solve_batch(probs, tol=1e-6)
    res8 = None
    for k, ((X, y, C), (x, w, info), r) in enumerate(zip(probs, res6, refs)):
        assert info["status_name"] == "OK", info
        Xr = X.astype(np.float64)
        xh = x.cpu().numpy()
        R, _ = ssnal.rkkt(Xr, y, C, xh)
        assert R <= 1e-6 * 1.0001
        assert np.all(xh >= 0.0) and np.all(xh <= C)
        w_ref = ssnal.atmul(Xr, y, xh)
        np.testing.assert_allclose(w.cpu().numpy(), w_ref, rtol=0,
                                   atol=1e-10 * (1 + np.abs(w_ref).max()))

        def rerun(k=k, Xr=Xr, y=y, C=C):
            nonlocal res8
            if res8 is None:
                res8 = solve_batch(probs, tol=1e-8)
            x8 = res8[k][0].cpu().numpy()
            assert res8[k][2]["status_name"] == "OK"
            return ssnal.dual_objective(Xr, y, x8), ssnal.rkkt(Xr, y, C, x8)[0]

        _objective_bar(ssnal.dual_objective(Xr, y, xh), r["f_star"], rerun)
