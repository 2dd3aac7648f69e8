"""End-to-end parity of the GPU SSsNAL solve against the CPU oracle (GPU only).

x* is generally not unique (rank Q <= q < n), so the comparison uses what is
unique: the optimal value f*, the primal weights w* = A^T x*, R_KKT
recomputed by the oracle on the GPU's x, feasibility, and b when p > 0.
Bars: R_KKT <= 1e-6 and |f - f*| / max(1, |f*|) <= 1e-8 against an oracle
reference that reached R_KKT <= 1e-8 (status OK asserted).  Both bars are
checked on ONE solution: the tol-1e-6 solve when its objective already meets
1e-8, else a tol-1e-8 solve (R_KKT <= 1e-8 <= 1e-6); the tol-1e-6 solve's
objective error is printed either way.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import bruteforce, ssnal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(*a, **k):
    from paper_1910_01312_amd.solver import Solver
    tol = k.pop("tol", 1e-6)
    x0 = k.pop("x0", None)
    with Solver(*a, tol=tol, **k) as s:
        x, w, info = s.solve(x0)
        return x.cpu().numpy(), w.cpu().numpy(), info


def _ref(X, y, C, **kw):
    """Oracle reference solved to R_KKT <= 1e-8, which it must reach (status
    OK).  In fp64 the method's attainable R_KKT floor at large sigma is a few
    1e-9 on some of these problems, so 1e-10 is not reachable there; at 1e-8
    the objective agrees with the best attainable one to ~1e-11 relative,
    three orders inside the 1e-8 objective bar."""
    r = ssnal.solve(X, y, C, tol=1e-8, **kw)
    assert r.status == "OK", (r.status, r.rkkt, r.outer)
    return r


def _check_one(X, y, C, x, w, info, tol):
    """R_KKT (recomputed by the oracle), feasibility and w = A^T x of one
    returned solution."""
    assert info["status_name"] == "OK", info
    assert np.all(x >= 0.0) and np.all(x <= C)
    R, _ = ssnal.rkkt(X, y, C, x)
    assert R <= tol * 1.0001, (R, info)
    assert abs(info["rkkt"] - R) <= 1e-3 * R + 1e-12
    w_ref = ssnal.atmul(X, y, x)
    np.testing.assert_allclose(w, w_ref, rtol=0, atol=1e-10 * (1 + np.abs(w_ref).max()))
    return R


def _check_solution(X, y, C, x, w, info, ref, tol=1e-6, rerun=None):
    """Both bars on one solution (see the module docstring)."""
    R = _check_one(X, y, C, x, w, info, tol)
    f = ssnal.dual_objective(X, y, x)
    rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
    print(f"tol {tol:g}: R_KKT {R:.2e}, relative objective error {rel:.2e}")
    if rel > 1e-8 and rerun is not None:
        x2, w2, info2 = rerun()
        R2 = _check_one(X, y, C, x2, w2, info2, 1e-8)
        f = ssnal.dual_objective(X, y, x2)
        rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
        print(f"tol 1e-08: R_KKT {R2:.2e}, relative objective error {rel:.2e}")
    assert rel <= 1e-8, (f, ref.obj, rel)
    return R


def test_c1_dense_fp64():
    X, y = synth.dense_two_gaussians()
    ref = _ref(X, y, 1.0)
    x, w, info = _solve(X, y, 1.0, tol=1e-6)
    _check_solution(X, y, 1.0, x, w, info, ref,
                    rerun=lambda: _solve(X, y, 1.0, tol=1e-8))
    # same number of ALM iterations as the oracle at the same tolerance
    r6 = ssnal.solve(X, y, 1.0, tol=1e-6)
    assert info["iters_outer"] == r6.outer
    np.testing.assert_allclose(w, ref.w, atol=1e-4)


@pytest.mark.parametrize("C", [0.01, 1.0, 100.0])
def test_dense_small_various_C(C):
    X, y = synth.dense_two_gaussians(n=600, q=12, shift=0.3, seed=77)
    ref = _ref(X, y, C)
    x, w, info = _solve(X, y, C, tol=1e-6)
    _check_solution(X, y, C, x, w, info, ref, rerun=lambda: _solve(X, y, C, tol=1e-8))


@pytest.mark.parametrize("seed", range(4))
def test_tiny_vs_enumeration(seed):
    X, y = synth.tiny_problem(7, 2 + seed % 2, 500 + seed)
    C = [0.5, 2.0][seed % 2]
    f_star, _, _ = bruteforce.qp_by_enumeration(X, y, C)
    x, w, info = _solve(X, y, C, tol=1e-9)
    f = ssnal.dual_objective(X, y, x)
    assert abs(f - f_star) <= 1e-8 * max(1.0, abs(f_star))


def test_golden_qp(golden):
    for case in golden["qp_cases"]:
        X = np.array(case["X"], dtype=np.float64)
        y = np.array(case["y"], dtype=np.int8)
        x, w, info = _solve(X, y, case["C"], tol=1e-10)
        assert ssnal.dual_objective(X, y, x) == pytest.approx(case["f_star"], abs=1e-9)
        np.testing.assert_allclose(w, case["w_star"], atol=1e-7)


def test_single_class():
    X = np.random.default_rng(0).standard_normal((50, 4))
    y = np.ones(50, np.int8)
    x, w, info = _solve(X, y, 1.0)
    assert np.all(x == 0.0)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_dense_low_precision_storage(dtype):
    X, y = synth.mixture_problem(4000, q=64, seed=3)
    if dtype == "bf16":
        Xs = synth.to_bf16_bits(X)
        Xr = synth.bf16_bits_to_f32(Xs).astype(np.float64)
        kw = {"bf16": True}
    else:
        Xs, Xr, kw = X, X.astype(np.float64), {}
    ref = _ref(Xr, y, 0.1)
    x, w, info = _solve(Xs, y, 0.1, tol=1e-6, **kw)
    _check_solution(Xr, y, 0.1, x, w, info, ref,
                    rerun=lambda: _solve(Xs, y, 0.1, tol=1e-8, **kw))


def test_csr_pcg_solve():
    vals, ci, rp, y = synth.sparse_text(n=20000, q=4000, seed=21)
    n, q = rp.size - 1, 4000
    Xr = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(n, q))
    ref = _ref(Xr, y, 1.0, newton="pcg", max_cg=2000)
    x, w, info = _solve(csr=(vals, ci, rp, n, q), y=y, C_=1.0, tol=1e-6)
    _check_solution(Xr, y, 1.0, x, w, info, ref,
                    rerun=lambda: _solve(csr=(vals, ci, rp, n, q), y=y, C_=1.0, tol=1e-8))


def test_warm_start_from_solution():
    X, y = synth.dense_two_gaussians(n=1000, q=20, seed=4)
    ref = _ref(X, y, 1.0)
    x, w, info = _solve(X, y, 1.0, tol=1e-6, x0=ref.x)
    assert info["status_name"] == "OK"
    assert info["iters_outer"] <= 2


def test_bad_arguments():
    from paper_1910_01312_amd._lib import SsnalmError
    from paper_1910_01312_amd.solver import Solver
    X = np.zeros((4, 2))
    with pytest.raises(SsnalmError):
        Solver(X, np.array([1, -1, 2, 1], np.int8), 1.0)
    with pytest.raises(SsnalmError):
        Solver(X, np.array([1, -1, 1, 1], np.int8), -1.0)
    Xn = np.array([[1.0, np.nan], [0, 1], [1, 1], [2, 0]])
    with pytest.raises(SsnalmError):
        Solver(Xn, np.array([1, -1, 1, 1], np.int8), 1.0, check_finite=1)


def test_deterministic_solve():
    X, y = synth.dense_two_gaussians(n=3000, q=30, seed=8)
    x1, w1, i1 = _solve(X, y, 1.0)
    x2, w2, i2 = _solve(X, y, 1.0)
    np.testing.assert_array_equal(x1, x2)
    assert i1["iters_inner"] == i2["iters_inner"]


@pytest.mark.parametrize("C", [0.1, 1.0])
def test_mixed_precision_bf16_solve(C):
    """Mixed precision (bf16 X, bf16 MFMA Gram, fp64 Cholesky + refinement,
    fp64 iterates): same bars as the fp64 path against the fp64 oracle on the
    same bf16 data."""
    bits, y = synth.dense_bf16_directions(n=8000, q=256, seed=41)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    ref = _ref(Xr, y, C)
    x, w, info = _solve(bits, y, C, tol=1e-6, bf16=True, precision="mixed")
    _check_solution(Xr, y, C, x, w, info, ref,
                    rerun=lambda: _solve(bits, y, C, tol=1e-8, bf16=True, precision="mixed"))
    x2, w2, info2 = _solve(bits, y, C, tol=1e-6, bf16=True)       # fp64 Gram
    _check_solution(Xr, y, C, x2, w2, info2, ref,
                    rerun=lambda: _solve(bits, y, C, tol=1e-8, bf16=True))
