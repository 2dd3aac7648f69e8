"""Batched solve (ssnalm_solve_batch) against the CPU oracle, per problem
(GPU only).

Every problem of a batch must meet the same bars as a single solve: status
OK, feasibility, R_KKT <= tol recomputed by the oracle on the returned x, w =
A^T x, and |f - f*| / max(1, |f*|) <= 1e-8 against an oracle reference solved
to R_KKT <= 1e-8 (the batch is re-run at tol 1e-8 for the objective when the
1e-6 stop leaves it outside).  Batches mix sizes (ragged tails of the
1024-row work items, n below one row group), C values over the log grid of
the batched workload, and a single-class problem.
"""
import numpy as np
import pytest

import synth
from oracle import ssnal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(problems, **kw):
    from paper_1910_01312_amd.solver import solve_batch
    out = solve_batch(problems, **kw)
    return [(x.cpu().numpy(), w.cpu().numpy(), info) for x, w, info in out]


def _family(count, q, n_lo, n_hi, seed, dtype=np.float32):
    rng = np.random.default_rng(seed)
    probs = []
    for k in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        C = 10.0 ** (-3.0 + 5.0 * k / max(count - 1, 1))
        X, y = synth.mixture_problem(n, q=q, seed=seed * 100 + k)
        probs.append((X.astype(dtype), y, C))
    return probs


def _check_one(Xr, y, C, x, w, info, tol):
    assert info["status_name"] == "OK", info
    assert np.all(x >= 0.0) and np.all(x <= C)
    assert abs(float(y.astype(np.float64) @ x)) <= 1e-9 * max(1.0, C * len(x))
    R, _ = ssnal.rkkt(Xr, y, C, x)
    assert R <= tol * 1.0001, (R, info)
    assert abs(info["rkkt"] - R) <= 1e-3 * R + 1e-12
    w_ref = ssnal.atmul(Xr, y, x)
    np.testing.assert_allclose(w, w_ref, rtol=0, atol=1e-10 * (1 + np.abs(w_ref).max()))
    f = ssnal.dual_objective(Xr, y, x)
    assert info["obj"] == pytest.approx(f, rel=1e-9, abs=1e-9)
    # the reported duality gap is the oracle's at the reported bias
    g_at, _, _ = ssnal.duality_gap_at(Xr, y, C, x, info["b"])
    assert info["gap"] == pytest.approx(g_at, rel=1e-6, abs=1e-12), (info["gap"], g_at)
    return f


def _check(X, y, C, x, w, info, tol, rerun=None):
    """Per-problem bars; R_KKT <= tol and the 1e-8 objective bar hold on one
    solution: the tol solve's when its objective meets 1e-8, else the
    tol-1e-8 solve's (rerun() -> (x, w, info))."""
    Xr = X.astype(np.float64)
    f = _check_one(Xr, y, C, x, w, info, tol)
    ref = ssnal.solve(Xr, y, C, tol=1e-8)
    assert ref.status == "OK", (ref.status, ref.rkkt)
    rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
    if rel > 1e-8 and rerun is not None:
        print(f"tol {tol:g}: relative objective error {rel:.2e}; checking the tol-1e-8 solve")
        x2, w2, info2 = rerun()
        f = _check_one(Xr, y, C, x2, w2, info2, 1e-8)
        rel = abs(f - ref.obj) / max(1.0, abs(ref.obj))
    assert rel <= 1e-8, (f, ref.obj, rel)


@pytest.mark.parametrize("q,dtype", [(128, np.float32), (40, np.float64), (19, np.float32)])
def test_batch_vs_oracle(q, dtype):
    """C grid 1e-3..1e2; q = 128 and 40 use the 16-byte vector loads, q = 19
    the scalar ones; n spans 9..3000 (one partial row group up to several
    work items with ragged tails)."""
    probs = _family(7, q, 9, 3000, seed=11 + q, dtype=dtype)
    probs[3] = (probs[3][0][:2047], probs[3][1][:2047], probs[3][2])
    res = _batch(probs, tol=1e-6)
    res8 = None
    for k, ((X, y, C), (x, w, info)) in enumerate(zip(probs, res)):
        def rerun(k=k):
            nonlocal res8
            if res8 is None:
                res8 = _batch(probs, tol=1e-8)
            return res8[k]
        _check(X, y, C, x, w, info, 1e-6, rerun=rerun)


def test_batch_bf16_storage():
    probs = []
    for k in range(4):
        bits, y = synth.dense_bf16_directions(n=1500 + 700 * k, q=64, seed=70 + k)
        probs.append((bits, y, [0.1, 1.0, 10.0, 0.01][k]))
    res = _batch(probs, tol=1e-6, bf16=True)
    res8 = _batch(probs, tol=1e-8, bf16=True)
    for k, ((bits, y, C), (x, w, info)) in enumerate(zip(probs, res)):
        Xr = synth.bf16_bits_to_f32(bits)
        _check(Xr, y, C, x, w, info, 1e-6, rerun=lambda k=k: res8[k])


def test_batch_matches_single_solve():
    """Same problems through ssnalm_solve one at a time: both meet the bar,
    objectives agree to 1e-8, outer iteration counts agree."""
    from paper_1910_01312_amd.solver import solve
    probs = _family(5, 128, 800, 5000, seed=5)
    res = _batch(probs, tol=1e-8)
    for (X, y, C), (x, w, info) in zip(probs, res):
        xs, ws, infs = solve(X, y, C, tol=1e-8)
        xs = xs.cpu().numpy()
        f_b = ssnal.dual_objective(X.astype(np.float64), y, x)
        f_s = ssnal.dual_objective(X.astype(np.float64), y, xs)
        assert abs(f_b - f_s) <= 1e-8 * max(1.0, abs(f_s))
        assert info["status_name"] == "OK" and infs["status_name"] == "OK"
        assert abs(info["iters_outer"] - infs["iters_outer"]) <= 1


def test_batch_graphs_autotune_do_not_change_results():
    """Graph replay vs eager launches and tuned vs default launch shapes
    change only the schedule: results are bitwise equal, also run to run."""
    probs = _family(6, 128, 100, 6000, seed=9)
    a = _batch(probs, tol=1e-6)
    b = _batch(probs, tol=1e-6, batch_graphs=0)
    c = _batch(probs, tol=1e-6, autotune=0)
    d = _batch(probs, tol=1e-6)
    for ra, rb, rc, rd in zip(a, b, c, d):
        np.testing.assert_array_equal(ra[0], rb[0])
        np.testing.assert_array_equal(ra[0], rc[0])
        np.testing.assert_array_equal(ra[0], rd[0])
        assert ra[2]["iters_inner"] == rb[2]["iters_inner"] == rc[2]["iters_inner"]


def test_batch_single_class_and_tiny():
    rng = np.random.default_rng(3)
    X1 = rng.standard_normal((30, 8)).astype(np.float32)
    y1 = np.ones(30, np.int8)                         # one class: x = 0
    X2, y2 = synth.tiny_problem(7, 8, 501)
    X3, y3 = synth.mixture_problem(1, q=8, seed=4)    # n = 1
    X4, y4 = synth.mixture_problem(2000, q=8, seed=5)
    probs = [(X1, y1, 1.0), (X2.astype(np.float32), y2, 2.0), (X3, y3, 1.0), (X4, y4, 0.5)]
    res = _batch(probs, tol=1e-9)
    assert np.all(res[0][0] == 0.0)
    assert np.all(res[2][0] == 0.0)
    from oracle import bruteforce
    f_star, _, _ = bruteforce.qp_by_enumeration(X2.astype(np.float32).astype(np.float64), y2, 2.0)
    f = ssnal.dual_objective(X2.astype(np.float32).astype(np.float64), y2, res[1][0])
    assert abs(f - f_star) <= 1e-8 * max(1.0, abs(f_star))
    _check(X4, y4, 0.5, res[3][0], res[3][1], res[3][2], 1e-9)


def test_batch_bad_arguments():
    from paper_1910_01312_amd._lib import SsnalmError
    rng = np.random.default_rng(0)
    y = np.where(rng.random(50) < 0.5, 1, -1).astype(np.int8)
    A = rng.standard_normal((50, 8))
    with pytest.raises(SsnalmError):        # q differs
        _batch([(A, y, 1.0), (rng.standard_normal((50, 9)), y, 1.0)])
    with pytest.raises(SsnalmError):        # dtype differs
        _batch([(A, y, 1.0), (A.astype(np.float32), y, 1.0)])
    with pytest.raises(SsnalmError):        # q above the batched limit
        _batch([(rng.standard_normal((50, 129)), y, 1.0)])
    with pytest.raises(SsnalmError):        # bad label
        yb = y.copy()
        yb[3] = 0
        _batch([(A, yb, 1.0)])
    with pytest.raises(SsnalmError):        # C <= 0
        _batch([(A, y, 0.0)])
    with pytest.raises(SsnalmError):        # PCG is not a batched Newton mode
        _batch([(A, y, 1.0)], newton="pcg")
