"""Host-forced exits and less travelled paths of the GPU solve against the
CPU oracle run with the same options (GPU only).

  * MAXITER (max_outer small): the best x seen is returned, as the oracle's;
  * LINESEARCH_FAIL (alpha = 1 only, Armijo constant 0.9 that a Newton step
    on a locally quadratic psi cannot meet): every inner loop ends in a
    failed line search, as in the oracle;
  * the steepest-descent fallback: with PCG capped at 0 iterations the
    Newton direction is d = 0 (not one of descent), replaced by -grad psi in
    every step on both sides;
  * PCG on dense X (the matrix-free Newton operator) against the oracle's
    Jacobi-preconditioned CG;
  * a mixed precision solve at q = 77 (the bf16 MFMA Gram product for q
    not a multiple of 8; its element-wise check is in test_gpu_ops);
  * the duality gap and the bias b_out against the oracle at the same b;
  * a problem whose arrays are written on a non-blocking side stream;
  * training labels computed by the library against the oracle's.
"""
import numpy as np
import pytest

import synth
from oracle import mlp, ssnal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(X, y, C, tol=1e-6, **kw):
    from paper_1910_01312_amd.solver import Solver
    with Solver(X, y, C, tol=tol, **kw) as s:
        x, w, info = s.solve()
        return x.cpu().numpy(), w.cpu().numpy(), info


def _same_iterate(X, y, C, x, info, ref, rtol=1e-7):
    """The GPU's x is the oracle's x up to rounding: same R_KKT, objective and
    weights (the iterates of both runs follow the same steps)."""
    R, _ = ssnal.rkkt(X, y, C, x)
    assert R == pytest.approx(ref.rkkt, rel=1e-4, abs=1e-12), (R, ref.rkkt)
    assert info["rkkt"] == pytest.approx(R, rel=1e-3, abs=1e-12)
    f = ssnal.dual_objective(X, y, x)
    assert f == pytest.approx(ref.obj, rel=rtol, abs=1e-12), (f, ref.obj)
    np.testing.assert_allclose(ssnal.atmul(X, y, x), ref.w, rtol=0,
                               atol=rtol * (1.0 + np.abs(ref.w).max()) * 100)


def test_maxiter_returns_best_x():
    X, y = synth.dense_two_gaussians(n=800, q=10, shift=0.3, seed=31)
    ref = ssnal.solve(X, y, 1.0, tol=1e-12, max_outer=2)
    assert ref.status == "MAXITER"
    x, w, info = _solve(X, y, 1.0, tol=1e-12, max_outer=2)
    assert info["status_name"] == "MAXITER"
    assert info["iters_outer"] == 2 == ref.outer
    assert info["iters_inner"] == ref.inner
    assert np.all(x >= 0.0) and np.all(x <= 1.0)
    _same_iterate(X, y, 1.0, x, info, ref)


def test_linesearch_fail():
    X, y = synth.dense_two_gaussians(n=800, q=10, shift=0.3, seed=32)
    opts = dict(max_outer=3, max_backtracks=0, mu=0.9)
    ref = ssnal.solve(X, y, 1.0, tol=1e-12, **opts)
    assert ref.ls_fail >= 1
    x, w, info = _solve(X, y, 1.0, tol=1e-12, **opts)
    assert info["ls_fail"] == ref.ls_fail
    assert info["iters_inner"] == ref.inner
    want = "LINESEARCH_FAIL" if ref.ls_fail >= ref.outer else ref.status
    assert info["status_name"] == want
    _same_iterate(X, y, 1.0, x, info, ref)


def test_gradient_fallback_when_pcg_is_capped():
    X, y = synth.dense_two_gaussians(n=600, q=8, shift=0.4, seed=33)
    opts = dict(newton="pcg", max_cg=0, max_outer=3)
    ref = ssnal.solve(X, y, 1.0, tol=1e-12, **opts)
    # every step with J nonempty falls back (a step with J empty is -g already)
    assert 0 < ref.grad_steps <= ref.inner
    x, w, info = _solve(X, y, 1.0, tol=1e-12, **opts)
    assert info["grad_steps"] == ref.grad_steps
    assert info["iters_inner"] == ref.inner
    assert info["cg_iters"] == 0
    _same_iterate(X, y, 1.0, x, info, ref, rtol=1e-6)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dense_pcg_solve(dtype):
    X, y = synth.dense_two_gaussians(n=3000, q=40, shift=0.3, seed=34)
    Xs = X.astype(dtype)
    Xr = Xs.astype(np.float64)
    ref8 = ssnal.solve(Xr, y, 1.0, tol=1e-8, newton="pcg")
    assert ref8.status == "OK"
    ref6 = ssnal.solve(Xr, y, 1.0, tol=1e-6, newton="pcg")
    x, w, info = _solve(Xs, y, 1.0, tol=1e-6, newton="pcg")
    assert info["status_name"] == "OK"
    R, _ = ssnal.rkkt(Xr, y, 1.0, x)
    assert R <= 1e-6 * 1.0001
    assert info["iters_outer"] == ref6.outer
    # the same CG (Jacobi, tolerance min(eta, |g|^(1+tau))) on both sides
    assert abs(info["cg_iters"] - ref6.cg_iters) <= max(2, 0.05 * ref6.cg_iters), \
        (info["cg_iters"], ref6.cg_iters)
    x8, w8, info8 = _solve(Xs, y, 1.0, tol=1e-8, newton="pcg")
    R8, _ = ssnal.rkkt(Xr, y, 1.0, x8)
    assert R8 <= 1e-8 * 1.0001
    f = ssnal.dual_objective(Xr, y, x8)
    assert abs(f - ref8.obj) <= 1e-8 * max(1.0, abs(ref8.obj))


def test_mixed_solve_q77():
    bits, y = synth.dense_bf16_directions(n=6000, q=77, seed=77)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    ref = ssnal.solve(Xr, y, 1.0, tol=1e-8)
    assert ref.status == "OK"
    x, w, info = _solve(bits, y, 1.0, tol=1e-8, bf16=True, precision="mixed")
    assert info["status_name"] == "OK"
    R, _ = ssnal.rkkt(Xr, y, 1.0, x)
    assert R <= 1e-8 * 1.0001
    f = ssnal.dual_objective(Xr, y, x)
    assert abs(f - ref.obj) <= 1e-8 * max(1.0, abs(ref.obj))


@pytest.mark.parametrize("C", [0.1, 1.0, 10.0])
def test_gap_and_bias(C):
    X, y = synth.dense_two_gaussians(n=2000, q=20, shift=0.3, seed=35)
    x, w, info = _solve(X, y, C, tol=1e-8)
    assert info["status_name"] == "OK"
    assert info["b_out"] == info["b"]
    _, b_ora = ssnal.rkkt(X, y, C, x)
    assert info["b"] == pytest.approx(b_ora, rel=1e-8, abs=1e-10)
    g_at, P, f = ssnal.duality_gap_at(X, y, C, x, info["b"])
    assert info["gap"] == pytest.approx(g_at, rel=1e-6, abs=1e-13), (info["gap"], g_at)
    g_best, _, _ = ssnal.duality_gap(X, y, C, x)
    assert info["gap"] >= g_best - 1e-12
    assert 0.0 <= g_best and info["gap"] <= 1e-6


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_arrays_written_on_a_side_stream(kind):
    """The problem arrays are produced by kernels queued on a non-blocking
    side stream behind a long product; ssnalm_create (which reads y, and the
    CSR arrays, from the host) must see their final values."""
    from paper_1910_01312_amd.solver import Solver
    dev = torch.device("cuda", torch.cuda.current_device())
    side = torch.cuda.Stream()
    if kind == "dense":
        X, y = synth.dense_two_gaussians(n=3000, q=16, shift=0.4, seed=36)
        Xr = X
    else:
        vals, ci, rp, y = synth.sparse_text(n=6000, q=1500, seed=37)
        import scipy.sparse as sp
        Xr = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(rp.size - 1, 1500))
    ref = ssnal.solve(Xr, y, 1.0, tol=1e-8, **({"newton": "pcg"} if kind == "csr" else {}))
    src_y = torch.from_numpy(y).to(dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        big = torch.ones((4096, 4096), device=dev)
        for _ in range(20):
            big = big @ big * (1.0 / 4096.0)
        yd = torch.zeros_like(src_y)
        yd.copy_(src_y)                               # written after the long product
        if kind == "dense":
            Xd = torch.from_numpy(X).to(dev) * 1.0
            s = Solver(Xd, yd, 1.0, tol=1e-6)
        else:
            v = torch.from_numpy(vals).to(dev) * 1.0
            c = torch.from_numpy(ci).to(dev) + 0
            r = torch.from_numpy(rp).to(dev) + 0
            s = Solver(csr=(v, c, r, rp.size - 1, 1500), y=yd, C_=1.0, tol=1e-6)
        with s:
            x, w, info = s.solve()
        torch.cuda.current_stream().synchronize()
    xh = x.cpu().numpy()
    assert info["status_name"] == "OK"
    R, _ = ssnal.rkkt(Xr, y, 1.0, xh)
    assert R <= 1e-6 * 1.0001
    f = ssnal.dual_objective(Xr, y, xh)
    assert abs(f - ref.obj) <= 1e-6 * max(1.0, abs(ref.obj))


def test_training_labels():
    from paper_1910_01312_amd.solver import Solver
    from paper_1910_01312_amd.warmstart import labels
    X, y = synth.dense_two_gaussians(n=500, q=6, seed=38)
    C = 2.0
    rng = np.random.default_rng(5)
    x = rng.choice([0.0, 1e-9 * C, 0.3 * C, (1 - 1e-9) * C, C, 1e-7 * C], size=500)
    with Solver(X, y, C) as s:
        st, tg = labels(s, torch.from_numpy(x).cuda())
    st_ref, tg_ref = mlp.labels(x, C)
    np.testing.assert_array_equal(st.cpu().numpy(), st_ref)
    np.testing.assert_array_equal(tg.cpu().numpy(), np.asarray(tg_ref, np.float32))


def test_warmstart_rejected_status():
    """A prediction that keeps more than half of the rows is set aside: the
    plain cold solve runs and the call reports WARMSTART_REJECTED."""
    from paper_1910_01312_amd.solver import Solver
    import ctypes as Cc
    from paper_1910_01312_amd import _lib as L
    X, y = synth.mixture_problem(3000, q=32, seed=39)
    out = torch.zeros((3000, 4), dtype=torch.float32, device="cuda")
    out[:, 1] = 1.0                                  # every row "inside": nothing screened
    with Solver(X, y, 0.5, tol=1e-6) as s:
        xd = torch.empty(3000, dtype=torch.float64, device="cuda")
        info, st = L.Info(), L.WsStats()
        status = s._lib.ssnalm_ws_solve(s._ctx, Cc.c_void_p(out.data_ptr()), 0.9, 3,
                                        Cc.c_void_p(xd.data_ptr()), None, Cc.byref(info),
                                        Cc.byref(st))
    assert status == L.WARMSTART_REJECTED and info.status == L.WARMSTART_REJECTED
    assert st.fallback == 1
    R, _ = ssnal.rkkt(X.astype(np.float64), y, 0.5, xd.cpu().numpy())
    assert R <= 1e-6 * 1.0001
