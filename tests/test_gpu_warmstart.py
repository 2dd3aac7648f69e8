"""Warm-start network and features on the GPU against the FP64 oracle
(oracle/mlp.py), and the solve from the learned initial point (GPU only).

Bars: fp32 kernels against fp64 references.  Forward probabilities within
2e-5 absolute; gradients within 2e-4 of the largest entry of each parameter
block; Adam within 1e-6 relative; features: the projected part within 1e-5
relative to the row scale (fp32 accumulation over q terms), margins within
1e-6 relative (fp64 arithmetic, fp32 storage).
"""
import math

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


def _theta(seed=0, noise=0.05):
    th = synth.mlp_init(seed).astype(np.float64)
    th += noise * np.random.default_rng(seed + 11).standard_normal(th.size)
    return th.astype(np.float32)


def _batch(n, seed=0):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, 66)).astype(np.float32)
    Z[:, 64] *= 3.0
    Z[:, 65] = 4.0
    s = rng.integers(0, 3, size=n).astype(np.int32)
    t = rng.uniform(0.01, 0.99, size=n).astype(np.float32)
    return Z, s, t


@pytest.mark.parametrize("n", [1, 63, 300, 4096])
def test_forward_vs_oracle(n):
    from paper_1910_01312_amd.warmstart import Net
    th = _theta()
    Z, _, _ = _batch(n, seed=n)
    out = Net(th).forward(Z).cpu().numpy()
    O, _ = mlp.forward(th.astype(np.float64), Z.astype(np.float64))
    P, mult = mlp.head(O)
    np.testing.assert_allclose(out[:, :3], P, rtol=0, atol=2e-5)
    np.testing.assert_allclose(out[:, 3], mult, rtol=0, atol=2e-5)


@pytest.mark.parametrize("n", [5, 700, 4096])
def test_gradient_vs_oracle(n):
    from paper_1910_01312_amd.warmstart import Net
    th = _theta(1)
    Z, s, t = _batch(n, seed=100 + n)
    net = Net(th)
    loss, g = net.gradient(Z, s, t, w_mse=1.5)
    g = g.cpu().numpy().astype(np.float64)
    L_ref, g_ref = mlp.backward(th.astype(np.float64), Z.astype(np.float64), s,
                                t.astype(np.float64), w_mse=1.5)
    assert float(loss.cpu()[0]) == pytest.approx(L_ref, rel=2e-5)
    o = 0
    for name, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        ref = g_ref[o:o + k]
        scale = max(np.abs(ref).max(), 1e-30)
        assert np.abs(g[o:o + k] - ref).max() <= 2e-4 * scale, name
        o += k


def test_gradient_deterministic():
    from paper_1910_01312_amd.warmstart import Net
    th = _theta(2)
    Z, s, t = _batch(2048, seed=5)
    a = Net(th).gradient(Z, s, t)[1].cpu().numpy()
    b = Net(th).gradient(Z, s, t)[1].cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_adam_vs_oracle():
    from paper_1910_01312_amd.warmstart import Net
    th = _theta(3)
    Z, s, t = _batch(512, seed=9)
    net = Net(th)
    ref = th.astype(np.float64)
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    for step in range(1, 4):
        _, g = net.gradient(Z, s, t)
        gh = g.cpu().numpy().astype(np.float64)
        net.adam(1e-3)
        ref, m, v = mlp.adam_step(ref, gh, m, v, 1e-3, 0.9, 0.999, 1e-8, step)
        got = net.theta.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-7)
        ref = got          # follow the GPU parameters (fp32 rounding) into the next step


@pytest.mark.parametrize("dtype,q,C", [("f32", 128, 1.0), ("f64", 40, 0.01), ("bf16", 256, 30.0)])
def test_features_vs_oracle(dtype, q, C):
    from paper_1910_01312_amd.solver import Solver
    from paper_1910_01312_amd.warmstart import features
    X, y = synth.mixture_problem(3001, q=q, seed=17)
    if dtype == "bf16":
        Xs = synth.to_bf16_bits(X)
        Xr = synth.bf16_bits_to_f32(Xs).astype(np.float64)
        kw = {"bf16": True}
    elif dtype == "f64":
        Xs = X.astype(np.float64)
        Xr = Xs
        kw = {}
    else:
        Xs, Xr, kw = X, X.astype(np.float64), {}
    R = synth.projection_matrix(q)
    with Solver(Xs, y, C, **kw) as s:
        Z = features(s, R).cpu().numpy().astype(np.float64)
    Zr = mlp.features(Xr, y, C, R)
    rowscale = np.sqrt((Xr ** 2).sum(axis=1))[:, None] * np.abs(R).max()
    assert np.all(np.abs(Z[:, :64] - Zr[:, :64]) <= 1e-5 * rowscale + 1e-6)
    np.testing.assert_allclose(Z[:, 64], Zr[:, 64], rtol=1e-6, atol=1e-6 * np.abs(Zr[:, 64]).max())
    np.testing.assert_allclose(Z[:, 65], Zr[:, 65], rtol=1e-7)


def test_initial_point_vs_oracle():
    from paper_1910_01312_amd.solver import Solver
    from paper_1910_01312_amd.warmstart import Net, initial_point
    X, y = synth.mixture_problem(1000, q=16, seed=3)
    Z, _, _ = _batch(1000, seed=4)
    net = Net(_theta(4, noise=0.5))
    with Solver(X, y, 2.5) as s:
        out = net.forward(Z)
        x0 = initial_point(s, out).cpu().numpy()
    O, _ = mlp.forward(net.theta.cpu().numpy().astype(np.float64), Z.astype(np.float64))
    P, _ = mlp.head(O)
    top = np.sort(P, axis=1)
    clear = top[:, 2] - top[:, 1] > 1e-4           # fp32 and fp64 agree on the most probable status
    assert clear.mean() > 0.9
    np.testing.assert_allclose(x0[clear], mlp.x0_from_output(O, 2.5)[clear], rtol=0, atol=1e-4)


def test_training_on_solved_instances():
    """Labels from ssnalm_solve_batch solutions (two of them checked by the
    oracle), features by the library, a few Adam epochs with the library's
    kernels: the loss falls."""
    from paper_1910_01312_amd.warmstart import Net, build_dataset, train, training_instances
    specs = training_instances(48, n=1024, seed=7)
    R = synth.projection_matrix(32)
    specs = [dict(sp, q=32) for sp in specs]
    make = lambda sp: synth.mixture_problem(sp["n"], q=sp["q"], seed=sp["seed"])
    Z, st, tg, recs = build_dataset(specs, R, make, chunk=16)
    assert all(r["status"] == "OK" for r in recs)
    assert Z.shape == (48 * 1024, 66)
    for k in (0, 47):
        X, y = make(specs[k])
        x = tg[k * 1024:(k + 1) * 1024].double().cpu().numpy() * specs[k]["C"]
        R_k, _ = ssnal.rkkt(X.astype(np.float64), y, specs[k]["C"], x)
        assert R_k <= 1e-6 * 1.01
    net = Net(synth.mlp_init(0))
    hist = train(net, Z, st, tg, epochs=4, batch=1024, lr=2e-3)
    assert hist[-1] < 0.8 * hist[0], hist


def _median_time(fn, reps=3):
    ts = []
    out = None
    for _ in range(reps):
        torch.cuda.synchronize()
        import time
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts)), out


def test_learned_screening_gain():
    """The committed network (trained by the library's own kernels on solved
    instances of the batched family's generator, see
    paper_1910_01312_amd/warmstart.py) against the plain cold solve on
    held-out n = 200,000, q = 256 instances: the warm path (features +
    network + screened solves + full-problem KKT check) returns solutions
    that meet the bars on the full problem (R_KKT recomputed by the oracle,
    objective within 1e-8 of the oracle's reference f* stored by
    tests/golden/make_refs.py), and does less row work than the cold solve
    (Newton steps times rows solved over).  Times are printed, not asserted:
    they are reported by the benchmark."""
    import json
    import os
    from paper_1910_01312_amd.solver import Solver
    from paper_1910_01312_amd.warmstart import Net, warm_solve
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = Net.load(os.path.join(root, "paper_1910_01312_amd", "data", "warmstart_q256.npz"))
    with open(os.path.join(root, "tests", "golden", "oracle_refs.json")) as f:
        refs = json.load(f)["warm_eval"]
    R = synth.projection_matrix(256)
    t_cold = t_warm = 0.0
    for ref in refs:
        C = ref["C"]
        X, y = synth.mixture_problem(ref["n"], q=ref["q"], seed=ref["seed"])
        assert float(np.sum(X, dtype=np.float64)) == ref["inputs"]["sum_x"]
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        with Solver(Xd, yd, C, tol=1e-6) as s:
            s.solve()                                            # first-call costs out of the timing
            tc, (xc, wc, ic) = _median_time(lambda: s.solve())
            tw, (xw, ww, iw, sw) = _median_time(lambda: warm_solve(s, net, R, keep_frac=0.15))
        assert ic["status_name"] == "OK"
        assert iw["status_name"] in ("OK", "WARMSTART_REJECTED")
        Xr = X.astype(np.float64)
        for x in (xc, xw):
            xh = x.cpu().numpy()
            Rk, _ = ssnal.rkkt(Xr, y, C, xh)
            assert Rk <= 1e-6 * 1.0001, (C, Rk, sw)
            f = ssnal.dual_objective(Xr, y, xh)
            rel = abs(f - ref["f_star"]) / max(1.0, abs(ref["f_star"]))
            print(f"C={C}: relative objective error {rel:.2e}")
            assert rel <= 1e-6, (C, f, ref["f_star"])
        work_cold = ic["iters_inner"] * ref["n"]
        work_warm = iw["iters_inner"] * sw["kept"] if not sw["fallback"] else work_cold
        print(f"C={C}: cold {tc:.3f} s ({ic['iters_inner']} Newton x {ref['n']} rows), "
              f"warm {tw:.3f} s ({iw['iters_inner']} Newton x {sw['kept']} rows, {sw})")
        assert work_warm < work_cold, (C, work_warm, work_cold)
        t_cold += tc
        t_warm += tw
    print(f"total cold {t_cold:.3f} s, warm {t_warm:.3f} s, gain {t_cold / t_warm:.2f}")
