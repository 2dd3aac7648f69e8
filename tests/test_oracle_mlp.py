"""Pins of the warm-start oracle (oracle/mlp.py) against things other than
itself: central finite differences of the loss, closed forms of GELU,
softmax cross-entropy and the first Adam step, a two-point problem where the
one-step margin is the exact hard-margin solution, and planted mistakes that
these checks must catch."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp
from oracle import ssnal


def _batch(n=24, seed=0):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, mlp.IN))
    s = rng.integers(0, 3, size=n).astype(np.int32)
    t = rng.uniform(0.05, 0.95, size=n)
    return Z, s, t


def _theta(seed=0):
    th = synth.mlp_init(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    th += 0.05 * rng.standard_normal(th.size)          # nonzero biases too
    return th


def _fd_check(loss_fn, grad, theta, idx, h=1e-6):
    worst = 0.0
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (loss_fn(tp) - loss_fn(tm)) / (2 * h)
        worst = max(worst, abs(fd - grad[i]) / max(1e-8, abs(fd) + abs(grad[i])))
    return worst


def _sample_idx(rng, k_per_block=40):
    idx, o = [], 0
    for _, shp in mlp.SHAPES:
        k = int(np.prod(shp))
        idx += list(o + rng.choice(k, size=min(k, k_per_block), replace=False))
        o += k
    return idx


def test_param_count():
    assert mlp.N_PARAMS == 66 * 256 + 256 + 256 * 256 + 256 + 256 * 4 + 4
    assert synth.mlp_init(0).size == mlp.N_PARAMS


def test_gradient_finite_differences():
    """Every parameter block, 40 entries each: relative error <= 1e-6."""
    Z, s, t = _batch()
    th = _theta()
    L, g = mlp.backward(th, Z, s, t, w_mse=1.5)
    assert L == pytest.approx(mlp.loss(th, Z, s, t, w_mse=1.5), rel=1e-14)
    idx = _sample_idx(np.random.default_rng(3))
    assert _fd_check(lambda v: mlp.loss(v, Z, s, t, w_mse=1.5), g, th, idx) <= 1e-6


def test_planted_gelu_grad_mistake_is_caught(monkeypatch):
    Z, s, t = _batch()
    th = _theta()
    monkeypatch.setattr(mlp, "gelu_grad", lambda a: 0.5 * (1.0 + np.tanh(a)))
    _, g = mlp.backward(th, Z, s, t)
    monkeypatch.undo()
    idx = _sample_idx(np.random.default_rng(3))
    assert _fd_check(lambda v: mlp.loss(v, Z, s, t), g, th, idx) > 1e-3


def test_planted_missing_sigmoid_derivative_is_caught(monkeypatch):
    """A backward pass that forgets the sigmoid derivative of the multiplier
    head fails the finite-difference check on W3 / b3."""
    Z, s, t = _batch()
    s[:] = 1                                           # every row inside: MSE term active
    th = _theta()
    real_head = mlp.head

    def bad_backward(theta, Z, s, t, w_mse=1.0):
        p = mlp.unpack(np.asarray(theta, np.float64))
        O, (Zc, A1, H1, A2, H2) = mlp.forward(theta, Z)
        P, mult = real_head(O)
        n = Zc.shape[0]
        dO = np.zeros_like(O)
        dO[:, :3] = P
        dO[np.arange(n), s] -= 1.0
        dO[:, 3] = 2.0 * w_mse * (mult - t)             # missing mult (1 - mult)
        dO /= n
        return np.concatenate([(H2.T @ dO).ravel(), dO.sum(axis=0)])

    gb = bad_backward(th, Z, s, t)
    o = mlp.N_PARAMS - (256 * 4 + 4)
    idx = list(range(o, mlp.N_PARAMS))
    gfull = np.zeros(mlp.N_PARAMS)
    gfull[o:] = gb
    assert _fd_check(lambda v: mlp.loss(v, Z, s, t), gfull, th, idx) > 1e-2


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-16)
    a = np.array([-40.0, 40.0])
    np.testing.assert_allclose(mlp.gelu(a), [0.0, 40.0], atol=1e-300)
    # Phi(1) = (1 + erf(1/sqrt 2)) / 2 = 0.8413447460685429
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    x = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, rtol=1e-8, atol=1e-10)


def test_uniform_logits_loss_is_log3():
    """W3 = 0, b3 = 0: P = 1/3 everywhere, mult = 1/2, so L = log 3 +
    w_mse * mean(inside * (1/2 - t)^2)."""
    Z, s, t = _batch()
    th = _theta()
    p = mlp.unpack(th)
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    expect = math.log(3.0) + 0.7 * np.mean((s == 1) * (0.5 - t) ** 2)
    assert mlp.loss(th, Z, s, t, w_mse=0.7) == pytest.approx(expect, rel=1e-14)


def test_adam_first_step_closed_form():
    """From m = v = 0 at step 1 the bias-corrected update is
    lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1e-2, 0.9, 0.999, 1e-8, 1)
    np.testing.assert_allclose(th, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 1e-3 * g * g)


def test_one_step_margin_two_points_is_hard_margin_solution():
    """x = +1 (y = +1), x = -1 (y = -1), C = 1: p = Pi(C e) = (1, 1),
    A^T p = 2, t* = 2 / 4 = 1/2, w1 = 1, b1 = 0: the max-margin separator,
    margins exactly 1."""
    X = np.array([[1.0], [-1.0]])
    y = np.array([1, -1], np.int8)
    w1, b1, m = mlp.one_step_margin(X, y, 1.0)
    assert w1[0] == 1.0 and b1 == 0.0
    np.testing.assert_array_equal(m, [1.0, 1.0])
    # small C: the step length is capped at 1 -> w1 = C A^T e
    w1, b1, m = mlp.one_step_margin(X, y, 0.1)
    assert w1[0] == pytest.approx(0.2)


def test_one_step_is_exact_line_search():
    """f(t p) is minimised over t in [0, 1] at t*: f there is below f at
    nearby t, and p is feasible."""
    X, y = synth.mixture_problem(300, q=6, seed=2)
    X = X.astype(np.float64)
    C = 0.05
    yf = y.astype(np.float64)
    w1, b1, m = mlp.one_step_margin(X, y, C)
    from oracle.projection import project_svm
    p, _, _ = project_svm(np.full(300, C), y, C)
    assert abs(yf @ p) <= 1e-12 and p.min() >= 0 and p.max() <= C
    wp = ssnal.atmul(X, y, p)
    tstar = float(w1 @ wp) / float(wp @ wp)
    f = lambda tt: ssnal.dual_objective(X, y, tt * p)
    for dt in (-1e-3, 1e-3):
        tt = min(max(tstar + dt, 0.0), 1.0)
        assert f(tstar) <= f(tt) + 1e-12
    # b1 centres the two class means of the scores
    s_ = X @ w1
    assert (s_[y > 0] + b1).mean() == pytest.approx(-(s_[y < 0] + b1).mean(), rel=1e-12)


def test_features_layout():
    X, y = synth.mixture_problem(50, q=10, seed=1)
    R = synth.projection_matrix(10)
    Z = mlp.features(X, y, 2.0, R)
    assert Z.shape == (50, 66)
    np.testing.assert_allclose(Z[:, :64], X.astype(np.float64) @ R.astype(np.float64), rtol=1e-12)
    assert np.all(Z[:, 65] == math.log10(100.0))


def test_labels_and_x0():
    s, t = mlp.labels(np.array([0.0, 1e-9, 0.5, 1.0 - 1e-9, 1.0]), 1.0)
    np.testing.assert_array_equal(s, [0, 0, 1, 2, 2])
    # the most probable status decides: 0, C * mult or C
    O = np.array([[0.3, 0.2, 0.1, 0.0],        # x = 0
                  [0.0, 0.5, 0.4, 0.0],        # inside, mult = 1/2
                  [0.0, 0.1, 0.2, 3.0],        # x = C
                  [0.7, 0.7, 0.0, 1.0]])       # tie 0 / inside: the lower index
    np.testing.assert_allclose(mlp.x0_from_output(O, 2.0), [0.0, 1.0, 2.0, 0.0], atol=1e-20)
