"""CPU FP64 oracle of the learned warm start: features, network, loss,
gradients, Adam, labels and the initial point.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

The paper starts its exact-kernel solves from a cheaper approximate solution
(the random-Fourier-feature warm start of its RBF experiments, Section 4) and
notes that a good initial point matters (Remark 2).  For the linear solve
this project learns the initial point instead: a small network predicts for
every sample whether x_i* is 0, strictly inside (0, C) or C, and x_i*/C when
inside.  Nothing here is fixed by the paper, so every definition below is
this project's, stated once and used by both implementations:

  features  z_i = [ R^T x_i (64),  m_i,  log10(n C) ]              (66 inputs)
            R: q x 64 Gaussian / sqrt(q) (an input, drawn by synth);
            p  = Pi(C e)  (projection onto {y^T x = 0, 0 <= x <= C});
            t* = clip(e^T p / |A^T p|^2, 0, 1) (exact line search of
                 f(x) = 1/2 x^T Q x - e^T x along x = t p: one projected-
                 gradient step from x = 0, since grad f(0) = -e);
            w1 = t* A^T p,  s_i = x_i^T w1,
            b1 = -(mean of s over y = +1  +  mean of s over y = -1) / 2,
            m_i = y_i (s_i + b1).
  network   A1 = Z W1 + b1, H1 = gelu(A1), A2 = H1 W2 + b2, H2 = gelu(A2),
            O = H2 W3 + b3 (66 -> 256 -> 256 -> 4),
            gelu(a) = a Phi(a) (Phi: standard normal CDF).
  head      P = softmax(O[:, 0:3]) over (x = 0, inside, x = C),
            mult = sigmoid(O[:, 3]).
  loss      L = mean_i[-log P_i,s_i] + w_mse * mean_i[ [s_i = inside] (mult_i - t_i)^2 ].
  labels    s_i = 0 if x_i <= 1e-8 C, 2 if x_i >= (1 - 1e-8) C, else 1; t_i = x_i / C.
  x0        the most probable status decides: x0_i = 0, C mult_i or C
            (ties to the lower index); then projected by the solver.
  Adam      the update of Kingma & Ba (2015) with bias correction.

Parameter vector layout (one flat array): W1 (66 x 256, row-major), b1 (256),
W2 (256 x 256), b2 (256), W3 (256 x 4), b3 (4).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .projection import project_svm

IN, HID, OUT = 66, 256, 4
NPROJ = 64
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, OUT)), ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Views of the flat parameter vector, in layout order."""
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


# ------------------------------------------------------------------ network
def gelu(a):
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    """d gelu / da = Phi(a) + a phi(a)."""
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def forward(theta, Z):
    p = unpack(np.asarray(theta, np.float64))
    Z = np.asarray(Z, np.float64)
    A1 = Z @ p["W1"] + p["b1"]
    H1 = gelu(A1)
    A2 = H1 @ p["W2"] + p["b2"]
    H2 = gelu(A2)
    O = H2 @ p["W3"] + p["b3"]
    return O, (Z, A1, H1, A2, H2)


def head(O):
    L = O[:, :3] - O[:, :3].max(axis=1, keepdims=True)
    E = np.exp(L)
    P = E / E.sum(axis=1, keepdims=True)
    mult = 1.0 / (1.0 + np.exp(-O[:, 3]))
    return P, mult


def loss(theta, Z, s, t, w_mse=1.0):
    O, _ = forward(theta, Z)
    P, mult = head(O)
    n = Z.shape[0]
    s = np.asarray(s)
    ce = -np.log(P[np.arange(n), s])
    free = (s == 1).astype(np.float64)
    return float(ce.mean() + w_mse * np.mean(free * (mult - np.asarray(t, np.float64)) ** 2))


def backward(theta, Z, s, t, w_mse=1.0):
    """(L, dL/dtheta) by the chain rule written out layer by layer."""
    theta = np.asarray(theta, np.float64)
    p = unpack(theta)
    O, (Zc, A1, H1, A2, H2) = forward(theta, Z)
    P, mult = head(O)
    n = Zc.shape[0]
    s = np.asarray(s)
    t = np.asarray(t, np.float64)
    free = (s == 1).astype(np.float64)
    L = float(-np.log(P[np.arange(n), s]).mean() + w_mse * np.mean(free * (mult - t) ** 2))
    dO = np.zeros_like(O)
    dO[:, :3] = P
    dO[np.arange(n), s] -= 1.0
    dO[:, 3] = free * 2.0 * w_mse * (mult - t) * mult * (1.0 - mult)
    dO /= n
    g = {}
    g["W3"] = H2.T @ dO
    g["b3"] = dO.sum(axis=0)
    dA2 = (dO @ p["W3"].T) * gelu_grad(A2)
    g["W2"] = H1.T @ dA2
    g["b2"] = dA2.sum(axis=0)
    dA1 = (dA2 @ p["W2"].T) * gelu_grad(A1)
    g["W1"] = Zc.T @ dA1
    g["b1"] = dA1.sum(axis=0)
    return L, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam_step(theta, grad, m, v, lr, beta1, beta2, eps, step):
    """One Adam update (bias-corrected moments); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ features, labels, x0
def one_step_margin(X, y, C):
    """(w1, b1, m) of the one projected-gradient step from x = 0."""
    yf = np.asarray(y, np.float64)
    n = yf.size
    p, _, _ = project_svm(np.full(n, float(C)), y, C)
    wp = np.asarray(X.T @ (yf * p)).ravel()
    den = float(wp @ wp)
    tstar = min(max(float(p.sum()) / den, 0.0), 1.0) if den > 0.0 else 0.0
    w1 = tstar * wp
    s_ = np.asarray(X @ w1).ravel()
    pos, neg = yf > 0, yf < 0
    if pos.any() and neg.any():
        b1 = -0.5 * (s_[pos].mean() + s_[neg].mean())
    else:
        b1 = -s_.mean()
    return w1, b1, yf * (s_ + b1)


def features(X, y, C, R):
    """Z (n x 66) of the definition in the module docstring."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    _, _, m = one_step_margin(X, y, C)
    Z = np.empty((n, IN))
    Z[:, :NPROJ] = X @ np.asarray(R, np.float64)
    Z[:, NPROJ] = m
    Z[:, NPROJ + 1] = math.log10(n * C)
    return Z


def labels(x, C, rel=1e-8):
    """Bound status (0: x = 0, 1: inside, 2: x = C) and x / C."""
    x = np.asarray(x, np.float64)
    s = np.ones(x.size, np.int32)
    s[x <= rel * C] = 0
    s[x >= (1.0 - rel) * C] = 2
    return s, x / C


def x0_from_output(O, C):
    P, mult = head(np.asarray(O, np.float64))
    k = np.argmax(P, axis=1)
    return np.where(k == 0, 0.0, np.where(k == 1, C * mult, C))
