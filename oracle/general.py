"""CPU FP64 oracle of SSsNAL on the unified problem (P) with a linear kernel.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

Problem (Section 1, eq. Problem_P1_classical1):
    min 1/2 x^T Q x + c^T x   s.t.  a^T x = d,  l <= x <= u,   l < u,
with Q = B B^T for a given B (n x q, dense or CSR); Q is never formed.
Two instances are built here:
  * C-SVC (eq. Def_Dual_of_C_SVM_Problem): B = diag(y) X, c = -e, a = y,
    d = 0, l = 0, u = C e;
  * eps-SVR (eq. Def_Dual_of_SVR_Problem): variables [x; z] in R^{2n},
    B = [X; -X] (so that [x; z]^T Q [x; z] = |X^T (x - z)|^2), c = [eps e + y;
    eps e - y], a = [e; -e], d = 0, l = 0, u = C e.

The method is the same omega-space Algorithm 1 + Algorithm 3 as the C-SVC
oracle, with general data (omega := B^T w, so Q w = B omega):
    u(omega)  = x^k - sigma (B omega + c)                        (eq. Def_psi)
    psi       = 1/2|omega|^2 + (|u|^2 - |u - Pi(u)|^2)/(2 sigma) - |x^k|^2/(2 sigma)
    grad psi  = omega - B^T Pi(u)                  (eq. Def_differential_of_psi)
    Newton    (I + sigma B^T P B) d = -grad psi     (eq. Newton_Linear_System),
              by Cholesky or (newton="pcg") by Jacobi-preconditioned CG to
              |M d + g| <= min(eta, |g|^(1+tau))
with P the HS-Jacobian of Theorem 3.1 at the free set J (eq. Def_HS_P):
    B^T P B = B_J^T B_J - s s^T / (a_J^T a_J),  s = B_J^T a_J    (a_J != 0)
    B^T P B = B_J^T B_J                                          (a_J = 0)
the x-update x^{k+1} = Pi(u(omega^{k+1})) (eq. Def_new_update_xkplus) and
R_KKT(x) = |x - Pi(x - Q x - c)| / (1 + |x|) (eq. Def_Rkkt).

The line search compares psi(omega + alpha d) - psi(omega) with
mu alpha <g, d>, the change evaluated term by term: with t = u - lam a and
x = clip(t, l, u) one has 1/2(|u|^2 - |u - x|^2) = sum_i h_i(t_i) + lam d,
h_i(t) = t clip(t) - clip(t)^2 / 2, since a^T x = d.  Parameter readings are
those of the C-SVC oracle (`ssnal.Options`).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .projection import project
from .ssnal import Options


@dataclass
class Problem:
    B: object            # (n, q) ndarray or CSR, FP64
    c: np.ndarray
    a: np.ndarray
    d: float
    l: np.ndarray
    u: np.ndarray


def _f64(M):
    return sp.csr_matrix(M, dtype=np.float64) if sp.issparse(M) else np.asarray(M, np.float64)


def csvc_problem(X, y, C):
    """The C-SVC dual as an instance of (P)."""
    X = _f64(X)
    yf = np.asarray(y, np.float64)
    n = yf.size
    B = sp.diags(yf) @ X if sp.issparse(X) else yf[:, None] * X
    return Problem(B=_f64(B), c=-np.ones(n), a=yf.copy(), d=0.0,
                   l=np.zeros(n), u=np.full(n, float(C)))


def svr_problem(X, yr, C, eps):
    """The eps-SVR dual (eq. Def_Dual_of_SVR_Problem) as an instance of (P),
    variables ordered [x; z]."""
    X = _f64(X)
    yr = np.asarray(yr, np.float64)
    n = yr.size
    B = sp.vstack([X, -X], format="csr") if sp.issparse(X) else np.vstack([X, -X])
    return Problem(B=B, c=np.concatenate([eps + yr, eps - yr]),
                   a=np.concatenate([np.ones(n), -np.ones(n)]), d=0.0,
                   l=np.zeros(2 * n), u=np.full(2 * n, float(C)))


def bmul(B, v):
    """B v."""
    return np.asarray(B @ v).ravel()


def btmul(B, r):
    """B^T r."""
    return np.asarray(B.T @ r).ravel()


def projection(prob, v):
    """Pi_{K∩L}(v) with its lam_hat and the strict interior set J of
    l < v - lam a < u (Theorem 3.1)."""
    x, lam = project(v, prob.a, prob.l, prob.u, prob.d)
    t = np.asarray(v, np.float64) - lam * prob.a
    free = (t > prob.l) & (t < prob.u)
    return x, lam, free


def objective(prob, x):
    """1/2 x^T Q x + c^T x = 1/2 |B^T x|^2 + c^T x."""
    w = btmul(prob.B, x)
    return 0.5 * float(w @ w) + float(prob.c @ x)


def rkkt(prob, x):
    """eq. Def_Rkkt."""
    v = x - bmul(prob.B, btmul(prob.B, x)) - prob.c
    px, _, _ = projection(prob, v)
    return float(np.linalg.norm(x - px) / (1.0 + np.linalg.norm(x)))


def h_piece(t, l, u):
    """h(t) = t clip(t, l, u) - clip(t, l, u)^2 / 2, elementwise."""
    t = np.asarray(t, np.float64)
    x = np.minimum(np.maximum(t, l), u)
    return t * x - 0.5 * x * x


def h_increment(t, dt, l, u):
    """h(t + dt) - h(t); both ends on one piece use that piece's closed form
    in dt (slope l below l, t in between, u above u)."""
    t = np.asarray(t, np.float64)
    dt = np.asarray(dt, np.float64)
    b = t + dt
    out = h_piece(b, l, u) - h_piece(t, l, u)
    up = (t >= u) & (b >= u)
    lo = (t <= l) & (b <= l)
    mid = (t > l) & (t < u) & (b > l) & (b < u)
    out = np.where(up, u * dt, out)
    out = np.where(lo, l * dt, out)
    return np.where(mid, dt * (t + 0.5 * dt), out)


def psi_literal(prob, omega, xk, sigma):
    """psi(omega) as eq. Def_psi reads (Q w = B omega)."""
    u = xk - sigma * (bmul(prob.B, omega) + prob.c)
    px, _, _ = projection(prob, u)
    return (0.5 * float(omega @ omega)
            + (float(u @ u) - float((u - px) @ (u - px))) / (2.0 * sigma)
            - float(xk @ xk) / (2.0 * sigma))


def psi_increment(prob, omega, d, alpha, u, lam, u_a, lam_a, sigma):
    """psi(omega + alpha d) - psi(omega) through per-term increments."""
    t = u - lam * prob.a
    dt = (u_a - u) - (lam_a - lam) * prob.a
    dh = float(np.sum(h_increment(t, dt, prob.l, prob.u))) + (lam_a - lam) * prob.d
    return alpha * float(omega @ d) + 0.5 * alpha * alpha * float(d @ d) + dh / sigma


def newton_direction(prob, free, g, sigma):
    """d = -(I + sigma B^T P B)^{-1} g by Cholesky, P from Theorem 3.1."""
    idx = np.flatnonzero(free)
    if idx.size == 0:
        return -g.copy()
    BJ = prob.B[idx]
    if sp.issparse(BJ):
        BJ = BJ.toarray()
    aJ = prob.a[idx]
    M = BJ.T @ BJ
    den = float(aJ @ aJ)
    if den != 0.0:
        s = BJ.T @ aJ
        M = M - np.outer(s, s) / den
    M = np.eye(g.size) + sigma * M
    return -sla.cho_solve(sla.cho_factor(M, lower=True), g)


def newton_pcg(prob, free, g, sigma, tol, maxit=500):
    """The same Newton system solved matrix-free by conjugate gradients with
    the Jacobi preconditioner diag(M) (floored at 1), to |M d + g| <= tol.
    Returns (d, iterations)."""
    idx = np.flatnonzero(free)
    if idx.size == 0:
        return -g.copy(), 0
    BJ = prob.B[idx]
    aJ = prob.a[idx]
    den = float(aJ @ aJ)
    s = btmul(BJ, aJ)
    sq = (np.asarray(BJ.multiply(BJ).sum(axis=0)).ravel() if sp.issparse(BJ)
          else (BJ * BJ).sum(axis=0))
    diag = 1.0 + sigma * (sq - (s * s / den if den != 0.0 else 0.0))
    diag = np.maximum(diag, 1.0)

    def apply(v):
        out = v + sigma * btmul(BJ, bmul(BJ, v))
        if den != 0.0:
            out -= sigma * s * (float(s @ v) / den)
        return out

    d = np.zeros_like(g)
    r = -g.copy()
    z = r / diag
    pdir = z.copy()
    rz = float(r @ z)
    it = 0
    while it < maxit and math.sqrt(float(r @ r)) > tol:
        Ap = apply(pdir)
        alpha = rz / float(pdir @ Ap)
        d += alpha * pdir
        r -= alpha * Ap
        z = r / diag
        rz_new = float(r @ z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
        it += 1
    return d, it


@dataclass
class Result:
    x: np.ndarray
    omega: np.ndarray
    obj: float
    rkkt: float
    outer: int
    inner: int
    status: str
    cg_iters: int
    time_s: float


def solve(prob, tol=1e-6, x0=None, **kw):
    """SSsNAL (Algorithm 1 + Algorithm 3) on (P) with Q = B B^T."""
    t_start = time.perf_counter()
    opt = Options(tol=tol, **kw)
    B = prob.B
    n = prob.c.size
    x = np.zeros(n) if x0 is None else projection(prob, np.asarray(x0, np.float64))[0]
    if x0 is None and (abs(prob.d) > 0.0 or np.any(prob.l > 0.0) or np.any(prob.u < 0.0)):
        x = projection(prob, x)[0]
    omega = btmul(B, x)
    sigma = opt.sigma0
    inner_total = 0
    cg_total = 0
    status = "MAXITER"
    R = math.inf
    best = None                  # (R, x): returned if the iteration cap is hit
    outer = 0
    for k in range(opt.max_outer):
        outer = k + 1
        eps_k = opt.eps_decay ** k
        Bomega = bmul(B, omega)
        xk = x
        for _ in range(opt.max_inner):
            u = xk - sigma * (Bomega + prob.c)
            xt, lam, free = projection(prob, u)
            g = omega - btmul(B, xt)
            gn = float(np.linalg.norm(g))
            crit = min(eps_k, eps_k * float(np.linalg.norm(xt - xk))) / math.sqrt(sigma)
            if gn <= max(crit, opt.floor * (1.0 + float(np.linalg.norm(omega)))):
                break
            if opt.newton == "pcg":
                d, it = newton_pcg(prob, free, g, sigma, min(opt.eta, gn ** (1.0 + opt.tau)), opt.max_cg)
                cg_total += it
            else:
                d = newton_direction(prob, free, g, sigma)
            inner_total += 1
            t = bmul(B, d)
            gd = float(g @ d)
            accepted = False
            alpha = 1.0
            for m in range(opt.max_backtracks + 1):
                alpha = opt.ls_delta ** m
                u_a = u - alpha * sigma * t
                _, lam_a, _ = projection(prob, u_a)
                if psi_increment(prob, omega, d, alpha, u, lam, u_a, lam_a, sigma) <= opt.mu * alpha * gd:
                    accepted = True
                    break
            if not accepted:
                break
            omega = omega + alpha * d
            Bomega = bmul(B, omega)
        u = xk - sigma * (Bomega + prob.c)
        x, _, _ = projection(prob, u)
        R = rkkt(prob, x)
        if R <= opt.tol:
            status = "OK"
            break
        if best is None or R < best[0]:
            best = (R, x.copy())
        sigma = min(opt.rho * sigma, opt.sigma_max)
    if status == "MAXITER" and best is not None and best[0] < R:
        R, x = best
    return Result(x=x, omega=omega, obj=objective(prob, x), rkkt=R, outer=outer,
                  inner=inner_total, status=status, cg_iters=cg_total,
                  time_s=time.perf_counter() - t_start)


def svr_weights(X, x, z):
    """w = X^T (z - x) for the eps-SVR primal (eq. Def_SVR_Problem): the
    stationarity condition of its Lagrangian, with x the multipliers of the
    rows whose slack is xi_i and z those of xi*_i."""
    return btmul(_f64(X), np.asarray(z) - np.asarray(x))


def svr_primal(X, yr, C, eps, w, b):
    """1/2|w|^2 + C sum max(0, |y_i - x_i^T w - b| - eps): eq. Def_SVR_Problem
    with the optimal slacks for fixed (w, b)."""
    r = np.asarray(yr, np.float64) - bmul(_f64(X), w) - b
    return 0.5 * float(w @ w) + C * float(np.sum(np.maximum(0.0, np.abs(r) - eps)))


def svr_best_bias(X, yr, C, eps, w):
    """b minimising the eps-insensitive loss sum for fixed w: the loss is
    convex piecewise linear in b with kinks at r_i +- eps, so its minimum is
    attained at a kink; every kink is evaluated (small n only)."""
    r = np.asarray(yr, np.float64) - bmul(_f64(X), w)
    kinks = np.concatenate([r - eps, r + eps])
    vals = [float(np.sum(np.maximum(0.0, np.abs(r - b) - eps))) for b in kinks]
    return float(kinks[int(np.argmin(vals))])
