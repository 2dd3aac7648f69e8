"""CPU FP64 oracle of the SSsNAL method for the linear C-SVC dual QP.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

Problem (Section 1, eq. Def_Dual_of_C_SVM_Problem):
    min 1/2 x^T Q x - e^T x   s.t.  y^T x = 0,  0 <= x <= C,
with the linear kernel Q = A A^T, A = diag(y) X (Q is never formed).

The method is Algorithm 1 (augmented Lagrangian on the restricted dual (D))
with Algorithm 3 (semismooth Newton) for its inner problem.  Everything here
is written in omega-space, omega := A^T w: the dual variable w enters psi,
its gradient and the Newton system only through Q w = A omega and
<w, Q w> = |omega|^2 (Section 3.2.4, the L^T d representation of eq. Def_Ld
with L = A), so
    u(omega)    = x^k + sigma (e - A omega)                      (eq. Def_psi)
    psi(omega)  = 1/2|omega|^2 + (|u|^2 - |u - Pi(u)|^2)/(2 sigma) - |x^k|^2/(2 sigma)
    grad psi    = omega - A^T Pi(u)                   (eq. Def_differential_of_psi)
    Newton      (I + sigma A^T P A) d = -grad psi     (eq. Newton_Linear_System
                                                       in L = A coordinates)
and with a = y the HS-Jacobian (Theorem 3.1) gives
    A^T P A = X_J^T X_J - s s^T / p,   s = X_J^T 1,  p = |J|,
because y_i^2 = 1 makes the labels cancel.  The x-update is
x^{k+1} = Pi(u(omega^{k+1})) (eq. Def_new_update_xkplus).

Readings of points the paper leaves open (all are keyword options):
  sigma0 = 1, sigma_{k+1} = min(rho sigma_k, sigma_max), rho = 2, sigma_max = 1e6;
  eps_k = delta_k = 0.5^k in (A') and (B'); the strong-convexity modulus of
  psi in omega-space is 1, so (A')+(B') read |g| <= min(eps_k, delta_k
  |x^{k+1}-x^k|)/sqrt(sigma), with an absolute floor 1e-14 (1 + |omega|);
  mu = 1e-4, line-search factor delta = 0.5, tau = 0.5, eta = 0.1;
  at most 200 outer and 50 inner iterations; x^0 = 0, omega^0 = 0;
  the Armijo test compares psi(omega + alpha d) - psi(omega), evaluated as a
  sum of per-component increments (an exact rewriting, see `psi_increment`),
  with mu*alpha*<g, d>.  A line search that exhausts its backtracks ends the
  inner loop at the current iterate.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .projection import project_svm


# --------------------------------------------------------------------------
# operations on the implicit Q = A A^T
# --------------------------------------------------------------------------

def amul(X, y, v):
    """A v = y ⊙ (X v)."""
    return np.asarray(y, np.float64) * np.asarray(X @ v).ravel()


def atmul(X, y, r):
    """A^T r = X^T (y ⊙ r)."""
    return np.asarray(X.T @ (np.asarray(y, np.float64) * r)).ravel()


def rows(X, idx):
    """X_J as an FP64 matrix (dense ndarray or CSR)."""
    if sp.issparse(X):
        return X[idx]
    return X[idx, :]


# --------------------------------------------------------------------------
# psi and its increments
# --------------------------------------------------------------------------

def huber_piece(t, C):
    """phi(t) = int_0^t clip(s, 0, C) ds, elementwise."""
    t = np.asarray(t, np.float64)
    return np.where(t <= 0.0, 0.0, np.where(t < C, 0.5 * t * t, C * (t - 0.5 * C)))


def huber_increment(t, dt, C):
    """phi(t + dt) - phi(t), evaluated without cancellation when t is large
    (both ends on the same piece use the piece's closed form in dt)."""
    t = np.asarray(t, np.float64)
    dt = np.asarray(dt, np.float64)
    b = t + dt
    out = huber_piece(b, C) - huber_piece(t, C)
    up = (t >= C) & (b >= C)
    lo = (t <= 0.0) & (b <= 0.0)
    mid = (t > 0.0) & (t < C) & (b > 0.0) & (b < C)
    out = np.where(up, C * dt, out)
    out = np.where(lo, 0.0, out)
    out = np.where(mid, dt * (t + 0.5 * dt), out)
    return out


def psi_literal(omega, u, xk, sigma, y, C):
    """psi(omega) exactly as eq. Def_psi (with Q w = A omega)."""
    xt, _, _ = project_svm(u, y, C)
    return (0.5 * float(omega @ omega)
            + (float(u @ u) - float((u - xt) @ (u - xt))) / (2.0 * sigma)
            - float(xk @ xk) / (2.0 * sigma))


def psi_increment(omega, d, alpha, u, lam, u_a, lam_a, sigma, y, C):
    """psi(omega + alpha d) - psi(omega).

    Uses 1/2(|u|^2 - |u - Pi(u)|^2) = sum_i phi(u_i - lam y_i) (which holds
    because y^T Pi(u) = 0), and writes the change of every term through its
    own increment, t_i(alpha) - t_i = (u_a - u)_i - (lam_a - lam) y_i."""
    yf = np.asarray(y, np.float64)
    t = u - lam * yf
    dt = (u_a - u) - (lam_a - lam) * yf
    dh = float(np.sum(huber_increment(t, dt, C)))
    return alpha * float(omega @ d) + 0.5 * alpha * alpha * float(d @ d) + dh / sigma


# --------------------------------------------------------------------------
# Newton direction (Proposition 5 in omega-space and cross-checks)
# --------------------------------------------------------------------------

def newton_qspace(X, free, g, sigma):
    """d = -(I + sigma (X_J^T X_J - s s^T/p))^{-1} g by Cholesky.
    p = 0 gives P = 0 (Theorem 3.1, a^T Sigma a = 0 case with Sigma = 0): d = -g."""
    idx = np.flatnonzero(free)
    p = idx.size
    if p == 0:
        return -g.copy()
    XJ = rows(X, idx)
    if sp.issparse(XJ):
        XJ = XJ.toarray()
    s = XJ.sum(axis=0)
    G = XJ.T @ XJ
    M = np.eye(g.size) + sigma * (G - np.outer(s, s) / p)
    return -sla.cho_solve(sla.cho_factor(M, lower=True), g)


def newton_pspace_centered(X, free, g, sigma):
    """p-space form of the same step (Woodbury on the centered rows):
    (I_p/sigma + Xc Xc^T) v = Xc g,  d = -g + Xc^T v,  Xc = (I - 11^T/p) X_J."""
    idx = np.flatnonzero(free)
    p = idx.size
    if p == 0:
        return -g.copy()
    XJ = rows(X, idx)
    if sp.issparse(XJ):
        XJ = XJ.toarray()
    Xc = XJ - XJ.mean(axis=0, keepdims=True)
    K = np.eye(p) / sigma + Xc @ Xc.T
    v = sla.cho_solve(sla.cho_factor(K, lower=True), Xc @ g)
    return -g + Xc.T @ v


def newton_lowrank(X, free, g, sigma, prev_free, prev_cho):
    """The same direction as `newton_qspace`, obtained from the Cholesky
    factor of the Newton matrix M0 of an earlier step at the same sigma:
    M = M0 + U S U^T, the columns of U being the rows entering J (weight
    +sigma), the rows leaving J (-sigma), s0/sqrt(p0) of the earlier J
    (+sigma) and s/sqrt(p) of the new J (-sigma), S the diagonal of those
    weights.  By the Woodbury
    identity M^{-1} g = M0^{-1} g - M0^{-1} U (S^{-1} + U^T M0^{-1} U)^{-1}
    U^T M0^{-1} g.  prev_cho is scipy's cho_factor of M0; the rank of the
    correction is (rows that changed) + 2 (the two centring terms)."""
    idx = np.flatnonzero(free)
    idx0 = np.flatnonzero(prev_free)
    add = np.flatnonzero(free & ~prev_free)
    rem = np.flatnonzero(prev_free & ~free)
    cols, sgn = [], []
    Xd = X.toarray() if sp.issparse(X) else X
    for i in add:
        cols.append(Xd[i]); sgn.append(sigma)
    for i in rem:
        cols.append(Xd[i]); sgn.append(-sigma)
    if idx0.size:                       # + sigma s0 s0^T / p0 (old centring removed)
        s0 = Xd[idx0].sum(axis=0)
        cols.append(s0 / math.sqrt(idx0.size)); sgn.append(sigma)
    if idx.size:                        # - sigma s s^T / p (new centring)
        s1 = Xd[idx].sum(axis=0)
        cols.append(s1 / math.sqrt(idx.size)); sgn.append(-sigma)
    y0 = sla.cho_solve(prev_cho, g)
    if not cols:
        return -y0
    U = np.array(cols).T                               # q x k
    Z = sla.cho_solve(prev_cho, U)                     # M0^{-1} U
    cap = np.diag(1.0 / np.array(sgn)) + U.T @ Z       # S^{-1} + U^T M0^{-1} U
    return -(y0 - Z @ np.linalg.solve(cap, U.T @ y0))


def apply_M(X, y_unused, idx, s, sigma, v):
    """(I + sigma (X_J^T X_J - s s^T / p)) v, matrix-free."""
    p = idx.size
    if p == 0:
        return v.copy()
    XJ = rows(X, idx)
    w = np.asarray(XJ @ v).ravel()
    return v + sigma * (np.asarray(XJ.T @ w).ravel() - s * (float(s @ v) / p))


def newton_pcg(X, free, g, sigma, tol, maxit=500):
    """Step 1 of Algorithm 3 by conjugate gradients (Jacobi-preconditioned)
    to |M d + g| <= tol.  Returns (d, iterations)."""
    idx = np.flatnonzero(free)
    p = idx.size
    if p == 0:
        return -g.copy(), 0
    XJ = rows(X, idx)
    s = np.asarray(XJ.sum(axis=0)).ravel()
    if sp.issparse(XJ):
        sq = np.asarray(XJ.multiply(XJ).sum(axis=0)).ravel()
    else:
        sq = (XJ * XJ).sum(axis=0)
    diag = 1.0 + sigma * (sq - s * s / p)
    diag = np.maximum(diag, 1.0)
    b = -g
    x = np.zeros_like(g)
    r = b.copy()
    z = r / diag
    pdir = z.copy()
    rz = float(r @ z)
    it = 0
    while it < maxit and math.sqrt(float(r @ r)) > tol:
        Ap = apply_M(X, None, idx, s, sigma, pdir)
        alpha = rz / float(pdir @ Ap)
        x += alpha * pdir
        r -= alpha * Ap
        z = r / diag
        rz_new = float(r @ z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
        it += 1
    return x, it


# --------------------------------------------------------------------------
# KKT residual, objective, primal quantities
# --------------------------------------------------------------------------

def rkkt(X, y, C, x):
    """Relative KKT residual (eq. Def_Rkkt) with c = -e:
    |x - Pi(x - Qx + e)| / (1 + |x|).  Returns (R, b) where b = the lam_hat
    of that projection (the bias estimate)."""
    Qx = amul(X, y, atmul(X, y, x))
    v = x - Qx + 1.0
    px, lam, _ = project_svm(v, y, C)
    return float(np.linalg.norm(x - px) / (1.0 + np.linalg.norm(x))), lam


def dual_objective(X, y, x):
    """f(x) = 1/2 |A^T x|^2 - e^T x."""
    w = atmul(X, y, x)
    return 0.5 * float(w @ w) - float(np.sum(x))


def primal_objective(X, y, C, w, b):
    """C-SVC primal (eq. Def_C_SVM_Problem) with the optimal slacks:
    1/2|w|^2 + C sum max(0, 1 - y_i (x_i^T w + b))."""
    m = np.asarray(X @ w).ravel() + b
    return 0.5 * float(w @ w) + C * float(np.sum(np.maximum(0.0, 1.0 - np.asarray(y, np.float64) * m)))


def best_bias(X, y, C, w):
    """b minimising the hinge sum for fixed w (exact 1-D search over the
    kinks b = y_i - x_i^T w; the objective is convex piecewise linear)."""
    yf = np.asarray(y, np.float64)
    m = np.asarray(X @ w).ravel()
    kinks = np.sort(yf - m)
    # subgradient in b: -sum_{active, y=+1} + sum_{active, y=-1}; evaluate at kinks
    best_b, best_v = 0.0, math.inf
    # evaluate convex function at a few candidates found by bisection on kinks
    lo, hi = 0, kinks.size - 1

    def val(b):
        return float(np.sum(np.maximum(0.0, 1.0 - yf * (m + b))))

    while hi - lo > 2:
        m1 = lo + (hi - lo) // 3
        m2 = hi - (hi - lo) // 3
        if val(kinks[m1]) <= val(kinks[m2]):
            hi = m2
        else:
            lo = m1
    for k in range(lo, hi + 1):
        vk = val(kinks[k])
        if vk < best_v:
            best_b, best_v = float(kinks[k]), vk
    return best_b


def duality_gap(X, y, C, x):
    """Relative gap (P(w,b) + f(x)) / (1 + |P| + |f|) with w = A^T x and the
    hinge-optimal b; P(w,b) + f(x) >= 0 by weak duality."""
    w = atmul(X, y, x)
    b = best_bias(X, y, C, w)
    return duality_gap_at(X, y, C, x, b)


def duality_gap_at(X, y, C, x, b):
    """The same relative gap at a given bias b (weak duality holds for every
    b, so it is >= the gap at the hinge-optimal b).  Returns (gap, P, f)."""
    w = atmul(X, y, x)
    P = primal_objective(X, y, C, w, b)
    f = dual_objective(X, y, x)
    return (P + f) / (1.0 + abs(P) + abs(f)), P, f


# --------------------------------------------------------------------------
# the solver
# --------------------------------------------------------------------------

@dataclass
class Options:
    tol: float = 1e-6
    sigma0: float = 1.0
    rho: float = 2.0
    sigma_max: float = 1e6
    max_outer: int = 200
    max_inner: int = 50
    max_backtracks: int = 40
    mu: float = 1e-4
    ls_delta: float = 0.5
    tau: float = 0.5
    eta: float = 0.1
    eps_decay: float = 0.5
    floor: float = 1e-14
    newton: str = "qspace"       # qspace | pspace | pcg
    max_cg: int = 500
    record: bool = False
    time_budget_s: float = 0.0    # > 0: stop (status "BUDGET") once exceeded


@dataclass
class Result:
    x: np.ndarray
    w: np.ndarray
    b: float
    obj: float
    rkkt: float
    outer: int
    inner: int
    p: int
    n_sv: int
    status: str
    sigma: float
    omega: np.ndarray
    history: list = field(default_factory=list)
    time_s: float = 0.0
    cg_iters: int = 0
    ls_fail: int = 0
    ls_trials: int = 0
    grad_steps: int = 0


def solve(X, y, C, tol=1e-6, x0=None, **kw):
    """SSsNAL (Algorithm 1 + Algorithm 3) on the linear C-SVC dual.

    X: (n,q) ndarray or scipy CSR (any float dtype; used in FP64),
    y: n labels in {+1,-1}, C > 0.  Returns a `Result`.
    """
    t_start = time.perf_counter()
    opt = Options(tol=tol, **kw)
    if sp.issparse(X):
        X = sp.csr_matrix(X, dtype=np.float64)
    else:
        X = np.asarray(X, np.float64)
    y = np.asarray(y)
    yf = y.astype(np.float64)
    n, q = X.shape

    if x0 is None:
        x = np.zeros(n)
    else:
        x, _, _ = project_svm(np.asarray(x0, np.float64), y, C)
    omega = atmul(X, y, x)
    sigma = opt.sigma0
    inner_total = 0
    cg_total = 0
    ls_fail = 0
    ls_trials = 0
    grad_steps = 0
    hist = []
    status = "MAXITER"
    R, b = math.inf, float("nan")
    best = None                  # (R, x, b): returned if the cap is hit
    outer = 0
    for k in range(opt.max_outer):
        outer = k + 1
        eps_k = opt.eps_decay ** k
        Aomega = amul(X, y, omega)
        xk = x
        if opt.time_budget_s > 0 and time.perf_counter() - t_start > opt.time_budget_s:
            status = "BUDGET"
            break
        for j in range(opt.max_inner):
            if opt.time_budget_s > 0 and time.perf_counter() - t_start > opt.time_budget_s:
                status = "BUDGET"
                break
            u = xk + sigma * (1.0 - Aomega)
            xt, lam, free = project_svm(u, y, C)
            g = omega - atmul(X, y, xt)
            gn = float(np.linalg.norm(g))
            crit = min(eps_k, eps_k * float(np.linalg.norm(xt - xk))) / math.sqrt(sigma)
            if gn <= max(crit, opt.floor * (1.0 + float(np.linalg.norm(omega)))):
                break
            # Step 1: Newton direction
            if opt.newton == "qspace":
                d = newton_qspace(X, free, g, sigma)
            elif opt.newton == "pspace":
                d = newton_pspace_centered(X, free, g, sigma)
            else:
                cg_tol = min(opt.eta, gn ** (1.0 + opt.tau))
                d, it = newton_pcg(X, free, g, sigma, cg_tol, opt.max_cg)
                cg_total += it
            inner_total += 1
            # Step 2: Armijo line search on psi.  Reading: a direction that
            # is not one of descent (possible only when the linear system is
            # solved inexactly) can never pass the Armijo test on the convex
            # psi, so the steepest-descent direction -g replaces it.
            t = amul(X, y, d)
            gd = float(g @ d)
            if not gd < 0.0 and gn > 0.0:
                d = -g
                t = amul(X, y, d)
                gd = float(g @ d)
                grad_steps += 1
            accepted = False
            alpha = 1.0
            for m in range(opt.max_backtracks + 1):
                alpha = opt.ls_delta ** m
                ls_trials += 1
                u_a = u - alpha * sigma * t
                _, lam_a, _ = project_svm(u_a, y, C)
                dpsi = psi_increment(omega, d, alpha, u, lam, u_a, lam_a, sigma, y, C)
                if dpsi <= opt.mu * alpha * gd:
                    accepted = True
                    break
            if not accepted:
                ls_fail += 1
                break
            # Step 3
            omega = omega + alpha * d
            Aomega = amul(X, y, omega)
        if status == "BUDGET":
            x = xk
            break
        # Step 2 of Algorithm 1
        u = xk + sigma * (1.0 - Aomega)
        x, _, free = project_svm(u, y, C)
        R, b = rkkt(X, y, C, x)
        if opt.record:
            hist.append({"k": k, "sigma": sigma, "rkkt": R, "inner": inner_total,
                         "p": int(free.sum())})
        if R <= opt.tol:
            status = "OK"
            break
        if best is None or R < best[0]:
            best = (R, x.copy(), b)
        sigma = min(opt.rho * sigma, opt.sigma_max)
    if status == "MAXITER" and best is not None and best[0] < R:
        R, x, b = best

    w = atmul(X, y, x)
    t_i = x  # free set at the returned x: 0 < x_i < C
    p = int(np.sum((t_i > 0.0) & (t_i < C)))
    return Result(x=x, w=w, b=b, obj=dual_objective(X, y, x), rkkt=R, outer=outer,
                  inner=inner_total, p=p, n_sv=int(np.sum(x > 0.0)), status=status,
                  sigma=sigma, omega=omega, history=hist,
                  time_s=time.perf_counter() - t_start, cg_iters=cg_total,
                  ls_fail=ls_fail, ls_trials=ls_trials, grad_steps=grad_steps)
