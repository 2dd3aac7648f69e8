"""CPU FP64 oracle of the C-SVC dual with a nonlinear kernel (Section 1,
eq. Def_Dual_of_C_SVM_Problem with Q_ij = y_i y_j k(x_i, x_j)), the problem
of Table 3.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

Two formulations of the same method:

* `solve`: Q is formed explicitly (small n only) and factored as Q = B B^T
  from its eigendecomposition (eigenvalues below zero by rounding are set to
  zero); the unified-form oracle then runs Algorithms 1 and 3 on it in
  omega-space (omega = B^T w).  For w in Ran(Q) these are the iterates of
  the w-space method the paper states.

* `solve_p5`: the method in the paper's own variable w in R^n, with Q used
  only through products and through Q_JJ, the Newton step taken by the
  p x p system of Proposition 5 (`newton_pspace`).  Inner products of the
  omega-space method become Q-inner products (|omega|^2 = w^T Q w,
  |grad|^2 = s^T Q s with s = w - Pi(u(w))), so both formulations take the
  same decisions; the tests pin one against the other.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import general
from .ssnal import Options


def kernel_q(K, y):
    """Q = diag(y) K diag(y)."""
    yf = np.asarray(y, np.float64)
    return yf[:, None] * np.asarray(K, np.float64) * yf[None, :]


def factor(Q):
    """B with B B^T = Q (PSD part of the symmetric Q)."""
    lam, V = np.linalg.eigh(0.5 * (Q + Q.T))
    return V * np.sqrt(np.maximum(lam, 0.0))[None, :]


def box_problem(y, C):
    """The constraints of the C-SVC dual, y^T x = 0, 0 <= x <= C, with c = -e
    (B is not needed by the projection)."""
    yf = np.asarray(y, np.float64)
    n = yf.size
    return general.Problem(B=None, c=-np.ones(n), a=yf.copy(), d=0.0,
                           l=np.zeros(n), u=np.full(n, float(C)))


def kernel_problem(K, y, C):
    prob = box_problem(y, C)
    prob.B = factor(kernel_q(K, y))
    return prob


def solve(K, y, C, tol=1e-6, **kw):
    """SSsNAL on the kernel C-SVC dual (omega-space, through the factor of Q);
    returns the unified-form result."""
    return general.solve(kernel_problem(K, y, C), tol=tol, **kw)


# --------------------------------------------------------------------------
# w-space formulation (Proposition 5)
# --------------------------------------------------------------------------

def newton_pspace(Q, a, free, s, sigma):
    """Newton step of Algorithm 3 for (Q + sigma Q P Q) d = -grad psi(w),
    grad psi(w) = Q s, d in Ran(Q) (eq. Newton system 1), through a p x p
    system on the free set J (Proposition 5).

    With Q = L L^T and P of Theorem 3.1, P restricted to J is the projector
    Pi = I_p - a_J a_J^T / (a_J^T a_J) (Pi = I_p when a_J = 0, part (b)).
    Then L^T d = -(I + sigma G^T G)^{-1} L^T s with G = Pi L_J, and the
    Woodbury identity gives
        (I_p + sigma Pi Q_JJ Pi) v = Pi g_J,   g = Q s,
        z = sigma Pi v,   L^T d = -L^T s + L_J^T z,
    so one representative of d is -s + E_J z (E_J: zero-fill from J) and
        Q d     = -g + Q_{:,J} z,
        d^T Q d = s^T Q s - 2 z^T g_J + z^T Q_JJ z.
    This is the solution of Proposition 5 (eq. Def_small_linear_eq and
    eq. Def_Qd_start1 apply Sherman-Morrison to the rank-one part instead of
    keeping the projector inside; the p x p matrix here is symmetric
    positive definite for every sigma > 0).

    Returns (d, Qd, dQd)."""
    Q = np.asarray(Q, np.float64)
    a = np.asarray(a, np.float64)
    s = np.asarray(s, np.float64)
    g = Q @ s
    J = np.flatnonzero(free)
    if J.size == 0:
        return -s, -g, float(s @ g)
    aJ = a[J]
    QJJ = Q[np.ix_(J, J)]
    p = J.size
    den = float(aJ @ aJ)

    def proj(V):
        # Pi V with Pi = I - a_J a_J^T / den applied as a rank-one update
        if den == 0.0:
            return V
        return V - np.multiply.outer(aJ, aJ @ V) / den

    PQP = proj(proj(QJJ).T).T                  # Pi Q_JJ Pi (Pi symmetric)
    M = np.eye(p) + sigma * PQP
    v = sla.cho_solve(sla.cho_factor(M, lower=True), proj(g[J]))
    z = sigma * proj(v)
    d = -s.copy()
    d[J] += z
    Qd = -g + Q[:, J] @ z
    dQd = float(s @ g) - 2.0 * float(z @ g[J]) + float(z @ QJJ @ z)
    return d, Qd, dQd


def objective_q(Q, x):
    """1/2 x^T Q x - e^T x."""
    return 0.5 * float(x @ Q @ x) - float(np.sum(x))


def rkkt_q(Q, y, C, x):
    """eq. Def_Rkkt with c = -e: |x - Pi(x - Q x + e)| / (1 + |x|).  Returns
    (R, lam) with lam the lam_hat of that projection (the bias reading)."""
    v = x - Q @ x + 1.0
    px, lam, _ = general.projection(box_problem(y, C), v)
    return float(np.linalg.norm(x - px) / (1.0 + np.linalg.norm(x))), lam


def duality_gap_at_q(Q, y, C, x, b):
    """Relative gap of the kernel C-SVC (eq. Def_C_SVM_Problem in the feature
    space): the primal at the expansion w = sum_i x_i y_i phi(x_i) and bias b
    is 1/2 x^T Q x + C sum_i max(0, 1 - (Q x)_i - y_i b), since
    y_i (w . phi(x_i) + b) = (Q x)_i + y_i b.  Returns (gap, P, f)."""
    yf = np.asarray(y, np.float64)
    Qx = Q @ x
    P = 0.5 * float(x @ Qx) + C * float(np.sum(np.maximum(0.0, 1.0 - Qx - yf * b)))
    f = 0.5 * float(x @ Qx) - float(np.sum(x))
    return (P + f) / (1.0 + abs(P) + abs(f)), P, f


def solve_p5(K, y, C, tol=1e-6, x0=None, **kw):
    """SSsNAL (Algorithm 1 + Algorithm 3) on the kernel C-SVC dual in w-space
    with the Newton step of `newton_pspace`.  Parameters as `ssnal.Options`
    (direct solves only; time_budget_s > 0 stops with status "BUDGET").
    Returns a `general.Result` (omega holds w)."""
    import time
    t_start = time.perf_counter()
    opt = Options(tol=tol, **kw)
    Q = kernel_q(K, y)
    prob = box_problem(y, C)
    a, c = prob.a, prob.c
    n = a.size
    x = np.zeros(n) if x0 is None else general.projection(prob, np.asarray(x0, np.float64))[0]
    w = x.copy()                      # omega^0 = B^T x^0 is w^0 = x^0
    sigma = opt.sigma0
    inner_total = 0
    status = "MAXITER"
    R = math.inf
    best = None
    outer = 0
    def over_budget():
        return opt.time_budget_s > 0 and time.perf_counter() - t_start > opt.time_budget_s

    for k in range(opt.max_outer):
        outer = k + 1
        eps_k = opt.eps_decay ** k
        Qw = Q @ w
        xk = x
        if over_budget():
            status = "BUDGET"
            break
        for _ in range(opt.max_inner):
            if over_budget():
                status = "BUDGET"
                break
            u = xk - sigma * (Qw + c)
            xt, lam, free = general.projection(prob, u)
            s = w - xt
            g = Q @ s
            gn = math.sqrt(max(float(s @ g), 0.0))
            crit = min(eps_k, eps_k * float(np.linalg.norm(xt - xk))) / math.sqrt(sigma)
            wn = math.sqrt(max(float(w @ Qw), 0.0))
            if gn <= max(crit, opt.floor * (1.0 + wn)):
                break
            d, Qd, dQd = newton_pspace(Q, a, free, s, sigma)
            inner_total += 1
            gd = float(d @ g)                 # <grad, d> in omega-space: s^T Q d
            od = float(w @ Qd)                # <omega, d>: w^T Q d
            accepted = False
            alpha = 1.0
            t = u - lam * a
            for m in range(opt.max_backtracks + 1):
                alpha = opt.ls_delta ** m
                u_a = u - alpha * sigma * Qd
                _, lam_a, _ = general.projection(prob, u_a)
                dt = (u_a - u) - (lam_a - lam) * a
                dh = float(np.sum(general.h_increment(t, dt, prob.l, prob.u))) + (lam_a - lam) * prob.d
                dpsi = alpha * od + 0.5 * alpha * alpha * dQd + dh / sigma
                if dpsi <= opt.mu * alpha * gd:
                    accepted = True
                    break
            if not accepted:
                break
            w = w + alpha * d
            Qw = Q @ w
        if status == "BUDGET":
            x = xk
            break
        u = xk - sigma * (Qw + c)
        x = general.projection(prob, u)[0]
        R = rkkt_q(Q, y, C, x)[0]
        if R <= opt.tol:
            status = "OK"
            break
        if best is None or R < best[0]:
            best = (R, x.copy())
        sigma = min(opt.rho * sigma, opt.sigma_max)
    if status == "MAXITER" and best is not None and best[0] < R:
        R, x = best
    return general.Result(x=x, omega=w, obj=objective_q(Q, x), rkkt=R, outer=outer,
                          inner=inner_total, status=status, cg_iters=0,
                          time_s=time.perf_counter() - t_start)
