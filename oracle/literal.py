"""The paper's Newton system in its original n-space form, for tiny checks.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

These functions work with the dual variable w in R^n and the explicit
Q = A A^T (dense, so n must be small).  They let the tests compare the
omega-space solver in `ssnal` against
  * the n-space Newton system (Q + sigma Q P Q) d = -grad psi(w), d in Ran(Q)
    (eq. Newton system 1, Section 3.2.4), solved in the minimum-norm sense;
  * Proposition 5 (a)/(b) as printed: the p x p system eq. Def_small_linear_eq
    (or Def_small_linear_eq_s) and the formulas eq. Def_Qd_start1 / Def_dQd
    for Q d and d^T Q d.
"""
from __future__ import annotations

import numpy as np

from .projection import hs_jacobian, project_svm


def state_nspace(X, y, w, xk, sigma, C):
    """u(w) = x^k - sigma (Q w + c) with c = -e; Pi(u); free set; grad psi."""
    yf = np.asarray(y, np.float64)
    A = yf[:, None] * np.asarray(X, np.float64)
    Q = A @ A.T
    u = xk - sigma * (Q @ w - 1.0)
    xt, lam, free = project_svm(u, y, C)
    grad = Q @ w - Q @ xt
    return Q, u, xt, free, grad


def newton_nspace(X, y, w, xk, sigma, C):
    """Minimum-norm solution d of (Q + sigma Q P Q) d = -grad psi(w)."""
    Q, u, xt, free, grad = state_nspace(X, y, w, xk, sigma, C)
    P = hs_jacobian(free, np.asarray(y, np.float64))
    M = Q + sigma * Q @ P @ Q
    d = np.linalg.pinv(M, rcond=1e-12, hermitian=True) @ (-grad)
    return d, Q


def prop5_paper(X, y, w, xk, sigma, C):
    """Q d and d^T Q d by Proposition 5 exactly as printed.
    Returns (Qd, dQd, case) with case 'a' (a^T Sigma a != 0) or 'b'."""
    yf = np.asarray(y, np.float64)
    Q, u, xt, free, grad = state_nspace(X, y, w, xk, sigma, C)
    J = np.flatnonzero(free)
    s = w - xt                                  # s(w) = w - Pi(u(w))
    sQs = float(s @ Q @ s)
    if J.size == 0:
        # case (b): Sigma a = 0, v_J empty
        return -grad, sQs, "b"
    QJ = Q[J, :]
    QJJ = Q[np.ix_(J, J)]
    aJ = yf[J]
    gJ = grad[J]
    p = J.size
    den = float(aJ @ aJ - sigma * aJ @ QJJ @ aJ)
    QJJa = QJJ @ aJ
    lhs = np.eye(p) / sigma + QJJ + sigma * np.outer(QJJa, QJJa) / den
    rhs = (np.eye(p) + sigma * np.outer(QJJa, aJ) / den) @ gJ
    vJ = np.linalg.solve(lhs, rhs)
    coef = float(aJ @ QJJ @ vJ - aJ @ gJ)
    Qd = QJ.T @ vJ - grad + sigma * coef / den * (QJ.T @ aJ)
    dQd = (float(vJ @ QJJ @ vJ) - 2.0 * float(vJ @ gJ) + sQs
           + (2.0 * sigma * float(aJ @ aJ) - sigma ** 2 * float(aJ @ QJJ @ aJ)) / den ** 2 * coef ** 2)
    return Qd, dQd, "a"
