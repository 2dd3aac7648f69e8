"""CPU FP64 oracle: Euclidean projection onto K ∩ L and its HS-Jacobian.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

K = {l <= x <= u}, L = {a^T x = d}  (Section 3.2.1, problem "Def proj_KL001").
The projection is Pi_K(v - lam*a) where lam is the zero of the nondecreasing
piecewise-linear function grad_phi(lam) = -a^T Pi_K(v - lam*a) + d, whose
breakpoints are (v_i - u_i)/a_i and (v_i - l_i)/a_i.  lam is found by the
breakpoint search of Algorithm 2 (sort the 2n breakpoints, bisect on their
index, interpolate linearly inside the final bracket).

Readings taken where the paper is silent:
  * `[.]` in Algorithm 2 is the floor.
  * Components with a_i = 0 have no breakpoints; they are excluded from the
    breakpoint set and clipped directly (never the case for C-SVC, a = y).
  * The free index set J of Theorem 3.1 / Proposition 5 is the strict
    interior l_i < v_i - lam*a_i < u_i: a component exactly at a bound
    counts as active (the active set I(v) is defined by equality).
"""
from __future__ import annotations

import numpy as np


def clip_box(t, l, u):
    """Pi_[l,u] componentwise (Section 3.2.1, final display)."""
    return np.minimum(np.maximum(t, l), u)


def grad_phi(lam, v, a, l, u, d):
    """grad phi(lam) = -a^T Pi_K(v - lam a) + d (Section 3.2.1)."""
    return -float(np.dot(a, clip_box(v - lam * a, l, u))) + d


def breakpoint_search(v, a, l, u, d=0.0):
    """Algorithm 2: zero of grad_phi by binary search over sorted breakpoints.

    Returns lam_hat.  Degenerate ends (root left of the first breakpoint or
    right of the last one) return that end breakpoint; they do not occur for
    feasible C-SVC data with both classes present.
    """
    v = np.asarray(v, np.float64)
    a = np.asarray(a, np.float64)
    l = np.broadcast_to(np.asarray(l, np.float64), v.shape)
    u = np.broadcast_to(np.asarray(u, np.float64), v.shape)
    nz = a != 0
    T = np.sort(np.concatenate([(v[nz] - u[nz]) / a[nz], (v[nz] - l[nz]) / a[nz]]))
    m = T.size
    if m == 0:
        return 0.0
    Il, Iu = 0, m - 1
    fl = grad_phi(T[Il], v, a, l, u, d)
    fu = grad_phi(T[Iu], v, a, l, u, d)
    if fl >= 0.0:
        return float(T[0])
    if fu < 0.0:
        return float(T[-1])
    while Iu - Il > 1 and T[Iu] > T[Il]:
        Im = (Il + Iu) // 2
        fm = grad_phi(T[Im], v, a, l, u, d)
        if fm >= 0.0:
            Iu, fu = Im, fm
        else:
            Il, fl = Im, fm
    if fu == 0.0 and fl == 0.0:
        return float(T[Il])
    return float(T[Il] - fl / (fu - fl) * (T[Iu] - T[Il]))


def project(v, a, l, u, d=0.0):
    """Pi_{K∩L}(v) = Pi_K(v - lam_hat*a).  Returns (x, lam_hat)."""
    lam = breakpoint_search(v, a, l, u, d)
    x = clip_box(np.asarray(v, np.float64) - lam * np.asarray(a, np.float64), l, u)
    return x, lam


def project_svm(v, y, C):
    """Projection onto {y^T x = 0, 0 <= x <= C} (a = y, d = 0, l = 0, u = C).
    Returns (x, lam_hat, free_mask) with free_mask the strict interior set J."""
    yf = np.asarray(y, np.float64)
    x, lam = project(v, yf, 0.0, C, 0.0)
    t = np.asarray(v, np.float64) - lam * yf
    free = (t > 0.0) & (t < C)
    return x, lam, free


def hs_jacobian(free, a):
    """The HS-Jacobian element of Theorem 3.1 (eq. Def_HS_P) as a dense matrix.

    Sigma = diag(free); P = Sigma (I - a a^T / (a^T Sigma a)) Sigma when
    a^T Sigma a != 0, else Sigma.  Dense: for small-n checks only.
    """
    Sig = np.diag(np.asarray(free, np.float64))
    a = np.asarray(a, np.float64)
    den = float(a @ Sig @ a)
    if den != 0.0:
        n = a.size
        return Sig @ (np.eye(n) - np.outer(a, a) / den) @ Sig
    return Sig
