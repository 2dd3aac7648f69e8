"""CPU FP64 oracle: Euclidean projection onto K ∩ L and its HS-Jacobian.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

K = {l <= x <= u}, L = {a^T x = d}  (Section 3.2.1, problem "Def proj_KL001").
The projection is Pi_K(v - lam*a) where lam is the zero of the nondecreasing
piecewise-linear function grad_phi(lam) = -a^T Pi_K(v - lam*a) + d, whose
breakpoints are (v_i - u_i)/a_i and (v_i - l_i)/a_i.  lam is the smallest
zero, the value Algorithm 2 returns: the breakpoints are sorted, the function
is evaluated at all of them by one sweep of running intercept and slope
sums, and the zero is interpolated linearly inside the first bracket where
its sign changes.

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
    """Smallest zero of grad_phi, located among the sorted breakpoints.

    grad_phi is continuous, nondecreasing and linear between consecutive
    breakpoints (Section 3.2.1).  Each component i with a_i != 0 is free
    (l_i < v_i - lam a_i < u_i) for lam between its two breakpoints
    e_i = min((v_i - u_i)/a_i, (v_i - l_i)/a_i) and f_i = max(...), and
    sits at a bound outside: for lam < e_i at u_i if a_i > 0 (else l_i), for
    lam > f_i at l_i if a_i > 0 (else u_i).  So a^T Pi_K(v - lam a) =
    c0 + c1 lam with an intercept c0 and a slope c1 that change only at
    breakpoints: entering the free range swaps a_i * bound for a_i v_i in c0
    and adds -a_i^2 to c1, leaving it does the reverse with the other bound.
    Sweeping the sorted breakpoints with running sums of those changes gives
    grad_phi at every breakpoint; the first breakpoint where it is >= 0
    closes the bracket, and the zero is the linear interpolation inside it
    (the value Algorithm 2 returns).  The bracket ends are then evaluated
    again directly from the definition (grad_phi), and the bracket moved if
    the running sums' rounding misplaced it, so the result depends only on
    the definition at two points.

    Degenerate ends (grad_phi >= 0 already at the first breakpoint, or < 0 at
    the last one) return that end breakpoint; they do not occur for feasible
    C-SVC data with both classes present.  Components with a_i = 0 contribute
    a constant and have no breakpoints.
    """
    v = np.asarray(v, np.float64)
    a = np.asarray(a, np.float64)
    l = np.broadcast_to(np.asarray(l, np.float64), v.shape)
    u = np.broadcast_to(np.asarray(u, np.float64), v.shape)
    nz = a != 0
    vz, az, lz, uz = v[nz], a[nz], l[nz], u[nz]
    b_u, b_l = (vz - uz) / az, (vz - lz) / az
    e = np.minimum(b_u, b_l)                      # enters the free range
    f = np.maximum(b_u, b_l)                      # leaves it
    left = np.where(az > 0, uz, lz)               # bound held for lam < e
    right = np.where(az > 0, lz, uz)              # bound held for lam > f
    m = 2 * vz.size
    if m == 0:
        return 0.0
    T = np.concatenate([e, f])
    d0 = np.concatenate([az * vz - az * left, az * right - az * vz])   # change of c0
    d1 = np.concatenate([-az * az, az * az])                            # change of c1
    order = np.argsort(T, kind="stable")
    T, d0, d1 = T[order], d0[order], d1[order]
    # a^T Pi_K at lam just left of the first breakpoint, plus the a_i = 0 part
    c0 = float(np.sum(az * left)) + float(np.dot(a[~nz], clip_box(v[~nz], l[~nz], u[~nz])))
    # values at each breakpoint (continuity: either side's line gives it)
    c0_run = c0 + np.cumsum(d0)
    c1_run = np.cumsum(d1)
    h = -(c0_run + c1_run * T) + d
    k = int(np.searchsorted(h >= 0.0, True))      # first index with h >= 0 (h is monotone)

    def g(i):
        return grad_phi(T[i], v, a, l, u, d)

    # confirm the bracket with the definition
    k = min(k, m)
    while k < m and g(k) < 0.0:
        k += 1
    while k > 0 and g(k - 1) >= 0.0:
        k -= 1
    if k == 0:
        return float(T[0])
    if k == m:
        return float(T[-1])
    fl, fu = g(k - 1), g(k)
    return float(T[k - 1] - fl / (fu - fl) * (T[k] - T[k - 1]))


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
