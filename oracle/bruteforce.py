"""Brute-force references for tiny C-SVC duals and projections.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

`qp_by_enumeration` enumerates all 3^n partitions (lower / free / upper) of
the dual QP of eq. Def_Dual_of_C_SVM_Problem and keeps the partitions whose
KKT system (stationarity on the free set, y^T x = 0, sign conditions on the
reduced costs of the bound sets) has a solution.  Every KKT point of a convex
QP is optimal, so all survivors share the optimal value f*.

`projection_by_enumeration` does the same for the projection problem
eq. Def proj_KL001 with a = y, d = 0, l = 0, u = C.

`general_qp_by_enumeration` does the same for the unified problem (P)
(eq. Problem_P1_classical1) with general Q, c, a, d, l, u.
"""
from __future__ import annotations

import itertools

import numpy as np


def qp_by_enumeration(X, y, C, tol=1e-9):
    """Returns (f_star, x_star, b_star_or_None) for min 1/2 x^T Q x - e^T x,
    y^T x = 0, 0 <= x <= C with Q = A A^T, A = diag(y) X.  n <= 10."""
    X = np.asarray(X, np.float64)
    yf = np.asarray(y, np.float64)
    n = X.shape[0]
    A = yf[:, None] * X
    Q = A @ A.T
    best = None
    for lab in itertools.product((0, 1, 2), repeat=n):   # 0 lower, 1 free, 2 upper
        lab = np.array(lab)
        F = np.flatnonzero(lab == 1)
        U = np.flatnonzero(lab == 2)
        L = np.flatnonzero(lab == 0)
        x = np.zeros(n)
        x[U] = C
        if F.size == 0:
            if abs(float(yf[U].sum()) * C) > tol:
                continue
            # b-interval from r_L >= 0, r_U <= 0, r = Qx - 1 + b y
            base = Q @ x - 1.0
            lo, hi = -np.inf, np.inf
            for i in L:
                # base_i + b y_i >= 0
                if yf[i] > 0:
                    lo = max(lo, -base[i])
                else:
                    hi = min(hi, base[i])
            for i in U:
                # base_i + b y_i <= 0
                if yf[i] > 0:
                    hi = min(hi, -base[i])
                else:
                    lo = max(lo, base[i])
            if lo > hi + tol:
                continue
            b = None
            f = 0.5 * x @ Q @ x - x.sum()
            cand = (f, x.copy(), b)
        else:
            m = F.size
            K = np.zeros((m + 1, m + 1))
            K[:m, :m] = Q[np.ix_(F, F)]
            K[:m, m] = yf[F]
            K[m, :m] = yf[F]
            rhs = np.zeros(m + 1)
            rhs[:m] = 1.0 - C * Q[np.ix_(F, U)].sum(axis=1)
            rhs[m] = -C * yf[U].sum()
            sol, *_ = np.linalg.lstsq(K, rhs, rcond=None)
            if np.linalg.norm(K @ sol - rhs) > tol * (1.0 + np.linalg.norm(rhs)):
                continue
            xF, b = sol[:m], sol[m]
            if np.any(xF < -tol) or np.any(xF > C + tol):
                continue
            x[F] = np.clip(xF, 0.0, C)
            r = Q @ x - 1.0 + b * yf
            if np.any(r[L] < -tol * 10) or np.any(r[U] > tol * 10):
                continue
            f = 0.5 * x @ Q @ x - x.sum()
            cand = (f, x.copy(), float(b))
        if best is None or cand[0] < best[0] - 1e-12:
            best = cand
    return best


def projection_by_enumeration(v, y, C, tol=1e-12):
    """Pi onto {y^T x = 0, 0 <= x <= C} by enumerating the 3^n partitions of
    the KKT system x = clip(v - lam y); the valid partition gives lam by one
    linear equation.  n <= 12."""
    v = np.asarray(v, np.float64)
    yf = np.asarray(y, np.float64)
    n = v.size
    best = None
    for lab in itertools.product((0, 1, 2), repeat=n):
        lab = np.array(lab)
        F = lab == 1
        U = lab == 2
        # y^T x = sum_F y_i (v_i - lam y_i) + C sum_U y_i = 0
        cnt = F.sum()
        rhs = float(yf[F] @ v[F]) + C * float(yf[U].sum())
        if cnt == 0:
            if abs(rhs) > tol * (1 + C * n):
                continue
            lams = [None]
        else:
            lams = [rhs / cnt]
        for lam in lams:
            if lam is None:
                # any lam consistent with the signs; check via interval
                lo, hi = -np.inf, np.inf
                for i in range(n):
                    # need v_i - lam y_i <= 0 for lower, >= C for upper
                    if lab[i] == 0:
                        if yf[i] > 0:
                            lo = max(lo, v[i])
                        else:
                            hi = min(hi, -v[i])
                    else:
                        if yf[i] > 0:
                            hi = min(hi, v[i] - C)
                        else:
                            lo = max(lo, C - v[i])
                if lo > hi + tol:
                    continue
                lam = lo if np.isfinite(lo) else hi
            t = v - lam * yf
            ok = np.all(t[lab == 0] <= tol) and np.all(t[U] >= C - tol) and \
                np.all((t[F] > -tol) & (t[F] < C + tol))
            if not ok:
                continue
            x = np.clip(t, 0.0, C)
            dist = float(np.sum((x - v) ** 2))
            if best is None or dist < best[0] - 1e-14:
                best = (dist, x, lam)
    return best[1], best[2]


def general_qp_by_enumeration(Q, c, a, d, l, u, tol=1e-9):
    """Returns (f_star, x_star) for the unified problem (P) of Section 1:
    min 1/2 x^T Q x + c^T x, a^T x = d, l <= x <= u, by enumerating the 3^n
    partitions into lower / free / upper and keeping the candidates that
    satisfy the KKT conditions (r = Q x + c - mu a: r_i >= 0 at a lower
    bound, <= 0 at an upper bound, = 0 when free).  n <= 8."""
    Q = np.asarray(Q, np.float64)
    c = np.asarray(c, np.float64)
    a = np.asarray(a, np.float64)
    l = np.asarray(l, np.float64)
    u = np.asarray(u, np.float64)
    n = c.size
    best = None
    for lab in itertools.product((0, 1, 2), repeat=n):
        lab = np.array(lab)
        F = np.flatnonzero(lab == 1)
        L = np.flatnonzero(lab == 0)
        U = np.flatnonzero(lab == 2)
        x = np.where(lab == 2, u, l).astype(np.float64)
        x[F] = 0.0
        fixed = np.concatenate([L, U])
        if F.size == 0:
            if abs(float(a @ x) - d) > tol * (1.0 + abs(d)):
                continue
            base = Q @ x + c
            lo, hi = -np.inf, np.inf
            ok = True
            for i in L:                       # base_i - mu a_i >= 0
                if a[i] > 0:
                    hi = min(hi, base[i] / a[i])
                elif a[i] < 0:
                    lo = max(lo, base[i] / a[i])
                elif base[i] < -tol:
                    ok = False
            for i in U:                       # base_i - mu a_i <= 0
                if a[i] > 0:
                    lo = max(lo, base[i] / a[i])
                elif a[i] < 0:
                    hi = min(hi, base[i] / a[i])
                elif base[i] > tol:
                    ok = False
            if not ok or lo > hi + tol:
                continue
        else:
            m = F.size
            K = np.zeros((m + 1, m + 1))
            K[:m, :m] = Q[np.ix_(F, F)]
            K[:m, m] = -a[F]
            K[m, :m] = a[F]
            rhs = np.zeros(m + 1)
            rhs[:m] = -c[F] - Q[np.ix_(F, fixed)] @ x[fixed]
            rhs[m] = d - float(a[fixed] @ x[fixed])
            sol, *_ = np.linalg.lstsq(K, rhs, rcond=None)
            if np.linalg.norm(K @ sol - rhs) > tol * (1.0 + np.linalg.norm(rhs)):
                continue
            xF, mu = sol[:m], sol[m]
            if np.any(xF < l[F] - tol) or np.any(xF > u[F] + tol):
                continue
            x[F] = np.clip(xF, l[F], u[F])
            r = Q @ x + c - mu * a
            if np.any(r[L] < -10 * tol) or np.any(r[U] > 10 * tol):
                continue
        f = 0.5 * float(x @ Q @ x) + float(c @ x)
        if best is None or f < best[0] - 1e-12:
            best = (f, x.copy())
    return best
