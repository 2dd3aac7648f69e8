"""CPU FP64 oracle of the C-SVC dual with a nonlinear kernel (Section 1,
eq. Def_Dual_of_C_SVM_Problem with Q_ij = y_i y_j k(x_i, x_j)), the problem
of Table 3.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

Q is formed explicitly (small n only) and factored as Q = B B^T from its
eigendecomposition (eigenvalues below zero by rounding are set to zero);
the unified-form oracle then runs Algorithms 1 and 3 on it.  For w in Ran(Q)
the omega-space iterates (omega = B^T w) are those of the w-space method the
paper states, so this is the method itself on the kernel problem; what a GPU
path would add is forming the rows of Q_J from kernel evaluations on demand
(Proposition 5) instead of holding Q.
"""
from __future__ import annotations

import numpy as np

from . import general


def kernel_q(K, y):
    """Q = diag(y) K diag(y)."""
    yf = np.asarray(y, np.float64)
    return yf[:, None] * np.asarray(K, np.float64) * yf[None, :]


def factor(Q):
    """B with B B^T = Q (PSD part of the symmetric Q)."""
    lam, V = np.linalg.eigh(0.5 * (Q + Q.T))
    return V * np.sqrt(np.maximum(lam, 0.0))[None, :]


def kernel_problem(K, y, C):
    yf = np.asarray(y, np.float64)
    n = yf.size
    return general.Problem(B=factor(kernel_q(K, y)), c=-np.ones(n), a=yf.copy(), d=0.0,
                           l=np.zeros(n), u=np.full(n, float(C)))


def solve(K, y, C, tol=1e-6, **kw):
    """SSsNAL on the kernel C-SVC dual; returns the unified-form result."""
    return general.solve(kernel_problem(K, y, C), tol=tol, **kw)
