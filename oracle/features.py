"""CPU FP64 oracle of the two kernel approximations of Section 4 that turn the
RBF-kernel C-SVC into a linear one (Tables 3_1 and 3_2).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.

RBF kernel (Section 1): k(x, y) = exp(-|x - y|^2 / (2 alpha)), alpha > 0.

Random Fourier features: by Bochner's theorem k is the Fourier transform of
the Gaussian density with covariance I / alpha; with N frequencies drawn from
it, row i of Z is [cos(w_1^T x_i), sin(w_1^T x_i), ..., cos(w_N^T x_i),
sin(w_N^T x_i)] (n x 2N, pairs interleaved as in the paper) and K ~ Z Z^T / N.

Nystroem: with landmark set I (r points), K ~ K_nr (K_rr + s I)^{-1} K_nr^T,
s = 1e-3 as in the paper; as features, Z = K_nr L^{-T} with
K_rr + s I = L L^T, so that Z Z^T is that approximation.

Either Z then replaces X in the linear C-SVC (the paper's R_KKT with Q
replaced by its approximation is the linear problem's R_KKT with X = Z).

Readings: the frequencies (and the landmark indices) are inputs, drawn by the
caller's seeded generator; the 1/N of the sample average is folded into Z as
a factor 1/sqrt(N) so that Z Z^T itself is the estimate; the paper picks
landmarks by k-means, a heuristic this oracle leaves to the caller.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def rbf_kernel(X, Y, alpha):
    """K_ij = exp(-|x_i - y_j|^2 / (2 alpha))."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    d2 = (X * X).sum(1)[:, None] + (Y * Y).sum(1)[None, :] - 2.0 * X @ Y.T
    return np.exp(-np.maximum(d2, 0.0) / (2.0 * alpha))


def rff_frequencies(rng, N, q, alpha):
    """N frequencies from the density with covariance I / alpha (q columns)."""
    return rng.standard_normal((N, q)) / np.sqrt(alpha)


def rff_features(X, W):
    """Z (n x 2N): cos / sin pairs of W x_i, scaled by 1/sqrt(N)."""
    X = np.asarray(X, np.float64)
    P = X @ np.asarray(W, np.float64).T            # n x N
    N = P.shape[1]
    Z = np.empty((X.shape[0], 2 * N))
    Z[:, 0::2] = np.cos(P)
    Z[:, 1::2] = np.sin(P)
    return Z / np.sqrt(N)


def nystroem_features(X, landmarks, alpha, shift=1e-3):
    """Z (n x r) with Z Z^T = K_nr (K_rr + shift I)^{-1} K_nr^T."""
    X = np.asarray(X, np.float64)
    L_pts = X[np.asarray(landmarks)]
    Knr = rbf_kernel(X, L_pts, alpha)
    Krr = rbf_kernel(L_pts, L_pts, alpha) + shift * np.eye(L_pts.shape[0])
    L = sla.cholesky(Krr, lower=True)
    return sla.solve_triangular(L, Knr.T, lower=True).T
