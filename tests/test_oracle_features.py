"""Pins of the kernel approximations of Section 4 (random Fourier features and
Nystroem) that turn the RBF C-SVC into a linear one: exact identities
(diag of the RFF estimate is 1, a Nystroem approximation with every point as
a landmark and no shift reproduces K), the Monte Carlo convergence of the RFF
estimate, and the linear C-SVC oracle on the features against brute force."""
import numpy as np
import pytest

from oracle import bruteforce, features, ssnal


def test_rbf_kernel_closed_forms():
    alpha = 0.7
    X = np.array([[0.0, 0.0], [np.sqrt(2 * alpha), 0.0], [0.0, 2.0 * np.sqrt(alpha)]])
    K = features.rbf_kernel(X, X, alpha)
    np.testing.assert_allclose(np.diag(K), 1.0, rtol=0, atol=1e-15)
    assert K[0, 1] == pytest.approx(np.exp(-1.0), rel=1e-14)      # |x-y|^2 = 2 alpha
    assert K[0, 2] == pytest.approx(np.exp(-2.0), rel=1e-14)      # |x-y|^2 = 4 alpha
    np.testing.assert_allclose(K, K.T, rtol=0, atol=0)


def test_rff_diagonal_is_exact():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 5))
    W = features.rff_frequencies(rng, 64, 5, alpha=2.0)
    Z = features.rff_features(X, W)
    assert Z.shape == (30, 128)
    np.testing.assert_allclose((Z * Z).sum(1), 1.0, rtol=0, atol=1e-14)   # cos^2 + sin^2


def test_rff_estimate_converges():
    rng = np.random.default_rng(2)
    alpha = 1.5
    X = rng.standard_normal((8, 3))
    K = features.rbf_kernel(X, X, alpha)
    errs = []
    for N in (256, 4096, 65536):
        W = features.rff_frequencies(np.random.default_rng(N), N, 3, alpha)
        Z = features.rff_features(X, W)
        errs.append(np.abs(Z @ Z.T - K).max())
    # Monte Carlo: each entry is a mean of N terms bounded by 1 in magnitude
    assert errs[-1] <= 5.0 / np.sqrt(65536)
    assert errs[-1] < errs[0]


def test_rff_wrong_bandwidth_is_caught():
    """A plausible slip (frequencies with covariance alpha I instead of
    I / alpha) misses K by far more than the Monte Carlo error."""
    rng = np.random.default_rng(3)
    alpha = 4.0
    X = rng.standard_normal((8, 3))
    K = features.rbf_kernel(X, X, alpha)
    W = np.random.default_rng(9).standard_normal((65536, 3)) * np.sqrt(alpha)
    Z = features.rff_features(X, W)
    assert np.abs(Z @ Z.T - K).max() > 0.1


def test_nystroem_all_landmarks_reproduces_k():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((12, 4)) * 3.0          # well separated: K well conditioned
    alpha = 0.5
    K = features.rbf_kernel(X, X, alpha)
    Z = features.nystroem_features(X, np.arange(12), alpha, shift=0.0)
    np.testing.assert_allclose(Z @ Z.T, K, atol=1e-10)
    # with the paper's shift the landmark block is K_rr (K_rr + sI)^{-1} K_rr
    Zs = features.nystroem_features(X, np.arange(12), alpha)
    np.testing.assert_allclose(Zs @ Zs.T, K, atol=5e-3)


def test_nystroem_low_rank_is_psd_and_below_k():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((40, 3))
    alpha = 2.0
    K = features.rbf_kernel(X, X, alpha)
    Z = features.nystroem_features(X, rng.choice(40, 10, replace=False), alpha)
    Kt = Z @ Z.T
    # K - K_nr (K_rr + sI)^{-1} K_nr^T is a Schur complement of a PSD matrix plus a shift: PSD
    assert np.linalg.eigvalsh(K - Kt).min() >= -1e-10


def test_rff_csvc_matches_enumeration():
    """The features go through the linear C-SVC oracle unchanged."""
    rng = np.random.default_rng(6)
    X = rng.standard_normal((7, 2))
    y = np.array([1, -1, 1, -1, 1, -1, 1], np.int8)
    X += 0.8 * y[:, None]
    W = features.rff_frequencies(rng, 4, 2, alpha=1.0)
    Z = features.rff_features(X, W)
    f_star, _, _ = bruteforce.qp_by_enumeration(Z, y, 1.0)
    r = ssnal.solve(Z, y, 1.0, tol=1e-10)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
