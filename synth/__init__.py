"""Seeded synthetic inputs for the linear C-SVC dual QP.

This module only draws data: it holds none of the solver's arithmetic, so the
CPU oracle and the GPU path can both take their inputs from it without sharing
any code of the method.  Every generator is a pure function of its seed.

The paper's own workloads (LIBSVM sets scaled to [0,1]^q, Section 4) are not
available; the workloads below stand in for them with the shapes, sparsity
and label structure described next to each function.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 20191003


def seed_for(config: int, instance: int = 0) -> int:
    """Seed of workload `config` (1..6), instance `instance`."""
    return SEED_BASE + config + 1000 * instance


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------

def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round an fp32 array to bfloat16 (round to nearest, ties to even).

    Returns the raw 16-bit patterns as uint16.  NaN/Inf are not expected in
    generated data and are not specially handled.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) >> 16
    return b.astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 patterns to fp32."""
    return (bits.astype(np.uint32) << 16).view(np.float32)


def _labels_from_score(rng, score: np.ndarray, noise: float) -> np.ndarray:
    s = score + noise * rng.standard_normal(score.shape[0])
    y = np.where(s >= 0.0, 1, -1).astype(np.int8)
    return y


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def dense_two_gaussians(n: int = 2000, q: int = 50, shift: float = 0.5,
                        seed: int | None = None):
    """Two Gaussian classes N(+shift*1, I) and N(-shift*1, I), n/2 each,
    rows shuffled.  Returns (X float64 [n,q], y int8 [n])."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    n_pos = n // 2
    n_neg = n - n_pos
    Xp = rng.standard_normal((n_pos, q)) + shift
    Xn = rng.standard_normal((n_neg, q)) - shift
    X = np.vstack([Xp, Xn])
    y = np.concatenate([np.ones(n_pos, np.int8), -np.ones(n_neg, np.int8)])
    perm = rng.permutation(n)
    return np.ascontiguousarray(X[perm]), np.ascontiguousarray(y[perm])


def sparse_text(n: int = 500_000, q: int = 100_000, mean_nnz: float = 60.0,
                zipf_s: float = 1.1, seed: int | None = None,
                w_support: float = 0.10, noise: float = 0.1):
    """Text-like CSR matrix.

    * row length ~ Poisson(mean_nnz), at least 1;
    * the distinct columns of a row are drawn by a Zipf(zipf_s) rank law,
      P(rank r) ~ r^-zipf_s, over a seeded permutation of the column ids
      (draws are repeated until the row has its length in distinct columns,
      capped at twice the length in draws);
    * values lognormal(0, 1), each row scaled to unit L2 norm;
    * labels y = sign(w^T x + noise*N(0,1)) (0 -> +1) for a w with
      `w_support` of its entries nonzero, N(0,1), scaled so std(Xw) = 1.

    Returns (values float32 [nnz], col_idx int32 [nnz], row_ptr int64 [n+1],
    y int8 [n]); columns within a row are sorted ascending.
    """
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    lens = np.maximum(rng.poisson(mean_nnz, size=n), 1).astype(np.int64)
    lens = np.minimum(lens, q)
    ranks = np.arange(1, q + 1, dtype=np.float64)
    pmf = ranks ** (-zipf_s)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    col_of_rank = rng.permutation(q).astype(np.int64)

    vals_out, cols_out, lens_out = [], [], []
    chunk = 50_000
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        L = lens[r0:r1]
        ndraw = 2 * L
        tot = int(ndraw.sum())
        row_of = np.repeat(np.arange(r1 - r0, dtype=np.int64), ndraw)
        draw_pos = np.arange(tot, dtype=np.int64) - np.repeat(np.cumsum(ndraw) - ndraw, ndraw)
        rk = np.searchsorted(cdf, rng.random(tot), side="right")
        rk = np.minimum(rk, q - 1)
        col = col_of_rank[rk]
        # first occurrence of each (row, col) in draw order
        key = row_of * q + col
        order = np.lexsort((draw_pos, key))
        ks = key[order]
        first = np.ones(tot, dtype=bool)
        first[1:] = ks[1:] != ks[:-1]
        keep_idx = order[first]
        # rank of each kept draw among the row's distinct draws, by draw order
        keep_idx.sort()
        krow = row_of[keep_idx]
        start = np.searchsorted(krow, np.arange(r1 - r0))
        rank_in_row = np.arange(keep_idx.size) - start[krow]
        sel = keep_idx[rank_in_row < L[krow]]
        srow = row_of[sel]
        scol = col[sel]
        o = np.lexsort((scol, srow))
        srow, scol = srow[o], scol[o]
        cnt = np.bincount(srow, minlength=r1 - r0)
        v = rng.lognormal(0.0, 1.0, size=scol.size)
        nrm = np.sqrt(np.bincount(srow, weights=v * v, minlength=r1 - r0))
        v = v / nrm[srow]
        vals_out.append(v.astype(np.float32))
        cols_out.append(scol.astype(np.int32))
        lens_out.append(cnt)
    values = np.concatenate(vals_out)
    col_idx = np.concatenate(cols_out)
    row_len = np.concatenate(lens_out)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])

    w = np.zeros(q)
    supp = rng.choice(q, size=max(1, int(round(w_support * q))), replace=False)
    w[supp] = rng.standard_normal(supp.size)
    vals64 = values.astype(np.float64)
    rows = np.repeat(np.arange(n), row_len)
    score = np.bincount(rows, weights=vals64 * w[col_idx], minlength=n)
    sd = score.std()
    if sd > 0:
        score = score / sd
    y = _labels_from_score(rng, score, noise)
    return values, col_idx, row_ptr, y


def dense_bf16_directions(n: int = 1_000_000, q: int = 512, k_dirs: int = 4,
                          flip: float = 0.05, noise: float = 0.1,
                          seed: int | None = None):
    """Dense N(0,1) features rounded to bfloat16, labels from a noisy linear
    rule on `k_dirs` random orthonormal directions, then `flip` of the labels
    flipped uniformly at random.

    The bfloat16 matrix is the problem: labels are computed from it.
    Returns (bits uint16 [n,q], y int8 [n]).
    """
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    V, _ = np.linalg.qr(rng.standard_normal((q, k_dirs)))
    direction = V.sum(axis=1)
    bits = np.empty((n, q), dtype=np.uint16)
    score = np.empty(n)
    blk = 65536
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        Xb = rng.standard_normal((r1 - r0, q), dtype=np.float32)
        bb = to_bf16_bits(Xb)
        bits[r0:r1] = bb
        score[r0:r1] = bf16_bits_to_f32(bb).astype(np.float64) @ direction
    sd = score.std()
    score /= sd if sd > 0 else 1.0
    y = _labels_from_score(rng, score, noise)
    flips = rng.random(n) < flip
    y[flips] = -y[flips]
    return bits, y


def mixture_problem(n: int, q: int = 128, seed: int = 0, n_comp: int = 3,
                    mean_scale: float = 0.5):
    """One problem of the batched family: two classes, each a mixture of
    `n_comp` Gaussians with means ~ N(0, mean_scale^2 I) and identity
    covariance; the positive-class share ~ U[0.3, 0.7]; rows in random
    order.  Draws in float32 (the workload's storage type).
    Returns (X float32 [n,q], y int8 [n])."""
    rng = np.random.default_rng(seed)
    frac = rng.uniform(0.3, 0.7)
    n_pos = int(round(frac * n))
    n_pos = min(max(n_pos, 1), n - 1)
    means = rng.normal(0.0, mean_scale, size=(2 * n_comp, q)).astype(np.float32)
    cls = np.ones(n, dtype=np.int64)
    cls[:n_pos] = 0
    rng.shuffle(cls)
    comp = rng.integers(0, n_comp, size=n)
    X = rng.standard_normal((n, q), dtype=np.float32)
    X += means[cls * n_comp + comp]
    y = np.where(cls == 0, 1, -1).astype(np.int8)
    return X, y


def batch_family(count: int = 256, q: int = 128, n_lo: int = 1000,
                 n_hi: int = 200_000, seed: int | None = None):
    """Sizes, C values and per-problem seeds of the batched workload:
    n_k ~ U{n_lo..n_hi}, C_k = 10^(-3 + 5k/(count-1)) (log grid 1e-3..1e2).
    Returns a list of dicts {n, q, C, seed}; use `mixture_problem` to draw
    each problem's data."""
    rng = np.random.default_rng(seed_for(4) if seed is None else seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    out = []
    for k in range(count):
        C = 10.0 ** (-3.0 + 5.0 * k / max(count - 1, 1))
        out.append({"n": int(ns[k]), "q": q, "C": float(C),
                    "seed": seed_for(4, k + 1)})
    return out


def tiny_problem(n: int, q: int, seed: int, integer: bool = False,
                 balanced: bool = True):
    """Small random C-SVC instance for brute-force checks.
    integer=True draws integer features in [-3, 3]."""
    rng = np.random.default_rng(seed)
    if integer:
        X = rng.integers(-3, 4, size=(n, q)).astype(np.float64)
    else:
        X = rng.standard_normal((n, q))
    if balanced:
        y = np.ones(n, np.int8)
        y[: n // 2] = -1
        rng.shuffle(y)
    else:
        y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
        if np.all(y == y[0]):
            y[0] = -y[0]
    X = X + (1.0 if integer else 0.5) * y[:, None]
    return X, y


def projection_matrix(q: int, k: int = 64, seed: int = 0) -> np.ndarray:
    """Seeded Gaussian q x k matrix scaled by 1/sqrt(q) (float32): the
    feature projection of the warm-start network."""
    rng = np.random.default_rng(SEED_BASE + 5000 + q + 100000 * seed)
    return (rng.standard_normal((q, k)) / np.sqrt(q)).astype(np.float32)


def mlp_init(seed: int = 0, sizes=(66, 256, 256, 4)) -> np.ndarray:
    """Seeded initial parameters of the warm-start network (float32, flat,
    layout W1, b1, W2, b2, W3, b3): weights ~ N(0, 2 / (fan_in + fan_out)),
    biases 0."""
    rng = np.random.default_rng(SEED_BASE + 7000 + seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal((a, b)) * np.sqrt(2.0 / (a + b))).ravel())
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def tiny_regression(n: int, q: int, seed: int, noise: float = 0.1):
    """Small random regression set (X Gaussian, y = X beta + Gaussian noise)
    for eps-SVR checks."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, q))
    beta = rng.standard_normal(q)
    y = X @ beta + 0.3 + noise * rng.standard_normal(n)
    return X, y


def tiny_general(n: int, q: int, seed: int, zero_a: int = 0):
    """Small random instance of the unified problem (P): B (n x q), c, a
    (mixed signs, `zero_a` entries set to 0), l < u, and d = a^T x for a
    point x drawn inside the box, so the feasible set is non-empty."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, q))
    c = rng.standard_normal(n)
    a = rng.uniform(0.5, 2.0, n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    if zero_a:
        a[rng.choice(n, zero_a, replace=False)] = 0.0
    l = rng.uniform(-1.0, 0.5, n)
    u = l + rng.uniform(0.2, 2.0, n)
    d = float(a @ rng.uniform(l, u))
    return B, c, a, d, l, u


def rbf_problem(n: int, q: int = 100, seed: int = 0, n_comp: int = 3, flip: float = 0.0):
    """Input of the nonlinear-kernel C-SVC (Table 3's shape): the two-class
    Gaussian mixture of `mixture_problem`, every feature rescaled to [0, 1]
    over the samples (the scaling Section 4 applies to the datasets); a
    fraction `flip` of the labels drawn at random is inverted (label noise:
    the datasets of Table 3 are classified at 82-99% accuracy).
    Returns (X float64 [n,q], y int8 [n])."""
    X, y = mixture_problem(n, q, seed=seed, n_comp=n_comp, mean_scale=1.0)
    if flip > 0.0:
        rng = np.random.default_rng(seed + 7)
        f = rng.random(n) < flip
        y = np.where(f, -y, y).astype(np.int8)
    X = X.astype(np.float64)
    lo, hi = X.min(axis=0), X.max(axis=0)
    X = (X - lo) / np.where(hi > lo, hi - lo, 1.0)
    return X, y
