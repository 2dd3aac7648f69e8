"""Step-level parity of the HIP library against the CPU oracle (GPU only).

Each step of the hot path is called through the C ABI on seeded inputs and
compared element by element with the oracle's FP64 result:
  * A v and A^T z (dense fp64/fp32/bf16 storage, CSR fp32/fp64): bitwise on
    integer-valued data (every partial sum is an exact integer in fp64),
    within 1e-12 relative to |X||v| otherwise (fp64 accumulation);
  * the projection onto {y^T x = 0, 0 <= x <= C} (Algorithm 2's multiplier);
  * the Newton direction (Proposition 5 in omega-space), Cholesky and PCG;
  * one line-search trial (the phi-increment sum of psi);
  * R_KKT (eq. Def_Rkkt).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import ssnal
from oracle.projection import project_svm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01312_amd import _lib
    _lib.load()


def _solver(*a, **k):
    from paper_1910_01312_amd.solver import Solver
    return Solver(*a, **k)


def _np(t):
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------ matvecs

@pytest.mark.parametrize("n,q", [(1, 1), (7, 3), (1000, 50), (2001, 129), (5000, 512), (333, 1000)])
def test_dense_matvec_integer_exact(n, q):
    rng = np.random.default_rng(n * 31 + q)
    X = rng.integers(-8, 9, size=(n, q)).astype(np.float64)
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    v = rng.integers(-8, 9, size=q).astype(np.float64)
    z = rng.integers(-8, 9, size=n).astype(np.float64)
    with _solver(X, y, 1.0) as s:
        t = _np(s.amul(v))
        r = _np(s.atmul(z))
    np.testing.assert_array_equal(t, y * (X @ v))
    np.testing.assert_array_equal(r, X.T @ (y * z))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,q", [(1000, 50), (4097, 256), (3000, 512), (1500, 77)])
def test_dense_matvec_gaussian(dtype, n, q):
    rng = np.random.default_rng(7 + n + q)
    X64 = rng.standard_normal((n, q))
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    if dtype == "f64":
        Xs, Xref, kw = X64, X64, {}
    elif dtype == "f32":
        Xs = X64.astype(np.float32)
        Xref, kw = Xs.astype(np.float64), {}
    else:
        Xs = synth.to_bf16_bits(X64.astype(np.float32))
        Xref, kw = synth.bf16_bits_to_f32(Xs).astype(np.float64), {"bf16": True}
    v = rng.standard_normal(q)
    z = rng.standard_normal(n) * (rng.random(n) < 0.6)     # many zero rows
    with _solver(Xs, y, 1.0, **kw) as s:
        t = _np(s.amul(v))
        r = _np(s.atmul(z))
    t_ref = y * (Xref @ v)
    r_ref = Xref.T @ (y * z)
    bound_t = 1e-12 * (np.abs(Xref) @ np.abs(v))
    bound_r = 1e-12 * (np.abs(Xref).T @ np.abs(z))
    assert np.all(np.abs(t - t_ref) <= bound_t + 1e-300)
    assert np.all(np.abs(r - r_ref) <= bound_r + 1e-300)


def _csr_case(n, q, seed, heavy=True, integer=False, f64=False):
    rng = np.random.default_rng(seed)
    lens = rng.poisson(6, size=n)
    lens[rng.random(n) < 0.05] = 0                      # empty rows
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = rng.choice(q, size=min(L, q), replace=False)
        if heavy and rng.random() < 0.9:
            c = np.union1d(c, [0])                       # column 0 in ~90% of rows
        rows.append(np.full(c.size, i))
        cols.append(np.sort(c))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = (rng.integers(-5, 6, size=rows.size).astype(np.float64) if integer
            else rng.standard_normal(rows.size))
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, q))
    M.sort_indices()
    data = M.data.astype(np.float64 if f64 else np.float32)
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return data, M.indices.astype(np.int32), M.indptr.astype(np.int64), y


@pytest.mark.parametrize("dtype,q", [("f64", 128), ("f32", 256), ("bf16", 512)])
@pytest.mark.parametrize("density", [0.0, 0.02, 0.125, 1.0])
def test_dense_atmul_sparse_coefficients(dtype, q, density):
    """X^T (y .* z) where z is zero on most rows: the row kernel for rows of one
    piece per lane skips every row whose coefficient is zero, so whole 64-row
    chunks with no nonzero (density 0.02), chunks with about one batch of 8
    (0.125), none at all and all of them are compared with the plain product
    (n = 5003: a ragged last chunk)."""
    n = 5003
    rng = np.random.default_rng(q + int(1000 * density))
    X64 = rng.standard_normal((n, q))
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    if dtype == "f64":
        Xs, Xref, kw = X64, X64, {}
    elif dtype == "f32":
        Xs = X64.astype(np.float32)
        Xref, kw = Xs.astype(np.float64), {}
    else:
        Xs = synth.to_bf16_bits(X64.astype(np.float32))
        Xref, kw = synth.bf16_bits_to_f32(Xs).astype(np.float64), {"bf16": True}
    z = rng.standard_normal(n) * (rng.random(n) < density)
    with _solver(Xs, y, 1.0, **kw) as s:
        r = _np(s.atmul(z))
    r_ref = Xref.T @ (y * z)
    bound = 1e-12 * (np.abs(Xref).T @ np.abs(z))
    assert np.all(np.abs(r - r_ref) <= bound + 1e-300)


@pytest.mark.parametrize("n,q,seed", [(1, 3, 1), (50, 20, 2), (3000, 500, 3), (20000, 3000, 4)])
@pytest.mark.parametrize("f64", [False, True])
def test_csr_matvec(n, q, seed, f64):
    data, ci, rp, y = _csr_case(n, q, seed, integer=(seed % 2 == 0), f64=f64)
    Xref = sp.csr_matrix((data.astype(np.float64), ci, rp), shape=(n, q))
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(q) if seed % 2 else rng.integers(-4, 5, size=q).astype(np.float64)
    z = rng.standard_normal(n) if seed % 2 else rng.integers(-4, 5, size=n).astype(np.float64)
    with _solver(csr=(data, ci, rp, n, q), y=y) as s:
        t = _np(s.amul(v))
        r = _np(s.atmul(z))
    t_ref = y * (Xref @ v)
    r_ref = Xref.T @ (y * z)
    if seed % 2 == 0:
        np.testing.assert_array_equal(t, t_ref)
        np.testing.assert_array_equal(r, r_ref)
    else:
        absX = abs(Xref)
        assert np.all(np.abs(t - t_ref) <= 1e-12 * (absX @ np.abs(v)) + 1e-300)
        assert np.all(np.abs(r - r_ref) <= 1e-12 * (absX.T @ np.abs(z)) + 1e-300)


@pytest.mark.parametrize("n,f64", [(131073, False), (140000, True), (262144, False)])
def test_csr_transpose_row_blocks(n, f64):
    """n >= 2^17 rows: A^T z runs over the CSC copy cut into row blocks (one
    per XCD) with the per-block column sums added afterwards (a column present
    in most rows, empty columns); integer data, so every sum is exact."""
    q = 5000
    rng = np.random.default_rng(n)
    lens = rng.poisson(5, size=n)
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(1, q - 10, size=rows.size)           # the last columns stay empty
    heavy = np.nonzero(rng.random(n) < 0.8)[0]
    rows = np.concatenate([rows, heavy])
    cols = np.concatenate([cols, np.zeros(heavy.size, np.int64)])
    vals = rng.integers(-3, 4, size=rows.size).astype(np.float64)
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, q))
    M.sum_duplicates()
    M.sort_indices()
    data = M.data.astype(np.float64 if f64 else np.float32)
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    z = rng.integers(-4, 5, size=n).astype(np.float64)
    v = rng.integers(-4, 5, size=q).astype(np.float64)
    Xref = sp.csr_matrix((data.astype(np.float64), M.indices, M.indptr), shape=(n, q))
    with _solver(csr=(data, M.indices.astype(np.int32), M.indptr.astype(np.int64), n, q), y=y) as s:
        r = _np(s.atmul(z))
        t = _np(s.amul(v))
    np.testing.assert_array_equal(r, Xref.T @ (y * z))
    np.testing.assert_array_equal(t, y * (Xref @ v))


@pytest.mark.parametrize("case", ["ell", "ell_wide", "long_row", "skewed"])
def test_csr_matvec_row_layouts(case):
    """A v over fp32 CSR rows in each row layout: rows of similar lengths (the
    sliced-ELL copy; empty rows, n not a multiple of 64, several 1024-row
    windows; with q = 40 000 also columns past the 16 384 whose v is read from
    LDS), one row past the copy's 1024-entry limit, and lengths so skewed that
    the copy's padding would pass a quarter of the entries (both on the
    merge-path plan).  Integer data, so every sum is exact."""
    n, q = 5037, (40000 if case == "ell_wide" else 3000)
    rng = np.random.default_rng({"ell": 1, "ell_wide": 4, "long_row": 2, "skewed": 3}[case])
    if case == "skewed":
        lens = np.where(rng.random(n) < 0.02, 600, 2)
    else:
        lens = rng.poisson(12, size=n)
        lens[rng.random(n) < 0.05] = 0
        if case == "long_row":
            lens[1234] = 2000
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, q, size=rows.size)
    M = sp.csr_matrix((rng.integers(1, 4, size=rows.size).astype(np.float64), (rows, cols)), shape=(n, q))
    M.sum_duplicates()
    M.sort_indices()
    data = M.data.astype(np.float32)
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    v = rng.integers(-4, 5, size=q).astype(np.float64)
    with _solver(csr=(data, M.indices.astype(np.int32), M.indptr.astype(np.int64), n, q), y=y) as s:
        t = _np(s.amul(v))
    np.testing.assert_array_equal(t, y * (M @ v))


def test_csr_text_like_sample():
    """Workload-shaped CSR (Zipf columns, L2-normalised rows), reduced n."""
    vals, ci, rp, y = synth.sparse_text(n=30000, q=8000, seed=11)
    n, q = rp.size - 1, 8000
    Xref = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(n, q))
    rng = np.random.default_rng(3)
    v = rng.standard_normal(q)
    z = rng.standard_normal(n)
    with _solver(csr=(vals, ci, rp, n, q), y=y) as s:
        t = _np(s.amul(v))
        r = _np(s.atmul(z))
    absX = abs(Xref)
    assert np.all(np.abs(t - y * (Xref @ v)) <= 1e-12 * (absX @ np.abs(v)) + 1e-300)
    assert np.all(np.abs(r - Xref.T @ (y * z)) <= 1e-12 * (absX.T @ np.abs(z)) + 1e-300)


def test_matvec_deterministic():
    X, y = synth.dense_two_gaussians(n=5000, q=64)
    rng = np.random.default_rng(0)
    z = rng.standard_normal(5000)
    with _solver(X, y, 1.0) as s:
        a = _np(s.atmul(z))
        b = _np(s.atmul(z))
    np.testing.assert_array_equal(a, b)


# ------------------------------------------------------------------ projection

@pytest.mark.parametrize("n,scale,seed", [(1, 1.0, 0), (2, 1.0, 1), (9, 3.0, 2), (1000, 5.0, 3),
                                          (100000, 50.0, 4), (100000, 1e6, 5), (333333, 2.0, 6)])
def test_projection_parity(n, scale, seed):
    rng = np.random.default_rng(seed)
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    if n >= 2 and np.all(y == y[0]):
        y[0] = -y[0]
    C = float(rng.uniform(0.1, 3))
    v = rng.standard_normal(n) * scale
    X = np.zeros((n, 1))
    with _solver(X, y, C) as s:
        x, m, lam, p, passes = s.project(v)
    x, m = _np(x), _np(m).astype(bool)
    x_ref, lam_ref, free_ref = project_svm(v, y, C)
    tol = 1e-12 * (np.abs(v).max() + C)
    assert abs(lam - lam_ref) <= tol
    assert np.all(np.abs(x - x_ref) <= 2 * tol)
    assert np.all(x >= 0) and np.all(x <= C)
    t_ref = v - lam_ref * y
    ties = np.minimum(np.abs(t_ref), np.abs(t_ref - C)) <= 4 * tol
    assert np.array_equal(m[~ties], free_ref[~ties])
    assert p == int(m.sum())


def test_projection_golden(golden):
    for case in golden["projection_cases"]:
        v = np.array(case["v"])
        y = np.array(case["y"], dtype=np.int8)
        with _solver(np.zeros((v.size, 1)), y, case["C"]) as s:
            x, m, lam, p, _ = s.project(v)
        assert lam == pytest.approx(case["lam"], abs=1e-14)
        np.testing.assert_allclose(_np(x), case["x"], atol=1e-14)
        assert list(_np(m).astype(bool)) == case["free"]


def test_projection_single_class_and_ties():
    n = 1000
    y = np.ones(n, np.int8)
    v = np.random.default_rng(0).standard_normal(n)
    with _solver(np.zeros((n, 1)), y, 1.0) as s:
        x, m, lam, p, _ = s.project(v)
    assert np.all(_np(x) == 0.0) and p == 0
    # all components equal (u = sigma e at the first ALM step)
    y2 = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int8)
    with _solver(np.zeros((n, 1)), y2, 1.0) as s:
        x, m, lam, p, _ = s.project(np.full(n, 1.0))
    x_ref, lam_ref, _ = project_svm(np.full(n, 1.0), y2, 1.0)
    np.testing.assert_allclose(_np(x), x_ref, atol=1e-14)


# ------------------------------------------------------------------ Newton

def _newton_state(X, y, C, sigma, seed):
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    xk, _, _ = project_svm(rng.random(n) * C, y, C)
    omega = ssnal.atmul(X, y, rng.standard_normal(n) * 0.05)
    u = xk + sigma * (1.0 - ssnal.amul(X, y, omega))
    xt, lam, free = project_svm(u, y, C)
    g = omega - ssnal.atmul(X, y, xt)
    return u, lam, free, g, omega, xk


@pytest.mark.parametrize("q,dtype", [(50, "f64"), (128, "f32"), (33, "f64")])
def test_newton_cholesky(q, dtype):
    X, y = synth.dense_two_gaussians(n=3000, q=q, seed=5)
    if dtype == "f32":
        X = X.astype(np.float32)
    Xr = X.astype(np.float64)
    sigma = 7.0
    u, lam, free, g, _, _ = _newton_state(Xr, y, 1.0, sigma, 1)
    d_ref = ssnal.newton_qspace(Xr, free, g, sigma)
    with _solver(X, y, 1.0, newton="chol") as s:
        d, _ = s.newton(free.astype(np.uint8), g, sigma)
    d = _np(d)
    assert np.linalg.norm(d - d_ref) <= 1e-10 * (1 + np.linalg.norm(d_ref))


def test_newton_empty_free_set():
    X, y = synth.dense_two_gaussians(n=200, q=10, seed=1)
    g = np.random.default_rng(1).standard_normal(10)
    with _solver(X, y, 1.0) as s:
        d, _ = s.newton(np.zeros(200, np.uint8), g, 3.0)
    np.testing.assert_array_equal(_np(d), -g)


@pytest.mark.parametrize("q", [3000, 40000])
@pytest.mark.parametrize("f64", [False, True])
def test_newton_pcg_csr(f64, q):
    """The Newton direction by PCG on a CSR X_J; at q = 40 000 the CG's row
    product reads v for the 16 384 most frequent columns from LDS and for the
    rest from global memory."""
    vals, ci, rp, y = synth.sparse_text(n=20000, q=q, seed=12)
    if f64:
        vals = vals.astype(np.float64)
    n = rp.size - 1
    Xr = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(n, q))
    sigma = 25.0
    u, lam, free, g, _, _ = _newton_state(Xr, y, 1.0, sigma, 2)
    d_ref, _ = ssnal.newton_pcg(Xr, free, g, sigma, 1e-13, 2000)
    with _solver(csr=(vals, ci, rp, n, q), y=y, newton="pcg", max_cg=2000) as s:
        d, it = s.newton(free.astype(np.uint8), g, sigma, cg_tol=1e-13)
    d = _np(d)
    assert it > 0
    assert np.linalg.norm(d - d_ref) <= 1e-8 * (1 + np.linalg.norm(d_ref))


# ------------------------------------------------------------------ line search

def test_linesearch_trial_increment():
    X, y = synth.dense_two_gaussians(n=4000, q=40, seed=9)
    sigma, C = 50.0, 1.0
    u, lam, free, g, omega, xk = _newton_state(X, y, C, sigma, 3)
    d = ssnal.newton_qspace(X, free, g, sigma)
    t = ssnal.amul(X, y, d)
    with _solver(X, y, C) as s:
        for alpha in (1.0, 0.25):
            lam_a, dh = s.linesearch_trial(u, t, lam, alpha, sigma)
            u_a = u - alpha * sigma * t
            _, lam_ref, _ = project_svm(u_a, y, C)
            yf = y.astype(np.float64)
            dt = -alpha * sigma * t - (lam_ref - lam) * yf
            dh_ref = float(np.sum(ssnal.huber_increment(u - lam * yf, dt, C)))
            assert abs(lam_a - lam_ref) <= 1e-12 * (np.abs(u_a).max() + C)
            assert abs(dh - dh_ref) <= 1e-9 * (1 + abs(dh_ref))


# ------------------------------------------------------------------ KKT

def test_rkkt_parity():
    X, y = synth.dense_two_gaussians(n=2000, q=50)
    r = ssnal.solve(X, y, 1.0, tol=1e-4)
    R_ref, b_ref = ssnal.rkkt(X, y, 1.0, r.x)
    with _solver(X, y, 1.0) as s:
        R, b = s.rkkt(r.x)
    assert abs(R - R_ref) <= 1e-10 * R_ref + 1e-14
    assert abs(b - b_ref) <= 1e-9


# ------------------------------------------------------------------ mixed precision

@pytest.mark.parametrize("q,p_frac", [(128, 0.3), (256, 0.05), (512, 0.2), (200, 0.5),
                                      (77, 0.4), (203, 0.3)])
def test_gram_mfma_bf16(q, p_frac):
    """bf16 MFMA SYRK with fp32 accumulation: exact on small-integer bf16
    data (every partial sum is an integer below 2^24), and within the fp32
    accumulation bound on Gaussian data."""
    n = 3000
    rng = np.random.default_rng(q)
    free = rng.random(n) < p_frac
    y = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    Xi = rng.integers(-4, 5, size=(n, q)).astype(np.float32)
    bits = synth.to_bf16_bits(Xi)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    with _solver(bits, y, 1.0, bf16=True, newton="chol", precision="mixed") as s:
        G = _np(s.gram(free.astype(np.uint8)))
    np.testing.assert_array_equal(G, Xr[free].T @ Xr[free])
    Xg = rng.standard_normal((n, q)).astype(np.float32)
    bits = synth.to_bf16_bits(Xg)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    with _solver(bits, y, 1.0, bf16=True, newton="chol", precision="mixed") as s:
        G = _np(s.gram(free.astype(np.uint8)))
    XJ = Xr[free]
    ref = XJ.T @ XJ
    bound = 4 * 2.0 ** -24 * free.sum() * (np.abs(XJ).T @ np.abs(XJ))
    assert np.all(np.abs(G - ref) <= bound + 1e-30)


@pytest.mark.parametrize("q", [160, 200, 512, 1000])
def test_newton_blocked_cholesky_fp64(q):
    X, y = synth.dense_two_gaussians(n=4000, q=q, seed=6)
    sigma = 3.0
    u, lam, free, g, _, _ = _newton_state(X, y, 1.0, sigma, 4)
    d_ref = ssnal.newton_qspace(X, free, g, sigma)
    with _solver(X, y, 1.0, newton="chol") as s:
        d, _ = s.newton(free.astype(np.uint8), g, sigma)
    d = _np(d)
    assert np.linalg.norm(d - d_ref) <= 1e-9 * (1 + np.linalg.norm(d_ref))


def test_newton_mixed_refined():
    """bf16 Gram + fp64 Cholesky + refinement reaches the fp64 direction."""
    bits, y = synth.dense_bf16_directions(n=6000, q=256, seed=31)
    Xr = synth.bf16_bits_to_f32(bits).astype(np.float64)
    sigma = 40.0
    u, lam, free, g, _, _ = _newton_state(Xr, y, 1.0, sigma, 5)
    d_ref = ssnal.newton_qspace(Xr, free, g, sigma)
    tol = 1e-10 * np.linalg.norm(g)
    with _solver(bits, y, 1.0, bf16=True, newton="chol", precision="mixed") as s:
        d, its = s.newton(free.astype(np.uint8), g, sigma, cg_tol=tol)
    d = _np(d)
    assert its <= 6
    assert np.linalg.norm(d - d_ref) <= 1e-8 * (1 + np.linalg.norm(d_ref))
