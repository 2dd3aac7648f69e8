"""ssnalm_project_noalloc (the projection with its scratch in a static device
array, no allocation) against ssnalm_op_project (the same kernels with a
context's workspace), called through the C ABI: bitwise equal results on two
calls in a row, the second with a smaller input, and the oracle's projection
as the reference for both (GPU only)."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle.projection import project_svm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc(v, y, Cb):
    from paper_1910_01312_amd import _lib as L
    lib = L.load()
    n = v.numel()
    x = torch.empty(n, dtype=torch.float64, device=v.device)
    m = torch.empty(n, dtype=torch.uint8, device=v.device)
    lam, p = C.c_double(), C.c_int64()
    st = lib.ssnalm_project_noalloc(C.c_void_p(v.data_ptr()), C.c_void_p(y.data_ptr()), n,
                                    float(Cb), C.c_void_p(x.data_ptr()), C.c_void_p(m.data_ptr()),
                                    C.byref(lam), C.byref(p),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(st, "ssnalm_project_noalloc")
    return x.cpu().numpy(), m.cpu().numpy(), lam.value, p.value


def _with_context(X, y, v, Cb):
    from paper_1910_01312_amd.solver import Solver
    with Solver(X, y, Cb) as s:
        x, m, lam, p, _ = s.project(v)
        return x.cpu().numpy(), m.cpu().numpy(), lam, p


def test_noalloc_matches_context_projection_twice():
    rng = np.random.default_rng(2024)
    for n, Cb in ((300_001, 1.5), (4_097, 0.25)):        # second call smaller
        X, y = synth.dense_two_gaussians(n=n, q=2, seed=n)
        v = rng.standard_normal(n) * 2.0
        vd = torch.from_numpy(v).cuda()
        yd = torch.from_numpy(y).cuda()
        xa, ma, la, pa = _noalloc(vd, yd, Cb)
        xb, mb, lb, pb = _with_context(X, y, vd, Cb)
        np.testing.assert_array_equal(xa, xb)
        np.testing.assert_array_equal(ma, mb)
        assert la == lb and pa == pb
        x_ref, lam_ref, free_ref = project_svm(v, y, Cb)
        assert abs(la - lam_ref) <= 1e-12 * (1.0 + np.abs(v).max())
        np.testing.assert_allclose(xa, x_ref, rtol=0, atol=1e-12 * (1.0 + np.abs(v).max()))
        assert pa == int(ma.sum())


def test_noalloc_rejects_bad_sizes():
    from paper_1910_01312_amd import _lib as L
    lib = L.load()
    v = torch.zeros(4, dtype=torch.float64, device="cuda")
    y = torch.ones(4, dtype=torch.int8, device="cuda")
    big = int(lib.ssnalm_noalloc_max_n()) + 1
    assert lib.ssnalm_project_noalloc(C.c_void_p(v.data_ptr()), C.c_void_p(y.data_ptr()), big,
                                      1.0, C.c_void_p(v.data_ptr()), None, None, None,
                                      None) == L.E_BADARG
    assert b"n must be" in lib.ssnalm_last_error()
    assert lib.ssnalm_project_noalloc(C.c_void_p(v.data_ptr()), C.c_void_p(y.data_ptr()), 0,
                                      1.0, C.c_void_p(v.data_ptr()), None, None, None,
                                      None) == L.E_BADARG
