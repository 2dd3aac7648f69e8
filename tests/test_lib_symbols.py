"""The C-ABI library builds for gfx950, loads on a host without a GPU, and
exports every entry point that include/ssnalm.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssnalm.h")
LIB = os.path.join(ROOT, "paper_1910_01312_amd", "libssnalm.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ssnalm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = _declared()
    for required in ("ssnalm_create", "ssnalm_solve", "ssnalm_solve_batch", "ssnalm_destroy",
                     "ssnalm_last_error", "ssnalm_default_options"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1910_01312_amd.build import build
        build()
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ssnalm_\w+)", out))
    assert set(_declared()) <= exported


def test_binding_lists_every_symbol():
    from paper_1910_01312_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_default_options_without_gpu():
    """ssnalm_default_options touches no device: callable on the CPU host."""
    from paper_1910_01312_amd import _lib
    o = _lib.default_options()
    assert o.sigma0 == 1.0 and o.rho == 2.0 and o.max_outer == 200 and o.max_inner == 50
    assert o.mu == 1e-4 and o.ls_delta == 0.5 and o.tau == 0.5 and o.eta == 0.1


def test_code_separation():
    """The product path never imports the oracle and the oracle never imports
    the product package."""
    pkg = os.path.join(ROOT, "paper_1910_01312_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", txt, re.M), f
                assert "oracle/" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1910_01312_amd" not in txt, f


def test_struct_layouts_match_header():
    """The ctypes mirrors of ssnalm_problem / ssnalm_options / ssnalm_info /
    ssnalm_kstat have exactly the header's fields, in order."""
    import ctypes
    from paper_1910_01312_amd import _lib

    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)

    def fields(struct_name):
        m = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct_name + r"\s*;", src, re.S)
        body = m.group(1)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            m2 = re.match(r"^(?:const\s+)?\w+\s*\**\s*(.*)$", decl, re.S)
            names = m2.group(1).replace("*", " ")
            for nm in names.split(","):
                nm = nm.strip()
                if nm:
                    out.append(nm)
        return out

    for cls, name in [(_lib.Problem, "ssnalm_problem"), (_lib.Options, "ssnalm_options"),
                      (_lib.Info, "ssnalm_info"), (_lib.KStat, "ssnalm_kstat"),
                      (_lib.WsStats, "ssnalm_ws_stats")]:
        assert [f for f, _ in cls._fields_] == fields(name), name


def test_create_rejects_bad_arguments_without_gpu():
    """ssnalm_create validates its arguments before any device call: each bad
    field gives SSNALM_E_BADARG and a message naming it, also on a host with
    no GPU (the pointers below are never dereferenced)."""
    import ctypes as C
    from paper_1910_01312_amd import _lib
    lib = _lib.load()
    buf = (C.c_byte * 64)()
    addr = C.addressof(buf)

    def problem(**kw):
        f = dict(kind=0, dtype=0, n=4, q=2, nnz=0, X=addr, row_ptr=None, col_idx=None,
                 y=addr, C=1.0, tol=1e-6)
        f.update(kw)
        return _lib.Problem(**f)

    ctx = C.c_void_p()
    assert lib.ssnalm_create(C.byref(ctx), None, None, None) == _lib.E_BADARG
    cases = [(dict(n=0), b"n and q"), (dict(q=0), b"n and q"), (dict(C=0.0), b"C must"),
             (dict(C=float("inf")), b"C must"), (dict(tol=0.0), b"tol"), (dict(kind=7), b"kind"),
             (dict(dtype=9), b"dtype"), (dict(y=None), b"y missing"), (dict(X=None), b"X missing")]
    for kw, msg in cases:
        pr = problem(**kw)
        st = lib.ssnalm_create(C.byref(ctx), C.byref(pr), None, None)
        assert st == _lib.E_BADARG, kw
        assert msg in lib.ssnalm_last_error(), (kw, lib.ssnalm_last_error())
        assert not ctx.value


def test_solve_batch_rejects_bad_arguments_without_gpu():
    """ssnalm_solve_batch validates every problem before any device call."""
    import ctypes as C
    from paper_1910_01312_amd import _lib
    lib = _lib.load()
    buf = (C.c_byte * 64)()
    addr = C.addressof(buf)

    def probs(k_bad=None, **kw):
        arr = (_lib.Problem * 3)()
        for k in range(3):
            f = dict(kind=0, dtype=0, n=4, q=8, nnz=0, X=addr, row_ptr=None, col_idx=None,
                     y=addr, C=1.0, tol=1e-6)
            if k == k_bad:
                f.update(kw)
            arr[k] = _lib.Problem(**f)
        return arr

    xs = (C.c_void_p * 3)(addr, addr, addr)
    infos = (_lib.Info * 3)()

    def call(pr, opt=None, count=3, x_out=xs):
        return lib.ssnalm_solve_batch(count, pr, C.byref(opt) if opt else None, None, x_out, None, infos)

    assert call(probs(), count=0) == _lib.E_BADARG
    assert call(probs(), x_out=None) == _lib.E_BADARG
    cases = [(dict(kind=1), b"problem 1: batched problems must be dense"),
             (dict(dtype=1), b"problem 1: dtype and q must match"),
             (dict(q=9), b"problem 1: dtype and q must match"),
             (dict(n=0), b"problem 1: n must be"),
             (dict(C=-1.0), b"problem 1: C must"),
             (dict(tol=0.0), b"problem 1: tol"),
             (dict(y=None), b"problem 1: X and y")]
    for kw, msg in cases:
        assert call(probs(1, **kw)) == _lib.E_BADARG, kw
        assert msg in lib.ssnalm_last_error(), (kw, lib.ssnalm_last_error())
    o = _lib.default_options()
    o.newton = 2
    assert call(probs(), opt=o) == _lib.E_BADARG
    assert b"Cholesky" in lib.ssnalm_last_error()
    o = _lib.default_options()
    o.precision = 1
    assert call(probs(), opt=o) == _lib.E_BADARG
    assert b"fp64" in lib.ssnalm_last_error()


def test_null_handles_and_sizes_without_gpu():
    """Entry points reject null handles and bad sizes before any device call;
    the network's parameter count matches the oracle's layout."""
    import ctypes as C
    import numpy as np
    import synth
    from oracle import mlp as omlp
    from paper_1910_01312_amd import _lib
    lib = _lib.load()
    buf = (C.c_byte * 64)()
    a = C.addressof(buf)
    info = _lib.Info()
    assert lib.ssnalm_solve(None, None, a, None, None, C.byref(info)) == _lib.E_BADARG
    assert lib.ssnalm_op_amul(None, a, a) == _lib.E_BADARG
    assert lib.ssnalm_op_atmul(None, a, a) == _lib.E_BADARG
    assert lib.ssnalm_ws_x0(None, a, a) == _lib.E_BADARG
    ks = _lib.KStat()
    assert lib.ssnalm_batch_kernel_stats(-1, C.byref(ks)) == _lib.E_BADARG
    n_params = omlp.IN * omlp.HID + omlp.HID + omlp.HID * omlp.HID + omlp.HID + omlp.HID * omlp.OUT + omlp.OUT
    assert lib.ssnalm_mlp_param_count() == n_params == synth.mlp_init(0).size
    assert lib.ssnalm_mlp_forward(a, a, 0, a, a, None) == _lib.E_BADARG
    assert b"n must be" in lib.ssnalm_last_error()
    assert lib.ssnalm_mlp_forward(None, a, 4, a, a, None) == _lib.E_BADARG
    assert lib.ssnalm_mlp_adam(None, a, a, a, 4, 1e-3, 0.9, 0.999, 1e-8, 1, None) == _lib.E_BADARG
