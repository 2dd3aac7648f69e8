"""Python front end of the HIP SSsNAL library.

PyTorch provides the device memory and the stream; every step of the solve
runs in the library's kernels (see include/ssnalm.h).  Inputs may be torch
tensors already on the GPU or NumPy arrays, which are copied to the GPU once.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the SSsNAL library runs on an MI355X (gfx950) only")
    return torch.device("cuda", torch.cuda.current_device())


def _to_dev(a, dtype=None):
    if isinstance(a, torch.Tensor):
        t = a if a.is_cuda else a.to(_dev())
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(_dev())
    if dtype is not None and t.dtype != dtype:
        t = t.to(dtype)
    return t.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_OPT_KEYS = {"sigma0", "rho", "sigma_max", "mu", "ls_delta", "tau", "eta", "eps_decay",
             "floor_rel", "max_outer", "max_inner", "max_backtracks", "newton", "precision",
             "max_cg", "verbose", "check_finite", "profile", "batch_graphs", "autotune", "lowrank"}


def make_options(**kw) -> L.Options:
    o = L.default_options()
    for k, v in kw.items():
        if k not in _OPT_KEYS:
            raise TypeError(f"unknown option {k}")
        if k == "newton" and isinstance(v, str):
            v = {"auto": L.NEWTON_AUTO, "chol": L.NEWTON_CHOL, "pcg": L.NEWTON_PCG}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": L.PREC_FP64, "mixed": L.PREC_MIXED}[v]
        setattr(o, k, v)
    return o


class Solver:
    """One problem bound to a library context.

    Dense: X is (n, q) float64 / float32 / bfloat16 (a torch.bfloat16 tensor
    or raw uint16 bit patterns with bf16=True).  CSR: pass values, col_idx and
    row_ptr.  y holds labels in {+1, -1}.
    """

    def __init__(self, X=None, y=None, C_=1.0, tol=1e-6, *, csr=None, bf16=False, **opts):
        lib = L.load()
        self._keep = []
        prob = L.Problem()
        if csr is not None:
            values, col_idx, row_ptr, n, q = csr
            v = _to_dev(values)
            if v.dtype not in (torch.float32, torch.float64):
                v = v.to(torch.float32)
            ci = _to_dev(col_idx, torch.int32)
            rp = _to_dev(row_ptr, torch.int64)
            prob.kind = L.CSR
            prob.dtype = L.F64 if v.dtype == torch.float64 else L.F32
            prob.n, prob.q, prob.nnz = int(n), int(q), int(v.numel())
            prob.X, prob.row_ptr, prob.col_idx = v.data_ptr(), rp.data_ptr(), ci.data_ptr()
            self._keep += [v, ci, rp]
        else:
            if isinstance(X, torch.Tensor) and X.dtype == torch.bfloat16:
                Xd = _to_dev(X).view(torch.int16)
                dt = L.BF16
            elif bf16:
                Xd = _to_dev(np.asarray(X).view(np.int16) if not isinstance(X, torch.Tensor) else X)
                dt = L.BF16
            else:
                Xd = _to_dev(X)
                if Xd.dtype == torch.float64:
                    dt = L.F64
                elif Xd.dtype == torch.float32:
                    dt = L.F32
                else:
                    raise TypeError(f"unsupported X dtype {Xd.dtype}")
            n, q = Xd.shape
            prob.kind = L.DENSE
            prob.dtype = dt
            prob.n, prob.q, prob.nnz = int(n), int(q), 0
            prob.X = Xd.data_ptr()
            self._keep.append(Xd)
        yd = _to_dev(y, torch.int8)
        self._keep.append(yd)
        prob.y = yd.data_ptr()
        prob.C = float(C_)
        prob.tol = float(tol)
        self.n, self.q, self.C, self.tol = int(prob.n), int(prob.q), float(C_), float(tol)
        self.y = yd
        self.problem = prob
        self.options = make_options(**opts)
        ctx = C.c_void_p()
        L.check(lib.ssnalm_create(C.byref(ctx), C.byref(prob), C.byref(self.options),
                                  _stream_handle()), "ssnalm_create")
        self._ctx = ctx
        self._lib = lib

    # ------------------------------------------------------------------ solve
    def solve(self, x0=None):
        """Returns (x, w, info) with x, w torch float64 tensors on the GPU."""
        dev = _dev()
        x = torch.empty(self.n, dtype=torch.float64, device=dev)
        w = torch.empty(self.q, dtype=torch.float64, device=dev)
        info = L.Info()
        x0d = _to_dev(x0, torch.float64) if x0 is not None else None
        b = C.c_double(float("nan"))
        st = self._lib.ssnalm_solve(self._ctx, _ptr(x0d), _ptr(x), _ptr(w), C.byref(b),
                                    C.byref(info))
        L.check(st, "ssnalm_solve")
        d = info.as_dict()
        d["b_out"] = b.value
        d["status_name"] = L.STATUS_NAMES.get(st, str(st))
        return x, w, d

    # ------------------------------------------------------------------ steps
    def amul(self, v):
        v = _to_dev(v, torch.float64)
        t = torch.empty(self.n, dtype=torch.float64, device=v.device)
        L.check(self._lib.ssnalm_op_amul(self._ctx, _ptr(v), _ptr(t)), "ssnalm_op_amul")
        return t

    def atmul(self, z):
        z = _to_dev(z, torch.float64)
        r = torch.empty(self.q, dtype=torch.float64, device=z.device)
        L.check(self._lib.ssnalm_op_atmul(self._ctx, _ptr(z), _ptr(r)), "ssnalm_op_atmul")
        return r

    def project(self, v):
        v = _to_dev(v, torch.float64)
        x = torch.empty(self.n, dtype=torch.float64, device=v.device)
        m = torch.empty(self.n, dtype=torch.uint8, device=v.device)
        lam, p, passes = C.c_double(), C.c_int64(), C.c_int32()
        L.check(self._lib.ssnalm_op_project(self._ctx, _ptr(v), _ptr(x), _ptr(m), C.byref(lam),
                                            C.byref(p), C.byref(passes)), "ssnalm_op_project")
        return x, m, lam.value, p.value, passes.value

    def newton(self, free_mask, g, sigma, cg_tol=1e-12):
        fm = _to_dev(free_mask, torch.uint8)
        g = _to_dev(g, torch.float64)
        d = torch.empty(self.q, dtype=torch.float64, device=g.device)
        it = C.c_int32()
        L.check(self._lib.ssnalm_op_newton(self._ctx, _ptr(fm), _ptr(g), float(sigma),
                                           float(cg_tol), _ptr(d), C.byref(it)),
                "ssnalm_op_newton")
        return d, it.value

    def gram(self, free_mask):
        fm = _to_dev(free_mask, torch.uint8)
        G = torch.empty(self.q * self.q, dtype=torch.float64, device=fm.device)
        L.check(self._lib.ssnalm_op_gram(self._ctx, _ptr(fm), _ptr(G)), "ssnalm_op_gram")
        return G.view(self.q, self.q)

    def linesearch_trial(self, u, t, lam, alpha, sigma):
        u = _to_dev(u, torch.float64)
        t = _to_dev(t, torch.float64)
        la, dh = C.c_double(), C.c_double()
        L.check(self._lib.ssnalm_op_linesearch_trial(self._ctx, _ptr(u), _ptr(t), float(lam),
                                                     float(alpha), float(sigma), C.byref(la),
                                                     C.byref(dh)), "ssnalm_op_linesearch_trial")
        return la.value, dh.value

    def rkkt(self, x):
        x = _to_dev(x, torch.float64)
        r, b = C.c_double(), C.c_double()
        L.check(self._lib.ssnalm_op_rkkt(self._ctx, _ptr(x), C.byref(r), C.byref(b)),
                "ssnalm_op_rkkt")
        return r.value, b.value

    def set_profile(self, profile):
        """HIP-event timing: 0 off, 1 all classes, or a mask with bit (k + 1)
        for class k of K_NAMES."""
        L.check(self._lib.ssnalm_set_profile(self._ctx, int(profile)), "ssnalm_set_profile")

    def kernel_stats(self, reset=False):
        """Per-class kernel statistics (needs profile=1): {name: {launches,
        seconds, bytes, flops}}."""
        out = {}
        for k, name in enumerate(L.K_NAMES):
            ks = L.KStat()
            L.check(self._lib.ssnalm_kernel_stats(self._ctx, k, C.byref(ks), 0),
                    "ssnalm_kernel_stats")
            out[name] = {"launches": ks.launches, "seconds": ks.seconds, "bytes": ks.bytes,
                         "flops": ks.flops}
        if reset:
            ks = L.KStat()
            L.check(self._lib.ssnalm_kernel_stats(self._ctx, 0, C.byref(ks), 1),
                    "ssnalm_kernel_stats")
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.ssnalm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class SVR(Solver):
    """eps-SVR (ssnalm_create_svr): dense X (n, q), regression targets y (n).
    solve() returns (xz, w, info) with xz = [x; z] (2n doubles), w the
    primal weights X^T (z - x) and info["b"] the bias of w^T x + b."""

    def __init__(self, X, y, C_=1.0, eps=0.1, tol=1e-6, *, bf16=False, **opts):
        lib = L.load()
        self._keep = []
        Xd, dt = _dense_dev(X, bf16)
        yd = _to_dev(y, torch.float64)
        self._keep += [Xd, yd]
        n, q = Xd.shape
        prob = L.SvrProblem()
        prob.kind, prob.dtype = L.DENSE, dt
        prob.n, prob.q = int(n), int(q)
        prob.X, prob.y = Xd.data_ptr(), yd.data_ptr()
        prob.C, prob.eps, prob.tol = float(C_), float(eps), float(tol)
        self.n, self.q, self.C, self.tol = 2 * int(n), int(q), float(C_), float(tol)
        self.problem = prob
        self.options = make_options(**opts)
        ctx = C.c_void_p()
        L.check(lib.ssnalm_create_svr(C.byref(ctx), C.byref(prob), C.byref(self.options),
                                      _stream_handle()), "ssnalm_create_svr")
        self._ctx = ctx
        self._lib = lib


class General(Solver):
    """The unified problem (P) (ssnalm_create_general): min 1/2 |B^T x|^2 +
    c^T x s.t. a^T x = d, l <= x <= u, with dense B (n, q) and vectors c, a,
    l, u (n).  solve() returns (x, w = B^T x, info); info["b"] is the
    multiplier of a^T x = d."""

    def __init__(self, B, c, a, l, u, d=0.0, tol=1e-6, *, bf16=False, **opts):
        lib = L.load()
        self._keep = []
        Bd, dt = _dense_dev(B, bf16)
        vecs = [_to_dev(v, torch.float64) for v in (c, a, l, u)]
        self._keep += [Bd, *vecs]
        n, q = Bd.shape
        prob = L.GeneralProblem()
        prob.kind, prob.dtype = L.DENSE, dt
        prob.n, prob.q = int(n), int(q)
        prob.B = Bd.data_ptr()
        prob.c, prob.a, prob.l, prob.u = (v.data_ptr() for v in vecs)
        prob.d, prob.tol = float(d), float(tol)
        self.n, self.q, self.C, self.tol = int(n), int(q), float("nan"), float(tol)
        self.problem = prob
        self.options = make_options(**opts)
        ctx = C.c_void_p()
        L.check(lib.ssnalm_create_general(C.byref(ctx), C.byref(prob), C.byref(self.options),
                                          _stream_handle()), "ssnalm_create_general")
        self._ctx = ctx
        self._lib = lib



class KernelSVC(Solver):
    """The C-SVC dual with a nonlinear kernel (ssnalm_create_kernel):
    Q_ij = y_i y_j k(x_i, x_j) with k = "rbf" (exp(-|x - z|^2 / (2 alpha)))
    or "linear" (x^T z), formed once on the GPU in fp64 and kept resident.
    solve() returns (x, None, info); amul(v) is Q v (n -> n); newton_step()
    is the Proposition 5 step."""

    def __init__(self, X, y, C_=1.0, alpha=1.0, tol=1e-6, *, kernel="rbf", bf16=False, **opts):
        lib = L.load()
        self._keep = []
        Xd, dt = _dense_dev(X, bf16)
        yd = _to_dev(y, torch.int8)
        self._keep += [yd]
        n, q = Xd.shape
        prob = L.KernelProblem()
        prob.kernel = {"rbf": L.KERNEL_RBF, "linear": L.KERNEL_LINEAR}[kernel]
        prob.dtype = dt
        prob.n, prob.q = int(n), int(q)
        prob.X, prob.y = Xd.data_ptr(), yd.data_ptr()
        prob.C, prob.alpha, prob.tol = float(C_), float(alpha), float(tol)
        self.n, self.q, self.C, self.tol = int(n), int(n), float(C_), float(tol)
        self.y = yd
        self.problem = prob
        self.options = make_options(**opts)
        ctx = C.c_void_p()
        L.check(lib.ssnalm_create_kernel(C.byref(ctx), C.byref(prob), C.byref(self.options),
                                         _stream_handle()), "ssnalm_create_kernel")
        self._ctx = ctx
        self._lib = lib
        del Xd                       # the samples are read only while Q is formed

    def solve(self, x0=None):
        dev = _dev()
        x = torch.empty(self.n, dtype=torch.float64, device=dev)
        info = L.Info()
        x0d = _to_dev(x0, torch.float64) if x0 is not None else None
        b = C.c_double(float("nan"))
        st = self._lib.ssnalm_solve(self._ctx, _ptr(x0d), _ptr(x), None, C.byref(b),
                                    C.byref(info))
        L.check(st, "ssnalm_solve")
        d = info.as_dict()
        d["b_out"] = b.value
        d["status_name"] = L.STATUS_NAMES.get(st, str(st))
        return x, None, d

    def newton_step(self, free_mask, s, sigma, cg_tol=1e-12):
        """Returns (d, Q d, d^T Q d, cg_iters)."""
        m = _to_dev(free_mask, torch.uint8)
        sv = _to_dev(s, torch.float64)
        d = torch.empty(self.n, dtype=torch.float64, device=sv.device)
        Qd = torch.empty_like(d)
        dQd = C.c_double()
        it = C.c_int32()
        L.check(self._lib.ssnalm_op_kernel_newton(self._ctx, _ptr(m), _ptr(sv), float(sigma),
                                                  float(cg_tol), _ptr(d), _ptr(Qd), C.byref(dQd),
                                                  C.byref(it)), "ssnalm_op_kernel_newton")
        return d, Qd, dQd.value, it.value

def solve(X, y, C_, tol=1e-6, x0=None, **opts):
    """One-shot solve: returns (x, w, info)."""
    with Solver(X, y, C_, tol, **opts) as s:
        return s.solve(x0)


def _dense_dev(X, bf16=False):
    """Device copy of a dense X and its library dtype code."""
    if isinstance(X, torch.Tensor) and X.dtype == torch.bfloat16:
        return _to_dev(X).view(torch.int16), L.BF16
    if bf16:
        return _to_dev(np.asarray(X).view(np.int16) if not isinstance(X, torch.Tensor) else X), L.BF16
    Xd = _to_dev(X)
    if Xd.dtype == torch.float64:
        return Xd, L.F64
    if Xd.dtype == torch.float32:
        return Xd, L.F32
    raise TypeError(f"unsupported X dtype {Xd.dtype}")


def solve_batch(problems, tol=1e-6, *, bf16=False, want_w=True, **opts):
    """Batched solve (ssnalm_solve_batch): `problems` is a sequence of
    (X, y, C) with dense X of one dtype and one q <= 128.  tol is a number or
    one value per problem.  Returns a list of (x, w, info) per problem."""
    lib = L.load()
    count = len(problems)
    tols = [float(tol)] * count if np.isscalar(tol) else [float(t) for t in tol]
    probs = (L.Problem * count)()
    keep, xs, ws = [], [], []
    dev = _dev()
    for k, (X, y, C_) in enumerate(problems):
        Xd, dt = _dense_dev(X, bf16)
        yd = _to_dev(y, torch.int8)
        keep += [Xd, yd]
        n, q = Xd.shape
        pr = probs[k]
        pr.kind, pr.dtype = L.DENSE, dt
        pr.n, pr.q, pr.nnz = int(n), int(q), 0
        pr.X, pr.y = Xd.data_ptr(), yd.data_ptr()
        pr.C, pr.tol = float(C_), tols[k]
        xs.append(torch.empty(int(n), dtype=torch.float64, device=dev))
        ws.append(torch.empty(int(q), dtype=torch.float64, device=dev) if want_w else None)
    xp = (C.c_void_p * count)(*[x.data_ptr() for x in xs])
    wp = (C.c_void_p * count)(*[w.data_ptr() for w in ws]) if want_w else None
    infos = (L.Info * count)()
    o = make_options(**opts)
    st = lib.ssnalm_solve_batch(count, probs, C.byref(o), _stream_handle(), xp, wp, infos)
    L.check(st, "ssnalm_solve_batch")
    out = []
    for k in range(count):
        d = infos[k].as_dict()
        d["status_name"] = L.STATUS_NAMES.get(infos[k].status, str(infos[k].status))
        out.append((xs[k], ws[k], d))
    return out


def batch_kernel_stats():
    """Kernel statistics of the last solve_batch call on this thread made
    with profile=1: {name: {launches, seconds, bytes, flops}}."""
    lib = L.load()
    out = {}
    for k, name in enumerate(L.K_NAMES):
        ks = L.KStat()
        L.check(lib.ssnalm_batch_kernel_stats(k, C.byref(ks)), "ssnalm_batch_kernel_stats")
        out[name] = {"launches": ks.launches, "seconds": ks.seconds, "bytes": ks.bytes,
                     "flops": ks.flops}
    return out
