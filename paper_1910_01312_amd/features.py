"""RBF kernels through explicit features (Section 4): random Fourier
features and Nystroem features computed by the library's kernels
(ssnalm_rff_features, ssnalm_nystroem_features).  The feature matrix Z is
then solved as a linear problem: Solver(Z, y, C).  Argument marshalling
only."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .solver import _dense_dev, _stream_handle, _to_dev


def _p(t):
    return C.c_void_p(t.data_ptr())


def rff(X, W, out_dtype=torch.float64, bf16=False):
    """Z (n x 2N): cos / sin pairs of X W^T scaled by 1/sqrt(N); W: N x q
    frequencies drawn from N(0, I / alpha)."""
    lib = L.load()
    Xd, dt = _dense_dev(X, bf16)
    Wd = _to_dev(W, torch.float64)
    n, q = Xd.shape
    N = Wd.shape[0]
    if Wd.shape[1] != q:
        raise ValueError("W must have q columns")
    Z = torch.empty((n, 2 * N), dtype=out_dtype, device=Xd.device)
    zdt = L.F64 if out_dtype == torch.float64 else L.F32
    L.check(lib.ssnalm_rff_features(_p(Xd), dt, n, q, _p(Wd), N, _p(Z), zdt, _stream_handle()),
            "ssnalm_rff_features")
    return Z


def nystroem(X, landmarks, alpha, shift=1e-3, out_dtype=torch.float64, bf16=False):
    """Z (n x r) = K_nr L^{-T} with K_rr + shift I = L L^T."""
    lib = L.load()
    Xd, dt = _dense_dev(X, bf16)
    lm = _to_dev(np.asarray(landmarks) if not isinstance(landmarks, torch.Tensor) else landmarks,
                 torch.int32)
    n, q = Xd.shape
    r = lm.numel()
    Z = torch.empty((n, r), dtype=out_dtype, device=Xd.device)
    zdt = L.F64 if out_dtype == torch.float64 else L.F32
    L.check(lib.ssnalm_nystroem_features(_p(Xd), dt, n, q, _p(lm), r, float(alpha), float(shift),
                                         _p(Z), zdt, _stream_handle()), "ssnalm_nystroem_features")
    return Z
