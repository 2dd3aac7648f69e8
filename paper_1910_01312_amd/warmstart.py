"""Learned warm start for the SSsNAL solve.

A small network (66 -> 256 -> 256 -> 4, GELU; definition in
include/ssnalm.h) predicts for every sample whether x_i* is 0, strictly
inside (0, C) or C, and x_i*/C when inside.  Its prediction becomes x^0 for
ssnalm_solve, which projects it onto {y^T x = 0, 0 <= x <= C} and sets
omega^0 = A^T x^0 (ssnalm_ws_x0).  The solve that uses the prediction,
ssnalm_ws_solve, leaves out the rows the network rules out as x_i* = 0,
solves the rest, and lets the KKT residual of the full problem judge the
result; plain cold start (x^0 = 0 on all rows) stays the fallback.

Every step runs in the library's HIP kernels: features (ssnalm_ws_features),
forward / backward / Adam (ssnalm_mlp_*), the initial point (ssnalm_ws_x0).
Training data are the method's own solutions of instances of the batched
workload's generator, solved by ssnalm_solve_batch.

    python -m paper_1910_01312_amd.warmstart --instances 4000 --q 256 --out weights.npz
"""
from __future__ import annotations

import argparse
import ctypes as C
import math
import time

import numpy as np
import torch

from . import _lib as L
from .solver import Solver, _dev, _stream_handle, _to_dev, solve_batch

IN, HID, OUT, NPROJ = 66, 256, 4, 64


def _p(t):
    return C.c_void_p(t.data_ptr())


class Net:
    """Parameters (one flat float32 vector on the GPU) and Adam state."""

    def __init__(self, theta):
        self.lib = L.load()
        self.n_params = int(self.lib.ssnalm_mlp_param_count())
        th = _to_dev(theta, torch.float32).reshape(-1).clone()
        if th.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {th.numel()}")
        self.theta = th
        self.m = torch.zeros_like(th)
        self.v = torch.zeros_like(th)
        self.grad = torch.zeros_like(th)
        self.step = 0
        self._work = {}

    def _bufs(self, n, scratch=False):
        key = (n, scratch)
        if key not in self._work:
            dev = self.theta.device
            work = torch.empty(int(self.lib.ssnalm_mlp_work_floats(n)), dtype=torch.float32, device=dev)
            out = torch.empty((n, OUT), dtype=torch.float32, device=dev)
            scr = (torch.empty(int(self.lib.ssnalm_mlp_scratch_floats(n)), dtype=torch.float32, device=dev)
                   if scratch else None)
            self._work = {key: (work, out, scr)}          # keep one shape only
        return self._work[key]

    def forward(self, Z, scratch=False):
        """out (n x 4) = (P0, P1, P2, mult) for features Z (n x 66)."""
        Z = _to_dev(Z, torch.float32)
        n = Z.shape[0]
        work, out, _ = self._bufs(n, scratch)
        L.check(self.lib.ssnalm_mlp_forward(_p(self.theta), _p(Z), n, _p(out), _p(work),
                                            _stream_handle()), "ssnalm_mlp_forward")
        return out

    def gradient(self, Z, status, target, w_mse=1.0):
        """(loss, grad) of the mean loss over the rows of Z."""
        Z = _to_dev(Z, torch.float32)
        st = _to_dev(status, torch.int32)
        tg = _to_dev(target, torch.float32)
        n = Z.shape[0]
        out = self.forward(Z, scratch=True)
        work, _, scr = self._bufs(n, True)
        loss = torch.empty(1, dtype=torch.float32, device=Z.device)
        L.check(self.lib.ssnalm_mlp_backward(_p(self.theta), _p(Z), n, _p(work), _p(out), _p(st),
                                             _p(tg), float(w_mse), _p(self.grad), _p(loss), _p(scr),
                                             _stream_handle()), "ssnalm_mlp_backward")
        return loss, self.grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        L.check(self.lib.ssnalm_mlp_adam(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v),
                                         self.n_params, float(lr), float(beta1), float(beta2),
                                         float(eps), self.step, _stream_handle()), "ssnalm_mlp_adam")

    def train_step(self, Z, status, target, lr, w_mse=1.0):
        loss, _ = self.gradient(Z, status, target, w_mse)
        self.adam(lr)
        return loss

    def save(self, path, **meta):
        np.savez(path, theta=self.theta.cpu().numpy(), **{k: np.asarray(v) for k, v in meta.items()})

    @classmethod
    def load(cls, path):
        with np.load(path, allow_pickle=False) as f:
            return cls(f["theta"])


def features(solver: Solver, R):
    """z (n x 66) of the solver's problem; R: q x 64 projection."""
    Rd = _to_dev(R, torch.float32)
    if Rd.shape != (solver.q, NPROJ):
        raise ValueError(f"R must be {solver.q} x {NPROJ}")
    Z = torch.empty((solver.n, IN), dtype=torch.float32, device=Rd.device)
    L.check(solver._lib.ssnalm_ws_features(solver._ctx, _p(Rd), _p(Z)), "ssnalm_ws_features")
    return Z


def initial_point(solver: Solver, out):
    x0 = torch.empty(solver.n, dtype=torch.float64, device=out.device)
    L.check(solver._lib.ssnalm_ws_x0(solver._ctx, _p(out), _p(x0)), "ssnalm_ws_x0")
    return x0


def labels(solver: Solver, x):
    """Bound status (0: x = 0, 1: inside, 2: x = C; relative threshold
    1e-8 C) and target x / C of a solution x of the solver's problem
    (ssnalm_ws_labels)."""
    xd = _to_dev(x, torch.float64)
    st = torch.empty(solver.n, dtype=torch.int32, device=xd.device)
    tg = torch.empty(solver.n, dtype=torch.float32, device=xd.device)
    L.check(solver._lib.ssnalm_ws_labels(solver._ctx, _p(xd), _p(st), _p(tg)), "ssnalm_ws_labels")
    return st, tg


def warm_solve(solver: Solver, net: Net, R, keep_frac=0.25, max_rounds=3):
    """Solve the solver's problem with the network's status prediction
    (ssnalm_ws_solve): only the keep_frac share of rows least surely at
    x_i* = 0 is kept, the rest is solved, the full-problem KKT residual judges
    the result, margin violators are added back, and the plain cold solve is
    the fallback.  Returns (x, w, info, stats); stats adds t_infer (features
    and network)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Z = features(solver, R)
    out = net.forward(Z)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    dev = out.device
    x = torch.empty(solver.n, dtype=torch.float64, device=dev)
    w = torch.empty(solver.q, dtype=torch.float64, device=dev)
    info = L.Info()
    st = L.WsStats()
    status = solver._lib.ssnalm_ws_solve(solver._ctx, _p(out), float(keep_frac), int(max_rounds),
                                         _p(x), _p(w), C.byref(info), C.byref(st))
    L.check(status, "ssnalm_ws_solve")
    d = info.as_dict()
    d["status_name"] = L.STATUS_NAMES.get(status, str(status))
    stats = {"t_infer": t_infer, "rounds": st.rounds, "kept": st.kept, "fallback": bool(st.fallback),
             "rkkt_full": st.rkkt_full, "t_reduced": st.t_reduced}
    return x, w, d, stats


# ------------------------------------------------------------------ training data
def training_instances(count, n=4096, q=128, seed=0, nc_lo=2e2, nc_hi=2e7):
    """Specs of the training instances: the batched workload's generator at
    n rows, with n C log-uniform in [nc_lo, nc_hi] (the range of n C over
    the evaluation instances), seeds disjoint from evaluation."""
    rng = np.random.default_rng(20191003 + 900_000 + seed)
    lognc = rng.uniform(math.log10(nc_lo), math.log10(nc_hi), size=count)
    return [{"n": n, "q": q, "C": float(10.0 ** lognc[k] / n), "seed": 20191003 + 1_000_000 + 1000 * seed + k}
            for k in range(count)]


def build_dataset(specs, R, make_problem, chunk=512, log=None):
    """Solve every instance (ssnalm_solve_batch for q <= 128, else one
    ssnalm_solve each), compute its features and labels; returns GPU tensors (Z, status, target) and per-instance
    solve records."""
    Zs, Ss, Ts, recs = [], [], [], []
    for c0 in range(0, len(specs), chunk):
        part = specs[c0:c0 + chunk]
        probs = []
        for sp in part:
            X, y = make_problem(sp)
            probs.append((torch.from_numpy(X).to(_dev()), torch.from_numpy(y).to(_dev()), sp["C"]))
        batched = probs[0][0].shape[1] <= 128          # the batched solver's q limit
        res = solve_batch(probs, tol=1e-6, want_w=False) if batched else [None] * len(probs)
        for (Xd, yd, C_), r in zip(probs, res):
            with Solver(Xd, yd, C_, tol=1e-6) as s:
                x, _, info = r if batched else s.solve()
                Zs.append(features(s, R))
                st, tg = labels(s, x)
            Ss.append(st)
            Ts.append(tg)
            recs.append({"status": info["status_name"], "newton": info["iters_inner"]})
        if log:
            log(f"[warmstart] solved and featurised {c0 + len(part)} / {len(specs)} instances")
    return torch.cat(Zs), torch.cat(Ss), torch.cat(Ts), recs


def train(net: Net, Z, status, target, epochs=3, batch=4096, lr=1e-3, w_mse=1.0, seed=0, log=None):
    """Adam over shuffled minibatches; returns the mean loss of every epoch."""
    n = Z.shape[0]
    g = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(g.permutation(n)).to(Z.device)
        tot, cnt = torch.zeros((), dtype=torch.float64, device=Z.device), 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            loss = net.train_step(Z[idx], status[idx], target[idx], lr, w_mse)
            tot += loss[0].double()
            cnt += 1
        hist.append(float(tot) / max(cnt, 1))
        if log:
            log(f"[warmstart] epoch {ep}: mean loss {hist[-1]:.4f}")
    return hist


def main():
    ap = argparse.ArgumentParser(description="train the warm-start network")
    ap.add_argument("--instances", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", required=True)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--q", type=int, default=256)
    args = ap.parse_args()
    import sys

    import synth

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    specs = training_instances(args.instances, q=args.q)
    R = synth.projection_matrix(args.q)
    t = time.perf_counter()
    Z, st, tg, recs = build_dataset(
        specs, R, lambda sp: synth.mixture_problem(sp["n"], q=sp["q"], seed=sp["seed"]), log=log)
    log(f"[warmstart] dataset {Z.shape[0]} rows in {time.perf_counter() - t:.1f} s; "
        f"status shares {[float((st == k).float().mean()) for k in range(3)]}")
    net = Net(synth.mlp_init(args.init_seed))
    hist = train(net, Z, st, tg, epochs=args.epochs, lr=args.lr, log=log)
    net.save(args.out, loss=np.array(hist), instances=args.instances, q=args.q,
             rows=specs[0]["n"], epochs=args.epochs, lr=args.lr)
    log(f"[warmstart] saved {args.out}")


if __name__ == "__main__":
    main()
