"""Writes tests/golden/oracle_refs.json: oracle reference solutions of the
full-size workloads that the GPU parity tests check against.

Every value here comes from the CPU FP64 oracle (`oracle/`) on inputs drawn
by `synth/`; nothing is taken from the HIP library.  The GPU tests draw the
same inputs again, compare the input checksums stored here, and check the
library's objective against the stored f* (relative 1e-8) next to R_KKT
recomputed by the oracle on the returned x.

The references are solved to R_KKT <= 1e-8 (the objective of such a solve
agrees with the best attainable one to ~1e-11 relative on these families).

    python tests/golden/make_refs.py [name ...]      # default: all

Each reference is added to the file when its job ends (the file is read
again at that moment), so jobs may run in separate processes side by side.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ssnal  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_refs.json")


def checksum_dense(X, y):
    return {"sum_x": float(np.sum(X, dtype=np.float64)), "sum_y": int(np.sum(y, dtype=np.int64)),
            "shape": list(X.shape)}


def checksum_csr(vals, ci, rp, y):
    return {"sum_x": float(np.sum(vals, dtype=np.float64)), "sum_col": int(np.sum(ci, dtype=np.int64)),
            "nnz": int(rp[-1]), "sum_y": int(np.sum(y, dtype=np.int64))}


def record(r, t):
    return {"f_star": float(r.obj), "rkkt": float(r.rkkt), "status": r.status, "outer": int(r.outer),
            "newton": int(r.inner), "b": float(r.b), "w_norm": float(np.linalg.norm(r.w)),
            "oracle_seconds": round(t, 1)}


def sparse_text_full():
    vals, ci, rp, y = synth.sparse_text()
    n, q = rp.size - 1, 100_000
    X = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(n, q))
    t = time.perf_counter()
    r = ssnal.solve(X, y, 1.0, tol=1e-8, newton="pcg", max_cg=2000)
    return {"inputs": checksum_csr(vals, ci, rp, y), "C": 1.0, **record(r, time.perf_counter() - t)}


def dense_bf16_full(C):
    bits, y = synth.dense_bf16_directions()
    X = synth.bf16_bits_to_f32(bits).astype(np.float64)
    del bits
    t = time.perf_counter()
    r = ssnal.solve(X, y, C, tol=1e-8)
    return {"inputs": checksum_dense(X, y), "C": C, **record(r, time.perf_counter() - t)}


# the batched workload's family at sizes that reach the batched Gram
# product's per-problem cap (|J| > 16384 in the first Newton step: C > 1
# leaves u = e strictly inside the box, so J is every row)
BATCH_CAP = [{"n": 120_000, "C": 10.0, "seed": 4_100_001},
             {"n": 1_000, "C": 0.01, "seed": 4_100_002},
             {"n": 5_003, "C": 1.0, "seed": 4_100_003}]

# held-out instances of the learned warm start's evaluation family
WARM_EVAL = [{"n": 200_000, "q": 256, "C": C, "seed": 880_000 + k}
             for k, C in enumerate([0.01, 10.0, 100.0])]


def batch_cap():
    out = []
    for p in BATCH_CAP:
        X, y = synth.mixture_problem(p["n"], q=128, seed=p["seed"])
        Xd = X.astype(np.float64)
        t = time.perf_counter()
        r = ssnal.solve(Xd, y, p["C"], tol=1e-8)
        out.append({**p, "inputs": checksum_dense(X, y), **record(r, time.perf_counter() - t)})
    return out


def warm_eval():
    out = []
    for p in WARM_EVAL:
        X, y = synth.mixture_problem(p["n"], q=p["q"], seed=p["seed"])
        Xd = X.astype(np.float64)
        t = time.perf_counter()
        r = ssnal.solve(Xd, y, p["C"], tol=1e-8)
        out.append({**p, "inputs": checksum_dense(X, y), **record(r, time.perf_counter() - t)})
    return out


JOBS = {
    "sparse_text_full": sparse_text_full,
    "dense_bf16_full_C0.1": lambda: dense_bf16_full(0.1),
    "dense_bf16_full_C1": lambda: dense_bf16_full(1.0),
    "batch_gram_cap": batch_cap,
    "warm_eval": warm_eval,
}


def _store(path, name, value):
    """Add one reference to the file at path, re-reading it first (several
    jobs may run side by side, each adding its own entries)."""
    refs = {}
    if os.path.exists(path):
        with open(path) as f:
            refs = json.load(f)
    refs[name] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(refs, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def main(names):
    for name in names or list(JOBS):
        t = time.perf_counter()
        value = JOBS[name]()
        print(f"{name}: {time.perf_counter() - t:.1f} s", flush=True)
        _store(OUT, name, value)


if __name__ == "__main__":
    main(sys.argv[1:])
