#!/usr/bin/env python3
"""Benchmark of the MI355X SSsNAL solver.

One step = one full solve of the linear C-SVC dual QP to R_KKT <= 1e-6
(Algorithm 1 with Algorithm 3 inside, every §-step of the hot path on the
GPU) with the data already resident in HBM.  The default workload is the
sparse text-like problem: CSR X with n = 500,000 rows, q = 100,000 columns,
~60 nonzeros per row with Zipf(1.1) column frequencies, lognormal values,
L2-normalised rows, noisy linear labels, C = 1.

Prints ONE JSON line with the metric, the per-solve time, the roofline of
the dominant kernel (HIP-event timing inside the library over the timed
solves, algorithmic bytes per launch) and a CPU baseline of the FP64 oracle
measured on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAKS_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
METRIC = "time-to-KKT≤1e-6 per SVM QP (s); matvec HBM GB/s; warm-start vs plain speedup"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of a kernel class per launch, from two rocprofv3 --pmc runs of
# `bench.py --traffic-op CLASS` (FETCH_SIZE, then WRITE_SIZE, KiB summed over
# the class's kernels and divided by the op calls), each scaled by what the
# same counter reads for a plain 1 GiB device copy (profiles/ records the
# commands and readings).  Reported only while the sources of those kernels
# are byte-identical to the ones measured (sha256 of each file below).
MEASURED_TRAFFIC = {
    # X_J^T w in the CG (k_keyed_tr<float, 0> + k_keyed_fix_list), sparse text
    # workload: counters summed over the dispatches of one warm-up and one
    # timed solve, divided by the 2 x 1328 CG iterations that did work
    # (profiles/sparse_text_atmul_J_hbm_traffic.md)
    ("sparse-text", "atmul_J"): {
        "fetch_kib": 52682109.125 + 1168507.875, "write_kib": 2634972.875 + 299527.5, "calls": 2656,
        "fetch_scale": 2.0, "write_scale": 1.0,
        "files": {
            "paper_1910_01312_amd/csrc/kernels_cg.hip":
                "8e85f733a7420d47c946802ee1dfa72364236f54a1c9160ddcf75daaca924fd8",
            "paper_1910_01312_amd/csrc/dev_common.h":
                "a34ef9e72788212b20fbb624e54dbe54c03922933c400472c434eed96aacfd9e",
        },
    },
}


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload, cls):
    m = MEASURED_TRAFFIC.get((workload, cls))
    if not m:
        return None
    for rel, digest in m["files"].items():
        if _sha256(os.path.join(ROOT, rel)) != digest:
            return None
    return (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024.0 / m["calls"]


# the kernels of each class that a traffic probe sums, and their sources, for
# CSR and for dense X
TRAFFIC_KERNELS = {
    "atmul": (["k_mul_y", "k_segsum<float, 0>", "k_segsum_fix", "k_reduce_cols"],
              ["paper_1910_01312_amd/csrc/kernels_sparse.hip", "paper_1910_01312_amd/csrc/kernels_vec.hip",
               "paper_1910_01312_amd/csrc/kernels_dense.hip", "paper_1910_01312_amd/csrc/dev_common.h"]),
    "amul": (["k_sell_amul", "k_segsum<float, 0>", "k_segsum_fix"],
             ["paper_1910_01312_amd/csrc/kernels_sell.hip", "paper_1910_01312_amd/csrc/kernels_sparse.hip",
              "paper_1910_01312_amd/csrc/dev_common.h"]),
    "atmul-dense": (["k_atmul_rows", "k_reduce_cols"],
                    ["paper_1910_01312_amd/csrc/kernels_dense.hip", "paper_1910_01312_amd/csrc/lane_ops.h",
                     "paper_1910_01312_amd/csrc/dev_common.h"]),
    "amul-dense": (["k_amul_rows"],
                   ["paper_1910_01312_amd/csrc/kernels_dense.hip", "paper_1910_01312_amd/csrc/dev_common.h"]),
}


def make_workload(name, C=None):
    import numpy as np
    import synth
    if name == "dense-bf16":
        bits, y = synth.dense_bf16_directions()
        Cv = 1.0 if C is None else C
        cfg = {"workload": f"dense bf16 n=1000000 q=512, 4 informative directions, 5% flips, C={Cv}",
               "n": 1_000_000, "q": 512, "C": Cv, "tol": 1e-6}
        return {"X": bits, "bf16": True, "y": y, "C": Cv, "cfg": cfg}
    if name == "sparse-text":
        vals, ci, rp, y = synth.sparse_text()
        n, q = rp.size - 1, 100_000
        cfg = {"workload": "sparse-text CSR n=500000 q=100000 ~60 nnz/row Zipf(1.1) fp32 values",
               "n": int(n), "q": q, "nnz": int(vals.size), "C": 1.0, "tol": 1e-6}
        return {"csr": (vals, ci, rp, n, q), "y": y, "C": 1.0, "cfg": cfg}
    if name == "dense-small":
        X, y = synth.dense_two_gaussians()
        cfg = {"workload": "dense two-Gaussian n=2000 q=50 fp64", "n": 2000, "q": 50,
               "C": 1.0, "tol": 1e-6}
        return {"X": X, "y": y, "C": 1.0, "cfg": cfg}
    raise SystemExit(f"unknown workload {name}")


def oracle_sample(wl, budget_s, gpu_newton_steps):
    """Time the FP64 oracle on the same workload for about budget_s seconds
    and scale its seconds per Newton step to the GPU solve's step count."""
    import numpy as np
    import psutil
    import scipy.sparse as sp
    from oracle import ssnal
    if "csr" in wl:
        vals, ci, rp, n, q = wl["csr"]
        X = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(n, q))
        mode = "pcg"
    elif wl.get("bf16"):
        import synth
        X = synth.bf16_bits_to_f32(wl["X"]).astype(np.float64)
        mode = "qspace"
    else:
        X = wl["X"]
        mode = "qspace"
    proc = psutil.Process()
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover - reporting only
        blas_threads = None
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    r = ssnal.solve(X, wl["y"], wl["C"], tol=1e-6, newton=mode, time_budget_s=budget_s,
                    max_cg=2000)
    wall = time.perf_counter() - t0
    c1 = proc.cpu_times()
    busy = ((c1.user - c0.user) + (c1.system - c0.system)) / max(wall, 1e-9)
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    steps = max(r.inner, 1)
    if r.status == "OK":
        est = wall
        sample = (f"full oracle solve of the same workload ({r.inner} Newton steps, "
                  f"{r.cg_iters} CG iterations, {wall:.1f} s)")
    else:
        est = wall / steps * gpu_newton_steps
        sample = (f"first {wall:.1f} s of the oracle solve of the same workload: {steps} Newton "
                  f"steps ({r.cg_iters} CG iterations, {r.outer} ALM iterations); seconds per "
                  f"Newton step x the {gpu_newton_steps} Newton steps of the GPU solve")
    return {"value": est, "unit": "s",
            "cores": int(blas_threads) if blas_threads else max(1, round(busy)),
            "kind": "oracle", "sample": sample,
            "nproc": os.cpu_count(), "cpu_model": cpu_model, "blas_threads": blas_threads,
            "avg_busy_cores": round(busy, 2)}


def run_batch(args):
    """Batched workload: 256 dense FP32 QPs (two-class Gaussian mixtures,
    q = 128, n_k uniform in [1000, 200000], C_k on the log grid 1e-3..1e2)
    solved by one ssnalm_solve_batch call per step; value = seconds per QP.
    Also times the same QPs one by one through ssnalm_solve (plain cold-start
    GPU solves) and checks sampled solutions with the oracle's KKT code."""
    import numpy as np
    import torch
    import synth
    from paper_1910_01312_amd import _lib
    from paper_1910_01312_amd.solver import Solver, batch_kernel_stats, solve_batch
    from oracle import ssnal

    _lib.load()
    fam = synth.batch_family(count=args.count)
    log(f"[bench] generating {len(fam)} problems (sum n = {sum(p['n'] for p in fam)})")
    t = time.perf_counter()
    probs = []
    for i, p in enumerate(fam):
        X, y = synth.mixture_problem(p["n"], q=p["q"], seed=p["seed"])
        probs.append((torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), p["C"]))
        if i % 32 == 31:
            log(f"[bench]   {i + 1} problems on the GPU ({time.perf_counter() - t:.1f} s)")
    torch.cuda.synchronize()
    log(f"[bench] generated in {time.perf_counter() - t:.1f} s")
    count = len(probs)
    ntot = sum(p["n"] for p in fam)
    for i in range(args.warmup):
        t = time.perf_counter()
        out = solve_batch(probs, tol=1e-6, want_w=False, profile=1)
        st = [o[2]["status_name"] for o in out]
        log(f"[bench] warmup {i}: {time.perf_counter() - t:.3f} s, OK {st.count('OK')}/{count}, "
            f"max newton {max(o[2]['iters_inner'] for o in out)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = solve_batch(probs, tol=1e-6, want_w=False, profile=1)
        log(f"[bench] step {i} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_batch = (t1 - t0) / args.steps
    ks = batch_kernel_stats()["amul"]
    roofline = None
    if ks["launches"]:
        avg = ks["seconds"] / ks["launches"]
        achieved = ks["bytes"] / ks["launches"] / avg / 1e9
        roofline = {"bound": "hbm", "kernel": "batched A v (all active problems)",
                    "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "bytes_per_launch": ks["bytes"] / ks["launches"],
                    "avg_launch_us": avg * 1e6, "launches": ks["launches"]}
    infos = [o[2] for o in out]
    # oracle KKT check on sampled problems: smallest and largest n, both C ends
    idx = sorted({int(np.argmin([p["n"] for p in fam])), int(np.argmax([p["n"] for p in fam])),
                  0, count - 1})
    checks = []
    for k in idx:
        X, y = synth.mixture_problem(fam[k]["n"], q=fam[k]["q"], seed=fam[k]["seed"])
        R, _ = ssnal.rkkt(X.astype(np.float64), y, fam[k]["C"], out[k][0].cpu().numpy())
        checks.append({"problem": k, "n": fam[k]["n"], "C": fam[k]["C"], "rkkt_oracle": R})
    seq = None
    if not args.no_seq:
        log("[bench] sequential single-problem GPU solves of the same QPs")
        tsum, st_ok = 0.0, 0
        for k, (Xd, yd, C_) in enumerate(probs):
            with Solver(Xd, yd, C_, tol=1e-6) as s:
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, _, inf = s.solve()
                torch.cuda.synchronize()
                tsum += time.perf_counter() - t
                st_ok += inf["status_name"] == "OK"
            if k % 32 == 31:
                log(f"[bench]   {k + 1} sequential solves, {tsum:.1f} s")
        seq = {"total_s": tsum, "per_qp_s": tsum / count, "ok": st_ok,
               "batched_speedup": tsum / per_batch}
    cpu = None
    if not args.no_cpu_baseline:
        import psutil
        log(f"[bench] cpu baseline: oracle solves for ~{args.cpu_budget:.0f} s")
        proc = psutil.Process()
        c0 = proc.cpu_times()
        w0 = time.perf_counter()
        tsolve, nrows, done = 0.0, 0, 0
        for p in fam:
            if time.perf_counter() - w0 > args.cpu_budget:
                break
            X, y = synth.mixture_problem(p["n"], q=p["q"], seed=p["seed"])
            Xo = X.astype(np.float64)
            t = time.perf_counter()
            r = ssnal.solve(Xo, y, p["C"], tol=1e-6)
            tsolve += time.perf_counter() - t
            nrows += p["n"]
            done += 1
        wall = time.perf_counter() - w0
        c1 = proc.cpu_times()
        cores = max(1, round(((c1.user - c0.user) + (c1.system - c0.system)) / max(wall, 1e-9)))
        est_total = tsolve / max(nrows, 1) * ntot
        cpu = {"value": est_total / count, "unit": "s", "cores": int(cores), "kind": "oracle",
               "sample": (f"oracle solves of the first {done} QPs of the family ({nrows} rows, "
                          f"{tsolve:.1f} s), seconds per row x the family's {ntot} rows / {count} QPs")}
    out_json = {
        "metric": METRIC,
        "value": per_batch / count,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_batch * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {count} dense fp32 QPs, q=128, n in [1000, 200000] "
                               f"(sum {ntot}), two-class Gaussian mixtures, C log grid 1e-3..1e2",
                   "count": count, "sum_n": ntot, "q": 128, "tol": 1e-6},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batch": {"seconds_per_batch": per_batch,
                  "ok": sum(i["status_name"] == "OK" for i in infos),
                  "newton_max": max(i["iters_inner"] for i in infos),
                  "newton_sum": sum(i["iters_inner"] for i in infos),
                  "outer_max": max(i["iters_outer"] for i in infos),
                  "oracle_checks": checks, "sequential_gpu": seq},
    }
    print(json.dumps(out_json), flush=True)


def run_warmstart(args):
    """Learned warm start: 16 held-out dense fp32 QPs (n = 200,000, q = 256,
    the batched family's generator, C on the log grid 1e-3..1e2), each
    solved cold (ssnalm_solve from x = 0) and with the committed network
    (features + inference + screened solves + full-problem KKT check);
    value = mean warm time per QP, speedup = T_cold / (T_infer + T_warm)."""
    import numpy as np
    import torch
    import synth
    from paper_1910_01312_amd import _lib
    from paper_1910_01312_amd.solver import Solver
    from paper_1910_01312_amd.warmstart import Net, warm_solve
    from oracle import ssnal

    _lib.load()
    net = Net.load(os.path.join(ROOT, "paper_1910_01312_amd", "data", "warmstart_q256.npz"))
    R = synth.projection_matrix(256)
    count = args.count if args.count != 256 else 16
    Cs = [10.0 ** (-3.0 + 5.0 * k / max(count - 1, 1)) for k in range(count)]
    rows = []
    tc_sum = tw_sum = ti_sum = 0.0
    for k, C in enumerate(Cs):
        X, y = synth.mixture_problem(200_000, q=256, seed=synth.seed_for(5, k + 1))
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        with Solver(Xd, yd, C, tol=1e-6) as s:
            s.solve()
            tcs, tws = [], []
            for _ in range(args.steps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                xc, _, ic = s.solve()
                torch.cuda.synchronize()
                tcs.append(time.perf_counter() - t)
                t = time.perf_counter()
                xw, _, iw, sw = warm_solve(s, net, R, keep_frac=args.keep_frac)
                torch.cuda.synchronize()
                tws.append(time.perf_counter() - t)
        tc, tw = float(np.median(tcs)), float(np.median(tws))
        tc_sum += tc
        tw_sum += tw
        ti_sum += sw["t_infer"]
        rec = {"C": C, "cold_s": tc, "warm_s": tw, "t_infer": sw["t_infer"], "kept": sw["kept"],
               "rounds": sw["rounds"], "fallback": sw["fallback"], "newton_cold": ic["iters_inner"],
               "newton_warm": iw["iters_inner"], "status": iw["status_name"]}
        if k in (0, count // 2, count - 1):
            rec["rkkt_oracle"] = ssnal.rkkt(X.astype(np.float64), y, C, xw.cpu().numpy())[0]
        rows.append(rec)
        log(f"[bench] C={C:.3g}: cold {tc:.3f} s, warm {tw:.3f} s, kept {sw['kept']}, rounds {sw['rounds']}")
    out = {
        "metric": METRIC,
        "value": tw_sum / count,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": tw_sum / count * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"learned warm start: {count} held-out dense fp32 QPs n=200000 q=256, "
                               "C log grid 1e-3..1e2", "count": count, "keep_frac": args.keep_frac},
        "roofline": None,
        "cpu_baseline": None,
        "warmstart": {"speedup": tc_sum / tw_sum, "cold_s_per_qp": tc_sum / count,
                      "warm_s_per_qp": tw_sum / count, "infer_s_per_qp": ti_sum / count,
                      "per_qp": rows},
    }
    print(json.dumps(out), flush=True)


def run_kernel(args):
    """Nonlinear-kernel workload (Table 3's problem, the a7a shape): the RBF
    C-SVC dual with n = 16100 samples of q = 122 features in [0, 1]
    (two-class Gaussian mixture, rescaled, 10% of the labels inverted),
    C = 32, alpha = 4 (a7a's parameters in Table 3).  Q is formed
    once when the context is created (reported as create_s); a step is one
    solve from x^0 = 0 with Q resident."""
    import numpy as np
    import torch
    import synth
    from paper_1910_01312_amd import _lib
    from paper_1910_01312_amd.solver import KernelSVC
    from oracle import features, kernel
    n, q = args.kernel_n, 122
    Cv = 32.0 if args.C is None else args.C
    alpha = 4.0
    log(f"[bench] generating workload rbf-kernel n={n}")
    X, y = synth.rbf_problem(n, q, seed=synth.seed_for(6), flip=0.1)
    cfg = {"workload": f"RBF-kernel C-SVC n={n} q={q} (a7a shape), features in [0,1], 10% label noise, "
                       f"alpha={alpha}, C={Cv}, Q resident in fp64",
           "n": n, "q": q, "C": Cv, "alpha": alpha, "tol": 1e-6}
    t = time.perf_counter()
    s = KernelSVC(X, y, Cv, alpha, tol=1e-6, verbose=1 if args.verbose else 0)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t
    log(f"[bench] create (Q formation) {create_s:.3f} s")
    K_NAMES = _lib.K_NAMES
    ks_all = None
    for i in range(max(args.warmup, 1)):
        s.set_profile(1)
        x, _, info = s.solve()
        ks_all = s.kernel_stats(reset=True)
        log(f"[bench] warmup {i}: {info['time_s']:.3f} s status={info['status_name']} "
            f"R_KKT={info['rkkt']:.2e} outer={info['iters_outer']} newton={info['iters_inner']} "
            f"cg={info['cg_iters']} p={info['p']}")
    best = None
    for name, k in ks_all.items():
        if k["launches"] == 0 or (k["bytes"] <= 0 and k["flops"] <= 0):
            continue
        if best is None or k["seconds"] > ks_all[best]["seconds"]:
            best = name
    s.set_profile((1 << (K_NAMES.index(best) + 1)) if best is not None else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        x, _, info = s.solve()
        infos.append(info)
        log(f"[bench] step {i}: {info['time_s']:.3f} s R_KKT={info['rkkt']:.2e}")
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / args.steps
    ks = s.kernel_stats()
    roofline = None
    if best is not None and ks[best]["launches"]:
        k = ks[best]
        avg = k["seconds"] / k["launches"]
        if best == "chol":
            achieved = k["flops"] / k["launches"] / avg / 1e12
            roofline = {"bound": "alu", "kernel": best, "achieved": achieved,
                        "peak": PEAKS_TFLOPS["f64"], "unit": "TFLOP/s",
                        "frac": achieved / PEAKS_TFLOPS["f64"], "traffic": None,
                        "flops_per_launch": k["flops"] / k["launches"], "avg_launch_us": avg * 1e6,
                        "launches": k["launches"]}
        else:
            achieved = k["bytes"] / k["launches"] / avg / 1e9
            roofline = {"bound": "hbm", "kernel": best, "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic("rbf-kernel", best),
                        "bytes_per_launch": k["bytes"] / k["launches"],
                        "avg_launch_us": avg * 1e6, "launches": k["launches"]}
    xh = x.cpu().numpy()
    s.close()
    K = features.rbf_kernel(X, X, alpha)
    Q = kernel.kernel_q(K, y)
    rk_oracle = kernel.rkkt_q(Q, y, Cv, xh)[0]
    del Q
    cpu = None
    if not args.no_cpu_baseline:
        import psutil
        log(f"[bench] cpu baseline: kernel oracle for ~{args.cpu_budget:.0f} s")
        proc = psutil.Process()
        c0 = proc.cpu_times()
        t0 = time.perf_counter()
        r = kernel.solve_p5(K, y, Cv, tol=1e-6, time_budget_s=args.cpu_budget)
        wall = time.perf_counter() - t0
        c1 = proc.cpu_times()
        busy = ((c1.user - c0.user) + (c1.system - c0.system)) / max(wall, 1e-9)
        steps = max(r.inner, 1)
        gpu_steps = infos[-1]["iters_inner"]
        if r.status == "OK":
            est, sample = wall, f"full w-space oracle solve ({r.inner} Newton steps, {wall:.1f} s)"
        else:
            est = wall / steps * gpu_steps
            sample = (f"first {wall:.1f} s of the w-space oracle solve: {r.inner} Newton steps; "
                      f"seconds per Newton step x the {gpu_steps} Newton steps of the GPU solve "
                      f"(the first steps, with the largest free sets, cost the most)")
        cpu = {"value": est, "unit": "s", "cores": max(1, round(busy)), "kind": "oracle",
               "sample": sample, "nproc": os.cpu_count(), "avg_busy_cores": round(busy, 2)}
    last = infos[-1]
    out = {
        "metric": "time to solve one kernel C-SVC dual to R_KKT <= 1e-6",
        "value": per, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": per * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
        "roofline": roofline, "cpu_baseline": cpu,
        "solve": {"status": last["status_name"], "rkkt": last["rkkt"], "rkkt_oracle": rk_oracle,
                  "outer": last["iters_outer"], "newton": last["iters_inner"],
                  "cg": last["cg_iters"], "p": last["p"], "n_sv": last["n_sv"], "obj": last["obj"],
                  "gap": last["gap"], "create_s": create_s},
        "kernels_profiled_warmup": {k: {"launches": v["launches"], "ms": v["seconds"] * 1e3,
                        "GBps": (v["bytes"] / v["seconds"] / 1e9) if v["seconds"] > 0 and v["bytes"] > 0 else None,
                        "TFLOPs": (v["flops"] / v["seconds"] / 1e12) if v["seconds"] > 0 and v["flops"] > 0 else None}
                    for k, v in ks_all.items() if v["launches"]},
    }
    print(json.dumps(out), flush=True)


# the other configurations, run after the headline one (each in a child
# process: one warm-up and one timed step, no CPU baseline) and summarised in
# the headline line; skipped once the run has taken OTHER_BUDGET_S
OTHER_WORKLOADS = [
    ("dense-bf16 C=1", ["--workload", "dense-bf16"]),
    ("dense-bf16 C=0.1", ["--workload", "dense-bf16", "--C", "0.1"]),
    ("batch", ["--workload", "batch", "--no-seq"]),
    ("warmstart", ["--workload", "warmstart"]),
    ("rbf-kernel", ["--workload", "rbf-kernel"]),
]
OTHER_BUDGET_S = 300.0
OTHER_TIMEOUT_S = 150.0


def _summary(d):
    r = d.get("roofline") or {}
    out = {"value": d["value"], "unit": d["unit"], "workload": d["config"]["workload"],
           "dtype": d.get("dtype")}
    if r:
        out["roofline"] = {k: r.get(k) for k in ("kernel", "bound", "achieved", "peak", "unit", "frac")}
    sv = d.get("solve")
    if sv:
        out["solve"] = {k: sv.get(k) for k in ("status", "rkkt", "rkkt_oracle", "outer", "newton")}
    if "batch" in d:
        b = d["batch"]
        out["batch"] = {k: b.get(k) for k in ("seconds_per_batch", "ok", "newton_max", "oracle_checks")}
    if "warmstart" in d:
        w = d["warmstart"]
        out["warmstart"] = {k: w.get(k) for k in ("speedup", "cold_s_per_qp", "warm_s_per_qp")}
    return out


def other_workloads(t0):
    import subprocess
    res = {}
    for name, extra in OTHER_WORKLOADS:
        if time.perf_counter() - t0 > OTHER_BUDGET_S:
            res[name] = {"skipped": f"the run had passed {OTHER_BUDGET_S:.0f} s"}
            continue
        cmd = [sys.executable, os.path.abspath(__file__), *extra, "--steps", "1", "--warmup", "1",
               "--no-cpu-baseline", "--no-other-workloads"]
        log(f"[bench] other workload: {name}")
        t = time.perf_counter()
        try:
            p = subprocess.run(cmd, capture_output=True, text=True, timeout=OTHER_TIMEOUT_S)
        except subprocess.TimeoutExpired:
            res[name] = {"skipped": f"no result within {OTHER_TIMEOUT_S:.0f} s"}
            log(f"[bench]   {name}: no result within {OTHER_TIMEOUT_S:.0f} s")
            continue
        lines = [ln for ln in p.stdout.splitlines() if ln.startswith("{")]
        if p.returncode != 0 or not lines:
            res[name] = {"error": f"exit status {p.returncode}", "stderr_tail": p.stderr[-400:]}
            log(f"[bench]   {name}: exit status {p.returncode}")
            continue
        res[name] = _summary(json.loads(lines[-1]))
        log(f"[bench]   {name}: {res[name]['value']:.4g} {res[name]['unit']} "
            f"({time.perf_counter() - t:.0f} s)")
    return res


def main():
    t0 = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sparse-text")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="headline workload: leave out the summaries of the other configurations")
    ap.add_argument("--C", type=float, default=None)
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--count", type=int, default=256, help="batched workload: number of QPs")
    ap.add_argument("--no-seq", action="store_true", help="batched workload: skip the one-by-one solves")
    ap.add_argument("--keep-frac", type=float, default=0.15, help="warm-start workload: rows kept")
    ap.add_argument("--traffic-op", default=None, choices=[None, "atmul", "amul"],
                    help="run only this kernel class (--reps times after one warm-up) for a "
                         "rocprofv3 --pmc traffic reading, then exit")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--kernel-n", type=int, default=16100, help="rbf-kernel workload: samples")
    ap.add_argument("--verbose", action="store_true", help="one line per ALM iteration on stderr")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device 3 times (a plain copy "
                         "kernel of known size, to scale HBM counter readings)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the solver runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1910_01312_amd import _lib
    from paper_1910_01312_amd.solver import Solver

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs the GPU")
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "warmstart":
        run_warmstart(args)
        return
    if args.workload == "rbf-kernel":
        run_kernel(args)
        return
    _lib.load()
    log(f"[bench] generating workload {args.workload}")
    t = time.perf_counter()
    wl = make_workload(args.workload, args.C)
    log(f"[bench] generated in {time.perf_counter() - t:.1f} s")

    kw = {}
    if "csr" in wl:
        kw["csr"] = wl["csr"]
    else:
        kw["X"] = wl["X"]
        if wl.get("bf16"):
            kw["bf16"] = True
            kw["precision"] = args.precision or "mixed"
        elif args.precision:
            kw["precision"] = args.precision
    if "precision" in kw:
        wl["cfg"]["precision"] = kw["precision"]
    t = time.perf_counter()
    s = Solver(y=wl["y"], C_=wl["C"], tol=1e-6, **kw)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t
    log(f"[bench] create {create_s:.2f} s")
    if args.traffic_op:
        # A^T z or A v with random vectors (either op reads every entry of X
        # whatever the vector holds)
        if args.traffic_op == "atmul":
            z = torch.rand(s.n, dtype=torch.float64, device="cuda")
            for _ in range(args.reps + 1):
                s.atmul(z)
        else:
            v = torch.rand(s.q, dtype=torch.float64, device="cuda")
            for _ in range(args.reps + 1):
                s.amul(v)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_op": args.traffic_op, "calls": args.reps + 1,
                          "kernels": TRAFFIC_KERNELS[args.traffic_op + ("-dense" if wl.get("X") is not None
                                                                        else "")][0]}), flush=True)
        s.close()
        calib(args)
        return

    # Warm-up solves time every kernel class; the timed solves time only the
    # dominant class (largest summed time), so the roofline comes from the
    # timed region itself.  The library leaves out of a class's statistics the
    # CG launches that passed through after convergence, so bytes and time
    # cover the same launches.
    K_NAMES = _lib.K_NAMES
    untimed = set()
    ks_all = None
    for i in range(max(args.warmup, 1)):
        s.set_profile(1)
        x, w, info = s.solve()
        ks_all = s.kernel_stats(reset=True)
        log(f"[bench] warmup {i}: {info['time_s']:.3f} s status={info['status_name']} "
            f"R_KKT={info['rkkt']:.2e} trials={info['ls_trials']} passes={info['proj_passes']} outer={info['iters_outer']} newton={info['iters_inner']} "
            f"cg={info['cg_iters']} p={info['p']}")
    # the CG's classes are timed on a sample of their launches (one CG
    # iteration in eight): their share of the solve is the sampled average
    # times the CG iterations that did work
    def class_total(name, k):
        if name in ("amul_J", "atmul_J") and k["launches"]:
            return k["seconds"] / k["launches"] * max(info["cg_iters"], k["launches"])
        return k["seconds"]

    best = None
    for name, k in ks_all.items():
        if name in untimed or k["launches"] == 0 or (k["bytes"] <= 0 and k["flops"] <= 0):
            continue
        if best is None or class_total(name, k) > class_total(best, ks_all[best]):
            best = name
    s.set_profile((1 << (K_NAMES.index(best) + 1)) if best is not None else 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        x, w, info = s.solve()
        infos.append(info)
        log(f"[bench] step {i}: {info['time_s']:.3f} s R_KKT={info['rkkt']:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = (t1 - t0) / args.steps
    ks = s.kernel_stats()

    roofline = None
    if best is not None and ks[best]["launches"]:
        k = ks[best]
        avg = k["seconds"] / k["launches"]
        if best in ("syrk", "chol"):
            achieved = k["flops"] / k["launches"] / avg / 1e12
            peak = PEAKS_TFLOPS["bf16"] if (best == "syrk" and kw.get("precision") == "mixed") else PEAKS_TFLOPS["f64"]
            roofline = {"bound": "mfma" if best == "syrk" else "alu", "kernel": best,
                        "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                        "frac": achieved / peak, "traffic": None,
                        "flops_per_launch": k["flops"] / k["launches"], "avg_launch_us": avg * 1e6,
                        "launches": k["launches"]}
        else:
            achieved = k["bytes"] / k["launches"] / avg / 1e9
            roofline = {"bound": "hbm", "kernel": best, "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic(args.workload, best),
                        "bytes_per_launch": k["bytes"] / k["launches"],
                        "avg_launch_us": avg * 1e6, "launches": k["launches"]}

    # correctness of the timed result, checked by the oracle's own KKT code
    rk_oracle = None
    try:
        import scipy.sparse as sp
        from oracle import ssnal
        xh = x.cpu().numpy()
        if wl.get("bf16"):
            import synth
            Xo = synth.bf16_bits_to_f32(wl["X"])
        elif "csr" in wl:
            vals, ci, rp, n, q = wl["csr"]
            Xo = sp.csr_matrix((vals.astype(np.float64), ci, rp), shape=(n, q))
        else:
            Xo = wl["X"]
        rk_oracle, _ = ssnal.rkkt(Xo, wl["y"], wl["C"], xh)
    except Exception as e:  # pragma: no cover - reporting only
        log(f"[bench] oracle KKT check failed: {e}")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle for ~{args.cpu_budget:.0f} s")
        cpu = oracle_sample(wl, args.cpu_budget, infos[-1]["iters_inner"])

    last = infos[-1]
    out = {
        "metric": METRIC,
        "value": per,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if kw.get("precision") != "mixed" else "bf16+f64",
        "data": "synthetic",
        "config": wl["cfg"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "solve": {"status": last["status_name"], "rkkt": last["rkkt"], "rkkt_oracle": rk_oracle,
                  "outer": last["iters_outer"], "newton": last["iters_inner"],
                  "cg": last["cg_iters"], "proj_passes": last["proj_passes"], "p": last["p"],
                  "n_sv": last["n_sv"], "obj": last["obj"], "lowrank_steps": last["lowrank_steps"],
                  "create_s": create_s},
        "kernels_profiled_warmup": {k: {"launches": v["launches"], "ms": v["seconds"] * 1e3,
                        "ms_per_solve": class_total(k, v) * 1e3,
                        "GBps": (v["bytes"] / v["seconds"] / 1e9) if v["seconds"] > 0 and v["bytes"] > 0 else None}
                    for k, v in ks_all.items() if v["launches"]},
    }
    s.close()
    if args.workload == "sparse-text" and not args.no_other_workloads and not args.calib_copy_mb:
        out["other_workloads"] = other_workloads(t0)
    print(json.dumps(out), flush=True)
    calib(args)


def calib(args):
    """Plain device-to-device copies of known size (scale of the counters)."""
    if not args.calib_copy_mb:
        return
    import torch
    nb = args.calib_copy_mb * (1 << 20)
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copies of {args.calib_copy_mb} MiB done")


if __name__ == "__main__":
    main()
