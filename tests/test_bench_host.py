"""Host logic of bench.py (CPU only, no GPU work): the one-GPU guard, the
summaries of the other configurations, the time budget that skips them, and
the HBM counter reading that is reported only while the measured sources are
unchanged."""
import importlib.util
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_summary_of_a_child_line():
    b = _bench()
    child = {
        "metric": "m", "value": 0.08, "unit": "s", "dtype": "bf16+f64",
        "config": {"workload": "dense bf16 n=1000000 q=512", "n": 1000000},
        "roofline": {"kernel": "chol", "bound": "alu", "achieved": 0.15, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": 0.002, "traffic": None, "launches": 3},
        "solve": {"status": "OK", "rkkt": 5e-7, "rkkt_oracle": 5e-7, "outer": 13, "newton": 66,
                  "cg": 70},
        "kernels_profiled_warmup": {"amul": {}},
    }
    s = b._summary(child)
    assert s["value"] == 0.08 and s["unit"] == "s" and s["workload"] == "dense bf16 n=1000000 q=512"
    assert s["roofline"] == {"kernel": "chol", "bound": "alu", "achieved": 0.15, "peak": 78.6,
                             "unit": "TFLOP/s", "frac": 0.002}
    assert s["solve"] == {"status": "OK", "rkkt": 5e-7, "rkkt_oracle": 5e-7, "outer": 13, "newton": 66}
    assert "kernels_profiled_warmup" not in s
    ws = b._summary({"value": 0.08, "unit": "s", "config": {"workload": "w"}, "roofline": None,
                     "warmstart": {"speedup": 0.97, "cold_s_per_qp": 0.078, "warm_s_per_qp": 0.081,
                                   "per_qp": []}})
    assert ws["warmstart"] == {"speedup": 0.97, "cold_s_per_qp": 0.078, "warm_s_per_qp": 0.081}
    assert "roofline" not in ws


def test_other_workloads_skipped_past_the_budget(monkeypatch):
    b = _bench()

    def no_child(*a, **k):
        raise AssertionError("no child process may start past the budget")

    monkeypatch.setattr(subprocess, "run", no_child)
    res = b.other_workloads(time.perf_counter() - b.OTHER_BUDGET_S - 1.0)
    assert list(res) == [name for name, _ in b.OTHER_WORKLOADS]
    assert all("skipped" in v for v in res.values())


def test_traffic_reading_follows_the_sources(tmp_path, monkeypatch):
    b = _bench()
    t = b.measured_traffic("sparse-text", "atmul_J")
    m = b.MEASURED_TRAFFIC[("sparse-text", "atmul_J")]
    expect = (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024.0 / m["calls"]
    assert t == expect
    assert b.measured_traffic("sparse-text", "no-such-class") is None
    # a source that differs from the measured one drops the reading
    for rel in m["files"]:
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        (tmp_path / rel).write_bytes(b"changed")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("sparse-text", "atmul_J") is None
