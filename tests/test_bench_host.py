"""Host logic of bench.py's timed leg, run on the CPU with a stand-in solver:
the loop, the per-solve record hand-off and the summary keys (no GPU)."""
from types import SimpleNamespace

import numpy as np

import bench


class _Solver:
    def __init__(self):
        self.closed = False

    def solve(self, b, x=None, tol=1e-8, log=None, extra=None):
        if log is not None:
            log.append(extra)
        return x, 12, 5e-9, 0

    def info(self):
        return {"spmv_ms": [1.2, 0.0], "spmv_launches": [12, 0], "bj_ms": [2.4, 0.0], "bj_launches": [12, 0],
                "outer_iters": 0, "fp64_fallbacks": 0, "restarts": 1, "nnz_kept": 7, "shifted_blocks": 0,
                "max_shift": 0.0, "spmv_bytes": [1000, 600], "bj_bytes": [800, 500], "bytes_per_iter": 2000}

    def residual(self, b, x):
        return None, 5e-9 * float(np.linalg.norm(b))

    def close(self):
        self.closed = True


def _fakes():
    made = []

    def from_system(system, opts):
        made.append(_Solver())
        return made[-1]

    sd = SimpleNamespace(FP64=0, FP32_IR=1, OK=0, from_system=from_system)
    torch = SimpleNamespace(
        cuda=SimpleNamespace(synchronize=lambda: None),
        as_tensor=lambda a, device=None: np.asarray(a, dtype=np.float64),
        empty_like=np.empty_like,
        linalg=SimpleNamespace(vector_norm=lambda v: SimpleNamespace(item=lambda: float(np.linalg.norm(v)))))
    return sd, torch, made


def test_run_mode_times_every_step_and_hands_records_on():
    sd, torch, made = _fakes()
    system = SimpleNamespace(b=np.ones(8), name="tiny")
    records = []
    res = bench.run_mode(sd, torch, system, SimpleNamespace(precision=sd.FP64), steps=3, warmup=1, tol=1e-8,
                         solve_log=records)
    assert [r["step"] for r in records] == [0, 1, 2] and all(r["config"] == "tiny" for r in records)
    assert res["iterations"] == [12, 12, 12]
    assert abs(res["relres"] - 5e-9) < 1e-15
    assert res["spmv_launches"] == 36 and abs(res["spmv_avg_us"] - 100.0) < 1e-9
    assert res["solves_per_s"] > 0 and res["p50_ms"] is not None
    assert made[0].closed


def test_run_mode_without_a_record_sink():
    sd, torch, _ = _fakes()
    system = SimpleNamespace(b=np.ones(4), name="tiny")
    res = bench.run_mode(sd, torch, system, SimpleNamespace(precision=sd.FP32_IR), steps=1, warmup=0, tol=1e-8)
    assert res["iterations"] == [12]


def test_traffic_is_reported_only_while_the_sources_match(tmp_path, monkeypatch):
    """roofline.traffic comes from a committed counter file that records a
    hash of the kernel sources; a changed source turns it off (None)."""
    import hashlib
    import json
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    (tmp_path / "profiles").mkdir()
    rec = {"hbm_bytes_per_launch": 123, "sources": ["k.hip"],
           "sources_sha256": hashlib.sha256(b"kernel v1\n").hexdigest()}
    (tmp_path / "profiles" / "traffic_k_bj_c2_fp64.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("bj", "fp64") == 123
    assert bench.measured_traffic("spmv", "fp64") is None  # no counter file
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("bj", "fp64") is None

