"""The per-solve JSONL record (host logic only)."""
import json

from paper_2604_23979_amd import solvelog
from paper_2604_23979_amd._binding import Options


class FakeSolver:
    n, nnz, nblocks, n_border = 1000, 9000, 4, 0

    def __init__(self):
        self.options = Options(filter=2, tau=1e-3, precision=1)

    def info(self):
        return dict(inner_iters=400, outer_iters=3, fp64_fallbacks=1, restarts=0, relres=8e-9, nnz_kept=5000,
                    pivot_fixes=0, shifted_blocks=2, max_shift=0.04, setup_ms=3.0, solve_ms=20.0,
                    bytes_per_iter=1_000_000, device_bytes=123456)


def test_record_fields_and_rates(tmp_path):
    rec = solvelog.record(FakeSolver(), 0, {"config": "C1", "seed": 0})
    assert rec["status"] == "OK" and rec["iterations"] == 400 and rec["precision"] == "FP32_IR"
    assert rec["filter"] == "GEOMEAN" and rec["config"] == "C1" and rec["refinement_points"] == 3
    assert abs(rec["gbps"] - 1e6 * 400 / 0.02 / 1e9) < 1e-9
    assert solvelog.record(FakeSolver(), 5)["status"] == "E_NOT_CONVERGED"


def test_jsonl_appends_one_object_per_line(tmp_path):
    path = tmp_path / "logs" / "solves.jsonl"
    with solvelog.JsonlLog(str(path)) as log:
        for k in range(3):
            log.write(solvelog.record(FakeSolver(), 0, {"step": k}))
    with solvelog.JsonlLog(str(path)) as log:        # appends
        log.write({"step": 3})
    lines = path.read_text().splitlines()
    assert len(lines) == 4 and all(json.loads(line) for line in lines)
    assert [r["step"] for r in solvelog.read(str(path))] == [0, 1, 2, 3]
