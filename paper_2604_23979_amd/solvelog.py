"""One JSON line per solve: what was solved, how, and what it cost.

A record holds the system's size and structure (n, nnz, blocks, border,
nnz kept by the filter, pivot fixes and shifts), the options that shape the
solve (method, Krylov method, precision, filter, tau), the result
(status, Krylov iterations, refinement points, FP64 fallbacks, restarts, the
true relative residual the library recomputed in compensated FP64), the
setup and solve times, the algorithmic bytes of one iteration and the
resulting GB/s, and any extra fields the caller adds (a config name and
seed, or a served request's arrival, admission and completion times)."""
from __future__ import annotations

import json
import os
import threading
import time
from typing import Optional

_NAMES = {"method": {0: "BJ", 1: "BBD"}, "krylov": {0: "PCG", 1: "GMRES", 2: "BiCGSTAB", 3: "GCR"},
          "precision": {0: "FP64", 1: "FP32_IR", 2: "FP32_IR_RESTART"},
          "filter": {0: "none", 1: "MIN", 2: "GEOMEAN"}, "factor": {0: "ILU0", 1: "COMPLETE"}}
_STATUS = {0: "OK", 1: "E_INVALID", 2: "E_STRUCTURE", 3: "E_NOMEM", 4: "E_BREAKDOWN", 5: "E_NOT_CONVERGED",
           6: "E_DEVICE", 7: "E_STATE"}


def record(solver, status: int, extra: Optional[dict] = None) -> dict:
    """The record of the last solve on ``solver`` (a Solver) that ended with
    ``status``."""
    inf = solver.info()
    o = solver.options
    its = int(inf["inner_iters"])
    ms = float(inf["solve_ms"])
    rec = {
        "time": time.time(), "n": solver.n, "nnz": solver.nnz, "nblocks": solver.nblocks,
        "n_border": solver.n_border,
        "method": _NAMES["method"].get(o.method, o.method), "krylov": _NAMES["krylov"].get(o.krylov, o.krylov),
        "precision": _NAMES["precision"].get(o.precision, o.precision),
        "filter": _NAMES["filter"].get(o.filter, o.filter), "tau": o.tau,
        "factor": _NAMES["factor"].get(o.factor, o.factor), "mc64": bool(o.mc64),
        "status": _STATUS.get(int(status), int(status)), "iterations": its,
        "refinement_points": int(inf["outer_iters"]), "fp64_fallbacks": int(inf["fp64_fallbacks"]),
        "restarts": int(inf["restarts"]), "relres": float(inf["relres"]),
        "nnz_kept": int(inf["nnz_kept"]), "pivot_fixes": int(inf["pivot_fixes"]),
        "shifted_blocks": int(inf["shifted_blocks"]), "max_shift": float(inf["max_shift"]),
        "setup_ms": float(inf["setup_ms"]), "solve_ms": ms,
        "bytes_per_iter": int(inf["bytes_per_iter"]),
        "gbps": (int(inf["bytes_per_iter"]) * its / (ms * 1e-3) / 1e9) if ms > 0 and its > 0 else None,
        "device_bytes": int(inf["device_bytes"]),
    }
    if extra:
        rec.update(extra)
    return rec


class JsonlLog:
    """Appends one JSON object per line to ``path`` (flushed per record;
    safe to share between threads)."""

    def __init__(self, path: str):
        d = os.path.dirname(os.path.abspath(path))
        os.makedirs(d, exist_ok=True)
        self.path = path
        self._f = open(path, "a")
        self._lock = threading.Lock()

    def write(self, rec: dict) -> None:
        line = json.dumps(rec, default=float)
        with self._lock:
            self._f.write(line + "\n")
            self._f.flush()

    def close(self) -> None:
        with self._lock:
            if not self._f.closed:
                self._f.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def read(path: str) -> list:
    """The records of a JSONL log."""
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]
