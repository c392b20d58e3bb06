"""Writes c2_full_counts.json: what the oracle does on the full-size C2 system
(200,000 rows, 64 blocks, 20 dense columns kept as a low-rank term) with the
benchmark's options (GEOMEAN filter tau = 1e-3 with the dropped magnitude
added to the diagonal, SHIFT breakdown policy from 1e-2, the dense columns
eliminated as a border, tolerance 1e-8 on the true relative residual): the
FP64 PCG iteration count and residual, and the mixed FP32/FP64 mode's
refinement points, iterations, FP64 solves of the residual equation and
decisions (refine_delta 0.3, a forced point every 500 iterations).

It calls only the oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_c2_counts.py   (a few minutes on
8 cores)."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from ipm_inputs import gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_full_counts.json")


def main():
    # the oracle's row and block loops on the host cores (no result depends
    # on the thread count)
    O.set_threads(min(16, len(os.sched_getaffinity(0))))
    t0 = time.time()
    s = gen.c2(1.0)
    P = O.BJ(s, mode=O.FILTER_GEOMEAN, tau=1e-3, flags=O.DIAG_DROPSUM, delta=0.0, spd=True, policy=O.PIVOT_SHIFT,
             shift0=1e-2, border=True)
    assert P.status == O.OK
    rec = {"system": "C2 scale 1.0, seed 0", "n": s.n, "nnz": s.nnz, "nnz_kept": int(P.ci.shape[0]),
           "options": "GEOMEAN tau=1e-3 + DROPSUM, SHIFT 1e-2, border, tol 1e-8",
           "shifts": [float(a) for a in P.shifts]}
    x, its, rr, st, _ = O.pcg_bj(s, P, tol=1e-8, maxit=60_000)
    rec["fp64"] = {"status": int(st), "iterations": int(its), "relres": float(rr)}
    print(f"FP64: {its} iterations, relres {rr:.3e} ({time.time() - t0:.0f} s)", flush=True)
    x, pts, its, fb, rr, st, hist = O.mx_pcg_bj(s, P, tol=1e-8, delta=0.3, every=500, maxit=60_000,
                                                with_history=True)
    rec["fp32_mixed"] = {"status": int(st), "points": int(pts), "iterations": int(its), "fp64_solves": int(fb),
                         "relres": float(rr), "decisions": [O.RF_NAMES[h["act"]] for h in hist],
                         "decision_iterations": [h["it"] for h in hist]}
    print(f"mixed: {pts} points, {its} iterations, {fb} FP64 solves, relres {rr:.3e} "
          f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
