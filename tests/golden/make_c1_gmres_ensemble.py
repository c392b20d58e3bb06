"""Writes c1_gmres_ensemble.json: how far rounding alone moves the iteration
count of restarted GMRES(30) with block-Jacobi ILU(0) on C1 (2,000 rows, 4
blocks, no filter, tolerance 1e-8).  The oracle solves the system as given
and then 12 times with one entry of b moved by one ulp (entries drawn with a
fixed seed); it also records the true relative residual after 30 and 300
iterations of the unperturbed solve, where the residual histories of all
runs still agree closely.

It calls only the oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_c1_gmres_ensemble.py  (about a
minute)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from ipm_inputs import gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_gmres_ensemble.json")


def main():
    s = gen.c1()
    P = O.BJ(s)
    b0 = s.b.copy()
    _, its, rr, st, hist = O.gmres_bj(s, P, tol=1e-8, m=30, maxit=20_000, hist=True)
    rec = {"system": "C1, seed 0, GMRES(30), block-Jacobi ILU(0), tol 1e-8", "iterations": int(its),
           "status": int(st)}
    for k in (30, 300):
        x, _, rrk, _, _ = O.gmres_bj(s, P, tol=1e-30, m=30, maxit=k)
        rec[f"relres_after_{k}"] = float(rrk)
    rng = np.random.default_rng(1)
    counts, spots, first_split = [], [], []
    for _ in range(12):
        b = b0.copy()
        i = int(rng.integers(0, s.n))
        b[i] = np.nextafter(b[i], np.inf)
        s.b = b
        _, its2, _, st2, h2 = O.gmres_bj(s, P, tol=1e-8, m=30, maxit=20_000, hist=True)
        assert st2 == O.OK
        m = min(len(hist), len(h2))
        d = np.abs(hist[:m] - h2[:m]) / np.abs(hist[:m])
        counts.append(int(its2))
        spots.append(i)
        first_split.append(int(np.argmax(d > 1e-3)))
    s.b = b0
    rec["one_ulp_counts"] = counts
    rec["one_ulp_entries"] = spots
    rec["first_iteration_histories_differ_by_1e-3"] = first_split
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(rec)


if __name__ == "__main__":
    main()
