"""Writes c3_full_samples.json: what the oracle computes on the full-size C3
system (32 banded-random blocks of 46,750 rows, a 4,096-row border, ILU(0)
blocks, the dense border Schur complement with partial pivoting, GMRES(30),
tolerance 1e-8): every pivot of the Schur LU, 1,000 sampled entries of its
LU factors, 1,000 sampled entries of z = P^{-1} r for r ~ N(0,1) drawn with
seed 7, and the GMRES iteration count, true relative residual and 1,000
sampled entries of the solution, with the norms the samples are compared
against.  Sample positions come from numpy's PCG64 with seed 11.

It calls only the oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_c3_full.py  (a few minutes)."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from ipm_inputs import gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_full_samples.json")
K = 1000


def main():
    O.set_threads(min(16, len(os.sched_getaffinity(0))))
    t0 = time.time()
    s = gen.c3(1.0)
    P = O.BBD(s)
    assert P.status == O.OK
    parts = P.parts()
    print(f"setup {time.time() - t0:.0f} s", flush=True)
    nbd = s.n_border
    rng = np.random.default_rng(11)
    lu_i = rng.integers(0, nbd, K)
    lu_j = rng.integers(0, nbd, K)
    S = parts["S"]
    z_idx = np.sort(rng.choice(s.n, K, replace=False))
    x_idx = np.sort(rng.choice(s.n, K, replace=False))
    r = np.random.default_rng(7).standard_normal(s.n)
    z = P.apply(r)
    x, its, rr, st, _ = O.gmres_bbd(s, P, tol=1e-8, m=30, maxit=10_000)
    print(f"GMRES {its} iterations, relres {rr:.3e} ({time.time() - t0:.0f} s)", flush=True)
    rec = {"system": "C3 scale 1.0, seed 0: 32 x 46,750 + 4,096 border, ILU(0) blocks, GMRES(30), tol 1e-8",
           "n": s.n, "n_border": nbd, "pivots": [int(p) for p in parts["piv"]],
           "lu_max_abs": float(np.max(np.abs(S))),
           "lu_samples": [[int(i), int(j), float(S[i, j])] for i, j in zip(lu_i, lu_j)],
           "apply_rhs_seed": 7, "apply_max_abs": float(np.max(np.abs(z))),
           "apply_samples": [[int(i), float(z[i])] for i in z_idx],
           "gmres": {"status": int(st), "iterations": int(its), "relres": float(rr),
                     "x_norm2": float(np.linalg.norm(x)), "x_max_abs": float(np.max(np.abs(x))),
                     "x_samples": [[int(i), float(x[i])] for i in x_idx]}}
    with open(OUT, "w") as f:
        json.dump(rec, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
