"""GPU path vs the CPU oracle on the same seeded inputs, through the C ABI.

Tolerances: the filtered pattern is compared bitwise (an integer decision
taken in FP64 on both sides); corrected values and ILU(0) factors within
1e-12 relative (both sides use the same operation order and explicit fma, so
they are expected to agree bitwise); SpMV per entry within 64 u (|M||x|)_i;
the triangular solves within 1e-12 relative (same order of operations);
solves: true relative residual <= 1e-8 recomputed by the oracle's compensated
residual and iteration counts within 10% of the oracle's."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from ipm_inputs import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2604_23979_amd as sd  # noqa: E402

DEV = "cuda:0"
U64 = np.finfo(np.float64).eps
U32 = np.finfo(np.float32).eps


def opts(**kw):
    return sd.Options(**kw)


def oracle_opts(o: sd.Options):
    return dict(mode=o.filter, tau=o.tau, flags=o.diag_flags, delta=o.delta, spd=bool(o.spd), policy=o.pivot,
                shift0=o.shift0, border=bool(o.border))


def tdev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def ragged_system(n=3000, nblocks=5, seed=0, maxrow=180):
    """Symmetric diagonally dominant matrix with row lengths from 1 to ~maxrow
    and uneven block sizes."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxrow, size=n)
    rows = np.repeat(np.arange(n), lens)
    cols = np.clip(rows + rng.integers(-400, 400, size=rows.shape[0]), 0, n - 1)
    a = sp.coo_matrix((rng.standard_normal(rows.shape[0]), (rows, cols)), shape=(n, n)).tocsr()
    a = a + a.T
    a.setdiag(0.0)
    a.eliminate_zeros()
    d = np.asarray(abs(a).sum(axis=1)).ravel() + 1.0
    a = (a + sp.diags(d)).tocsr()
    a.sort_indices()
    cuts = np.sort(rng.choice(np.arange(1, n), size=nblocks - 1, replace=False))
    bp = np.r_[0, cuts, n].astype(np.int32)
    return gen.System("ragged", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                      rng.standard_normal(n), bp)


def big_block_system(n=20000, seed=1):
    """One block larger than the LDS solution ring (so the triangular solves
    read evicted values back from global memory), banded plus far entries."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), 6)
    off = rng.integers(1, 3000, size=rows.shape[0])
    far = rng.random(rows.shape[0]) < 0.1
    off = np.where(far, rng.integers(1, n, size=rows.shape[0]), off)
    cols = (rows + off) % n
    a = sp.coo_matrix((rng.standard_normal(rows.shape[0]), (rows, cols)), shape=(n, n)).tocsr()
    a = a + a.T
    a.setdiag(0.0)
    a.eliminate_zeros()
    d = np.asarray(abs(a).sum(axis=1)).ravel() * 1.2 + 1.0
    a = (a + sp.diags(d)).tocsr()
    a.sort_indices()
    return gen.System("bigblock", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                      rng.standard_normal(n), np.array([0, 7000, n], dtype=np.int32))


CASES = {
    "C1": (lambda: gen.c1(), opts()),
    "C2x0.02": (lambda: gen.c2(0.02), opts(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)),
    "ragged-min-delta": (lambda: ragged_system(), opts(filter=sd.FILTER_MIN, tau=5e-2, diag_flags=sd.DIAG_DELTA,
                                                       delta=1e-3)),
    "bigblock": (lambda: big_block_system(), opts(filter=sd.FILTER_GEOMEAN, tau=1e-2,
                                                  diag_flags=sd.DIAG_DROPSUM | sd.DIAG_DELTA, delta=1e-12)),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    mk, o = CASES[request.param]
    s = mk()
    solver = sd.from_system(s, o)
    P = O.BJ(s, **oracle_opts(o))
    yield request.param, s, o, solver, P
    solver.close()


def test_factor_parity(case):
    name, s, o, solver, P = case
    assert P.status == O.OK
    f = solver.factors()
    n = s.n
    assert np.array_equal(f["row_ptr"][: n + 1], P.rp), "filtered pattern row pointers"
    assert np.array_equal(f["col"], P.ci), "filtered pattern columns"
    assert np.array_equal(f["corrected"], P.corrected), "filter + correction values"
    rel = np.abs(f["lu"] - P.v) / np.maximum(np.abs(P.v), 1e-300)
    assert rel.max() <= 1e-12, f"ILU(0) factors: max rel diff {rel.max():.3e}"
    assert np.array_equal(f["shifts"], P.shifts)
    print(f"{name}: kept {P.rp[-1]} entries, bitwise factors: {np.array_equal(f['lu'], P.v)}, "
          f"shifts {sorted(set(P.shifts.tolist()))}")


def test_spmv_parity(case):
    name, s, o, solver, P = case
    rng = np.random.default_rng(5)
    x = rng.standard_normal(s.n)
    y = solver.spmv(tdev(x)).cpu().numpy()
    ref = O.spmv(s.row_ptr, s.col, s.val, x, lowrank=s.lowrank)
    M = s.scipy()
    scale = abs(M) @ np.abs(x)
    if s.lowrank is not None:
        U, c = s.lowrank
        scale = scale + abs(U) @ (np.abs(c) * (abs(U).T @ np.abs(x)))
    err = np.abs(y - ref) / scale
    assert err.max() <= 64 * U64, f"{name}: FP64 SpMV {err.max():.3e}"
    x32 = x.astype(np.float32)
    y32 = solver.spmv(tdev(x32, torch.float32), fp32=True).cpu().numpy().astype(np.float64)
    v32 = s.val.astype(np.float32).astype(np.float64)
    lr32 = None
    if s.lowrank is not None:
        U, c = s.lowrank
        U32m = sp.csr_matrix((U.data.astype(np.float32).astype(np.float64), U.indices, U.indptr), shape=U.shape)
        lr32 = (U32m, c.astype(np.float32).astype(np.float64))
    ref32 = O.spmv(s.row_ptr, s.col, v32, x32.astype(np.float64), lowrank=lr32)
    err32 = np.abs(y32 - ref32) / scale
    assert err32.max() <= 512 * U32, f"{name}: FP32 SpMV {err32.max():.3e}"


def test_precond_apply_parity(case):
    name, s, o, solver, P = case
    r = np.random.default_rng(6).standard_normal(s.n)
    z = solver.precond_apply(tdev(r)).cpu().numpy()
    zo = P.apply(r)
    rel = np.abs(z - zo) / np.maximum(np.abs(zo), 1e-300)
    assert np.max(np.abs(z - zo)) <= 1e-12 * np.max(np.abs(zo)), f"{name}: apply rel {rel.max():.3e}"
    # FP32 apply against the FP64 oracle on rounded factors: close to FP32 rounding
    r32 = r.astype(np.float32)
    z32 = solver.precond_apply(tdev(r32, torch.float32), fp32=True).cpu().numpy().astype(np.float64)
    if P.border is None:
        zo32 = O.lu_solve(P.rp, P.ci, P.v.astype(np.float32).astype(np.float64), P.dp, r32.astype(np.float64))
    else:
        zo32 = P.apply(r32.astype(np.float64))
    assert np.max(np.abs(z32 - zo32)) <= 1e-3 * np.max(np.abs(zo32)), f"{name}: FP32 apply"


def test_residual_parity(case):
    name, s, o, solver, P = case
    rng = np.random.default_rng(7)
    x = rng.standard_normal(s.n)
    r, nr = solver.residual(tdev(s.b), tdev(x))
    ro, nro = O.residual(s.row_ptr, s.col, s.val, x, s.b, s.lowrank)
    r = r.cpu().numpy()
    assert np.max(np.abs(r - ro)) <= 1e-15 * np.max(np.abs(ro)) + 1e-300
    assert abs(nr - nro) <= 1e-14 * nro


def test_pcg_fp64_matches_oracle(case):
    name, s, o, solver, P = case
    xo, its_o, rr_o, st_o, _ = O.pcg_bj(s, P, tol=1e-8, maxit=50_000)
    assert st_o == O.OK
    b = tdev(s.b)
    # the residual of a converged solution, where b and M x cancel to 1e-8
    _, nr_g = solver.residual(b, tdev(xo))
    assert abs(nr_g / np.linalg.norm(s.b) - rr_o) <= 1e-6 * rr_o, (nr_g / np.linalg.norm(s.b), rr_o)
    x, its, rr, st = solver.solve(b, tol=1e-8)
    x = x.cpu().numpy()
    true_rr = O.relres(s, x)
    print(f"{name}: FP64 PCG gpu {its} its relres {true_rr:.2e} | oracle {its_o} its {rr_o:.2e}")
    assert st == sd.OK
    assert true_rr <= 1e-8
    assert abs(rr - true_rr) <= 1e-3 * true_rr + 1e-15
    assert abs(its - its_o) <= max(1, 0.10 * its_o)
    check_solution_gate(name, s, x, xo)


def smallest_eigenvalue(s):
    """A lower bound for lambda_min of the explicit sparse part of M (itself
    a lower bound for the operator's when a positive semidefinite low-rank
    term is added): Gershgorin's when it is positive (diagonally dominant
    matrices), else the eigenvalue itself by shift-invert Lanczos (small IPM
    systems only: a sparse LU of a large random pattern would not finish)."""
    import scipy.sparse.linalg as sla
    M = s.scipy().tocsr()
    d = M.diagonal()
    gersh = float(np.min(d - (np.asarray(abs(M).sum(axis=1)).ravel() - np.abs(d))))
    if gersh > 0:
        return gersh
    assert s.n <= 8000, "no cheap lambda_min bound for this system"
    return float(sla.eigsh(M.tocsc(), k=1, sigma=0, which="LM", return_eigenvectors=False)[0])


def check_solution_gate(name, s, x, xo):
    """Solution parity (the 1e-6 gate where it is attainable).  Two
    solutions with residuals r and r_o differ by M^{-1}(r_o - r), so
    ||x - x_o|| <= (||r|| + ||r_o||) / lambda_min(M): the difference must
    respect that bound, and must be below 1e-6 relative wherever the bound
    itself is."""
    _, nr = O.residual(s.row_ptr, s.col, s.val, x, s.b, s.lowrank)
    _, nro = O.residual(s.row_ptr, s.col, s.val, xo, s.b, s.lowrank)
    lam = smallest_eigenvalue(s)
    bound = (nr + nro) / lam / np.linalg.norm(xo)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"{name}: ||x - x_oracle|| / ||x_oracle|| = {rel:.2e}; residual bound {bound:.2e} "
          f"(lambda_min {lam:.2e}); 1e-6 gate {'applies' if bound <= 1e-6 else 'not attainable'}")
    assert rel <= 1.01 * bound + 1e-15
    if bound <= 1e-6:
        assert rel <= 1e-6


@pytest.mark.parametrize("prec", ["refine", "restart"])
def test_fp32_inner_refinement(case, prec):
    name, s, o, solver, P = case
    mode = sd.FP32_IR if prec == "refine" else sd.FP32_IR_RESTART
    o2 = sd.Options(**{**o.__dict__, "precision": mode})
    sv = sd.from_system(s, o2)
    try:
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        true_rr = O.relres(s, x.cpu().numpy())
        inf = sv.info()
        if prec == "refine":
            xo, outer_o, inner_o, fb_o, rr_o, st_o = O.mx_pcg_bj(s, P, tol=1e-8, delta=o2.refine_delta,
                                                                  every=o2.refine_every, maxit=100_000)
        else:
            xo, outer_o, inner_o, fb_o, rr_o, st_o = O.ir_pcg_bj(s, P, tol=1e-8, inner_tol=o2.inner_tol,
                                                                  maxit=100_000)
        print(f"{name}: FP32 {prec} gpu points {inf['outer_iters']} iterations {its} fallbacks "
              f"{inf['fp64_fallbacks']} relres {true_rr:.2e} | oracle points {outer_o} iterations {inner_o} "
              f"fallbacks {fb_o}")
        assert st == sd.OK and true_rr <= 1e-8
        assert abs(rr - true_rr) <= 1e-3 * true_rr + 1e-15
        # the library's decisions are the rule's on its own residual history
        O.replay_refine(sv.rf_history(), 0 if prec == "refine" else 1, inf["rf_nb"], 1e-8, o2.max_iter)
        if prec == "refine" and inf["fp64_fallbacks"] == 0 and fb_o == 0:
            # FP32 sums in a different order than the oracle's perturb the
            # recurrence; the counts stay within 10% plus a few iterations
            assert abs(its - inner_o) <= max(4, 0.10 * inner_o)
        # the error against the FP64 oracle's solution, stated and bounded
        check_solution_gate(f"{name} FP32 {prec}", s, x.cpu().numpy(),
                            O.pcg_bj(s, P, tol=1e-8, maxit=50_000)[0])
    finally:
        sv.close()


@pytest.mark.parametrize("prec", ["refine", "restart"])
@pytest.mark.parametrize("which", ["stall", "breakdown"])
def test_fp32_decisions_follow_the_rule(prec, which):
    """Late IPM systems on which the FP32 recurrence stalls (D spread about
    1e8: FP64 solves of the residual equation follow) or breaks down (rows
    holding only the 1e-8 regularisation): every decision the library took is
    the rule's on its own residual history, and the solve meets the
    tolerance (oracle residual)."""
    q = gen.IPMSequence(m=20000, nblocks=4 if which == "stall" else 1, steps=30)
    s = q.system(16 if which == "stall" else 1)
    print(f"\n[FP32 decisions: {which}, {prec}]", flush=True)
    mode = sd.FP32_IR if prec == "refine" else sd.FP32_IR_RESTART
    o = opts(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM, precision=mode, max_iter=60_000,
             refine_delta=0.3)
    sv = sd.from_system(s, o)
    try:
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        inf = sv.info()
        hist = sv.rf_history()
        print(f"  gpu: {its} iterations, {inf['fp64_fallbacks']} FP64 solves, decisions "
              f"{[O.RF_NAMES[h['act']] for h in hist]}")
        O.replay_refine(hist, 0 if prec == "refine" else 1, inf["rf_nb"], 1e-8, o.max_iter)
        assert st == sd.OK and O.relres(s, x.cpu().numpy()) <= 1e-8
        assert inf["fp64_fallbacks"] >= 1 or prec == "restart"
    finally:
        sv.close()


# ------------------------------------------------------------------ full size

# the options the benchmark times on the full C2 system
BENCH_C2 = dict(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM, pivot=sd.PIVOT_SHIFT, shift0=1e-2,
                kernel_timing=True, max_iter=60_000, refine_delta=0.3, border=True)


@pytest.fixture(scope="module")
def c2_full():
    print("\n[case C2 at full size, benchmark options]", flush=True)
    s = gen.c2(1.0)
    o = opts(**BENCH_C2)
    solver = sd.from_system(s, o)
    P = O.BJ(s, **oracle_opts(o))
    yield "C2-full", s, o, solver, P
    solver.close()


def test_full_c2_setup_spmv_apply_residual(c2_full):
    """At the benchmark's size and launch configuration, every output the
    oracle computes in seconds: the filtered pattern (bitwise), corrected
    values and factors, the FP64/FP32 SpMV with the low-rank term, the
    bordered preconditioner apply, and the compensated residual."""
    test_factor_parity(c2_full)
    test_spmv_parity(c2_full)
    test_precond_apply_parity(c2_full)
    test_residual_parity(c2_full)
    # sdsl_info's sweep depth: levels of 512-row chunks (forward chunks from
    # each block's top, backward ones from its bottom), recounted here from
    # the factor pattern
    name, s, o, solver, P = c2_full
    f = solver.factors()
    rp, ci = f["row_ptr"], f["col"]
    per_block = []
    for b in range(s.nblocks):
        lo, hi = int(s.block_ptr[b]), int(s.block_ptr[b + 1])
        total = 0
        for fwd in (True, False):
            m = 0
            while (lo + m * 512 < hi) if fwd else (hi - m * 512 > lo):
                a, e = (lo + m * 512, min(hi, lo + (m + 1) * 512)) if fwd else (max(lo, hi - (m + 1) * 512),
                                                                              hi - m * 512)
                lev = {}
                rows = range(a, e) if fwd else range(e - 1, a - 1, -1)
                for i in rows:
                    cols = ci[rp[i]:rp[i + 1]]
                    dep = cols[(cols >= a) & (cols < i)] if fwd else cols[(cols > i) & (cols < e)]
                    lev[i] = 1 + max(lev[j] for j in dep) if dep.size else 0
                total += 1 + max(lev.values())
                m += 1
        per_block.append(total)
    inf = solver.info()
    print(f"  sweep levels per block: max {inf['sweep_levels_max']}, mean {inf['sweep_levels_mean']:.1f}")
    assert inf["sweep_levels_max"] == max(per_block)
    assert inf["sweep_levels_mean"] == pytest.approx(np.mean(per_block), rel=1e-12)


def test_full_c4_samples_match_oracle():
    """C4's first system at its full size (5.2M rows, 256 blocks, the bench's
    filter and breakdown policy), on outputs the oracle computes piece by
    piece: the FP64 SpMV at 2,000 sampled rows (each row a plain dot
    product), and for five sampled blocks (one of them shifted by the
    breakdown policy, where there is one) the filtered pattern (bitwise),
    corrected values (bitwise), factors (1e-12) and shifts, and those
    blocks' part of one preconditioner apply (1e-12 of the block's largest
    entry).  The blocks are independent in the preconditioner, so each is
    factored by the oracle on its own."""
    print("\n[C4 at full size]", flush=True)
    s = gen.IPMSequence(steps=30).system(0)
    assert s.n == 5_200_000 and s.nblocks == 256
    o = opts(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
    sv = sd.from_system(s, o)
    try:
        rng = np.random.default_rng(40)
        x = rng.standard_normal(s.n)
        y = sv.spmv(tdev(x)).cpu().numpy()
        rows = rng.choice(s.n, 2000, replace=False)
        for i in rows:
            a, e = s.row_ptr[i], s.row_ptr[i + 1]
            ref = float(np.dot(s.val[a:e], x[s.col[a:e]]))
            scale = float(np.dot(np.abs(s.val[a:e]), np.abs(x[s.col[a:e]])))
            assert abs(y[i] - ref) <= 64 * U64 * scale, i
        r = rng.standard_normal(s.n)
        z = sv.precond_apply(tdev(r)).cpu().numpy()
        f = sv.factors()
        # also the first block the library had to shift (SHIFT policy), if any
        shifted = [int(q) for q in np.flatnonzero(f["shifts"] > 0)[:1]]
        for b in [0, 77, 160, 255] + shifted:
            lo, hi = int(s.block_ptr[b]), int(s.block_ptr[b + 1])
            blk = s_sub(s, lo, hi)
            sub = gen.System(f"C4-block{b}", blk.indptr.astype(np.int64), blk.indices.astype(np.int32), blk.data,
                             r[lo:hi], np.array([0, hi - lo], dtype=np.int32))
            P = O.BJ(sub, **oracle_opts(o))
            assert P.status == O.OK
            a0, a1 = int(f["row_ptr"][lo]), int(f["row_ptr"][hi])
            assert np.array_equal(f["row_ptr"][lo:hi + 1] - a0, P.rp), b
            assert np.array_equal(f["col"][a0:a1] - lo, P.ci), b
            assert np.array_equal(f["corrected"][a0:a1], P.corrected), b
            rel = np.abs(f["lu"][a0:a1] - P.v) / np.maximum(np.abs(P.v), 1e-300)
            assert rel.max() <= 1e-12, (b, rel.max())
            assert f["shifts"][b] == P.shifts[0], b
            zo = P.apply(r[lo:hi])
            assert np.max(np.abs(z[lo:hi] - zo)) <= 1e-12 * np.max(np.abs(zo)), b
            print(f"  block {b}: {hi - lo} rows, kept {P.rp[-1]}, shift {P.shifts[0]}", flush=True)
    finally:
        sv.close()


def s_sub(s, lo, hi):
    """Rows and columns [lo, hi) of the system's matrix (CSR, sorted)."""
    a, e = int(s.row_ptr[lo]), int(s.row_ptr[hi])
    rp = s.row_ptr[lo:hi + 1] - a
    ci, v = s.col[a:e], s.val[a:e]
    keep = (ci >= lo) & (ci < hi)
    cnt = np.add.reduceat(keep.astype(np.int64), rp[:-1]) if hi > lo else np.zeros(0, np.int64)
    cnt[np.diff(rp) == 0] = 0
    rp2 = np.concatenate([[0], np.cumsum(cnt)])
    return sp.csr_matrix((v[keep], ci[keep] - lo, rp2), shape=(hi - lo, hi - lo))


def test_full_c2_solves(c2_full):
    """The first PCG iterations against the oracle's (a full oracle solve
    takes minutes), then complete FP64 and FP32-inner solves, whose true
    residual the oracle recomputes at full size.  The recurrence on this
    system amplifies rounding quickly: in the oracle itself, a one-ulp change
    of b moves the iterate by 1e-14 after 5 iterations, 3e-11 after 10 and
    2e-2 after 20, so the iterates are compared after 5."""
    name, s, o, solver, P = c2_full
    b = tdev(s.b)
    k = 5
    solver.set_max_iter(k)
    x, its, rr, st = solver.solve(b, tol=1e-8)
    solver.set_max_iter(o.max_iter)
    xo, its_o, rr_o, st_o, _ = O.pcg_bj(s, P, tol=1e-8, maxit=k)
    xg = x.cpu().numpy()
    dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"  {k} iterations: GPU relres {rr:.9e}, oracle {rr_o:.9e}, |x - x_oracle| / |x_oracle| = {dx:.2e}")
    assert st == sd.E_NOT_CONVERGED and its == its_o == k
    assert abs(rr - rr_o) <= 1e-9 * rr_o and dx <= 1e-9
    # the oracle's complete solves on this system (tests/golden/c2_full_counts.json,
    # written by make_c2_counts.py: minutes of oracle time, so stored)
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2_full_counts.json")) as f:
        gold = json.load(f)
    assert gold["n"] == s.n and gold["nnz"] == s.nnz and gold["nnz_kept"] == solver.info()["nnz_kept"]
    x, its, rr, st = solver.solve(b, tol=1e-8)
    true_rr = O.relres(s, x.cpu().numpy())
    print(f"  FP64: {its} iterations (oracle {gold['fp64']['iterations']}), relres {true_rr:.2e}")
    assert st == sd.OK and true_rr <= 1e-8 and abs(rr - true_rr) <= 1e-3 * true_rr
    assert abs(its - gold["fp64"]["iterations"]) <= 0.10 * gold["fp64"]["iterations"]
    sv = sd.from_system(s, sd.Options(**{**o.__dict__, "precision": sd.FP32_IR}))
    try:
        x, its32, rr, st = sv.solve(b, tol=1e-8)
        true_rr = O.relres(s, x.cpu().numpy())
        inf = sv.info()
        mx = gold["fp32_mixed"]
        print(f"  FP32-inner: {its32} iterations, {inf['outer_iters']} points, {inf['fp64_fallbacks']} FP64 solves "
              f"(oracle {mx['iterations']}, {mx['points']}, {mx['fp64_solves']}), relres {true_rr:.2e}")
        assert st == sd.OK and true_rr <= 1e-8 and abs(rr - true_rr) <= 1e-3 * true_rr
        O.replay_refine(sv.rf_history(), 0, inf["rf_nb"], 1e-8, o.max_iter)
    finally:
        sv.close()


# ------------------------------------------------------------------ edge cases

def _tiny(a, bp, o=None, b=None):
    m = sp.csr_matrix(np.asarray(a, dtype=np.float64))
    m.sort_indices()
    n = m.shape[0]
    s = gen.System("tiny", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                   np.ones(n) if b is None else b, np.asarray(bp, dtype=np.int32))
    return s


def test_one_row_blocks_is_jacobi_and_single_row():
    rng = np.random.default_rng(3)
    n = 700
    a = np.diag(rng.uniform(1, 2, n)) + np.diag(0.1 * rng.standard_normal(n - 1), 1)
    a = a + a.T
    s = _tiny(a, np.arange(n + 1))
    sv = sd.from_system(s)
    r = rng.standard_normal(n)
    z = sv.precond_apply(tdev(r)).cpu().numpy()
    assert np.array_equal(z, r / np.diag(a))
    sv.close()
    s1 = _tiny([[4.0]], [0, 1], b=np.array([2.0]))
    sv = sd.from_system(s1)
    x, its, rr, st = sv.solve(tdev(s1.b))
    assert st == sd.OK and abs(x.item() - 0.5) < 1e-15 and its == 1
    sv.close()


def test_exact_preconditioner_one_iteration():
    """Tridiagonal SPD in one block: ILU(0) is exact, PCG takes one step."""
    rng = np.random.default_rng(4)
    n = 5000
    off = rng.standard_normal(n - 1)
    a = sp.diags([off, np.abs(np.r_[off, 0]) + np.abs(np.r_[0, off]) + 0.5, off], [-1, 0, 1]).tocsr()
    a.sort_indices()
    s = gen.System("tri", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                   rng.standard_normal(n), np.array([0, n], dtype=np.int32))
    sv = sd.from_system(s)
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-12)
    assert st == sd.OK and its == 1 and O.relres(s, x.cpu().numpy()) <= 1e-12
    sv.close()


def test_zero_rhs():
    s = gen.c1()
    sv = sd.from_system(s)
    x, its, rr, st = sv.solve(torch.zeros(s.n, dtype=torch.float64, device=DEV))
    assert st == sd.OK and its == 0 and rr == 0.0 and torch.count_nonzero(x).item() == 0
    sv.close()


def test_invalid_inputs_are_rejected():
    a = np.array([[2.0, 1.0], [1.0, 2.0]])
    s = _tiny(a, [0, 2])
    bad = s.val.copy()
    bad[1] = np.nan
    with pytest.raises(sd.SdslError) as e:
        sd.Solver(s.row_ptr, s.col, bad, s.block_ptr)
    assert e.value.status == sd.E_INVALID
    col = s.col.copy()
    col[0], col[1] = col[1], col[0]
    with pytest.raises(sd.SdslError) as e:
        sd.Solver(s.row_ptr, col, s.val, s.block_ptr)
    assert e.value.status == sd.E_INVALID
    nodiag = _tiny([[0.0, 1.0], [1.0, 2.0]], [0, 2])
    with pytest.raises(sd.SdslError) as e:
        sd.Solver(nodiag.row_ptr, nodiag.col, nodiag.val, nodiag.block_ptr)
    assert e.value.status == sd.E_INVALID
    for bp in ([0, 1], [0, 2, 2], [1, 2]):
        with pytest.raises(sd.SdslError) as e:
            sd.Solver(s.row_ptr, s.col, s.val, np.array(bp))
        assert e.value.status == sd.E_INVALID
    sv = sd.Solver(s.row_ptr, s.col, s.val, s.block_ptr)
    with pytest.raises(sd.SdslError):
        sv.refactor(tdev(bad))
    sv.close()


def test_breakdown_policies_on_device():
    a = np.array([[1.0, -0.6, 0.1, 0.2, -0.6],
                  [-0.6, 1.0, 0.0, 0.4, 0.0],
                  [0.1, 0.0, 1.0, -0.1, 0.0],
                  [0.2, 0.4, -0.1, 1.0, -0.7],
                  [-0.6, 0.0, 0.0, -0.7, 1.0]])
    s = _tiny(a, [0, 5])
    with pytest.raises(sd.SdslError) as e:
        sd.from_system(s, sd.Options(pivot=sd.PIVOT_FAIL))
    assert e.value.status == sd.E_BREAKDOWN
    sv = sd.from_system(s, sd.Options(pivot=sd.PIVOT_SHIFT, shift0=0.01))
    P = O.BJ(s, policy=O.PIVOT_SHIFT, shift0=0.01)
    f = sv.factors()
    assert np.array_equal(f["shifts"], P.shifts) and np.array_equal(f["lu"], P.v)
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-12)
    assert st == sd.OK and O.relres(s, x.cpu().numpy()) <= 1e-12
    sv.close()
    sv = sd.from_system(s, sd.Options(pivot=sd.PIVOT_REPLACE))
    P = O.BJ(s, policy=O.PIVOT_REPLACE)
    assert np.array_equal(sv.factors()["lu"], P.v) and sv.info()["pivot_fixes"] == P.nfix == 1
    assert P.v[P.dp[4]] == a[4, 4]
    sv.close()
    # non-unit diagonal and a small first shift: the relative shift d + a d
    # after several doublings, bit for bit as in the oracle
    sc = np.array([2.0, 0.5, 3.0, 1.5, 0.25])
    s = _tiny(sc[:, None] * a * sc[None, :], [0, 5])
    sv = sd.from_system(s, sd.Options(pivot=sd.PIVOT_SHIFT, shift0=1e-4))
    P = O.BJ(s, policy=O.PIVOT_SHIFT, shift0=1e-4)
    f = sv.factors()
    assert P.shifts[0] > 1e-4
    assert np.array_equal(f["shifts"], P.shifts) and np.array_equal(f["lu"], P.v)
    sv.close()
    # an exactly zero pivot is a breakdown in SPD mode
    with pytest.raises(sd.SdslError) as e:
        sd.from_system(_tiny([[1.0, 1.0], [1.0, 1.0]], [0, 2]), sd.Options(pivot=sd.PIVOT_FAIL))
    assert e.value.status == sd.E_BREAKDOWN


def test_not_converged_and_max_iter():
    s = gen.c1()
    sv = sd.from_system(s, sd.Options(max_iter=3, check_every=2))
    x, its, rr, st = sv.solve(tdev(s.b))
    assert st == sd.E_NOT_CONVERGED and its == 3
    assert abs(rr - O.relres(s, x.cpu().numpy())) <= 1e-10
    sv.close()


def test_pcg_stops_on_the_true_residual_only():
    """An IPM system on which the recurrence residual of PCG meets 1e-10
    before the true residual does (both the oracle, which stalls near 5e-10,
    and the GPU restart from the true residual).  Whatever the rounding
    history, OK means the true residual meets the tolerance, anything else
    ends at max_iter, and the reported residual is the true one (checked in
    x86 extended precision)."""
    q = gen.IPMSequence(m=3000, nblocks=4, steps=30)
    s = q.system(5)
    o = opts(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM, max_iter=1000)
    sv = sd.from_system(s, o)
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-10)
    xs = x.cpu().numpy()
    M = s.scipy()
    ld = np.longdouble
    res = s.b.astype(ld) - np.add.reduceat(M.data.astype(ld) * xs[M.indices].astype(ld), M.indptr[:-1])
    true = float(np.sqrt(np.sum(res * res)) / np.sqrt(np.sum(s.b.astype(ld) ** 2)))
    print(f"  its {its} status {st} relres {rr:.3e} (extended {true:.3e}) restarts {sv.info()['restarts']}")
    assert sv.info()["restarts"] >= 1
    assert rr == pytest.approx(true, rel=1e-3)
    if st == sd.OK:
        assert true <= 1e-10 and its < 1000
    else:
        assert st == sd.E_NOT_CONVERGED and its == 1000 and true > 1e-10
    sv.close()


def test_refactor_update_values_and_reuse():
    q = gen.IPMSequence(m=12000, nblocks=8, steps=4, seed=1)
    o = sd.Options(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
    s0 = q.system(0)
    sv = sd.from_system(s0, o)
    for k in (1, 2, 3):
        sk = q.system(k)
        vals = tdev(sk.val)
        if k == 2:
            sv.update_values(vals)      # keep the factors of step 1
        else:
            sv.refactor(vals)
            P = O.BJ(sk, **oracle_opts(o))
            f = sv.factors()
            assert np.array_equal(f["col"], P.ci) and np.array_equal(f["lu"], P.v)
        x, its, rr, st = sv.solve(tdev(sk.b))
        assert st == sd.OK and O.relres(sk, x.cpu().numpy()) <= 1e-8
    sv.close()


def test_solve_batch_equals_solo():
    systems = [gen.c2(0.01, seed=s, dense_cols=0) for s in range(3)]
    o = sd.Options(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
    streams = [torch.cuda.Stream() for _ in systems]
    solvers = [sd.from_system(s, o, stream=st) for s, st in zip(systems, streams)]
    solo = []
    for sv, s in zip(solvers, systems):
        x, its, rr, st = sv.solve(tdev(s.b))
        solo.append((x.cpu().numpy(), its))
    bs = [tdev(s.b) for s in systems]
    xs = [torch.empty_like(b) for b in bs]
    torch.cuda.synchronize()
    its, rr, st = sd.solve_batch(solvers, bs, xs)
    assert st == sd.OK
    for i in range(3):
        assert its[i] == solo[i][1]
        assert np.array_equal(xs[i].cpu().numpy(), solo[i][0])
    for sv in solvers:
        sv.close()


def nonsym_system(n=6000, nblocks=4, seed=3):
    """Nonsymmetric, weakly diagonally dominant banded system (random band
    entries, diagonal 0.6 x the row's magnitude sum, diagonal included)."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), 9)
    cols = np.clip(rows + rng.integers(-300, 300, size=rows.shape[0]), 0, n - 1)
    a = sp.coo_matrix((rng.standard_normal(rows.shape[0]), (rows, cols)), shape=(n, n)).tocsr()
    a.setdiag(0.0)
    a.eliminate_zeros()
    off = np.asarray(abs(a).sum(axis=1)).ravel()
    a = (a + sp.diags(1.5 * off + 1e-3)).tocsr()
    a.sort_indices()
    bp = np.linspace(0, n, nblocks + 1).astype(np.int32)
    return gen.System("nonsym", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                      rng.standard_normal(n), bp)


@pytest.mark.parametrize("which", ["nonsym", "nonsym-7blocks"])
def test_gmres_bj_matches_oracle(which):
    """Right-preconditioned GMRES(30) with the block-Jacobi preconditioner on
    nonsymmetric systems: true relres <= 1e-8 and inner iterations within
    10% (or 2) of the oracle's; both orthogonalise with classical
    Gram-Schmidt applied twice."""
    print(f"[gmres {which}]", flush=True)
    s = nonsym_system() if which == "nonsym" else nonsym_system(n=9000, nblocks=7, seed=4)
    o = opts(krylov=sd.GMRES, spd=False)
    sv = sd.from_system(s, o)
    P = O.BJ(s, **oracle_opts(o))
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
    x_o, its_o, rr_o, st_o, _ = O.gmres_bj(s, P, tol=1e-8, m=30, maxit=20_000)
    true_rr = O.relres(s, x.cpu().numpy())
    print(f"  GPU its {its} relres {true_rr:.2e}; oracle its {its_o} relres {rr_o:.2e}")
    assert st == sd.OK and st_o == O.OK
    assert true_rr <= 1e-8 and abs(rr - true_rr) <= 1e-3 * true_rr + 1e-15
    assert abs(its - its_o) <= max(2, 0.1 * its_o)
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - x_o) <= 1e-6 * np.linalg.norm(x_o)
    sv.close()


@pytest.mark.parametrize("which", ["nonsym", "nonsym-7blocks"])
def test_bicgstab_matches_oracle(which):
    """Right-preconditioned BiCGSTAB (the paper's block-Jacobi solver, Sec.
    4.3) on nonsymmetric systems whose count does not move under one-ulp
    changes of b (oracle: 6 iterations for each of 6 draws): true relres <=
    1e-8, iterations within 10% (or 2) of the oracle's, solution within
    1e-6."""
    print(f"[bicgstab {which}]", flush=True)
    s = nonsym_system() if which == "nonsym" else nonsym_system(n=9000, nblocks=7, seed=4)
    o = opts(krylov=sd.BICGSTAB, spd=False)
    sv = sd.from_system(s, o)
    try:
        P = O.BJ(s, **oracle_opts(o))
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        x_o, its_o, rr_o, st_o, _ = O.bicgstab_bj(s, P, tol=1e-8, maxit=20_000)
        x = x.cpu().numpy()
        true_rr = O.relres(s, x)
        print(f"  GPU its {its} relres {true_rr:.2e}; oracle its {its_o} relres {rr_o:.2e}")
        assert st == sd.OK and st_o == O.OK
        assert true_rr <= 1e-8 and abs(rr - true_rr) <= 1e-3 * true_rr + 1e-15
        assert abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x - x_o) <= 1e-6 * np.linalg.norm(x_o)
    finally:
        sv.close()


def test_bicgstab_c1_and_low_rank_against_oracle():
    """C1 (SPD, D spread 1e8) and C2 x 0.004 (low-rank term eliminated as a
    border): the first iterations follow the oracle's (true residual after
    10 iterations within 1e-6 relative), which exercises the product with
    the low-rank term and the bordered apply.  On C1 the complete solve
    meets 1e-8 with a count inside 10% of the range the oracle spans when
    one entry of b moves by one ulp (8 draws; BiCGSTAB there is as sensitive
    to rounding as GMRES)."""
    for name, s, o in (("C1", gen.c1(), opts(krylov=sd.BICGSTAB)),
                       ("C2x0.004", gen.c2(0.004), opts(krylov=sd.BICGSTAB, filter=sd.FILTER_GEOMEAN, tau=1e-3,
                                                        diag_flags=sd.DIAG_DROPSUM))):
        sv = sd.from_system(s, o)
        try:
            P = O.BJ(s, **oracle_opts(o))
            sv.set_max_iter(10)
            _, its, rr, st = sv.solve(tdev(s.b), tol=1e-30)
            _, its_o, rr_o, _, _ = O.bicgstab_bj(s, P, tol=1e-30, maxit=10)
            print(f"  {name} after 10: GPU relres {rr:.12e}, oracle {rr_o:.12e}")
            assert its == its_o == 10 and abs(rr - rr_o) <= 1e-6 * rr_o
            if name != "C1":
                continue
            sv.set_max_iter(20_000)
            x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
            b0 = s.b.copy()
            rng = np.random.default_rng(3)
            counts = [O.bicgstab_bj(s, P, tol=1e-8, maxit=20_000)[1]]
            for _ in range(8):
                bb = b0.copy()
                i = rng.integers(0, s.n)
                bb[i] = np.nextafter(bb[i], np.inf)
                s.b = bb
                counts.append(O.bicgstab_bj(s, P, tol=1e-8, maxit=20_000)[1])
            s.b = b0
            true_rr = O.relres(s, x.cpu().numpy())
            print(f"  C1 BiCGSTAB: GPU its {its} relres {true_rr:.2e}; oracle {counts[0]}, one-ulp range "
                  f"{min(counts)}-{max(counts)}")
            assert st == sd.OK and true_rr <= 1e-8
            assert 0.9 * min(counts) <= its <= 1.1 * max(counts)
        finally:
            sv.close()


@pytest.mark.parametrize("which", ["nonsym", "nonsym-7blocks"])
def test_gcr_matches_oracle(which):
    """Right-preconditioned restarted GCR(30) (the paper's solver with BBD and
    on single nodes, Sec. 4.2-4.3) with block Jacobi: true relres <= 1e-8,
    iterations within 10% (or 2) of the oracle's, solution within 1e-6; the
    first 10 steps follow the oracle's residual within 1e-8 relative."""
    print(f"[gcr {which}]", flush=True)
    s = nonsym_system() if which == "nonsym" else nonsym_system(n=9000, nblocks=7, seed=4)
    o = opts(krylov=sd.GCR, spd=False)
    sv = sd.from_system(s, o)
    try:
        P = O.BJ(s, **oracle_opts(o))
        sv.set_max_iter(10)
        _, its, rr, st = sv.solve(tdev(s.b), tol=1e-30)
        _, its_o, rr_o, _, _ = O.gcr_bj(s, P, tol=1e-30, m=30, maxit=10)
        print(f"  after 10: GPU relres {rr:.12e}, oracle {rr_o:.12e}")
        assert its == its_o == 10 and abs(rr - rr_o) <= 1e-8 * rr_o
        sv.set_max_iter(20_000)
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        x_o, its_o, rr_o, st_o, _ = O.gcr_bj(s, P, tol=1e-8, m=30, maxit=20_000)
        x = x.cpu().numpy()
        true_rr = O.relres(s, x)
        print(f"  GPU its {its} relres {true_rr:.2e}; oracle its {its_o} relres {rr_o:.2e}")
        assert st == sd.OK and st_o == O.OK
        assert true_rr <= 1e-8 and abs(rr - true_rr) <= 1e-3 * true_rr + 1e-15
        assert abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x - x_o) <= 1e-6 * np.linalg.norm(x_o)
    finally:
        sv.close()


def test_gcr_exact_preconditioner_and_breakdown():
    """A tridiagonal single block (ILU(0) exact) converges in one GCR step; a
    2 x 2 system whose residual is orthogonal to M P^-1 r repeats its first
    direction, which adds nothing: SDSL_E_BREAKDOWN after one step with x
    unchanged (the oracle says the same)."""
    rng = np.random.default_rng(5)
    n = 4000
    lo, up = rng.standard_normal(n - 1), rng.standard_normal(n - 1)
    dg = np.abs(np.r_[lo, 0]) + np.abs(np.r_[0, up]) + 1.0
    a = sp.diags([lo, dg, up], [-1, 0, 1]).tocsr()
    a.sort_indices()
    s = gen.System("tri-ns", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                   rng.standard_normal(n), np.array([0, n], dtype=np.int32))
    sv = sd.from_system(s, opts(krylov=sd.GCR, spd=False))
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-12)
    assert st == sd.OK and its == 1 and O.relres(s, x.cpu().numpy()) <= 1e-12
    sv.close()
    m = sp.csr_matrix(np.array([[1.0, 3.0], [-1.0, 1.0]]))
    bd = gen.System("bd", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, np.array([1.0, -1.0]),
                    np.array([0, 1, 2], dtype=np.int32))
    o = opts(krylov=sd.GCR, spd=False, pivot=sd.PIVOT_FAIL)
    sv = sd.from_system(bd, o)
    x, its, rr, st = sv.solve(tdev(bd.b), tol=1e-12)
    _, its_o, _, st_o, _ = O.gcr_bj(bd, O.BJ(bd, **oracle_opts(o)), tol=1e-12, maxit=10)
    assert st == sd.E_BREAKDOWN and st_o == O.BREAKDOWN and its == its_o == 1
    assert np.all(x.cpu().numpy() == 0.0)
    sv.close()


COMPLETE_CASES = {
    "C2x0.004-filtered": lambda: (gen.c2(0.004, dense_cols=0),
                                  opts(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM,
                                       factor=sd.FACT_COMPLETE)),
    "ragged": lambda: (ragged_system(), opts(factor=sd.FACT_COMPLETE)),
    "nonsym-banded": lambda: (nonsym_system(n=3000, nblocks=4, seed=5),
                              opts(krylov=sd.GMRES, spd=False, pivot=sd.PIVOT_FAIL, factor=sd.FACT_COMPLETE)),
}


@pytest.mark.parametrize("case", sorted(COMPLETE_CASES))
def test_complete_factors_and_solve_match_oracle(case):
    """COMPLETE factorisation (complete LU of every filtered, corrected
    block: Sec. 3.1, Alg. 2): the library's factor on its symbolic fill
    pattern equals the oracle's elimination over the dense block pattern
    within 1e-12 (relative to the largest entry), every entry the oracle has
    outside the library's pattern is exactly zero, and the solve takes the
    oracle's iterations within 10% (or 2) with the solution within 1e-6."""
    print(f"[complete {case}]", flush=True)
    s, o = COMPLETE_CASES[case]()
    sv = sd.from_system(s, o)
    try:
        P = O.BJ(s, **oracle_opts(o), complete=True)
        assert P.status == O.OK
        f = sv.factors()
        rp, ci, lu = f["row_ptr"], f["col"], f["lu"]
        n = s.n
        rows = np.repeat(np.arange(n), np.diff(rp[:n + 1]))
        blk_lo = np.repeat(s.block_ptr[:-1], np.diff(s.block_ptr))
        ref = P.v[P.rp[rows] + (ci - blk_lo[rows])]
        big = np.abs(P.v).max()
        d = np.abs(lu - ref).max()
        mask = np.ones(P.v.shape[0], dtype=bool)
        mask[P.rp[rows] + (ci - blk_lo[rows])] = False
        outside = np.abs(P.v[mask]).max() if mask.any() else 0.0
        print(f"  factor entries {lu.shape[0]} (dense blocks {P.v.shape[0]}), max diff {d / big:.2e}, "
              f"largest oracle entry outside the pattern {outside:.1e}")
        assert d <= 1e-12 * big and outside == 0.0
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        if o.krylov == sd.GMRES:
            x_o, its_o, rr_o, st_o, _ = O.gmres_bj(s, P, tol=1e-8, m=30)
        else:
            x_o, its_o, rr_o, st_o, _ = O.pcg_bj(s, P, tol=1e-8)
        x = x.cpu().numpy()
        print(f"  GPU its {its}, oracle its {its_o}")
        assert st == sd.OK and st_o == O.OK and O.relres(s, x) <= 1e-8
        assert abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x - x_o) <= 1e-6 * np.linalg.norm(x_o)
    finally:
        sv.close()


def test_bbd_with_complete_blocks_matches_oracle():
    """The paper's BBD preconditioner proper: complete LU of the interior
    blocks (Sec. 3.1) with the dense Schur complement.  Without a filter it
    is M itself (one GMRES step on a small bordered system); on C3 x 0.004
    the Schur LU takes the oracle's pivots, LU and apply agree within
    1e-10, and GMRES(30) takes the oracle's iterations within 10% (or 2)."""
    s = gen.bbd_system(nblocks=4, block_rows=300, n_border=48, nnz_off=4, half_band=10, tail_frac=0.2,
                       border_c=2, seed=14, name="bbd-small")
    sv = sd.from_system(s, opts(**dict(BBD_OPTS, factor=sd.FACT_COMPLETE)))
    try:
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-10)
        assert st == sd.OK and its == 1 and O.relres(s, x.cpu().numpy()) <= 1e-10
    finally:
        sv.close()
    s = gen.c3(0.004)
    sv = sd.from_system(s, opts(**dict(BBD_OPTS, factor=sd.FACT_COMPLETE)))
    try:
        P = O.BBD(s, complete=True)
        assert P.status == O.OK
        lu, piv, _ = sv.schur()
        parts = P.parts()
        assert np.array_equal(piv, parts["piv"].astype(np.int32))
        assert np.max(np.abs(lu - parts["S"])) <= 1e-10 * np.max(np.abs(parts["S"]))
        r = np.random.default_rng(22).standard_normal(s.n)
        z = sv.precond_apply(tdev(r)).cpu().numpy()
        zo = P.apply(r)
        assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        x_o, its_o, rr_o, st_o, _ = O.gmres_bbd(s, P, tol=1e-8, m=30)
        _, its_i, _, _, _ = O.gmres_bbd(s, O.BBD(s), tol=1e-8, m=30)
        print(f"  C3x0.004 complete BBD: GPU its {its}, oracle its {its_o} (ILU(0) blocks: {its_i})")
        assert st == sd.OK and st_o == O.OK and abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x.cpu().numpy() - x_o) <= 1e-6 * np.linalg.norm(x_o)
    finally:
        sv.close()


def test_complete_single_block_is_exact():
    """Without a filter the complete LU of the one block is the matrix's own
    LU: PCG on C1 (2,000 rows, nearly full fill) converges in one step, and
    refactor with new values refills and refactors the same way."""
    s = gen.c1()
    one = gen.System("c1-one", s.row_ptr, s.col, s.val, s.b, np.array([0, s.n], dtype=np.int32))
    sv = sd.from_system(one, opts(factor=sd.FACT_COMPLETE))
    try:
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        print(f"  C1 one block: its {its}, factor entries {sv.info()['nnz_kept']}")
        assert st == sd.OK and its == 1 and O.relres(one, x.cpu().numpy()) <= 1e-8
        rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
        v2 = s.val.copy()
        v2[s.col == rows] *= 2.0
        sv.refactor(tdev(v2))
        two = gen.System("c1-one-2", s.row_ptr, s.col, v2, s.b, np.array([0, s.n], dtype=np.int32))
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        assert st == sd.OK and its == 1 and O.relres(two, x.cpu().numpy()) <= 1e-8
    finally:
        sv.close()


def scrambled_system(n=1200, nblocks=6, seed=8):
    """The banded nonsymmetric system with its rows randomly permuted and
    rows / columns scaled over 1e-4..1e4: its diagonal is mostly empty, so
    block Jacobi cannot run on it as it stands; MC64 (Alg. 3) recovers a
    permutation with a heavy unit diagonal."""
    s = nonsym_system(n=n, nblocks=nblocks, seed=seed)
    rng = np.random.default_rng(seed + 100)
    a = s.scipy()
    a = sp.diags(10.0 ** rng.uniform(-4, 4, n)) @ a[rng.permutation(n)] @ sp.diags(10.0 ** rng.uniform(-2, 2, n))
    a = a.tocsr()
    a.sort_indices()
    return gen.System("scrambled", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                      rng.standard_normal(n), s.block_ptr)


def test_mc64_matching_scaling_and_solve_match_oracle():
    """MC64 on the host of the library (sparse shortest augmenting paths)
    against the oracle's dense Hungarian method: the same matching (unique
    for these random values), scalings that bound every scaled entry by 1
    with the matched ones equal to 1, and block-Jacobi GMRES through Alg. 3
    (A' y = Q Dr b, x = Dc y) that solves the original system like the
    oracle: iterations within 10% (or 2), solution within 1e-6."""
    print("[mc64 nonsymmetric]", flush=True)
    s = scrambled_system()
    o = opts(krylov=sd.GMRES, spd=False, pivot=sd.PIVOT_FAIL, mc64=True)
    sv = sd.from_system(s, o)
    try:
        row_of, dr, dc = sv.mc64()
        match_o, dr_o, dc_o, st_o = O.mc64(s)
        assert st_o == O.OK
        inv = np.empty_like(match_o)
        inv[match_o] = np.arange(s.n, dtype=match_o.dtype)
        assert np.array_equal(row_of, inv)
        a = s.scipy().tocoo()
        sc = np.abs(dr[a.row] * a.data * dc[a.col])
        assert sc.max() <= 1.0 + 1e-12
        matched = a.col == match_o[a.row]
        np.testing.assert_allclose(sc[matched], 1.0, rtol=1e-12)
        assert sv.info()["mc64_moved"] == int(np.count_nonzero(match_o != np.arange(s.n)))
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-10)
        s2, x_of = O.mc64_transform(s, match_o, dr_o, dc_o)
        P = O.BJ(s2, **oracle_opts(o))
        y_o, its_o, rr_o, st2, _ = O.gmres_bj(s2, P, tol=1e-10, m=30, maxit=5000)
        x_o = x_of(y_o)
        x = x.cpu().numpy()
        print(f"  GPU its {its} relres(A') {rr:.2e}; oracle its {its_o} relres(A') {rr_o:.2e}; "
              f"moved rows {sv.info()['mc64_moved']}")
        assert st == sd.OK and st2 == O.OK
        assert abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x - x_o) <= 1e-6 * np.linalg.norm(x_o)
        # the tolerance is that of A' y = b'; on A x = b the residual is the
        # oracle's (rows of A are scaled over 1e-4..1e4, so ||Dr^-1|| ||Dr||
        # bounds the ratio of the two relative residuals)
        rr_a, rr_ao = O.relres(s, x), O.relres(s, x_o)
        print(f"  relres on A x = b: GPU {rr_a:.2e}, oracle {rr_ao:.2e}")
        assert rr_a <= 2.0 * rr_ao + 1e-14
        assert rr_a <= 1e-10 * (dr.max() / dr.min())
    finally:
        sv.close()


def test_mc64_spd_is_jacobi_scaling_and_refactor_reuses_it():
    """SPD mode: the identity matching with 1/sqrt(a_ii) on both sides (the
    oracle's Hungarian method finds the identity and sqrt(dr dc) equals it);
    PCG on S A S matches the oracle on its transformed system; refactor with
    new values maps them through the same transform (the result equals a
    fresh handle on the new values scaled by the old diagonal)."""
    s = gen.c1()
    o = opts(mc64=True)
    sv = sd.from_system(s, o)
    try:
        row_of, dr, dc = sv.mc64()
        d = s.scipy().diagonal()
        assert np.array_equal(row_of, np.arange(s.n))
        np.testing.assert_allclose(dr, 1.0 / np.sqrt(d), rtol=1e-15)
        assert np.array_equal(dr, dc)
        match_o, dr_o, dc_o, _ = O.mc64(s)
        assert np.array_equal(match_o, np.arange(s.n))
        np.testing.assert_allclose(np.sqrt(dr_o * dc_o), dr, rtol=1e-10)
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        s2, x_of = O.mc64_transform(s, match_o, dr_o, dc_o, spd=True)
        y_o, its_o, rr_o, st_o, _ = O.pcg_bj(s2, O.BJ(s2, **oracle_opts(o)), tol=1e-8)
        x = x.cpu().numpy()
        print(f"  C1 MC64 (SPD): GPU its {its}, oracle its {its_o}")
        assert st == sd.OK and st_o == O.OK and abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x - x_of(y_o)) <= 1e-6 * np.linalg.norm(x_of(y_o))
        # refactor: new values (the diagonal raised by half the row's
        # magnitude sum), mapped through the transform of the old ones
        M = s.scipy()
        rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
        v2 = s.val.copy()
        on_diag = s.col == rows
        v2[on_diag] += 0.5 * np.asarray(abs(M).sum(axis=1)).ravel()[rows[on_diag]]
        sv.refactor(tdev(v2))
        x2, its2, rr2, st2 = sv.solve(tdev(s.b), tol=1e-8)
        s3 = gen.System("c1-new", s.row_ptr, s.col, v2, s.b, s.block_ptr)
        s_old = 1.0 / np.sqrt(d)
        s3b, x_of3 = O.mc64_transform(s3, np.arange(s.n, dtype=np.int32), s_old, s_old, spd=False)
        y3, its3, _, st3, _ = O.pcg_bj(s3b, O.BJ(s3b, **oracle_opts(o)), tol=1e-8)
        print(f"  after refactor: GPU its {its2}, oracle on the old transform its {its3}")
        assert st2 == sd.OK and st3 == O.OK and abs(its2 - its3) <= max(2, 0.1 * its3)
        assert np.linalg.norm(x2.cpu().numpy() - x_of3(y3)) <= 1e-6 * np.linalg.norm(x_of3(y3))
    finally:
        sv.close()


def test_mc64_rejects_what_it_cannot_transform():
    """A structurally singular matrix (no matching of nonzeros) is
    SDSL_E_STRUCTURE; a low-rank term or a BBD border is SDSL_E_INVALID."""
    a = sp.csr_matrix(np.array([[1.0, 0.0, 2.0], [3.0, 0.0, 1.0], [0.0, 0.0, 4.0]]))
    a = (a + sp.csr_matrix((np.array([0.0]), (np.array([1]), np.array([1]))), shape=(3, 3))).tocsr()
    a.sort_indices()
    bad = gen.System("sing", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data, np.ones(3),
                     np.array([0, 3], dtype=np.int32))
    with pytest.raises(sd.SdslError) as e:
        sd.from_system(bad, opts(krylov=sd.GMRES, spd=False, mc64=True))
    assert e.value.status == sd.E_STRUCTURE
    with pytest.raises(sd.SdslError) as e:
        sd.from_system(gen.c2(0.004), opts(mc64=True))
    assert e.value.status == sd.E_INVALID


def _row_scaled_system(seed, n=400):
    """Nonsymmetric, weakly dominant, rows scaled over 1e-5..1e5: GMRES(60)
    makes slow progress, which keeps a long run of cycles meaningful."""
    rng = np.random.default_rng(100 + seed)
    a = sp.random(n, n, density=0.02, random_state=rng, data_rvs=rng.standard_normal).toarray()
    np.fill_diagonal(a, 0.0)
    np.fill_diagonal(a, 0.05 * np.abs(a).sum(axis=1) + 1.0)
    a = np.diag(10.0 ** rng.uniform(-5, 5, n)) @ a
    m = sp.csr_matrix(a)
    m.sort_indices()
    return gen.System("rowscaled", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                      rng.standard_normal(n), gen.contiguous_blocks(n, 40))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gmres_long_run_on_row_scaled_system(seed):
    """600 steps of GMRES(60) that do not converge: the true residual after
    the run matches the oracle's (both orthogonalise with classical
    Gram-Schmidt applied twice; a basis that lost orthogonality would let
    the residual drift by factors of 2-10) and stays below ||b||."""
    s = _row_scaled_system(seed)
    o = opts(krylov=sd.GMRES, spd=False, pivot=sd.PIVOT_FAIL, restart=60, max_iter=600)
    sv = sd.from_system(s, o)
    P = O.BJ(s, **oracle_opts(o))
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-13)
    x_o, its_o, rr_o, st_o, _ = O.gmres_bj(s, P, tol=1e-13, m=60, maxit=600)
    print(f"  seed {seed}: GPU its {its} relres {rr:.4e}; oracle its {its_o} relres {rr_o:.4e}")
    assert st == sd.E_NOT_CONVERGED and its == its_o == 600
    assert rr <= 1.0 and abs(rr - rr_o) <= 0.05 * rr_o
    sv.close()


def test_gmres_c1_matches_oracle_within_rounding_spread():
    """C1 with GMRES(30).  Restarted GMRES on this SPD system (D spread 1e8)
    stagnates between restarts, and rounding alone moves its count: in the
    oracle, one ulp of one entry of b takes the 4,632 iterations to anywhere
    in 3,029-3,899 (12 draws, tests/golden/c1_gmres_ensemble.json, written by
    make_c1_gmres_ensemble.py), while the residual histories agree to 1e-12
    for the first 300 iterations and separate only after 1,200.  Gates: the
    true residual after 30 and 300 iterations equals the oracle's (1e-6
    relative), the solve meets 1e-8, and its count lies within 10% of the
    range the oracle spans under one-ulp changes of b."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_gmres_ensemble.json")) as f:
        ens = json.load(f)
    s = gen.c1()
    o = opts(krylov=sd.GMRES, max_iter=20_000)
    sv = sd.from_system(s, o)
    try:
        b = tdev(s.b)
        for k in (30, 300):
            sv.set_max_iter(k)
            _, its, rr, st = sv.solve(b, tol=1e-30)
            ref = ens[f"relres_after_{k}"]
            print(f"  after {k}: GPU relres {rr:.12e}, oracle {ref:.12e}")
            assert its == k and abs(rr - ref) <= 1e-6 * ref
        sv.set_max_iter(o.max_iter)
        x, its, rr, st = sv.solve(b, tol=1e-8)
        true_rr = O.relres(s, x.cpu().numpy())
        lo, hi = min(ens["one_ulp_counts"] + [ens["iterations"]]), max(ens["one_ulp_counts"] + [ens["iterations"]])
        print(f"  C1 GMRES: GPU its {its} relres {true_rr:.2e}; oracle {ens['iterations']}, one-ulp range {lo}-{hi}")
        assert st == sd.OK and true_rr <= 1e-8
        assert 0.9 * lo <= its <= 1.1 * hi
    finally:
        sv.close()


def test_gmres_exact_preconditioner_one_step():
    """Tridiagonal nonsymmetric single block: ILU(0) is exact, so right-
    preconditioned GMRES converges in one step."""
    rng = np.random.default_rng(5)
    n = 4000
    lo, up = rng.standard_normal(n - 1), rng.standard_normal(n - 1)
    dg = np.abs(np.r_[lo, 0]) + np.abs(np.r_[0, up]) + 1.0
    a = sp.diags([lo, dg, up], [-1, 0, 1]).tocsr()
    a.sort_indices()
    s = gen.System("tri-ns", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data,
                   rng.standard_normal(n), np.array([0, n], dtype=np.int32))
    sv = sd.from_system(s, opts(krylov=sd.GMRES, spd=False))
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-12)
    assert st == sd.OK and its == 1 and O.relres(s, x.cpu().numpy()) <= 1e-12
    sv.close()


# ------------------------------------------------------------------ BBD

BBD_OPTS = dict(method=sd.BBD, krylov=sd.GMRES, spd=False)


@pytest.fixture(scope="module", params=["C3x0.004", "C3x0.02"])
def bbd_case(request):
    print(f"\n[bbd case {request.param}]", flush=True)
    s = gen.c3(float(request.param[3:]))
    sv = sd.from_system(s, opts(**BBD_OPTS))
    P = O.BBD(s)
    assert P.status == O.OK
    yield request.param, s, sv, P
    sv.close()


def test_bbd_schur_lu_matches_oracle(bbd_case):
    """Dense border Schur complement: GPU (MFMA assembly, blocked LU) and
    oracle (column-by-column assembly, unblocked LU) take the same pivots and
    agree to rounding; the GPU inverse inverts the oracle's S."""
    name, s, sv, P = bbd_case
    lu, piv, inv = sv.schur()
    parts = P.parts()
    lu_o, piv_o = parts["S"], parts["piv"]
    m = s.n_border
    assert np.array_equal(piv, piv_o.astype(np.int32))
    assert np.max(np.abs(lu - lu_o)) <= 1e-10 * np.max(np.abs(lu_o))
    L = np.tril(lu_o, -1) + np.eye(m)
    U = np.triu(lu_o)
    S = L @ U
    for k in reversed(range(m)):           # undo the row swaps
        S[[k, piv_o[k]]] = S[[piv_o[k], k]]
    assert np.max(np.abs(inv @ S - np.eye(m))) <= 1e-9
    print(f"  {name}: border {m}, max |LU - LU_oracle| / max |LU| = "
          f"{np.max(np.abs(lu - lu_o)) / np.max(np.abs(lu_o)):.2e}")


def test_bbd_apply_matches_oracle(bbd_case):
    name, s, sv, P = bbd_case
    r = np.random.default_rng(21).standard_normal(s.n)
    z = sv.precond_apply(tdev(r)).cpu().numpy()
    zo = P.apply(r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)


def test_bbd_gmres_matches_oracle(bbd_case):
    name, s, sv, P = bbd_case
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
    x_o, its_o, rr_o, st_o, _ = O.gmres_bbd(s, P, tol=1e-8, m=30)
    true_rr = O.relres(s, x.cpu().numpy())
    print(f"  {name}: GPU its {its} relres {true_rr:.2e}; oracle its {its_o} relres {rr_o:.2e}")
    assert st == sd.OK and st_o == O.OK and true_rr <= 1e-8
    assert abs(its - its_o) <= max(2, 0.1 * its_o)
    assert np.linalg.norm(x.cpu().numpy() - x_o) <= 1e-6 * np.linalg.norm(x_o)


def test_bbd_gcr_matches_oracle(bbd_case):
    """GCR(30) with the BBD preconditioner, the pairing of the paper's
    ill-conditioned runs (Sec. 4.3): iterations within 10% (or 2) of the
    oracle's, true relres <= 1e-8, solution within 1e-6."""
    name, s, _, P = bbd_case
    sv = sd.from_system(s, opts(**dict(BBD_OPTS, krylov=sd.GCR)))
    try:
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        x_o, its_o, rr_o, st_o, _ = O.gcr_bbd(s, P, tol=1e-8, m=30)
        true_rr = O.relres(s, x.cpu().numpy())
        print(f"  {name} GCR: GPU its {its} relres {true_rr:.2e}; oracle its {its_o} relres {rr_o:.2e}")
        assert st == sd.OK and st_o == O.OK and true_rr <= 1e-8
        assert abs(its - its_o) <= max(2, 0.1 * its_o)
        assert np.linalg.norm(x.cpu().numpy() - x_o) <= 1e-6 * np.linalg.norm(x_o)
    finally:
        sv.close()


def test_full_c3_bbd_matches_oracle_samples():
    """C3 at full size (1,500,096 rows, 32 blocks, 4,096-row border): the
    Schur LU takes the oracle's pivots, sampled LU entries and sampled
    entries of one preconditioner apply agree within 1e-10 of the largest
    magnitude, GMRES(30) takes the oracle's iteration count within 10%, and
    the solution meets 1e-8 (oracle residual) and agrees with the oracle's
    sampled entries within 1e-6 of its largest.  The oracle's numbers take it
    a minute, so they are stored: tests/golden/c3_full_samples.json, written
    by make_c3_full.py."""
    import json
    import os
    print("\n[C3 at full size]", flush=True)
    with open(os.path.join(os.path.dirname(__file__), "golden", "c3_full_samples.json")) as f:
        gold = json.load(f)
    s = gen.c3(1.0)
    assert s.n == gold["n"] and s.n_border == gold["n_border"]
    sv = sd.from_system(s, opts(**BBD_OPTS))
    try:
        lu, piv, _ = sv.schur()
        assert np.array_equal(piv, np.asarray(gold["pivots"]))
        smp = np.asarray(gold["lu_samples"])
        ii, jj = smp[:, 0].astype(np.int64), smp[:, 1].astype(np.int64)
        d = np.max(np.abs(lu[ii, jj] - smp[:, 2]))
        print(f"  Schur LU: pivots equal, sampled max diff {d:.2e} (max |LU| {gold['lu_max_abs']:.2e})")
        assert d <= 1e-10 * gold["lu_max_abs"]
        del lu
        r = np.random.default_rng(gold["apply_rhs_seed"]).standard_normal(s.n)
        z = sv.precond_apply(tdev(r)).cpu().numpy()
        smp = np.asarray(gold["apply_samples"])
        d = np.max(np.abs(z[smp[:, 0].astype(np.int64)] - smp[:, 1]))
        print(f"  apply: sampled max diff {d:.2e} (max |z| {gold['apply_max_abs']:.2e})")
        assert d <= 1e-10 * gold["apply_max_abs"]
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        x = x.cpu().numpy()
        g = gold["gmres"]
        true_rr = O.relres(s, x)
        smp = np.asarray(g["x_samples"])
        d = np.max(np.abs(x[smp[:, 0].astype(np.int64)] - smp[:, 1]))
        print(f"  GMRES: {its} iterations (oracle {g['iterations']}), relres {true_rr:.2e}, sampled solution "
              f"max diff {d:.2e} (max |x| {g['x_max_abs']:.2e})")
        assert st == sd.OK and true_rr <= 1e-8
        assert abs(its - g["iterations"]) <= max(1, 0.10 * g["iterations"])
        assert d <= 1e-6 * g["x_max_abs"]
    finally:
        sv.close()


def test_alg1_switch_through_the_library():
    """Alg. 1 through the library: on a bordered system whose border couples
    strongly to its blocks (gen.strong_border_system), block-Jacobi GMRES
    fails with fresh factors, the sequence driver switches to BBD for good,
    and BBD GMRES converges with the oracle's count (10% or 2); the oracle's
    block-Jacobi GMRES fails on the system too.  The next two systems of the
    sequence (scaled values) stay on BBD and reuse its factors."""
    from paper_2604_23979_amd.ipm import SequenceSolver
    s = gen.strong_border_system(20.0)
    bj = gen.as_block_jacobi(s)
    _, its_j, rr_j, st_j, _ = O.gmres_bj(bj, O.BJ(bj, spd=False), tol=1e-8, m=30, maxit=300)
    _, its_b, rr_b, st_b, _ = O.gmres_bbd(s, O.BBD(s), tol=1e-8, m=30, maxit=300)
    print(f"\n  oracle: BJ {its_j} its relres {rr_j:.2e} (status {st_j}); BBD {its_b} its relres {rr_b:.2e}")
    assert st_j == O.NOT_CONVERGED and st_b == O.OK
    o_bj = opts(krylov=sd.GMRES, spd=False, max_iter=300)
    o_bbd = opts(method=sd.BBD, krylov=sd.GMRES, spd=False, max_iter=300)
    make = lambda sys_, o: sd.from_system(gen.as_block_jacobi(sys_) if o.method == sd.BJ else sys_, o)
    seq = SequenceSolver(make, o_bj, bbd_options=o_bbd)
    try:
        for k in range(3):
            vals = s.val * (1.0 + 0.25 * k)
            sk = gen.System(f"sb{k}", s.row_ptr, s.col, vals, s.b, s.block_ptr, n_border=s.n_border)
            x, rec = seq.step(k, sk, tdev(vals), tdev(s.b), tol=1e-8)
            true_rr = O.relres(sk, x.cpu().numpy())
            print(f"  step {k}: {rec.kind} {rec.method} {rec.iterations} its, status {rec.status}, relres {true_rr:.2e}")
            assert rec.status == sd.OK and true_rr <= 1e-8 and rec.method == "BBD"
            if k == 0:
                assert rec.kind == "setup+bbd" and seq.switched
                assert abs((rec.iterations - 300) - its_b) <= max(2, 0.1 * its_b)
            else:
                assert rec.kind == "reuse"
    finally:
        seq.close()


def test_bbd_exact_blocks_one_step():
    """Tridiagonal interior blocks: ILU(0) is exact, the BBD preconditioner
    is M itself and GMRES converges in one step."""
    s = gen.bbd_system(nblocks=4, block_rows=500, n_border=96, nnz_off=1, half_band=1, tail_frac=0.1,
                       border_c=2, seed=16, name="bbd-tri")
    sv = sd.from_system(s, opts(**BBD_OPTS))
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-10)
    assert st == sd.OK and its == 1 and O.relres(s, x.cpu().numpy()) <= 1e-10
    sv.close()


def test_bbd_early_border_rows_match_oracle():
    """Border rows that reach interior columns far left of every row with a
    border-column entry: the tails start at those columns (nearly whole
    blocks), and the Schur LU, the apply and the GMRES solve still match the
    oracle."""
    s = gen.bbd_system(nblocks=3, block_rows=600, n_border=96, nnz_off=4, half_band=10, tail_frac=0.1,
                       border_c=2, seed=14, name="bbd-early")
    M = s.scipy().tolil()
    ni = s.n - s.n_border
    M[ni, 1] = 0.3
    M[ni + 5, 1207] = -0.4
    M = M.tocsr()
    M.sort_indices()
    s = gen.System("bbd-early", M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data, s.b,
                   s.block_ptr, n_border=s.n_border)
    sv = sd.from_system(s, opts(**BBD_OPTS))
    P = O.BBD(s)
    assert P.status == O.OK
    assert list(P.parts()["tail"][[0, 2]]) == [1, 1207]
    lu, piv, inv = sv.schur()
    parts = P.parts()
    assert np.array_equal(piv, parts["piv"].astype(np.int32))
    assert np.max(np.abs(lu - parts["S"])) <= 1e-10 * np.max(np.abs(parts["S"]))
    r = np.random.default_rng(22).standard_normal(s.n)
    z = sv.precond_apply(tdev(r)).cpu().numpy()
    zo = P.apply(r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
    x_o, its_o, rr_o, st_o, _ = O.gmres_bbd(s, P, tol=1e-8, m=30)
    print(f"  GPU its {its} relres {rr:.2e}; oracle its {its_o} relres {rr_o:.2e}")
    assert st == sd.OK and st_o == O.OK and O.relres(s, x.cpu().numpy()) <= 1e-8
    assert abs(its - its_o) <= max(2, 0.1 * its_o)
    sv.close()


@pytest.mark.parametrize("row,col", [(0, 450), (299, 300), (300, 299)],
                         ids=["inside", "next-block-first-column", "previous-block-last-column"])
def test_bbd_rejects_block_coupling(row, col):
    s = gen.bbd_system(nblocks=2, block_rows=300, n_border=64, nnz_off=2, half_band=4, tail_frac=0.2,
                       border_c=1, seed=17)
    M = s.scipy().tolil()
    M[row, col] = 1.0  # an interior row of one block -> an interior column of another
    M = M.tocsr()
    M.sort_indices()
    s2 = gen.System("bad", M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data, s.b,
                    s.block_ptr, n_border=s.n_border)
    with pytest.raises(sd.SdslError) as e:
        sd.from_system(s2, opts(**BBD_OPTS))
    assert e.value.status == sd.E_STRUCTURE


# ------------------------------------------------------------------ serving

@pytest.mark.parametrize("mode", ["shared-graphs", "shared", "streams"])
def test_serving_mix_equals_alone(mode):
    """Continuous batching: requests of different sizes admitted while
    others run (shared launches on one stream, with or without graph replay,
    or one stream per request); every result is bitwise the one the same
    request gets when solved alone."""
    from paper_2604_23979_amd.serve import Request, Server
    reqs = gen.c5_requests(count=6, seed=3, m_lo=3000, m_hi=30000)
    systems = [gen.c5_system(r) for r in reqs]
    o = opts(precision=sd.FP32_IR, filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
    alone = []
    for s in systems:
        sv = sd.from_system(s, o)
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        alone.append((x.cpu().numpy(), its, st))
        sv.close()
    srv = Server(options=o, tol=1e-8, max_active=4, shared=mode != "streams", graphs=mode == "shared-graphs")
    done = srv.run([Request(s, arrival=0.002 * i, tag=i) for i, s in enumerate(systems)])
    stats = srv.stats()
    print(f"  serving ({mode}): {stats}")
    assert stats["requests"] == len(systems) and stats["max_concurrency"] >= 2
    if mode != "streams":
        g = stats["group"]
        assert g["slot_issues"] > g["flushes"] > 0           # launches were shared
        assert (g["graph_launches"] > g["captures"] > 0) == (mode == "shared-graphs")
    for r in done:
        xa, its_a, st_a = alone[r.tag]
        assert r.status == st_a == sd.OK and r.iters == its_a
        assert np.array_equal(r.x.cpu().numpy(), xa)
        assert O.relres(systems[r.tag], xa) <= 1e-8


@pytest.mark.parametrize("graphs", [True, False], ids=["graphs", "launches"])
def test_group_steps_equal_solo_solves(graphs):
    """A group advancing handles of every kind on one stream: FP64 PCG,
    FP32-inner PCG, classical refinement (their PCG iterations share
    launches), a low-rank handle and a GMRES handle (stepped on their own);
    solves begin at different steps and end at different steps.  Every
    result (solution, iterations, residual) is bitwise that of a solve alone."""
    geo = dict(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
    cases = [
        ("c1-fp64", gen.c1(), opts()),
        ("ragged-fp64", ragged_system(), opts()),
        ("c2-fp32ir", gen.c2(0.004, dense_cols=0), opts(precision=sd.FP32_IR, **geo)),
        ("c1-restart", gen.c1(), opts(precision=sd.FP32_IR_RESTART)),
        ("ragged2-fp32ir", ragged_system(n=5000, nblocks=9, seed=7), opts(precision=sd.FP32_IR)),
        ("c2-lowrank", gen.c2(0.004), opts(**geo)),
        ("gmres", nonsym_system(), opts(krylov=sd.GMRES, spd=False)),
    ]
    solo = {}
    for name, s, o in cases:
        sv = sd.from_system(s, o)
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
        solo[name] = (x.cpu(), its, rr, st)
        sv.close()
    stream = torch.cuda.Stream()
    grp = sd.Group(stream, graphs=graphs)
    svs, bufs = {}, {}
    for name, s, o in cases:
        svs[name] = sd.from_system(s, o, stream=stream)
        with torch.cuda.stream(stream):
            bufs[name] = (tdev(s.b), torch.empty(s.n, dtype=torch.float64, device=DEV))
    running, results, steps = [], {}, 0
    late = {name: 3 * i for i, (name, _, _) in enumerate(cases)}   # staggered joins
    while len(results) < len(cases):
        for name in [n for n, at in late.items() if at == steps]:
            b, x = bufs[name]
            if steps % 2:
                grp.begin(svs[name], b, x, 1e-8)
            else:
                svs[name].solve_begin(b, x, 1e-8)
            running.append(name)
        if running:
            done = grp.step([svs[n] for n in running])
            for n, d in zip(list(running), done):
                if d:
                    results[n] = svs[n].solve_end()
                    running.remove(n)
        steps += 1
        assert steps < 100_000
    stream.synchronize()
    st_g = grp.stats()
    print(f"  group stats ({'graphs' if graphs else 'launches'}): {st_g}")
    for name, _, _ in cases:
        x, its, rr, st = results[name]
        xs, its_s, rr_s, st_s = solo[name]
        assert st == st_s == sd.OK and its == its_s and rr == rr_s, name
        assert torch.equal(x.cpu(), xs), name
    assert st_g["slot_issues"] > st_g["flushes"] > 0
    assert (st_g["graph_launches"] > 0) == graphs
    for sv in svs.values():
        sv.close()
    grp.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32ir", "restart"])
def test_graph_replayed_solve_equals_plain_solve(prec):
    """graphs = 1: sdsl_solve issues each check interval's PCG iterations as
    one replayed HIP graph of the shared-launch kernels; the solution,
    iterations and residual are bitwise those of the plain launches (C1 and
    a ragged system, every precision form)."""
    mode = {"fp64": sd.FP64, "fp32ir": sd.FP32_IR, "restart": sd.FP32_IR_RESTART}[prec]
    for s in (gen.c1(), ragged_system()):
        res = []
        for graphs in (False, True):
            sv = sd.from_system(s, opts(precision=mode, graphs=graphs))
            try:
                x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
                x2, its2, rr2, st2 = sv.solve(tdev(s.b), tol=1e-8)   # the cached graphs again
                assert (its2, rr2, st2) == (its, rr, st) and torch.equal(x, x2)
                res.append((x.cpu(), its, rr, st))
            finally:
                sv.close()
        (xa, ia, ra, sa), (xb, ib, rb, sb) = res
        print(f"  {s.name} {prec}: its {ia}, graphs {ib}")
        assert sa == sb == sd.OK and ia == ib and ra == rb and torch.equal(xa, xb)


def test_group_refuses_misuse():
    """A handle on another stream and a handle with no running solve are
    refused (the others in the step still advance); a solve begun in a group
    cannot be stepped alone before the group's next step."""
    s = gen.c1()
    stream = torch.cuda.Stream()
    grp = sd.Group(stream)
    a = sd.from_system(s, stream=stream)
    other = sd.from_system(s)                     # default stream
    b = tdev(s.b)
    x = torch.empty_like(b)
    with pytest.raises(sd.SdslError) as e:
        grp.begin(other, b, x)
    assert e.value.status == sd.E_INVALID
    with pytest.raises(sd.SdslError) as e:
        grp.step([a])                             # nothing begun
    assert e.value.status == sd.E_STATE
    grp.begin(a, b, x)
    with pytest.raises(sd.SdslError) as e:
        a.solve_step()
    assert e.value.status == sd.E_STATE
    while not grp.step([a])[0]:
        pass
    _, its, rr, st = a.solve_end()
    assert st == sd.OK and rr <= 1e-8
    for h in (a, other):
        h.close()
    grp.close()


def test_solve_writes_a_jsonl_record(tmp_path):
    """One JSON line per solve with what the library reports, and one per
    served request with its arrival, admission and completion times."""
    from paper_2604_23979_amd.serve import Request, Server
    from paper_2604_23979_amd.solvelog import JsonlLog, read
    s = gen.c1()
    path = str(tmp_path / "solves.jsonl")
    with JsonlLog(path) as log:
        sv = sd.from_system(s)
        x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8, log=log, extra={"config": "C1"})
        sv.close()
        srv = Server(options=sd.Options(), max_active=2, log=log)
        srv.run([Request(s, 0.0, "a"), Request(s, 0.0, "b")])
    recs = read(path)
    assert len(recs) == 3
    r = recs[0]
    assert r["config"] == "C1" and r["status"] == "OK" and r["iterations"] == its and r["relres"] == rr
    assert r["n"] == s.n and r["nnz"] == s.nnz and r["gbps"] > 0 and r["tol"] == 1e-8
    for q in recs[1:]:
        assert q["request"] in ("a", "b") and q["iterations"] == its and q["finished_s"] >= q["admitted_s"] >= 0


def test_async_solve_equals_solve():
    s = gen.c1()
    sv = sd.from_system(s)
    b = tdev(s.b)
    x1, its1, rr1, st1 = sv.solve(b)
    x2 = torch.empty_like(b)
    sv.solve_begin(b, x2)
    while not sv.solve_step():
        pass
    x2, its2, rr2, st2 = sv.solve_end()
    assert st1 == st2 == sd.OK and its1 == its2 and rr1 == rr2
    assert torch.equal(x1, x2)
    sv.close()


def test_calls_refused_while_an_async_solve_runs():
    """One running solve per handle: while an asynchronous solve is
    unfinished, every call that would share its vectors or factors returns
    SDSL_E_STATE, and a batch may not name a handle twice."""
    s = gen.c1()
    sv = sd.from_system(s, opts())
    try:
        b = tdev(s.b)
        x = torch.empty_like(b)
        sv.solve_begin(b, x, 1e-8)
        calls = {"solve": lambda: sv.solve(b), "refactor": lambda: sv.refactor(tdev(s.val)),
                 "update_values": lambda: sv.update_values(tdev(s.val)), "spmv": lambda: sv.spmv(b),
                 "precond_apply": lambda: sv.precond_apply(b), "residual": lambda: sv.residual(b, x),
                 "set_max_iter": lambda: sv.set_max_iter(10), "solve_begin": lambda: sv.solve_begin(b, x)}
        for name, call in calls.items():
            with pytest.raises(sd.SdslError) as e:
                call()
            assert e.value.status == sd.E_STATE, name
        while not sv.solve_step():
            pass
        _, its, rr, st = sv.solve_end()
        assert st == sd.OK and rr <= 1e-8
        x2 = torch.empty_like(b)
        its2, rr2, st2 = sd.solve_batch([sv, sv], [b, b], [x, x2])
        assert st2 == sd.E_STATE and its2[0] == its
    finally:
        sv.close()


def test_handle_memory_comes_from_the_torch_allocator():
    """With the allocator hook the handle's device memory is PyTorch's: it
    shows in torch.cuda.memory_allocated() while the handle lives and goes
    back to the caching allocator (not to hipFree) when it is destroyed."""
    s = gen.c2(0.02)
    o = opts(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    sv = sd.from_system(s, o)
    held = torch.cuda.memory_allocated() - base
    dev = sv.info()["device_bytes"]
    assert dev > 0 and dev <= held <= 1.5 * dev + (64 << 20), (dev, held)
    x, its, rr, st = sv.solve(tdev(s.b), tol=1e-8)
    assert st == sd.OK
    del x
    reserved = torch.cuda.memory_reserved()
    sv.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= base + 8 * s.n + 512
    assert torch.cuda.memory_reserved() == reserved  # cached, not freed
    plain = sd.from_system(s, o, torch_memory=False)
    try:
        assert torch.cuda.memory_allocated() <= base + 8 * s.n + 512
        _, its2, _, st2 = plain.solve(tdev(s.b), tol=1e-8)
        assert st2 == sd.OK and its2 == its
    finally:
        plain.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_set_max_iter_caps_a_solve(prec):
    """A capped solve stops at the cap with E_NOT_CONVERGED; raising the cap
    again gives the uncapped result (the handle keeps no state of the capped
    solve)."""
    s = gen.c1()
    p = {"fp64": sd.FP64, "fp32ir": sd.FP32_IR}[prec]
    sv = sd.from_system(s, sd.Options(precision=p))
    b = tdev(s.b)
    x0, its0, rr0, st0 = sv.solve(b)
    assert st0 == sd.OK and its0 > 20
    sv.set_max_iter(10)
    _, its1, rr1, st1 = sv.solve(b)
    assert st1 == sd.E_NOT_CONVERGED and its1 <= 11 and rr1 > 1e-8  # an FP64 fallback may take one more
    sv.set_max_iter(100_000)
    x2, its2, rr2, st2 = sv.solve(b)
    assert st2 == sd.OK and its2 == its0 and rr2 == rr0
    assert torch.equal(x0, x2)
    with pytest.raises(sd.SdslError):
        sv.set_max_iter(0)
    sv.close()


@pytest.mark.parametrize("name", ["C1", "C2x0.02", "C1-gmres", "C3x0.05-bbd"])
def test_footprint_prediction_covers_the_handle(name):
    """The admission control's prediction (sdsl_footprint_bytes) is at least
    what a handle really holds on the device after a solve, the Krylov
    workspace (the GMRES basis) and, for BBD, the Schur complement, its
    inverse and the tail factors included."""
    from paper_2604_23979_amd.serve import footprint
    if name == "C3x0.05-bbd":
        s = gen.c3(0.05)
        o = sd.Options(**BBD_OPTS)
    else:
        s = gen.c2(0.02) if name == "C2x0.02" else gen.c1()
        o = sd.Options(filter=sd.FILTER_GEOMEAN, tau=1e-3, diag_flags=sd.DIAG_DROPSUM)
        if name == "C1-gmres":
            o = sd.Options(krylov=sd.GMRES, spd=False)
    sv = sd.from_system(s, o)
    sv.solve(tdev(s.b))
    held = sv.info()["device_bytes"]
    pred = footprint(s, o)
    print(f"  {name}: predicted {pred / 1e6:.1f} MB, held {held / 1e6:.1f} MB")
    assert pred >= held
    sv.close()
