"""Pins of the CPU oracle against things other than itself: hand-worked
fixtures, dense linear algebra, closed forms, invariants and brute force on
tiny inputs.  A plausible slip anywhere in the oracle (a dropped term, a wrong
sign or index, a transposed operand, a wrong tie rule) fails one of these."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import oracle as O
from ipm_inputs import gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def csr_of(a):
    m = sp.csr_matrix(np.asarray(a, dtype=np.float64))
    m.sort_indices()
    return m


def with_diag(m):
    """CSR with an explicit diagonal entry in every row."""
    m = sp.csr_matrix(m)
    d = m.diagonal()
    m = m + sp.diags(np.where(d == 0, 1.0, 0.0))
    m = sp.csr_matrix(m)
    m.sort_indices()
    return m


def rand_sparse(n, density, rng, sym=False, dd=1.5):
    a = sp.random(n, n, density=density, random_state=rng, data_rvs=rng.standard_normal).toarray()
    if sym:
        a = np.triu(a, 1)
        a = a + a.T
    np.fill_diagonal(a, 0.0)
    np.fill_diagonal(a, dd * np.abs(a).sum(axis=1) + 1.0)
    return a


def unpack_lu(rp, ci, v, n):
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            j = ci[p]
            if j < i:
                L[i, j] = v[p]
            else:
                U[i, j] = v[p]
    return L, U


# --------------------------------------------------------------- SpMV / residual

def test_spmv_matches_scipy():
    rng = np.random.default_rng(1)
    a = csr_of(rand_sparse(300, 0.05, rng))
    x = rng.standard_normal(300)
    y = O.spmv(a.indptr, a.indices, a.data, x)
    ref = a @ x
    assert np.max(np.abs(y - ref) / (np.abs(a) @ np.abs(x))) < 4e-16 * 20


def test_lowrank_reading_equals_explicit_ada():
    """M_s + U diag(D_d) U^T equals the explicit A D A^T with the dense columns
    kept inside A (the dense-column reading of paper Sec. 2.1)."""
    s = gen.ada_system(200, 500, 3, -2.0, 2.0, 4, model="loc", dense_cols=2, dense_p=0.3, seed=3)
    r_pat, r_val, r_d, _, _, _ = gen.streams(3)
    col_ptr, rows = gen.a_pattern(r_pat, 200, 500, 3, "loc")
    vals = r_val.standard_normal(rows.shape[0])
    d_all = gen.log_uniform(r_d, 502, -2.0, 2.0)
    A = sp.csc_matrix((vals, rows, col_ptr), shape=(200, 500)).toarray()
    mask = r_pat.random((200, 2)) < 0.3
    ri, ci = np.nonzero(mask)
    Ud = np.zeros((200, 2))
    Ud[ri, ci] = r_val.standard_normal(ri.shape[0])
    Afull = np.hstack([A, Ud])
    Mexp = Afull @ np.diag(d_all) @ Afull.T + 1e-8 * np.eye(200)
    x = np.random.default_rng(0).standard_normal(200)
    y = O.spmv(s.row_ptr, s.col, s.val, x, lowrank=s.lowrank)
    assert np.allclose(y, Mexp @ x, rtol=1e-12, atol=1e-12 * np.abs(Mexp).max())


def test_compensated_residual_is_exact_to_rounding():
    """The Dot2 residual equals the exactly rounded rational residual to
    within a couple of ulps even under heavy cancellation."""
    rng = np.random.default_rng(2)
    n = 40
    a = rand_sparse(n, 0.2, rng)
    x = rng.standard_normal(n)
    b = a @ x  # residual is pure cancellation
    b = b + 1e-10 * rng.standard_normal(n)
    m = csr_of(a)
    r, _ = O.residual(m.indptr, m.indices, m.data, x, b)
    for i in range(n):
        exact = Fraction(b[i])
        for p in range(m.indptr[i], m.indptr[i + 1]):
            exact -= Fraction(m.data[p]) * Fraction(x[m.indices[p]])
        ex = float(exact)
        assert abs(r[i] - ex) <= 4 * np.finfo(float).eps * abs(ex) + 1e-300


def test_compensated_residual_low_rank_projection_is_exact_to_rounding():
    """With the low-rank term the projections U^T x are themselves compensated
    sums: when they cancel almost completely, the residual still equals the
    exact rational one up to the rounding of each projection and of c_j
    (a few ulps of |u_ip| c_j |t_j|) and of the final row sum."""
    rng = np.random.default_rng(3)
    n, k = 40, 3
    a = rand_sparse(n, 0.2, rng)
    x = rng.standard_normal(n)
    Ud = np.where(rng.random((n, k)) < 0.4, rng.standard_normal((n, k)), 0.0)
    Ud[-1] = 1.0
    for j in range(k):
        # last entry of each column makes sum_i u_ij x_i cancel to ~1e-10
        Ud[-1, j] = (1e-10 - Ud[:-1, j] @ x[:-1]) / x[-1]
    c = rng.uniform(0.5, 2.0, k)
    U = sp.csr_matrix(Ud)
    U.sort_indices()
    b = a @ x + 1e-10 * rng.standard_normal(n)
    m = csr_of(a)
    r, _ = O.residual(m.indptr, m.indices, m.data, x, b, lowrank=(U, c))
    t = []
    for j in range(k):
        tj = Fraction(0)
        for i in range(n):
            if Ud[i, j] != 0.0:
                tj += Fraction(Ud[i, j]) * Fraction(x[i])
        t.append(tj)
    assert max(abs(float(tj)) for tj in t) < 1e-8  # the projections do cancel
    eps = np.finfo(float).eps
    for i in range(n):
        exact = Fraction(b[i])
        for p in range(m.indptr[i], m.indptr[i + 1]):
            exact -= Fraction(m.data[p]) * Fraction(x[m.indices[p]])
        slack = 0.0
        for j in range(k):
            if Ud[i, j] != 0.0:
                exact -= Fraction(Ud[i, j]) * Fraction(c[j]) * t[j]
                slack += abs(Ud[i, j]) * c[j] * abs(float(t[j]))
        ex = float(exact)
        assert abs(r[i] - ex) <= 4 * eps * abs(ex) + 4 * eps * slack + 1e-300


# --------------------------------------------------------------- filter / correction

def _golden_filter(mode, kept_key, ds_key, diag_key):
    g = json.load(open(os.path.join(GOLD, "filter_4x4.json")))
    m = csr_of(g["matrix"])
    bp = np.array([0, 4], dtype=np.int32)
    rp, ci, v, ds = O.filter_correct(m.indptr, m.indices, m.data, bp, mode, g["tau"], 0, 0.0)
    kept = sorted((i, int(ci[p])) for i in range(4) for p in range(rp[i], rp[i + 1]))
    assert kept == sorted(tuple(t) for t in g[kept_key])
    assert np.allclose(ds, g[ds_key], rtol=1e-15, atol=0)
    rp2, ci2, v2, _ = O.filter_correct(m.indptr, m.indices, m.data, bp, mode, g["tau"], O.DIAG_DROPSUM, 0.0)
    dg = [v2[p] for i in range(4) for p in range(rp2[i], rp2[i + 1]) if ci2[p] == i]
    assert np.allclose(dg, g[diag_key], rtol=1e-15, atol=0)


def test_filter_min_hand_example():
    _golden_filter(O.FILTER_MIN, "kept_min", "dropsum_min", "diag_dropsum_min")


def test_filter_geomean_hand_example():
    _golden_filter(O.FILTER_GEOMEAN, "kept_geomean", "dropsum_geomean", "diag_dropsum_geomean")


def test_filter_tie_keeps_entry():
    """Strict '<' in Eq. (filter): |a_ij| == tau |a_ii| keeps the entry."""
    a = np.array([[4.0, 1.0], [1.0, 4.0]])  # tau = 0.25: 1 == 0.25 * 4
    m = csr_of(a)
    for mode in (O.FILTER_MIN, O.FILTER_GEOMEAN):
        rp, ci, v, ds = O.filter_correct(m.indptr, m.indices, m.data, np.array([0, 2]), mode, 0.25)
        assert rp[-1] == 4 and np.all(ds == 0)


def test_filter_extremes_and_blocks():
    rng = np.random.default_rng(4)
    a = csr_of(rand_sparse(120, 0.1, rng, sym=True))
    bp = gen.contiguous_blocks(120, 5)
    for mode in (O.FILTER_MIN, O.FILTER_GEOMEAN):
        # tau = 0: nothing dropped, the pattern is exactly the in-block pattern
        rp, ci, v, ds = O.filter_correct(a.indptr, a.indices, a.data, bp, mode, 0.0)
        dense = a.toarray()
        blk = np.searchsorted(bp, np.arange(120), side="right") - 1
        inblock = (blk[:, None] == blk[None, :]) & (dense != 0)
        assert rp[-1] == inblock.sum() and np.all(ds == 0)
        # tau = inf: only the diagonal remains; DROPSUM gives l1-Jacobi on the block
        rp, ci, v, ds = O.filter_correct(a.indptr, a.indices, a.data, bp, mode, np.inf, O.DIAG_DROPSUM)
        assert rp[-1] == 120 and np.all(ci == np.arange(120))
        l1 = np.abs(np.where(inblock, dense, 0.0)).sum(axis=1)
        assert np.allclose(v, l1, rtol=1e-14)
    # monotone in tau
    prev = None
    for tau in (1e-3, 1e-2, 1e-1, 0.5):
        rp, ci, _, _ = O.filter_correct(a.indptr, a.indices, a.data, bp, O.FILTER_MIN, tau)
        cur = {(i, int(ci[p])) for i in range(120) for p in range(rp[i], rp[i + 1])}
        if prev is not None:
            assert cur <= prev
        prev = cur


def test_geomean_is_min_rule_on_unit_diagonal_scaling():
    """GEOMEAN on M equals Eq. (filter) on D^-1/2 M D^-1/2 (unit diagonal)."""
    rng = np.random.default_rng(5)
    a = rand_sparse(150, 0.08, rng, sym=True)
    a = a * np.exp(rng.uniform(-6, 6, 150))[:, None]
    a = (a + a.T) / 2
    np.fill_diagonal(a, np.abs(a).sum(axis=1))
    d = np.sqrt(np.diag(a))
    s = a / d[:, None] / d[None, :]
    bp = np.array([0, 75, 150], dtype=np.int32)
    m1, m2 = csr_of(a), csr_of(s)
    for tau in (1e-3, 3e-2, 0.2):
        rp1, ci1, _, _ = O.filter_correct(m1.indptr, m1.indices, m1.data, bp, O.FILTER_GEOMEAN, tau)
        rp2, ci2, _, _ = O.filter_correct(m2.indptr, m2.indices, m2.data, bp, O.FILTER_MIN, tau)
        assert np.array_equal(rp1, rp2) and np.array_equal(ci1, ci2)


def test_dropsum_correction_dominates_block():
    """With DROPSUM the corrected matrix minus the in-block part of M is
    diag(dropsum) - E: symmetric, weakly diagonally dominant with a
    non-negative diagonal, hence positive semidefinite."""
    s = gen.c2(0.004, dense_cols=0)
    rp, ci, v, ds = O.filter_correct(s.row_ptr, s.col, s.val, s.block_ptr, O.FILTER_GEOMEAN, 1e-2,
                                     O.DIAG_DROPSUM)
    n = s.n
    Phat = sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()
    M = s.scipy().toarray()
    blk = np.searchsorted(s.block_ptr, np.arange(n), side="right") - 1
    Mb = np.where(blk[:, None] == blk[None, :], M, 0.0)
    diff = Phat - Mb
    assert np.allclose(diff, diff.T, rtol=0, atol=1e-12 * np.abs(M).max())
    lam = np.linalg.eigvalsh((diff + diff.T) / 2)
    assert lam.min() >= -1e-12 * np.abs(M).max()


def test_delta_correction_sign_rule():
    a = np.array([[-3.0, 0.1], [0.1, 0.0 + 2.0]])
    a[1, 1] = 0.0
    m = sp.csr_matrix(a)
    m = sp.csr_matrix((np.array([-3.0, 0.1, 0.1, 0.0]), np.array([0, 1, 0, 1]), np.array([0, 2, 4])))
    rp, ci, v, _ = O.filter_correct(m.indptr, m.indices, m.data, np.array([0, 2]), O.FILTER_NONE, 0.0,
                                    O.DIAG_DELTA, 1e-12)
    dg = {i: v[p] for i in range(2) for p in range(rp[i], rp[i + 1]) if ci[p] == i}
    assert dg[0] == -3.0 - 1e-12  # sign(-3) = -1
    assert dg[1] == 1e-12         # sign(0) = +1 (reading)


def test_delta_and_dropsum_corrections_add():
    """Both flags: the diagonal moves away from zero by delta plus the row's
    dropped magnitude (Eq. (diagcorr) with the drop-sum variant)."""
    a = np.array([[4.0, 0.01, 1.0], [0.01, -5.0, 0.0], [1.0, 0.0, 3.0]])
    m = csr_of(a)
    rp, ci, v, ds = O.filter_correct(m.indptr, m.indices, m.data, np.array([0, 3]), O.FILTER_MIN, 0.1,
                                     O.DIAG_DELTA | O.DIAG_DROPSUM, 0.5)
    dg = {i: v[p] for i in range(3) for p in range(rp[i], rp[i + 1]) if ci[p] == i}
    assert list(ds) == [0.01, 0.01, 0.0]
    assert dg[0] == pytest.approx(4.51, rel=1e-15)
    assert dg[1] == pytest.approx(-5.51, rel=1e-15)
    assert dg[2] == pytest.approx(3.5, rel=1e-15)


# --------------------------------------------------------------- ILU(0)

def test_ilu0_hand_example_tridiagonal():
    g = json.load(open(os.path.join(GOLD, "ilu0_tridiag_3x3.json")))
    m = csr_of(g["matrix"])
    v, dp, st, _, _ = O.ilu0(m.indptr, m.indices, m.data)
    assert st == O.OK
    L, U = unpack_lu(m.indptr, m.indices, v, 3)
    assert np.allclose(L, g["L"], rtol=1e-15) and np.allclose(U, g["U"], rtol=1e-15)


def test_ilu0_pattern_identity():
    """(LU)_ij = p_ij on every pattern position (the defining property of
    ILU(0)), up to rounding."""
    rng = np.random.default_rng(6)
    for sym in (False, True):
        a = rand_sparse(200, 0.04, rng, sym=sym, dd=0.6)
        m = csr_of(a)
        v, dp, st, _, _ = O.ilu0(m.indptr, m.indices, m.data)
        assert st == O.OK
        L, U = unpack_lu(m.indptr, m.indices, v, 200)
        LU = L @ U
        mask = a != 0
        err = np.abs(LU - a)[mask] / (np.abs(L) @ np.abs(U))[mask]
        assert err.max() < 1e-13
        if sym:
            # symmetric input: u_ij = u_ii l_ji
            for i in range(200):
                for j in range(i + 1, 200):
                    if mask[i, j]:
                        assert abs(U[i, j] - U[i, i] * L[j, i]) <= 1e-12 * abs(U[i, j]) + 1e-300


def test_ilu0_tridiagonal_and_dense_equal_exact_lu():
    rng = np.random.default_rng(7)
    for kind in ("tri", "dense"):
        n = 60
        if kind == "tri":
            a = np.diag(rng.uniform(4, 5, n)) + np.diag(rng.standard_normal(n - 1), 1) + np.diag(rng.standard_normal(n - 1), -1)
        else:
            a = rng.standard_normal((n, n))
            np.fill_diagonal(a, np.abs(a).sum(axis=1) + 1)
        m = csr_of(a)
        v, dp, st, _, _ = O.ilu0(m.indptr, m.indices, m.data)
        L, U = unpack_lu(m.indptr, m.indices, v, n)
        P, Ls, Us = sl.lu(a)  # diagonally dominant -> no row exchanges
        assert np.array_equal(P, np.eye(n))
        assert np.allclose(L, Ls, rtol=1e-12, atol=1e-14) and np.allclose(U, Us, rtol=1e-12, atol=1e-12)


def test_ilu0_breakdown_policies():
    """An SPD matrix whose ILU(0) meets a non-positive pivot: FAIL reports
    it, SHIFT refactors the block with a strengthened diagonal (d + a d) and
    the result is the ILU(0) of that shifted block."""
    # SPD (lambda_min ~ 0.146) with a zero (1,4) entry: the fill that
    # eliminating row 0 would put there is dropped, and the last pivot of
    # ILU(0) goes negative (exact LU pivots stay positive).
    a = np.array([[1.0, -0.6, 0.1, 0.2, -0.6],
                  [-0.6, 1.0, 0.0, 0.4, 0.0],
                  [0.1, 0.0, 1.0, -0.1, 0.0],
                  [0.2, 0.4, -0.1, 1.0, -0.7],
                  [-0.6, 0.0, 0.0, -0.7, 1.0]])
    assert np.linalg.eigvalsh(a).min() > 0.1
    assert np.all(np.diag(sl.lu(a)[2]) > 0)
    s = gen.System("t", *(lambda m: (m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data))(csr_of(a)),
                   b=np.ones(5), block_ptr=np.array([0, 5], dtype=np.int32))
    fail = O.BJ(s, policy=O.PIVOT_FAIL)
    assert fail.status == O.BREAKDOWN
    # REPLACE: the failed (last) pivot becomes the corrected diagonal, counted
    rep = O.BJ(s, policy=O.PIVOT_REPLACE)
    assert rep.status == O.OK and rep.nfix == 1 and rep.v[rep.dp[4]] == a[4, 4]
    # SHIFT on a non-unit diagonal (symmetric scaling keeps SPD and the
    # breakdown): the shift is relative, d + a d, and the doubling from a
    # small shift0 stops at the first a that works
    sc = np.array([2.0, 0.5, 3.0, 1.5, 0.25])
    a = sc[:, None] * a * sc[None, :]
    s = gen.System("t", *(lambda m: (m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data))(csr_of(a)),
                   b=np.ones(5), block_ptr=np.array([0, 5], dtype=np.int32))
    shift0 = 1e-4
    sh = O.BJ(s, policy=O.PIVOT_SHIFT, shift0=shift0)
    assert sh.status == O.OK and sh.shifts[0] > shift0
    j = np.log2(sh.shifts[0] / shift0)
    assert j == np.round(j)  # shift0 * 2^j
    a2 = a + np.diag(sh.shifts[0] * np.diag(a))
    m2 = csr_of(a2)
    v, dp, st, _, _ = O.ilu0(m2.indptr, m2.indices, m2.data, spd=True)
    assert st == O.OK and np.allclose(v, sh.v, rtol=1e-14)
    # the smaller shift a/2 still breaks down (first success of the doubling)
    a3 = a + np.diag(sh.shifts[0] / 2 * np.diag(a))
    m3 = csr_of(a3)
    assert O.ilu0(m3.indptr, m3.indices, m3.data, spd=True)[2] == O.BREAKDOWN


def test_ilu0_zero_pivot_is_a_breakdown_in_spd_mode():
    """A positive semidefinite block whose elimination gives an exactly zero
    pivot: SPD mode needs a positive pivot, so FAIL reports a breakdown."""
    a = np.array([[1.0, 1.0], [1.0, 1.0]])
    m = csr_of(a)
    v, dp, st, nfix, bad = O.ilu0(m.indptr, m.indices, m.data, spd=True)
    assert st == O.BREAKDOWN and bad == 1


# --------------------------------------------------------------- BJ apply

def test_bj_apply_equals_dense_block_solve():
    s = gen.c2(0.004, dense_cols=0)
    P = O.BJ(s, O.FILTER_GEOMEAN, 1e-2, O.DIAG_DROPSUM)
    assert P.status == O.OK
    n = s.n
    L, U = unpack_lu(P.rp, P.ci, P.v, n)
    r = np.random.default_rng(8).standard_normal(n)
    z = P.apply(r)
    zz = sl.solve_triangular(U, sl.solve_triangular(L, r, lower=True, unit_diagonal=True))
    assert np.allclose(z, zz, rtol=1e-9, atol=1e-12 * np.abs(zz).max())
    # block structure: L U is block diagonal
    blk = np.searchsorted(s.block_ptr, np.arange(n), side="right") - 1
    LU = L @ U
    assert np.all(LU[blk[:, None] != blk[None, :]] == 0)


def test_bj_with_one_row_blocks_is_jacobi():
    rng = np.random.default_rng(9)
    a = csr_of(rand_sparse(50, 0.1, rng, sym=True))
    s = gen.System("j", a.indptr.astype(np.int64), a.indices.astype(np.int32), a.data, np.ones(50),
                   np.arange(51, dtype=np.int32))
    P = O.BJ(s)
    r = rng.standard_normal(50)
    assert np.allclose(P.apply(r), r / a.diagonal(), rtol=1e-15)


# --------------------------------------------------------------- PCG

def _small_spd(n, seed):
    rng = np.random.default_rng(seed)
    a = rand_sparse(n, 0.15, rng, sym=True, dd=0.3)
    a = a + a.T
    w = np.linalg.eigvalsh(a)
    a = a + (1e-2 - min(w.min(), 0)) * np.eye(n) * (w.min() < 1e-2)
    m = csr_of(a)
    b = rng.standard_normal(n)
    return gen.System("spd", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, b,
                      gen.contiguous_blocks(n, 3)), a


def test_pcg_iterates_are_krylov_minimisers_and_monotone():
    """x_k minimises the M-norm error over K_k(P^-1 M, P^-1 b) (x0 = 0), and
    that error never increases (paper Sec. 2.2, CG)."""
    s, a = _small_spd(40, 10)
    P = O.BJ(s, policy=O.PIVOT_FAIL, spd=True)
    assert P.status == O.OK
    n = s.n
    L, U = unpack_lu(P.rp, P.ci, P.v, n)
    Pm = L @ U
    Pinv = np.linalg.inv(Pm)
    xs = np.linalg.solve(a, s.b)
    errs = []
    for k in range(1, 9):
        x, its, rr, st, _ = O.pcg_bj(s, P, tol=1e-30, maxit=k)
        assert its == k
        K = [Pinv @ s.b]
        for _ in range(k - 1):
            K.append(Pinv @ (a @ K[-1]))
        Q, _ = np.linalg.qr(np.array(K).T)
        y = np.linalg.solve(Q.T @ a @ Q, Q.T @ s.b)
        xb = Q @ y
        assert np.linalg.norm(x - xb) <= 1e-7 * np.linalg.norm(xb)
        e = x - xs
        errs.append(np.sqrt(e @ a @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_pcg_exact_preconditioner_converges_in_one_step():
    """Tridiagonal SPD matrix in one block: ILU(0) is the exact LU, so PCG
    converges in one iteration."""
    n = 300
    rng = np.random.default_rng(11)
    off = rng.standard_normal(n - 1)
    a = np.diag(np.abs(np.r_[off, 0]) + np.abs(np.r_[0, off]) + 0.5) + np.diag(off, 1) + np.diag(off, -1)
    m = csr_of(a)
    s = gen.System("tri", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                   rng.standard_normal(n), np.array([0, n], dtype=np.int32))
    P = O.BJ(s)
    x, its, rr, st, _ = O.pcg_bj(s, P, tol=1e-12)
    assert st == O.OK and its == 1 and rr <= 1e-12


def test_pcg_c1_true_residual():
    s = gen.c1()
    P = O.BJ(s)
    x, its, rr, st, _ = O.pcg_bj(s, P)
    assert st == O.OK and rr <= 1e-8
    # true residual recomputed independently with scipy
    M = s.scipy()
    assert np.linalg.norm(s.b - M @ x) / np.linalg.norm(s.b) <= 1.5e-8
    # against a direct solve: ||x - x*||_M / ||x*||_M is bounded by kappa * relres
    xs = sp.linalg.spsolve(M.tocsc(), s.b)
    e = x - xs
    assert np.sqrt(e @ (M @ e)) / np.sqrt(xs @ (M @ xs)) < 1e-4


def test_pcg_stops_on_the_true_residual_only():
    """An IPM system on which this PCG's true residual stalls near 5e-10
    while its recurrence residual falls below the requested 1e-10: PCG only
    stops when the true residual meets the tolerance, so the solve ends not
    converged and reports the true residual."""
    q = gen.IPMSequence(m=3000, nblocks=4, steps=30)
    s = q.system(5)
    P = O.BJ(s, mode=O.FILTER_GEOMEAN, tau=1e-3, flags=O.DIAG_DROPSUM)
    x, its, rr, st, h = O.pcg_bj(s, P, tol=1e-10, maxit=1000, hist=True)
    assert np.any(h <= 1e-10)  # the recurrence met the tolerance
    assert st == O.NOT_CONVERGED and its == 1000
    # the true residual at this level needs more than FP64 (a plain FP64
    # product is ~10% off here): x86 extended precision, 64-bit mantissa
    M = s.scipy()
    ld = np.longdouble
    prod = M.data.astype(ld) * x[M.indices].astype(ld)
    res = s.b.astype(ld) - np.add.reduceat(prod, M.indptr[:-1])
    true = float(np.sqrt(np.sum(res * res)) / np.sqrt(np.sum(s.b.astype(ld) ** 2)))
    assert rr > 1e-10 and rr == pytest.approx(true, rel=1e-3)


# --------------------------------------------------------------- GMRES

def test_gmres_iterates_minimise_residual():
    rng = np.random.default_rng(12)
    n = 50
    a = rand_sparse(n, 0.15, rng, dd=0.4)
    m = csr_of(a)
    s = gen.System("ns", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                   rng.standard_normal(n), gen.contiguous_blocks(n, 4))
    P = O.BJ(s, spd=False, policy=O.PIVOT_FAIL)
    L, U = unpack_lu(P.rp, P.ci, P.v, n)
    Pinv = np.linalg.inv(L @ U)
    prev = np.inf
    for k in range(1, 10):
        x, its, rr, st, hist = O.gmres_bj(s, P, tol=1e-30, m=30, maxit=k, hist=True)
        # brute force: min ||b - M P^-1 y|| over y in K_k(M P^-1, b)
        K = [s.b]
        for _ in range(k - 1):
            K.append(a @ (Pinv @ K[-1]))
        Q, _ = np.linalg.qr(np.array(K).T)
        B = a @ Pinv @ Q
        c, *_ = np.linalg.lstsq(B, s.b, rcond=None)
        xb = Pinv @ (Q @ c)
        assert np.linalg.norm(x - xb) <= 1e-8 * max(1.0, np.linalg.norm(xb))
        assert rr <= prev * (1 + 1e-12)
        prev = rr


def test_gmres_full_dimension_converges():
    rng = np.random.default_rng(13)
    n = 25
    a = rng.standard_normal((n, n)) + 3 * np.eye(n)
    m = csr_of(a)
    s = gen.System("g", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                   rng.standard_normal(n), np.arange(n + 1, dtype=np.int32))
    P = O.BJ(s, spd=False, policy=O.PIVOT_FAIL)
    x, its, rr, st, _ = O.gmres_bj(s, P, tol=1e-10, m=30)
    assert st == O.OK and its <= n


def test_gmres_cycles_keep_the_arnoldi_residual_true():
    """Restarted GMRES on badly row-scaled systems it cannot solve in 600
    steps: in exact arithmetic the least-squares residual |g_{j+1}| at the end
    of a cycle is the true residual of the updated iterate, and no cycle
    raises the residual above that of the previous one.  Both survive
    rounding only while the Krylov basis stays orthogonal to working
    accuracy, which classical Gram-Schmidt applied twice provides and a
    single pass does not (there the two differ by factors of 2-10)."""
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        n = 400
        a = rand_sparse(n, 0.02, rng, dd=0.05)
        a = np.diag(10.0 ** rng.uniform(-5, 5, n)) @ a
        m = csr_of(a)
        s = gen.System("ns", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                       rng.standard_normal(n), gen.contiguous_blocks(n, 40))
        P = O.BJ(s, spd=False, policy=O.PIVOT_FAIL)
        prev = 1.0
        for cycles in (2, 5, 10):
            x, its, rr, st, h = O.gmres_bj(s, P, tol=1e-13, m=60, maxit=60 * cycles, hist=True)
            assert its == 60 * cycles
            true = np.linalg.norm(s.b - a @ x) / np.linalg.norm(s.b)
            assert rr == pytest.approx(true, rel=1e-8)
            assert abs(h[-1] / rr - 1.0) <= 1e-2, (seed, cycles, h[-1], rr)
            assert rr <= prev * (1 + 1e-6)
            prev = rr


# --------------------------------------------------------------- BBD

def _bbd_dense_parts(s, P):
    n, nb = s.n, s.n_border
    ni = n - nb
    M = s.scipy().toarray()
    parts = P.parts()
    L, U = unpack_lu(parts["lrp"], parts["lci"], parts["lv"], ni)
    E, F, Cc = M[:ni, ni:], M[ni:, :ni], M[ni:, ni:]
    return M, L, U, E, F, Cc, parts


def _with_early_border_rows(s):
    """Border rows that reach interior columns left of every row with a
    border-column entry: the tail must start at those columns."""
    M = s.scipy().tolil()
    ni = s.n - s.n_border
    M[ni, int(s.block_ptr[0]) + 1] = 0.3
    M[ni + 5, int(s.block_ptr[2]) + 7] = -0.4
    M = M.tocsr()
    M.sort_indices()
    return gen.System("bbd-early", M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data, s.b,
                      s.block_ptr, n_border=s.n_border)


@pytest.mark.parametrize("early", [False, True], ids=["generated", "early-border-rows"])
def test_bbd_schur_and_apply_match_dense(early):
    s = gen.bbd_system(nblocks=3, block_rows=60, n_border=12, nnz_off=4, half_band=10, tail_frac=0.2,
                       border_c=2, seed=14, name="bbd-tiny")
    if early:
        s = _with_early_border_rows(s)
    P = O.BBD(s)
    assert P.status == O.OK
    M, L, U, E, F, Cc, parts = _bbd_dense_parts(s, P)
    S = Cc - F @ np.linalg.solve(L @ U, E)
    # oracle LU of S with its pivots reproduces S
    lu, piv = parts["S"], parts["piv"]
    nb = s.n_border
    Ls = np.tril(lu, -1) + np.eye(nb)
    Us = np.triu(lu)
    Sp = S.copy()
    for k in range(nb):
        Sp[[k, piv[k]]] = Sp[[piv[k], k]]
    assert np.linalg.norm(Sp - Ls @ Us) <= 1e-12 * np.linalg.norm(S) * nb
    # pivots are LAPACK's (first maximum)
    lu_ref, piv_ref = sl.lu_factor(S)
    assert np.array_equal(piv, piv_ref)
    # apply = solve with the assembled M_BBD
    Mbbd = np.block([[L @ U, E], [F, Cc]])
    r = np.random.default_rng(15).standard_normal(s.n)
    z = P.apply(r)
    zz = np.linalg.solve(Mbbd, r)
    assert np.allclose(z, zz, rtol=1e-9, atol=1e-11 * np.abs(zz).max())
    # tail = first local index coupled to the border
    ni = s.n - nb
    for b in range(3):
        lo, hi = s.block_ptr[b], s.block_ptr[b + 1]
        rows_e = np.nonzero(np.any(E[lo:hi] != 0, axis=1))[0]
        cols_f = np.nonzero(np.any(F[:, lo:hi] != 0, axis=0))[0]
        assert parts["tail"][b] == lo + min(rows_e.min(), cols_f.min())
    if early:
        assert parts["tail"][0] == s.block_ptr[0] + 1 and parts["tail"][2] == s.block_ptr[2] + 7


def test_bbd_exact_blocks_gmres_one_step():
    """Tridiagonal interior blocks: ILU(0) is exact, M_BBD = M, and
    right-preconditioned GMRES converges in one step."""
    s = gen.bbd_system(nblocks=4, block_rows=80, n_border=16, nnz_off=1, half_band=1, tail_frac=0.1,
                       border_c=2, seed=16, name="bbd-tri")
    P = O.BBD(s)
    assert P.status == O.OK
    x, its, rr, st, _ = O.gmres_bbd(s, P, tol=1e-10)
    assert st == O.OK and its == 1 and rr <= 1e-10


def test_bbd_with_complete_blocks_is_exact():
    """With complete LU blocks and no filter the BBD preconditioner is M
    itself for any blocks (the Schur complement is exact for M_BBD), so
    right-preconditioned GMRES and GCR converge in one step, and the apply
    inverts M."""
    s = gen.bbd_system(nblocks=3, block_rows=60, n_border=12, nnz_off=4, half_band=10, tail_frac=0.2,
                       border_c=2, seed=14, name="bbd-tiny")
    P = O.BBD(s, complete=True)
    assert P.status == O.OK
    r = np.random.default_rng(19).standard_normal(s.n)
    np.testing.assert_allclose(s.scipy() @ P.apply(r), r, atol=1e-10 * np.abs(r).max())
    for fn in (O.gmres_bbd, O.gcr_bbd):
        x, its, rr, st, _ = fn(s, P, tol=1e-10)
        assert st == O.OK and its == 1 and rr <= 1e-10


@pytest.mark.parametrize("row,col", [(0, 45), (29, 30), (30, 29)],
                         ids=["inside", "next-block-first-column", "previous-block-last-column"])
def test_bbd_rejects_block_coupling(row, col):
    s = gen.bbd_system(nblocks=2, block_rows=30, n_border=6, nnz_off=2, half_band=4, tail_frac=0.2,
                       border_c=1, seed=17)
    M = s.scipy().tolil()
    M[row, col] = 1.0  # an interior row of one block -> an interior column of another
    M = M.tocsr()
    M.sort_indices()
    s2 = gen.System("bad", M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data, s.b,
                    s.block_ptr, n_border=s.n_border)
    assert O.BBD(s2).status == O.STRUCTURE


def test_dense_lu_matches_lapack():
    rng = np.random.default_rng(18)
    a = rng.standard_normal((70, 70))
    lu, piv, st = O.dense_lu(a)
    lu_ref, piv_ref = sl.lu_factor(a)
    assert st == O.OK and np.array_equal(piv, piv_ref)
    assert np.allclose(lu, lu_ref, rtol=1e-12, atol=1e-13)
    b = rng.standard_normal(70)
    assert np.allclose(O.dense_lu_solve(lu, piv, b), np.linalg.solve(a, b), rtol=1e-10)
    # ties in the first column: the first row of largest magnitude is taken
    a[:, 0] = rng.choice([-3.0, -2.0, 1.0, 2.0, 3.0], 70)
    lu, piv, st = O.dense_lu(a)
    lu_ref, piv_ref = sl.lu_factor(a)
    assert st == O.OK and piv[0] == np.flatnonzero(np.abs(a[:, 0]) == 3.0)[0]
    assert np.array_equal(piv, piv_ref)


# --------------------------------------------------------------- BiCGSTAB

def _small_nonsym(n, seed, blocks=3):
    rng = np.random.default_rng(seed)
    a = rand_sparse(n, 0.2, rng, sym=False, dd=0.6)
    m = csr_of(a)
    b = rng.standard_normal(n)
    return gen.System("ns", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, b,
                      gen.contiguous_blocks(n, blocks)), a


def test_bicgstab_first_step_is_petrov_galerkin_then_minimal_residual():
    """One BiCGSTAB step (paper Sec. 4.3's solver for block Jacobi), right
    preconditioned (Sec. 2.2) with x0 = 0 and shadow r^ = b: x1 lies in
    span{u1, u2}, u1 = P^-1 b, u2 = P^-1 M u1, as x1 = (a + w) u1 - a w u2,
    where a makes the half-step residual b - a M u1 orthogonal to b
    (Petrov-Galerkin) and w minimises ||s - w M P^-1 s|| over w (the
    stabilising step); both are checked from x1 alone."""
    s, a = _small_nonsym(30, 50)
    P = O.BJ(s, policy=O.PIVOT_FAIL, spd=False)
    assert P.status == O.OK
    L, U = unpack_lu(P.rp, P.ci, P.v, s.n)
    pinv = np.linalg.inv(L @ U)
    b = s.b
    u1 = pinv @ b
    u2 = pinv @ (a @ u1)
    x1, its, rr, st, _ = O.bicgstab_bj(s, P, tol=1e-30, maxit=1)
    assert its == 1 and st == O.NOT_CONVERGED
    coef, res, *_ = np.linalg.lstsq(np.c_[u1, u2], x1, rcond=None)
    assert np.linalg.norm(np.c_[u1, u2] @ coef - x1) <= 1e-12 * np.linalg.norm(x1)
    # coef = (alpha + omega, -alpha omega): alpha is the Petrov-Galerkin step
    alpha = (b @ b) / (b @ (a @ u1))
    omega = coef[0] - alpha
    assert abs(-alpha * omega - coef[1]) <= 1e-10 * abs(coef[1])
    sres = b - alpha * (a @ u1)
    assert abs(b @ sres) <= 1e-12 * np.linalg.norm(b) * np.linalg.norm(sres)
    t = a @ (pinv @ sres)
    assert abs(omega - (t @ sres) / (t @ t)) <= 1e-12 * abs(omega)


def test_bicgstab_iterates_stay_in_the_right_krylov_space():
    """Each step adds two dimensions: x_k lies in P^-1 K_2k(M P^-1, b) and
    not in P^-1 K_(2k-1) (a step with one product, or a left-preconditioned
    form, fails one of the two)."""
    s, a = _small_nonsym(40, 51)
    P = O.BJ(s, policy=O.PIVOT_FAIL, spd=False)
    L, U = unpack_lu(P.rp, P.ci, P.v, s.n)
    pinv = np.linalg.inv(L @ U)
    K = [s.b]
    for _ in range(8):
        K.append(a @ (pinv @ K[-1]))
    for k in (1, 2, 3):
        x, its, rr, st, _ = O.bicgstab_bj(s, P, tol=1e-30, maxit=k)
        for dim, inside in ((2 * k, True), (2 * k - 1, False)):
            B = pinv @ np.array(K[:dim]).T
            Q, _ = np.linalg.qr(B)
            off = np.linalg.norm(x - Q @ (Q.T @ x)) / np.linalg.norm(x)
            assert (off <= 1e-9) if inside else (off >= 1e-6), (k, dim, off)


def test_bicgstab_exact_preconditioner_terminates_and_small_systems_converge():
    """A single tridiagonal block (ILU(0) exact) converges in one step; a
    12-unknown nonsymmetric system converges within 12 steps (the BiCG
    polynomial inside the residual annihilates r0 by step n in exact
    arithmetic); an indefinite case with (r^, M P^-1 r0) = 0 is a
    breakdown."""
    n = 200
    rng = np.random.default_rng(52)
    lo, up = rng.standard_normal(n - 1), rng.standard_normal(n - 1)
    a = np.diag(np.abs(np.r_[lo, 0]) + np.abs(np.r_[0, up]) + 1.0) + np.diag(lo, -1) + np.diag(up, 1)
    m = csr_of(a)
    t = gen.System("tri", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, rng.standard_normal(n),
                   np.array([0, n], dtype=np.int32))
    x, its, rr, st, _ = O.bicgstab_bj(t, O.BJ(t, spd=False), tol=1e-12, maxit=10)
    assert st == O.OK and its == 1 and rr <= 1e-12
    s, a = _small_nonsym(12, 53, blocks=2)
    x, its, rr, st, _ = O.bicgstab_bj(s, O.BJ(s, spd=False), tol=1e-10, maxit=50)
    assert st == O.OK and its <= 12 and np.linalg.norm(s.b - a @ x) <= 1e-9 * np.linalg.norm(s.b)
    m = csr_of([[1.0, 3.0], [-1.0, 1.0]])
    bd = gen.System("bd", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, np.array([1.0, -1.0]),
                    np.array([0, 1, 2], dtype=np.int32))
    x, its, rr, st, _ = O.bicgstab_bj(bd, O.BJ(bd, spd=False), tol=1e-12, maxit=10)
    assert st == O.BREAKDOWN


def test_bicgstab_solves_c1_and_stops_on_the_true_residual():
    s = gen.c1()
    P = O.BJ(s)
    x, its, rr, st, h = O.bicgstab_bj(s, P, tol=1e-8, maxit=20_000, hist=True)
    assert st == O.OK and rr <= 1e-8
    assert np.linalg.norm(s.b - s.scipy() @ x) / np.linalg.norm(s.b) <= 1.5e-8


# --------------------------------------------------------------- GCR(m)

def test_gcr_iterates_minimise_residual_brute_force():
    """GCR (the paper's single-node and BBD solver, Sec. 4.2-4.3), right
    preconditioned (Sec. 2.2): after k steps from x0 = 0 the iterate is
    the minimiser of ||b - M P^-1 y|| over y in K_k(M P^-1, b), checked
    against a dense least-squares solve; the residual never grows."""
    rng = np.random.default_rng(60)
    n = 50
    a = rand_sparse(n, 0.15, rng, dd=0.4)
    m = csr_of(a)
    s = gen.System("ns", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                   rng.standard_normal(n), gen.contiguous_blocks(n, 4))
    P = O.BJ(s, spd=False, policy=O.PIVOT_FAIL)
    L, U = unpack_lu(P.rp, P.ci, P.v, n)
    Pinv = np.linalg.inv(L @ U)
    prev = np.inf
    for k in range(1, 10):
        x, its, rr, st, hist = O.gcr_bj(s, P, tol=1e-30, m=30, maxit=k, hist=True)
        assert its == k
        K = [s.b]
        for _ in range(k - 1):
            K.append(a @ (Pinv @ K[-1]))
        Q, _ = np.linalg.qr(np.array(K).T)
        c, *_ = np.linalg.lstsq(a @ Pinv @ Q, s.b, rcond=None)
        xb = Pinv @ (Q @ c)
        assert np.linalg.norm(x - xb) <= 1e-8 * max(1.0, np.linalg.norm(xb)), k
        assert rr <= prev * (1 + 1e-12)
        # the recurrence residual is the true one
        assert hist[-1] == pytest.approx(np.linalg.norm(s.b - a @ x) / np.linalg.norm(s.b), rel=1e-8)
        prev = rr


@pytest.mark.parametrize("m", [40, 7])
def test_gcr_follows_gmres_step_by_step(m):
    """GCR(m) and GMRES(m) minimise the same residual over the same space in
    every cycle, so from the same start their residual histories agree step
    by step, with restarts too (two independent recurrences: Arnoldi with
    Givens rotations against orthogonalised directions)."""
    rng = np.random.default_rng(61)
    n = 300
    a = rand_sparse(n, 0.03, rng, dd=0.3)
    mm = csr_of(a)
    s = gen.System("ns", mm.indptr.astype(np.int64), mm.indices.astype(np.int32), mm.data,
                   rng.standard_normal(n), gen.contiguous_blocks(n, 10))
    P = O.BJ(s, spd=False, policy=O.PIVOT_FAIL)
    _, its_g, rr_g, st_g, h_g = O.gmres_bj(s, P, tol=1e-10, m=m, maxit=2000, hist=True)
    _, its_c, rr_c, st_c, h_c = O.gcr_bj(s, P, tol=1e-10, m=m, maxit=2000, hist=True)
    assert st_g == O.OK and st_c == O.OK
    assert abs(its_c - its_g) <= 1
    k = min(its_c, its_g) - 1
    assert its_g > m or m == 40
    np.testing.assert_allclose(h_c[:k], h_g[:k], rtol=1e-6)


def test_gcr_small_cases_and_breakdown():
    """A single tridiagonal block (ILU(0) exact) converges in one step; a
    dense 25-unknown system within 25 steps; a residual orthogonal to
    M P^-1 r gives alpha = 0, the next direction repeats the last one, and
    the empty projection is a breakdown."""
    n = 200
    rng = np.random.default_rng(62)
    lo, up = rng.standard_normal(n - 1), rng.standard_normal(n - 1)
    a = np.diag(np.abs(np.r_[lo, 0]) + np.abs(np.r_[0, up]) + 1.0) + np.diag(lo, -1) + np.diag(up, 1)
    m = csr_of(a)
    t = gen.System("tri", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, rng.standard_normal(n),
                   np.array([0, n], dtype=np.int32))
    x, its, rr, st, _ = O.gcr_bj(t, O.BJ(t, spd=False), tol=1e-12)
    assert st == O.OK and its == 1 and rr <= 1e-12
    n = 25
    a = rng.standard_normal((n, n)) + 3 * np.eye(n)
    m = csr_of(a)
    g = gen.System("g", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                   rng.standard_normal(n), np.arange(n + 1, dtype=np.int32))
    x, its, rr, st, _ = O.gcr_bj(g, O.BJ(g, spd=False, policy=O.PIVOT_FAIL), tol=1e-10, m=30)
    assert st == O.OK and its <= n and np.linalg.norm(g.b - a @ x) <= 1e-9 * np.linalg.norm(g.b)
    m = csr_of([[1.0, 3.0], [-1.0, 1.0]])
    bd = gen.System("bd", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, np.array([1.0, -1.0]),
                    np.array([0, 1, 2], dtype=np.int32))
    x, its, rr, st, _ = O.gcr_bj(bd, O.BJ(bd, spd=False), tol=1e-12, maxit=10)
    assert st == O.BREAKDOWN and its == 1 and np.all(x == 0.0)


def test_gcr_with_bbd_matches_gmres_and_exact_blocks_take_one_step():
    s = gen.bbd_system(nblocks=4, block_rows=80, n_border=16, nnz_off=1, half_band=1, tail_frac=0.1,
                       border_c=2, seed=16, name="bbd-tri")
    P = O.BBD(s)
    x, its, rr, st, _ = O.gcr_bbd(s, P, tol=1e-10)
    assert st == O.OK and its == 1 and rr <= 1e-10
    s = gen.bbd_system(nblocks=3, block_rows=60, n_border=12, nnz_off=4, half_band=10, tail_frac=0.2,
                       border_c=2, seed=14, name="bbd-tiny")
    P = O.BBD(s)
    _, its_g, _, st_g, h_g = O.gmres_bbd(s, P, tol=1e-10, m=5, hist=True)
    x, its_c, rr, st_c, h_c = O.gcr_bbd(s, P, tol=1e-10, m=5, hist=True)
    assert st_g == O.OK and st_c == O.OK and abs(its_c - its_g) <= 1
    k = min(its_c, its_g) - 1
    np.testing.assert_allclose(h_c[:k], h_g[:k], rtol=1e-6)
    assert np.linalg.norm(s.b - s.scipy() @ x) <= 1.5e-10 * np.linalg.norm(s.b)


# --------------------------------------------------------------- complete factorisation

def test_complete_lu_reproduces_the_filtered_block_and_lapack():
    """COMPLETE (Sec. 3.1 complete LU, Alg. 2 complete factorisation of the
    filtered matrix): per block, L U equals the filtered, corrected block to
    rounding, and L, U equal SciPy's LU (LAPACK) where partial pivoting keeps
    the diagonal (a diagonally dominant block)."""
    s = gen.c2(0.004, dense_cols=0)
    P = O.BJ(s, O.FILTER_GEOMEAN, 1e-3, O.DIAG_DROPSUM, policy=O.PIVOT_FAIL, complete=True)
    F = O.BJ(s, O.FILTER_GEOMEAN, 1e-3, O.DIAG_DROPSUM, policy=O.PIVOT_FAIL)
    assert P.status == O.OK
    L, U = unpack_lu(P.rp, P.ci, P.v, s.n)
    Ph = sp.csr_matrix((F.corrected, F.ci, F.rp), shape=(s.n, s.n)).toarray()
    for b in range(s.nblocks):
        lo, hi = s.block_ptr[b], s.block_ptr[b + 1]
        blk = Ph[lo:hi, lo:hi]
        Lb, Ub = L[lo:hi, lo:hi], U[lo:hi, lo:hi]
        assert np.abs(Lb @ Ub - blk).max() <= 1e-12 * np.abs(blk).max()
    rng = np.random.default_rng(80)
    a = rand_sparse(150, 0.05, rng, dd=2.5)
    m = csr_of(a)
    t = gen.System("dd", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, rng.standard_normal(150),
                   np.array([0, 150], dtype=np.int32))
    Q = O.BJ(t, spd=False, policy=O.PIVOT_FAIL, complete=True)
    L, U = unpack_lu(Q.rp, Q.ci, Q.v, 150)
    p_, l_ref, u_ref = sl.lu(a)
    assert np.array_equal(p_, np.eye(150))
    np.testing.assert_allclose(L, l_ref, atol=1e-13)
    np.testing.assert_allclose(U, u_ref, atol=1e-12 * np.abs(u_ref).max())


def test_complete_lu_without_filter_is_exact_and_filtered_beats_ilu0():
    """Without a filter each block's complete LU is the block itself, so on
    one block PCG and GMRES converge in one step; with the filter and 4
    blocks it takes fewer PCG steps than ILU(0) of the same filtered
    blocks."""
    s = gen.c1()
    one = gen.System("c1-one", s.row_ptr, s.col, s.val, s.b, np.array([0, s.n], dtype=np.int32))
    x, its, rr, st, _ = O.pcg_bj(one, O.BJ(one, complete=True), tol=1e-8)
    assert st == O.OK and its == 1
    rng = np.random.default_rng(81)
    a = rand_sparse(300, 0.03, rng, dd=0.3)
    m = csr_of(a)
    g = gen.System("ns", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, rng.standard_normal(300),
                   np.array([0, 300], dtype=np.int32))
    x, its, rr, st, _ = O.gmres_bj(g, O.BJ(g, spd=False, policy=O.PIVOT_FAIL, complete=True), tol=1e-10)
    assert st == O.OK and its == 1
    s2 = gen.c2(0.004, dense_cols=0)
    kw = dict(mode=O.FILTER_GEOMEAN, tau=1e-3, flags=O.DIAG_DROPSUM)
    _, its_c, _, st_c, _ = O.pcg_bj(s2, O.BJ(s2, complete=True, **kw), tol=1e-8)
    _, its_i, _, st_i, _ = O.pcg_bj(s2, O.BJ(s2, **kw), tol=1e-8)
    assert st_c == st_i == O.OK and its_c < its_i


# --------------------------------------------------------------- MC64 (Alg. 3 step 1)

def _scrambled(n, seed, density=0.15):
    """Nonsymmetric sparse matrix whose large entries sit off the diagonal:
    a random permutation of rows of a diagonally heavy matrix, with entry
    magnitudes spread over 1e-4..1e4 by row and column scalings."""
    rng = np.random.default_rng(seed)
    a = rand_sparse(n, density, rng, dd=0.8)
    a = a[rng.permutation(n)]
    a = np.diag(10.0 ** rng.uniform(-4, 4, n)) @ a @ np.diag(10.0 ** rng.uniform(-2, 2, n))
    m = csr_of(a)
    return gen.System("scr", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data,
                      rng.standard_normal(n), gen.contiguous_blocks(n, 3)), a


@pytest.mark.parametrize("seed", [70, 71, 72])
def test_mc64_matching_maximises_the_diagonal_product(seed):
    """The matching maximises prod |a_{i,sigma(i)}| (Duff-Koster maximum
    product): its log-sum equals the optimum of SciPy's assignment solver on
    -log|a| (an independent algorithm), and it uses nonzeros only."""
    from scipy.optimize import linear_sum_assignment
    s, a = _scrambled(60, seed)
    match, dr, dc, st = O.mc64(s)
    assert st == O.OK
    assert np.all(a[np.arange(60), match] != 0.0)
    cost = np.where(a != 0.0, -np.log(np.abs(np.where(a != 0.0, a, 1.0))), 1e6)
    r, c = linear_sum_assignment(cost)
    best = -cost[r, c].sum()
    assert np.sum(np.log(np.abs(a[np.arange(60), match]))) == pytest.approx(best, abs=1e-9)


def test_mc64_brute_force_on_seven_unknowns():
    import itertools
    rng = np.random.default_rng(73)
    a = rng.standard_normal((7, 7)) * 10.0 ** rng.uniform(-3, 3, (7, 7))
    a[rng.random((7, 7)) < 0.3] = 0.0
    np.fill_diagonal(a, 0.0)
    a[np.arange(7), (np.arange(7) + 1) % 7] = 1.0   # keeps one nonzero matching
    m = csr_of(a)
    s = gen.System("bf", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, np.ones(7),
                   np.array([0, 7], dtype=np.int32))
    match, dr, dc, st = O.mc64(s)
    best, arg = -np.inf, None
    for perm in itertools.permutations(range(7)):
        vals = np.abs(a[np.arange(7), perm])
        if np.all(vals > 0):
            lv = np.sum(np.log(vals))
            if lv > best:
                best, arg = lv, perm
    assert st == O.OK and tuple(match) == arg


@pytest.mark.parametrize("seed", [74, 75])
def test_mc64_scaling_is_dual_feasible(seed):
    """The scalings from the assignment's duals make every scaled entry at
    most 1 in magnitude and every matched one exactly 1 (MC64's scaling);
    then the transformed system A' = Q Dr A Dc has a unit diagonal with no
    larger entry, b' = Q Dr b, and x = Dc y solves A x = b."""
    s, a = _scrambled(80, seed)
    match, dr, dc, st = O.mc64(s)
    sc = np.abs(dr[:, None] * a * dc[None, :])
    assert np.max(sc[a != 0.0]) <= 1.0 + 1e-12
    np.testing.assert_allclose(sc[np.arange(80), match], 1.0, rtol=1e-12)
    s2, x_of = O.mc64_transform(s, match, dr, dc)
    A2 = s2.scipy().toarray()
    np.testing.assert_allclose(np.abs(np.diag(A2)), 1.0, rtol=1e-12)
    assert np.max(np.abs(A2)) <= 1.0 + 1e-12
    y = np.linalg.solve(A2, s2.b)
    x = x_of(y)
    assert np.linalg.norm(a @ x - s.b) <= 1e-9 * np.linalg.norm(s.b) * np.linalg.cond(A2)


def test_mc64_of_spd_matrix_is_the_identity_with_jacobi_scaling():
    """|a_ij| <= sqrt(a_ii a_jj) for SPD matrices, so the identity has the
    largest diagonal product; the symmetric scaling sqrt(dr dc) is then
    1/sqrt(a_ii), the unit-diagonal scaling under which Eq. (filter) is the
    GEOMEAN rule."""
    s = gen.c1()
    match, dr, dc, st = O.mc64(s)
    assert st == O.OK and np.array_equal(match, np.arange(s.n))
    d = s.scipy().diagonal()
    np.testing.assert_allclose(np.sqrt(dr * dc), 1.0 / np.sqrt(d), rtol=1e-10)
    s2, x_of = O.mc64_transform(s, match, dr, dc, spd=True)
    np.testing.assert_allclose(s2.scipy().diagonal(), 1.0, rtol=1e-10)


def test_mc64_structurally_singular_and_transformed_solve():
    """An empty column has no matching (STRUCTURE).  A row-permuted, badly
    scaled system whose diagonal is mostly empty (so block Jacobi cannot
    factor it as it stands) is solved through Alg. 3: block-Jacobi GMRES on
    A', then x = Dc y."""
    a = np.array([[1.0, 0.0, 2.0], [3.0, 0.0, 1.0], [0.0, 0.0, 4.0]])
    m = csr_of(a)
    bad = gen.System("sing", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, np.ones(3),
                     np.array([0, 3], dtype=np.int32))
    assert O.mc64(bad)[3] == O.STRUCTURE
    s, a = _scrambled(600, 76, density=0.02)
    match, dr, dc, st = O.mc64(s)
    s2, x_of = O.mc64_transform(s, match, dr, dc)
    s.block_ptr = s2.block_ptr = gen.contiguous_blocks(600, 20)
    P2 = O.BJ(s2, spd=False, policy=O.PIVOT_FAIL)
    y, its2, rr2, st2, _ = O.gmres_bj(s2, P2, tol=1e-10, m=60, maxit=3000)
    assert st2 == O.OK
    x = x_of(y)
    assert np.linalg.norm(a @ x - s.b) <= 1e-8 * np.linalg.norm(s.b) * 1e4
    assert np.count_nonzero(np.diag(a)) < 600 // 4


# --------------------------------------------------------------- IR

def test_ir_reaches_tolerance_and_matches_fp64_solution():
    s = gen.c2(0.004, dense_cols=0)
    P = O.BJ(s, O.FILTER_GEOMEAN, 1e-3, O.DIAG_DROPSUM)
    x, outer, inner, fb, rr, st = O.ir_pcg_bj(s, P, tol=1e-8)
    assert st == O.OK and rr <= 1e-8 and outer >= 2
    M = s.scipy()
    assert np.linalg.norm(s.b - M @ x) / np.linalg.norm(s.b) <= 1.5e-8
    x64, its, rr64, st64, _ = O.pcg_bj(s, P, tol=1e-8)
    e = x - x64
    den = np.sqrt(x64 @ (M @ x64))
    assert np.sqrt(e @ (M @ e)) / den < 1e-3


# --------------------------------------------------------------- border, reliable updates

def test_border_correction_is_exact_inverse_of_bordered_preconditioner():
    """With the dense columns as a border, the preconditioner applies
    (P + U C U^T)^{-1} exactly (Sherman-Morrison-Woodbury of the bordered
    block elimination)."""
    s = gen.c2(0.004)
    P = O.BJ(s, O.FILTER_GEOMEAN, 1e-3, O.DIAG_DROPSUM, border=True)
    assert P.status == O.OK and P.border_status == O.OK
    n = s.n
    L, Uf = unpack_lu(P.rp, P.ci, P.v, n)
    U, c = s.lowrank
    Ud = U.toarray()
    Pfull = L @ Uf + Ud @ np.diag(c) @ Ud.T
    r = np.random.default_rng(30).standard_normal(n)
    z = P.apply(r)
    zz = np.linalg.solve(Pfull, r)
    assert np.linalg.norm(z - zz) <= 1e-8 * np.linalg.norm(zz)


def test_border_removes_low_rank_outliers():
    """The border preconditioner needs fewer PCG iterations than the block
    preconditioner that ignores the low-rank term (no more than the system
    without the dense columns needs, plus a few)."""
    s = gen.c2(0.004)
    s0 = gen.c2(0.004, dense_cols=0)
    its = {}
    for key, sys_, border in (("plain", s, False), ("border", s, True), ("nodense", s0, False)):
        P = O.BJ(sys_, O.FILTER_GEOMEAN, 1e-3, O.DIAG_DROPSUM, border=border)
        x, it, rr, st, _ = O.pcg_bj(sys_, P, tol=1e-8, maxit=50_000)
        assert st == O.OK and rr <= 1e-8
        its[key] = it
    assert its["border"] < its["plain"]
    assert its["border"] <= 1.5 * its["nodense"] + 20


def test_refine_rule_mixed_mode_scripted_histories():
    """The mixed mode's decision at a refinement point (a tuned rule; the
    paper states no precision): a point is weak when the true residual is
    above half the previous point's; three weak points in a row send the rest
    to FP64 solves of the residual equation; a breakdown reverts to the last
    point first; meeting the tolerance ends the solve before anything else."""
    assert O.refine_constants() == (0.5, 3.0, 2.0, 4.0, 0.5)
    tol = 1e-8

    def run(rel, bd=()):
        slow, acts, prev = 0, [], 1.0
        for e, nr in enumerate(rel):
            a, slow = O.refine_decide(0, nr, prev, tol, e in bd, slow)
            acts.append(O.RF_NAMES[a])
            prev = nr
        return acts, slow
    # halving exactly is not weak; a hair above half is
    assert run([0.5, 0.25])[0] == ["continue", "continue"]
    assert run([0.5, 0.2500001]) == (["continue", "continue"], 1)
    # three weak points in a row: FP64 at the third, not earlier
    assert run([0.9, 0.8]) == (["continue", "continue"], 2)
    assert run([0.9, 0.8, 0.7]) == (["continue", "continue", "fallback"], 3)
    # a strong point in between resets the count
    assert run([0.9, 0.8, 0.3, 0.25, 0.2])[0] == ["continue"] * 5
    assert run([0.9, 0.8, 0.3, 0.25, 0.2, 0.15])[0] == ["continue"] * 5 + ["fallback"]
    # breakdown: revert, whatever the count; convergence wins over breakdown
    assert run([0.1, 0.05], bd={1})[0] == ["continue", "revert"]
    assert run([0.1, 5e-9], bd={1})[0] == ["continue", "done"]
    assert run([0.9, 0.8, 1e-8])[0] == ["continue", "continue", "done"]
    # just above the tolerance is not done: three weak points there go to FP64
    assert run([1.5e-8, 1.2e-8, 1.1e-8, 1.0000001e-8]) == (["continue", "continue", "continue", "fallback"], 3)


def test_refine_rule_restart_mode_and_fallback_scripted_histories():
    """Classical refinement: two weak steps in a row send the rest to an FP64
    solve of the residual equation; an inner solve that broke down is
    discarded (revert) before that; after such a solve, another one follows
    only when it converged and fewer than four were run."""
    tol = 1e-8

    def run(rel, bd=()):
        slow, acts, prev = 0, [], 1.0
        for e, nr in enumerate(rel):
            a, slow = O.refine_decide(1, nr, prev, tol, e in bd, slow)
            acts.append(O.RF_NAMES[a])
            prev = nr
        return acts
    assert run([0.9, 0.8]) == ["continue", "fallback"]
    assert run([0.9, 0.3, 0.2]) == ["continue"] * 3
    assert run([0.9, 0.3, 0.2, 0.15]) == ["continue"] * 3 + ["fallback"]
    assert run([0.1, 0.01, 0.001]) == ["continue"] * 3
    assert run([0.5, 0.25, 0.125]) == ["continue"] * 3
    assert run([0.1], bd={0}) == ["revert"]
    assert run([0.9, 0.9], bd={1}) == ["continue", "revert"]
    assert run([1e-9], bd={0}) == ["done"]
    fb = lambda nr, st, k: O.RF_NAMES[O.fallback_decide(nr, tol, st, k)]
    assert fb(1e-8, O.OK, 1) == "done"
    assert fb(2e-8, O.OK, 1) == "fallback"
    assert fb(2e-8, O.OK, 3) == "fallback"
    assert fb(2e-8, O.OK, 4) == "fail"
    assert fb(2e-8, O.BREAKDOWN, 1) == "fail"
    assert fb(2e-8, O.NOT_CONVERGED, 1) == "fail"


def test_fp32_solvers_apply_the_refine_rule():
    """Both FP32 solvers take exactly the rule's decisions on their own
    residual histories, on late IPM systems that stall the FP32 recurrence
    (FP64 solves of the residual equation follow), and still meet the
    tolerance, checked with scipy."""
    q = gen.IPMSequence(m=20000, nblocks=4, steps=30)
    for k in (16, 20):
        s = q.system(k)
        P = O.BJ(s, mode=O.FILTER_GEOMEAN, tau=1e-3, flags=O.DIAG_DROPSUM)
        nb = np.linalg.norm(s.b)
        x, pts, its, fb, rr, st, hist = O.mx_pcg_bj(s, P, tol=1e-8, delta=0.3, every=500, maxit=60000,
                                                    with_history=True)
        assert st == O.OK and fb >= 1 and len(hist) >= 4
        assert np.linalg.norm(s.b - s.scipy() @ x) / nb <= 1.5e-8
        O.replay_refine(hist, 0, nb, 1e-8, 60000)
        x, outer, its, fb, rr, st, hist = O.ir_pcg_bj(s, P, tol=1e-8, inner_tol=1e-4, max_outer=30, maxit=60000,
                                                      with_history=True)
        assert st == O.OK and len(hist) >= 1
        O.replay_refine(hist, 1, nb, 1e-8, 60000)


def _mixed_case(lowrank, border, n=60, seed=40):
    s, a = _small_spd(n, seed)
    md = a.copy()
    if lowrank:
        rng = np.random.default_rng(seed + 1)
        U = sp.random(n, 3, density=0.5, random_state=rng, data_rvs=rng.standard_normal, format="csr")
        U.sort_indices()
        c = rng.uniform(0.5, 2.0, 3)
        s.lowrank = (U, c)
        ud = U.toarray()
        md = md + ud @ np.diag(c) @ ud.T
    P = O.BJ(s, policy=O.PIVOT_FAIL, spd=True, border=border)
    assert P.status == O.OK
    L, Uf = unpack_lu(P.rp, P.ci, P.v, n)
    pm = L @ Uf
    if lowrank and border:
        pm = pm + ud @ np.diag(c) @ ud.T
    return s, P, md, np.linalg.inv(pm)


@pytest.mark.parametrize("lowrank,border", [(False, False), (True, False), (True, True)],
                         ids=["plain", "lowrank", "border"])
def test_mixed_recurrence_is_fp64_cg_up_to_fp32_rounding(lowrank, border):
    """Before its first refinement point the mixed recurrence is preconditioned
    CG (Sec. 2.2) whose operator product and preconditioner apply are rounded
    to FP32: its k-th iterate is the M-norm minimiser over
    K_k(P^-1 M, P^-1 b), computed here in FP64 with dense algebra, up to a
    perturbation of order k * u32 * kappa(P^-1 M) (u32 = 2^-24).  Both
    halves are pinned: the iterate is that close (a dropped term, a wrong
    sign or a transposed factor is off by O(1)), and no closer than FP64
    rounding allows (the FP32 rounding really happens)."""
    s, P, md, pinv = _mixed_case(lowrank, border)
    kappa = np.linalg.cond(pinv @ md)
    u32 = 2.0 ** -24
    devs = []
    for k in range(1, 7):
        # delta 0 and no periodic refresh: no refinement point before maxit
        x, points, its, fallbacks, rr, st = O.mx_pcg_bj(s, P, tol=1e-30, delta=0.0, every=0, maxit=k)
        assert (points, its, fallbacks, st) == (0, k, 0, O.NOT_CONVERGED)
        K = [pinv @ s.b]
        for _ in range(k - 1):
            K.append(pinv @ (md @ K[-1]))
        Q, _ = np.linalg.qr(np.array(K).T)
        xb = Q @ np.linalg.solve(Q.T @ md @ Q, Q.T @ s.b)
        e = x - xb
        devs.append(np.sqrt(e @ md @ e) / np.sqrt(xb @ md @ xb))
        assert devs[-1] <= k * u32 * kappa, (k, devs[-1], k * u32 * kappa)
        assert rr == pytest.approx(np.linalg.norm(s.b - md @ x) / np.linalg.norm(s.b), rel=1e-10)
    assert min(devs) >= 1e-10


def _krylov_minimiser(md, pinv, b, k):
    K = [pinv @ b]
    for _ in range(k - 1):
        K.append(pinv @ (md @ K[-1]))
    Q, _ = np.linalg.qr(np.array(K).T)
    return Q @ np.linalg.solve(Q.T @ md @ Q, Q.T @ b)


@pytest.mark.parametrize("lowrank,border", [(False, False), (True, False), (True, True)],
                         ids=["plain", "lowrank", "border"])
def test_mixed_refinement_point_when_residual_falls_below_delta(lowrank, border):
    """A refinement point is taken at the first iteration whose recurrence
    residual is below delta times its value at the previous point (here
    ||b||).  With delta at the geometric midpoint of the exact CG residuals
    after 2 and 3 steps, no point is taken in 2 iterations and exactly one
    in 3."""
    s, P, md, pinv = _mixed_case(lowrank, border)
    nb = np.linalg.norm(s.b)
    h = [np.linalg.norm(s.b - md @ _krylov_minimiser(md, pinv, s.b, k)) / nb for k in (1, 2, 3)]
    assert h[2] < 0.8 * h[1] and h[2] < h[0]
    delta = np.sqrt(h[1] * h[2])
    for maxit, points_expected in ((2, 0), (3, 1)):
        x, points, its, fallbacks, rr, st = O.mx_pcg_bj(s, P, tol=1e-30, delta=delta, every=0, maxit=maxit)
        assert (points, its, fallbacks) == (points_expected, maxit, 0)


@pytest.mark.parametrize("lowrank,border", [(False, False), (True, False), (True, True)],
                         ids=["plain", "lowrank", "border"])
def test_fp32_inner_pcg_is_fp64_cg_up_to_fp32_rounding(lowrank, border):
    """One refinement step of k inner FP32 PCG iterations gives ||b|| times
    the k-th FP32 iterate for M d = b / ||b||: the FP64 Krylov minimiser up
    to k * u32 * kappa(P^-1 M), now with FP32 vectors, FP32 step lengths,
    the FP32 low-rank term and the FP32 border correction (a dropped term, a
    wrong sign or a missing rescaling by ||b|| is off by O(1))."""
    s, P, md, pinv = _mixed_case(lowrank, border)
    kappa = np.linalg.cond(pinv @ md)
    u32 = 2.0 ** -24
    for k in range(1, 7):
        x, outer, inner, fb, rr, st = O.ir_pcg_bj(s, P, tol=1e-30, inner_tol=1e-30, max_outer=1, maxit=k)
        assert (outer, inner, fb, st) == (1, k, 0, O.NOT_CONVERGED)
        xb = _krylov_minimiser(md, pinv, s.b, k)
        e = x - xb
        dev = np.sqrt(e @ md @ e) / np.sqrt(xb @ md @ xb)
        assert 1e-10 < dev <= k * u32 * kappa, (k, dev, k * u32 * kappa)


def test_mixed_first_step_rounds_only_the_sparse_product_to_fp32():
    """One-row blocks with power-of-two diagonals and FP32-representable
    data: the FP32 preconditioner apply is exact, so after one step the mixed
    iterate differs from FP64 CG (x1 = (b,z)/(z,Mz) z with z = D^-1 b) only
    through the FP32 sparse product.  The textbook bound for a rounded
    product, |fl(Az) - Az| <= gamma_m |A||z| (m = longest row), limits the
    relative change of the step length to gamma_m (|z|,|A||z|)/(z,Mz); the
    low-rank term, kept in FP64, adds nothing to it (its weights are large, so
    an FP32 rounding of that term would exceed the bound).  The change must
    also be above FP64 rounding: the product really is rounded to FP32."""
    n = 80
    rng = np.random.default_rng(42)
    off = sp.random(n, n, density=0.08, random_state=rng, data_rvs=rng.standard_normal).toarray()
    off = np.triu(off, 1)
    off = (off + off.T).astype(np.float32).astype(np.float64)
    d = 2.0 ** np.ceil(np.log2(np.abs(off).sum(axis=1) + 1.0))
    a = off + np.diag(d)
    m = csr_of(a)
    b = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    U = sp.random(n, 2, density=0.6, random_state=rng, data_rvs=rng.standard_normal, format="csr")
    U.sort_indices()
    c = np.array([4000.0, 2500.0])
    s = gen.System("jac", m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data, b,
                   np.arange(n + 1, dtype=np.int32), lowrank=(U, c))
    P = O.BJ(s, policy=O.PIVOT_FAIL, spd=True)
    assert P.status == O.OK
    ud = U.toarray()
    md = a + ud @ np.diag(c) @ ud.T
    z = b / d
    x1 = (b @ z) / (z @ md @ z) * z
    x, points, its, fallbacks, rr, st = O.mx_pcg_bj(s, P, tol=1e-30, delta=0.0, every=0, maxit=1)
    assert (points, its, fallbacks) == (0, 1, 0)
    rows = np.diff(m.indptr).max()
    u32 = 2.0 ** -24
    gamma = rows * u32 / (1 - rows * u32)
    bound = gamma * (np.abs(z) @ (np.abs(a) @ np.abs(z))) / (z @ md @ z) + 1e-13
    dev = np.linalg.norm(x - x1) / np.linalg.norm(x1)
    assert 1e-12 < dev <= bound, (dev, bound)


def test_mixed_recurrence_stall_hands_over_and_still_converges():
    """A late IPM system (D spread about 1e9): the refinement points stop
    halving the true residual, the recurrence is handed to the FP64 operator
    and factors (and, if it stalls again, to an FP64 solve of the residual
    equation), and the result still meets the tolerance, checked with scipy."""
    q = gen.IPMSequence(m=20000, nblocks=4, steps=30)
    s = q.system(20)
    P = O.BJ(s, mode=O.FILTER_GEOMEAN, tau=1e-3, flags=O.DIAG_DROPSUM)
    x, points, its, fallbacks, rr, st = O.mx_pcg_bj(s, P, tol=1e-8, delta=0.3, every=500, maxit=60000)
    assert st == O.OK and points >= 3 and fallbacks >= 1
    assert np.linalg.norm(s.b - s.scipy() @ x) / np.linalg.norm(s.b) <= 1.5e-8


def test_mixed_recurrence_breakdown_falls_back_to_fp64():
    """An IPM system whose FP32 rounding is not positive definite (rows of M
    that hold only the 1e-8 regularisation): the mixed recurrence breaks down
    and the FP64 residual-equation solve, started from the solution of the
    last refinement point, still reaches the tolerance."""
    q = gen.IPMSequence(m=20000, nblocks=1, steps=30)
    s = q.system(1)
    P = O.BJ(s, mode=O.FILTER_GEOMEAN, tau=1e-3, flags=O.DIAG_DROPSUM)
    x, points, its, fallbacks, rr, st = O.mx_pcg_bj(s, P, tol=1e-8, delta=0.3, every=500, maxit=20000)
    assert st == O.OK and fallbacks >= 1 and its < 1000
    assert O.relres(s, x) <= 1e-8
