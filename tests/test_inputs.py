"""The seeded generators: determinism, requested shapes and structure."""
import numpy as np
import scipy.sparse as sp

from ipm_inputs import gen


def test_c1_shape_determinism_symmetry():
    a, b = gen.c1(), gen.c1()
    assert a.n == 2000 and a.nblocks == 4
    assert np.array_equal(a.val, b.val) and np.array_equal(a.col, b.col) and np.array_equal(a.b, b.b)
    M = a.scipy()
    assert (M != M.T).nnz == 0                      # bitwise symmetric
    assert np.all(M.diagonal() > 0)
    assert all(np.all(np.diff(a.col[a.row_ptr[i]:a.row_ptr[i + 1]]) > 0) for i in range(a.n))
    assert 90_000 < a.nnz < 110_000


def test_pattern_models_distinct_rows_and_locality():
    rng = np.random.default_rng(0)
    cp, rows = gen.a_pattern(rng, 5000, 12000, 8, "loc")
    assert np.all(np.diff(cp) == 8)
    r = rows.reshape(-1, 8)
    assert np.all(np.diff(r, axis=1) > 0)          # distinct and sorted
    home = ((np.arange(12000) + 0.5) * 5000 / 12000).astype(int)
    lo = np.clip(home - 1024, 0, 5000 - 2048)       # the window, shifted inside at the ends
    near = (r >= lo[:, None]) & (r < lo[:, None] + 2048)
    assert 0.9 < near.mean() < 0.96               # 0.9 local + chance hits of the far draws
    # no row collects more than its share (the window is never clipped)
    counts = np.bincount(rows, minlength=5000)
    assert counts.max() < 3 * counts.mean()


def test_c2_low_rank_term_shape():
    s = gen.c2(0.01)
    U, c = s.lowrank
    assert U.shape == (s.n, 20) and c.shape == (20,)
    dens = U.nnz / (s.n * 20)
    assert 0.27 < dens < 0.33
    assert np.all(c > 0)


def test_ipm_sequence_values_are_ada():
    q = gen.IPMSequence(m=1500, nblocks=4, steps=4, seed=2)
    r_pat, r_val, _, _, _, _ = gen.streams(2)
    cp, rows = gen.a_pattern(r_pat, 1500, q.n_a, 4, "loc")
    vals = r_val.standard_normal(rows.shape[0])
    A = sp.csc_matrix((vals, rows, cp), shape=(1500, q.n_a))
    for k in range(4):
        Mk = gen.normal_equations(A, q.d[k])
        v = q.values(k)
        assert np.array_equal(Mk.indptr, q.row_ptr) and np.array_equal(Mk.indices, q.col)
        assert np.max(np.abs(Mk.data - v) / np.abs(Mk.data).max()) < 1e-14
        S = sp.csr_matrix((v, q.col, q.row_ptr))
        assert (S != S.T).nnz == 0
    spread = [np.log10(d.max() / d.min()) for d in q.d]
    assert abs(spread[0] - 2) < 0.1 and abs(spread[-1] - 12) < 1e-9


def test_bbd_structure():
    s = gen.c3(0.02)
    ni = s.n - s.n_border
    M = s.scipy()
    bp = s.block_ptr
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    cols = s.col
    interior = rows < ni
    rb = np.searchsorted(bp, rows[interior], side="right") - 1
    cb = np.where(cols[interior] < ni, np.searchsorted(bp, cols[interior], side="right") - 1, -1)
    assert np.all((cb == rb) | (cb == -1))         # no block-to-block coupling
    d = M.diagonal()
    off = np.asarray(abs(M).sum(axis=1)).ravel() - np.abs(d)
    assert np.allclose(np.abs(d), 1.5 * off)


def test_c5_requests():
    reqs = gen.c5_requests(50)
    assert len(reqs) == 50
    assert all(10_000 <= r["m"] <= 500_000 and 6 <= r["c"] <= 10 and r["nblocks"] in (8, 16, 32, 64, 128)
               for r in reqs)
    assert reqs == gen.c5_requests(50)
