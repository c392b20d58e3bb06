"""Seeded synthetic inputs shaped like interior-point-method linear systems.

This module only *builds inputs*: constraint-matrix patterns, the diagonal
scalings of an IPM iterate, the normal-equations matrix that a solver is handed,
right-hand sides, block partitions and request streams.  It holds none of the
solver's arithmetic (no filtering, factorisation, preconditioning or Krylov
steps), so the CPU oracle and the GPU path can both read its output without
sharing any method code.

The normal-equations form follows the reduction of the augmented IPM system to
its Schur complement (paper Sec. 2.1, Eq. (schur)): with constraint matrix ``A``
(the paper's ``B``) and positive diagonal ``D`` (the paper's ``D^{-1}``) the
system matrix is ``M = A D A^T + 1e-8 I``.  The ``1e-8 I`` regularisation is a
workload choice, not part of the paper.

Every random draw comes from numpy's PCG64 ``default_rng`` seeded through
``SeedSequence(seed).spawn(6)``; the six child streams are used, in order, for
the nonzero pattern, the A values, D, b, block counts and arrivals.

Two pattern models:

* ``uni``: each column's ``c`` distinct rows are uniform over ``[0, m)``.
* ``loc``: column ``j`` has a home row ``floor((j + 0.5) m / n_A)``; each of its
  nonzeros lands uniformly in the 2048-row window ``[home - 1024, home + 1024)``
  (shifted, not clipped, to stay inside ``[0, m)`` near the ends, so no row
  collects the overflow) with probability 0.9 and uniformly over ``[0, m)``
  otherwise; rows are distinct.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np
import scipy.sparse as sp

REG = 1e-8          # the ``+ 1e-8 I`` term of M
HALF_WINDOW = 1024  # half width of the ``loc`` model's home window
P_LOCAL = 0.9       # probability that a ``loc`` nonzero lands in the window


@dataclasses.dataclass
class System:
    """One linear system ``M x = b`` with its block partition.

    ``row_ptr`` (int64, n+1), ``col`` (int32, sorted per row, diagonal
    present) and ``val`` (float64) are M in CSR.  ``block_ptr`` (int32,
    nblocks+1) gives contiguous row blocks of the first ``n - n_border`` rows;
    ``n_border`` trailing rows form a BBD border (0 for block Jacobi).
    ``lowrank`` is ``None`` or ``(U, c)`` with ``U`` an n x k CSR matrix and
    ``c`` a length-k vector, meaning the operator is ``M + U diag(c) U^T``.
    """
    name: str
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray
    block_ptr: np.ndarray
    n_border: int = 0
    lowrank: Optional[tuple] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def nblocks(self) -> int:
        return int(self.block_ptr.shape[0] - 1)

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def streams(seed: int, k: int = 6):
    """Child generators of ``SeedSequence(seed)`` in the fixed order
    pattern, A values, D, b, block counts, arrivals."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def contiguous_blocks(n: int, nblocks: int) -> np.ndarray:
    """Block boundaries ``floor(b n / B)`` for b = 0..B (contiguous row blocks)."""
    b = np.arange(nblocks + 1, dtype=np.int64)
    return (b * n // nblocks).astype(np.int32)


def _draw_rows(rng, m, n_cols, c, model, home):
    """``n_cols x c`` row indices, drawn per the pattern model."""
    if model == "uni":
        return rng.integers(0, m, size=(n_cols, c), dtype=np.int64)
    local = rng.random((n_cols, c)) < P_LOCAL
    width = min(2 * HALF_WINDOW, m)
    lo = np.clip(home - HALF_WINDOW, 0, m - width)
    off = rng.integers(0, width, size=(n_cols, c), dtype=np.int64)
    near = lo[:, None] + off
    far = rng.integers(0, m, size=(n_cols, c), dtype=np.int64)
    return np.where(local, near, far)


def a_pattern(rng, m: int, n_a: int, c, model: str) -> tuple[np.ndarray, np.ndarray]:
    """Row indices of A, column-major: returns (col_ptr, rows) with every
    column holding distinct sorted rows.  ``c`` is an int or a per-column
    int array."""
    if m < 1 or n_a < 1:
        raise ValueError("empty shape")
    cnt = np.full(n_a, c, dtype=np.int64) if np.isscalar(c) else np.asarray(c, dtype=np.int64)
    if int(cnt.max()) > m:
        raise ValueError("more nonzeros per column than rows")
    cmax = int(cnt.max())
    home = ((np.arange(n_a, dtype=np.float64) + 0.5) * m / n_a).astype(np.int64)
    rows = _draw_rows(rng, m, n_a, cmax, model, home)
    # mask of slots that are in use for each column
    used = np.arange(cmax)[None, :] < cnt[:, None]
    big = np.int64(1) << 62
    while True:
        key = np.where(used, rows, big)
        order = np.argsort(key, axis=1, kind="stable")
        srt = np.take_along_axis(key, order, axis=1)
        dup_sorted = np.zeros_like(used)
        dup_sorted[:, 1:] = (srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] != big)
        if not dup_sorted.any():
            break
        dup = np.zeros_like(used)
        np.put_along_axis(dup, order, dup_sorted, axis=1)
        ci, si = np.nonzero(dup)
        fresh = _draw_rows(rng, m, ci.shape[0], 1, model, home[ci])[:, 0]
        rows[ci, si] = fresh
    # unused slots hold ``big`` and sort last, so each column's rows lead
    rows = np.sort(np.where(used, rows, big), axis=1)
    flat = rows[used]
    col_ptr = np.zeros(n_a + 1, dtype=np.int64)
    np.cumsum(cnt, out=col_ptr[1:])
    return col_ptr, flat


def log_uniform(rng, size, lo_exp: float, hi_exp: float) -> np.ndarray:
    """``10 ** U(lo_exp, hi_exp)``."""
    return np.power(10.0, rng.uniform(lo_exp, hi_exp, size=size))


def normal_equations(A: sp.csc_matrix, d: np.ndarray, reg: float = REG) -> sp.csr_matrix:
    """``A diag(d) A^T + reg I`` in CSR with sorted columns, a stored
    diagonal in every row and bitwise-symmetric values (the upper triangle is
    computed once and mirrored)."""
    m = A.shape[0]
    Ad = A @ sp.diags(d)
    M = (Ad @ A.T.tocsc()).tocsr()
    M = M + reg * sp.identity(m, format="csr")
    up = sp.triu(M, k=0, format="csr")
    strict = sp.triu(M, k=1, format="csr")
    M = (up + strict.T).tocsr()
    M.sort_indices()
    M.sum_duplicates()
    return M


def _system_from_csr(name, M, b, block_ptr, n_border=0, lowrank=None, meta=None) -> System:
    return System(name=name,
                  row_ptr=M.indptr.astype(np.int64),
                  col=M.indices.astype(np.int32),
                  val=M.data.astype(np.float64),
                  b=np.ascontiguousarray(b, dtype=np.float64),
                  block_ptr=np.ascontiguousarray(block_ptr, dtype=np.int32),
                  n_border=int(n_border), lowrank=lowrank, meta=dict(meta or {}))


def ada_system(m: int, n_a: int, c, d_lo: float, d_hi: float, nblocks: int,
               model: str = "loc", dense_cols: int = 0, dense_p: float = 0.3,
               seed: int = 0, name: str = "ada") -> System:
    """A normal-equations system ``M = A_s D_s A_s^T + 1e-8 I`` (+ a low-rank
    term for dense columns) with ``nblocks`` contiguous row blocks.

    ``A_s`` is m x n_a with ``c`` N(0,1) nonzeros per column (pattern model
    ``model``), D log-uniform with log10 in ``[d_lo, d_hi]``.  ``dense_cols``
    extra columns of A have Bernoulli(``dense_p``) rows; they are kept apart as
    ``U`` with ``c = D_dense`` so that the operator is
    ``M_s + U diag(D_dense) U^T`` (the dense columns relocated out of the
    sparse product, as in paper Sec. 2.1)."""
    r_pat, r_val, r_d, r_b, _, _ = streams(seed)
    col_ptr, rows = a_pattern(r_pat, m, n_a, c, model)
    vals = r_val.standard_normal(rows.shape[0])
    A = sp.csc_matrix((vals, rows, col_ptr), shape=(m, n_a))
    d_all = log_uniform(r_d, n_a + dense_cols, d_lo, d_hi)
    M = normal_equations(A, d_all[:n_a])
    lowrank = None
    if dense_cols:
        mask = r_pat.random((m, dense_cols)) < dense_p
        ri, ci = np.nonzero(mask)
        uv = r_val.standard_normal(ri.shape[0])
        U = sp.csr_matrix((uv, (ri, ci)), shape=(m, dense_cols))
        U.sort_indices()
        lowrank = (U, d_all[n_a:].copy())
    b = r_b.standard_normal(m)
    meta = dict(m=m, n_a=n_a, c=c if np.isscalar(c) else "per-column", d_lo=d_lo, d_hi=d_hi,
                model=model, dense_cols=dense_cols, seed=seed)
    return _system_from_csr(name, M, b, contiguous_blocks(m, nblocks), lowrank=lowrank, meta=meta)


# --------------------------------------------------------------------------
# The five workloads, each with a scale knob.  ``scale=1`` is the full size;
# smaller scales keep the structure and the per-row densities.
# --------------------------------------------------------------------------

def c1(seed: int = 0) -> System:
    """2,000 x 5,000 A, 5 N(0,1) per column at uniform rows, D log-uniform
    [1e-4, 1e4], 4 contiguous blocks (unfiltered ILU(0), FP64 PCG)."""
    return ada_system(2000, 5000, 5, -4.0, 4.0, 4, model="uni", seed=seed, name="C1")


def c2(scale: float = 1.0, seed: int = 0, dense_cols: int = 20) -> System:
    """200,000 x 500,000 A with 8 N(0,1) per column (``loc`` model), 20 dense
    columns at 30% density as a low-rank term, D log-uniform [1e-6, 1e6],
    64 contiguous blocks.  ``scale`` shrinks rows and columns together."""
    m = max(256, int(round(200_000 * scale)))
    n_a = int(round(2.5 * m))
    nb = 64 if scale == 1.0 else max(2, int(round(64 * scale)))
    return ada_system(m, n_a, 8, -6.0, 6.0, nb, model="loc", dense_cols=dense_cols,
                      seed=seed, name="C2" if scale == 1.0 else f"C2x{scale:g}")


def bbd_system(nblocks: int = 32, block_rows: int = 46_750, n_border: int = 4096,
               nnz_off: int = 11, half_band: int = 1024, tail_frac: float = 0.02,
               border_c: int = 4, seed: int = 0, name: str = "C3") -> System:
    """A nonsymmetric, weakly diagonally dominant system already in bordered
    block diagonal form (interior blocks first, border rows last).

    Block row i (local index) gets ``nnz_off`` distinct off-diagonals uniform in
    ``[i - half_band, i + half_band]`` clipped to the block, N(0,1) values.  The
    last ``t = round(tail_frac * block_rows)`` local indices of each block form
    its tail; each tail row gets 1-2 border-column entries and each tail column
    1-2 border-row entries (uniform over the border, N(0,1), drawn
    independently).  Each border row gets ``border_c`` off-diagonal entries in
    the border block.  Every diagonal is ``1.5 * sum_j |a_ij|`` over the row's
    off-diagonals (the 0.6x-of-row-sum reading with the diagonal included)."""
    r_pat, r_val, _, r_b, _, _ = streams(seed)
    nb, br, nbd = nblocks, block_rows, n_border
    n_int = nb * br
    n = n_int + nbd
    t = max(1, int(round(tail_frac * br)))
    t = min(t, br)
    rows_l, cols_l = [], []
    # interior band entries, per block (vectorised over rows)
    li = np.arange(br, dtype=np.int64)
    lo = np.maximum(li - half_band, 0)
    hi = np.minimum(li + half_band, br - 1)
    width = hi - lo + 1 - 1  # candidates excluding the diagonal
    k = np.minimum(nnz_off, width)
    kmax = int(k.max())
    for blk in range(nb):
        # draw kmax candidates per row, redraw duplicates/diagonal
        cand = lo[:, None] + (r_pat.random((br, kmax)) * (hi - lo)[:, None]).astype(np.int64)
        cand = np.where(cand >= li[:, None], cand + 1, cand)  # skip the diagonal
        used = np.arange(kmax)[None, :] < k[:, None]
        big = np.int64(1) << 62
        while True:
            key = np.where(used, cand, big)
            order = np.argsort(key, axis=1, kind="stable")
            srt = np.take_along_axis(key, order, axis=1)
            ds = np.zeros_like(used)
            ds[:, 1:] = (srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] != big)
            if not ds.any():
                break
            dup = np.zeros_like(used)
            np.put_along_axis(dup, order, ds, axis=1)
            ri, si = np.nonzero(dup)
            f = lo[ri] + (r_pat.random(ri.shape[0]) * (hi - lo)[ri]).astype(np.int64)
            f = np.where(f >= li[ri], f + 1, f)
            cand[ri, si] = f
        rr = np.broadcast_to(li[:, None], cand.shape)[used] + blk * br
        cc = cand[used] + blk * br
        rows_l.append(rr)
        cols_l.append(cc)
        # E: tail rows -> border columns ; F: border rows -> tail columns
        tail = np.arange(br - t, br, dtype=np.int64) + blk * br
        ne = r_pat.integers(1, 3, size=t)
        er = np.repeat(tail, ne)
        ec = n_int + r_pat.integers(0, nbd, size=er.shape[0])
        nf = r_pat.integers(1, 3, size=t)
        fc = np.repeat(tail, nf)
        fr = n_int + r_pat.integers(0, nbd, size=fc.shape[0])
        rows_l += [er, fr]
        cols_l += [ec, fc]
    # border block C: border_c off-diagonals per border row
    brow = np.repeat(np.arange(nbd, dtype=np.int64), border_c)
    boff = r_pat.integers(1, nbd, size=brow.shape[0])
    bcol = (brow + boff) % nbd
    rows_l.append(brow + n_int)
    cols_l.append(bcol + n_int)
    R = np.concatenate(rows_l)
    C = np.concatenate(cols_l)
    V = r_val.standard_normal(R.shape[0])
    M = sp.csr_matrix((V, (R, C)), shape=(n, n))
    M.sum_duplicates()  # coinciding border draws add up
    M.sort_indices()
    M.setdiag(0.0)
    M.eliminate_zeros()
    off_sum = np.asarray(np.abs(M).sum(axis=1)).ravel()
    diag = 1.5 * off_sum
    diag[diag == 0.0] = 1.0
    M = (M + sp.diags(diag)).tocsr()
    M.sort_indices()
    b = r_b.standard_normal(n)
    block_ptr = (np.arange(nb + 1, dtype=np.int64) * br).astype(np.int32)
    meta = dict(nblocks=nb, block_rows=br, n_border=nbd, tail=t, half_band=half_band, seed=seed)
    return _system_from_csr(name, M, b, block_ptr, n_border=nbd, meta=meta)


def strong_border_system(gamma: float = 20.0, seed: int = 5) -> System:
    """A small bordered system whose border couples strongly to its blocks:
    the bbd_system layout (4 blocks of 400 rows, 40 border rows) with every
    interior-border coupling multiplied by ``gamma``; interior diagonals are
    1.5x their row's off-diagonal magnitude sum, border diagonals 1.5x the
    sum over the border block only (+1e-3).  Block Jacobi, which drops the
    couplings, stalls on it; the bordered form keeps them (the situation in
    which Alg. 1 of the paper switches preconditioners)."""
    s = bbd_system(nblocks=4, block_rows=400, n_border=40, nnz_off=6, half_band=60, tail_frac=0.1,
                   border_c=2, seed=seed, name="strong-border")
    n, ni = s.n, s.n - s.n_border
    M = s.scipy().tocoo()
    r, c, v = M.row, M.col, M.data.copy()
    cross = (r != c) & (((r < ni) & (c >= ni)) | ((r >= ni) & (c < ni)))
    v[cross] *= gamma
    A = sp.csr_matrix((v, (r, c)), shape=(n, n))
    A.setdiag(0.0)
    A.eliminate_zeros()
    off = np.asarray(abs(A).sum(axis=1)).ravel()
    border_only = np.asarray(abs(A[:, ni:]).sum(axis=1)).ravel()
    d = np.where(np.arange(n) < ni, 1.5 * off, 1.5 * border_only + 1e-3)
    A = (A + sp.diags(d)).tocsr()
    A.sort_indices()
    return _system_from_csr(f"strong-border-x{gamma:g}", A, s.b, s.block_ptr, n_border=s.n_border,
                            meta=dict(gamma=gamma, seed=seed))


def as_block_jacobi(s: System) -> System:
    """The same system with its border rows taken as one more contiguous
    block (the partition block Jacobi needs)."""
    if s.n_border == 0:
        return s
    bp = np.r_[s.block_ptr, s.n].astype(np.int32)
    return System(name=s.name + "-bj", row_ptr=s.row_ptr, col=s.col, val=s.val, b=s.b, block_ptr=bp,
                  n_border=0, lowrank=s.lowrank, meta=dict(s.meta))


def c3(scale: float = 1.0, seed: int = 0) -> System:
    """BBD workload: 32 blocks of 46,750 rows, 4,096-row border.  ``scale``
    shrinks block rows (and the border proportionally, at least 64)."""
    if scale == 1.0:
        return bbd_system(seed=seed)
    br = max(200, int(round(46_750 * scale)))
    nbd = max(64, int(round(4096 * scale)))
    hb = min(1024, br // 4)
    return bbd_system(nblocks=32 if scale >= 0.05 else 8, block_rows=br, n_border=nbd,
                      half_band=hb, seed=seed, name=f"C3x{scale:g}")


class IPMSequence:
    """Consecutive IPM systems ``A D_k A^T + 1e-8 I`` on one fixed pattern.

    ``D_0`` is log-uniform with log10 in [-1, 1].  Step k draws
    ``z = ln D_{k-1} + N(0, 0.5^2)`` and rescales ``log10`` of ``exp(z)``
    affinely onto ``[-s_k/2, s_k/2]`` with ``s_k = 2 + 10 k / (K - 1)`` so the
    spread widens from 1e2 to 1e12 over K systems.  The values of every M_k
    are ``G d_k`` (+1e-8 on the diagonal) for a fixed sparse G, so the
    pattern never changes.
    """

    def __init__(self, m: int = 5_200_000, ratio: float = 1.6, c: int = 4, nblocks: int = 256,
                 steps: int = 30, seed: int = 0, model: str = "loc", progress=None):
        say = progress or (lambda msg: None)
        r_pat, r_val, r_d, r_b, _, _ = streams(seed)
        self.m, self.steps, self.nblocks = m, steps, nblocks
        n_a = int(round(ratio * m))
        self.n_a = n_a
        col_ptr, rows = a_pattern(r_pat, m, n_a, c, model)
        say(f"pattern of A: {rows.shape[0]} nonzeros")
        vals = r_val.standard_normal(rows.shape[0])
        A = sp.csc_matrix((vals, rows, col_ptr), shape=(m, n_a))
        # pattern of M (upper triangle incl. diagonal) via a structural product
        M0 = normal_equations(A, np.ones(n_a))
        self.row_ptr = M0.indptr.astype(np.int64)
        self.col = M0.indices.astype(np.int32)
        say(f"pattern of M: {self.col.shape[0]} nonzeros")
        n = m
        nnz = self.col.shape[0]
        rows_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(self.row_ptr))
        # G: for every column k of A and every ordered pair (ra, rb) with
        # ra <= rb of its rows, entry (ra, rb) of M gains A[ra,k] A[rb,k] d_k.
        cnt = np.diff(col_ptr)
        gi, gj, gk, gv = [], [], [], []
        for a in range(int(cnt.max())):
            for bb in range(a, int(cnt.max())):
                sel = np.nonzero(cnt > bb)[0]
                ra = rows[col_ptr[sel] + a]
                rb = rows[col_ptr[sel] + bb]
                gi.append(ra)
                gj.append(rb)
                gk.append(sel)
                gv.append(vals[col_ptr[sel] + a] * vals[col_ptr[sel] + bb])
        ri = np.concatenate(gi)
        rj = np.concatenate(gj)
        key_start = self.row_ptr[ri]
        # position of (ri, rj) inside row ri
        pos = np.empty(ri.shape[0], dtype=np.int64)
        order = np.argsort(ri, kind="stable")
        ri_s, rj_s = ri[order], rj[order]
        starts = self.row_ptr[ri_s]
        # searchsorted within each row: global search on (row * n + col) keys
        keys = rows_of * np.int64(n) + self.col.astype(np.int64)
        pos_s = np.searchsorted(keys, ri_s * np.int64(n) + rj_s)
        pos[order] = pos_s
        del key_start, starts, keys
        self.G = sp.csr_matrix((np.concatenate(gv), (pos, np.concatenate(gk))), shape=(nnz, n_a))
        say(f"value map G: {self.G.nnz} entries")
        self.is_diag = (rows_of == self.col.astype(np.int64))
        # mirror map: lower entries copy their transposed upper entry
        lower = np.nonzero(rows_of > self.col)[0]
        t_keys = self.col[lower].astype(np.int64) * np.int64(n) + rows_of[lower]
        keys = rows_of * np.int64(n) + self.col.astype(np.int64)
        self.lower = lower
        self.lower_src = np.searchsorted(keys, t_keys)
        self.b = r_b.standard_normal(m)
        self.block_ptr = contiguous_blocks(m, nblocks)
        # D sequence
        logd = r_d.uniform(-1.0, 1.0, size=n_a) * math.log(10.0)
        self.d = [np.exp(logd)]
        for k in range(1, steps):
            z = np.log(self.d[-1]) + r_d.normal(0.0, 0.5, size=n_a)
            l10 = z / math.log(10.0)
            s_k = 2.0 + 10.0 * k / (steps - 1)
            lo_, hi_ = l10.min(), l10.max()
            l10 = (l10 - lo_) / (hi_ - lo_) * s_k - s_k / 2.0
            self.d.append(np.power(10.0, l10))

    def values(self, k: int) -> np.ndarray:
        v = self.G @ self.d[k]
        v = v + REG * self.is_diag
        v[self.lower] = v[self.lower_src]
        return v

    def system(self, k: int) -> System:
        return System(name=f"C4[{k}]", row_ptr=self.row_ptr, col=self.col, val=self.values(k),
                      b=self.b, block_ptr=self.block_ptr, meta=dict(step=k, m=self.m))


def c5_requests(count: int = 2000, seed: int = 0, m_lo: int = 10_000, m_hi: int = 500_000):
    """Parameters of a served request stream: per request the row count
    (log-uniform in [m_lo, m_hi]), nonzeros per column of A (6-10), the block
    count (one of 8..128) and a per-request seed.  Systems are built on
    demand with :func:`c5_system`."""
    _, _, _, _, r_blk, _ = streams(seed)
    kids = np.random.SeedSequence(seed).spawn(6 + count)[6:]
    ms = np.round(np.exp(r_blk.uniform(math.log(m_lo), math.log(m_hi), size=count))).astype(np.int64)
    cs = r_blk.integers(6, 11, size=count)
    nbs = r_blk.choice(np.array([8, 16, 32, 64, 128]), size=count)
    return [dict(idx=i, m=int(ms[i]), c=int(cs[i]), nblocks=int(nbs[i]),
                 seed=int(kids[i].generate_state(1)[0])) for i in range(count)]


def c5_system(req: dict) -> System:
    m = req["m"]
    return ada_system(m, int(round(2.5 * m)), req["c"], -4.0, 4.0, req["nblocks"], model="loc",
                      seed=req["seed"], name=f"C5[{req['idx']}]")


def poisson_arrivals(count: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    _, _, _, _, _, r_arr = streams(seed)
    return np.cumsum(r_arr.exponential(1.0 / rate, size=count))


def cache_dir() -> str:
    d = os.environ.get("SDSL_INPUT_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sdsl_inputs"))
    os.makedirs(d, exist_ok=True)
    return d
