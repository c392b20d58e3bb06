"""Python access to the plain-C FP64 oracle (``sdsl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package; the solver library never does.  It shares
no code with the GPU path; both only read the seeded inputs of
``ipm_inputs``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdsl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, INVALID, STRUCTURE, BREAKDOWN, NOT_CONVERGED = 0, 1, 2, 4, 5
PIVOT_FAIL, PIVOT_REPLACE, PIVOT_SHIFT = 0, 1, 2
FILTER_NONE, FILTER_MIN, FILTER_GEOMEAN = 0, 1, 2
DIAG_DELTA, DIAG_DROPSUM = 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
        _lib.or_set_threads(1)
    return _lib


def set_threads(t: int) -> None:
    """Threads of the oracle's row and block loops (results do not depend on
    it: every sum keeps its sequential order)."""
    lib().or_set_threads(int(t))


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
D = C.c_double


def _declare(L):
    L.or_spmv.argtypes = [I64, P, P, P, P, P]
    L.or_lowrank_add.argtypes = [I64, I32, P, P, P, P, P, P]
    L.or_residual.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P]
    L.or_residual.restype = D
    L.or_filter.argtypes = [I64, P, P, P, I32, P, I32, D, C.c_uint32, D, P, P, P, P]
    L.or_filter.restype = I64
    L.or_ilu0.argtypes = [I64, P, P, P, I32, I32, P, P, P]
    L.or_ilu0.restype = C.c_int
    L.or_bj_factor.argtypes = [I64, P, P, P, I32, P, I32, I32, D, P, P, P, P, P]
    L.or_bj_factor.restype = C.c_int
    L.or_lu_solve.argtypes = [I64, I64, P, P, P, P, P, P]
    L.or_bj_apply.argtypes = [I64, P, P, P, P, P, P]
    L.or_dense_lu.argtypes = [I64, P, P]
    L.or_dense_lu.restype = C.c_int
    L.or_dense_lu_solve.argtypes = [I64, P, P, P]
    L.or_bbd_setup.argtypes = [I64, P, P, P, I32, P, I64, I32, D, C.c_uint32, D, I32, I32, P, P]
    L.or_bbd_setup.restype = P
    L.or_bbd_free.argtypes = [P]
    L.or_bbd_apply.argtypes = [P, P, P]
    L.or_bbd_get.argtypes = [P, P, P, P, P, P, P]
    L.or_pcg_bj.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, I32, P, P, P, P, D, I32, P, P, P]
    L.or_pcg_bj.restype = C.c_int
    L.or_gmres_bj.argtypes = [I64, P, P, P, P, P, P, P, I32, P, P, P, D, I32, I32, P, P, P]
    L.or_gmres_bj.restype = C.c_int
    L.or_bicgstab_bj.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, I32, P, P, P, P, D, I32, P, P, P]
    L.or_bicgstab_bj.restype = C.c_int
    L.or_gcr_bj.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, I32, P, P, P, P, D, I32, I32, P, P, P]
    L.or_gcr_bj.restype = C.c_int
    L.or_gcr_bbd.argtypes = [I64, P, P, P, P, P, P, D, I32, I32, P, P, P]
    L.or_gcr_bbd.restype = C.c_int
    L.or_mc64.argtypes = [I64, P, P, P, P, P, P]
    L.or_mc64.restype = C.c_int
    L.or_gmres_bbd.argtypes = [I64, P, P, P, P, P, P, D, I32, I32, P, P, P]
    L.or_gmres_bbd.restype = C.c_int
    L.or_ir_pcg_bj.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, I32, P, P, P, P, D, D, I32, I32,
                               I32, P, P, I32, P, P, P, P]
    L.or_ir_pcg_bj.restype = C.c_int
    L.or_mx_pcg_bj.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, I32, P, P, P, P, D, D, I32, I32,
                               P, P, I32, P, P, P, P]
    L.or_mx_pcg_bj.restype = C.c_int
    L.or_refine_decide.argtypes = [I32, D, D, D, I32, P]
    L.or_refine_decide.restype = C.c_int
    L.or_fallback_decide.argtypes = [D, D, I32, I32]
    L.or_fallback_decide.restype = C.c_int
    L.or_refine_constants.argtypes = [P]
    L.or_border_setup.argtypes = [I64, P, P, P, P, I32, P, I32, P, P, P, P, P]
    L.or_set_threads.argtypes = [I32]
    L.or_border_setup.restype = P
    L.or_border_free.argtypes = [P]
    L.or_border_apply.argtypes = [P, P, P]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _csr(rp, ci, v):
    return (np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(ci, dtype=np.int32),
            np.ascontiguousarray(v, dtype=np.float64))


def spmv(rp, ci, v, x, lowrank=None):
    rp, ci, v = _csr(rp, ci, v)
    n = rp.shape[0] - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n)
    lib().or_spmv(n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    if lowrank is not None:
        U, c = lowrank
        urp, uci, uv = _csr(U.indptr, U.indices, U.data)
        c = np.ascontiguousarray(c, dtype=np.float64)
        lib().or_lowrank_add(n, U.shape[1], _p(urp), _p(uci), _p(uv), _p(c), _p(x), _p(y))
    return y


def residual(rp, ci, v, x, b, lowrank=None):
    """Compensated true residual r = b - M x; returns (r, ||r||_2)."""
    rp, ci, v = _csr(rp, ci, v)
    n = rp.shape[0] - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.empty(n)
    if lowrank is not None:
        U, c = lowrank
        urp, uci, uv = _csr(U.indptr, U.indices, U.data)
        c = np.ascontiguousarray(c, dtype=np.float64)
        nr = lib().or_residual(n, _p(rp), _p(ci), _p(v), U.shape[1], _p(urp), _p(uci), _p(uv),
                               _p(c), _p(x), _p(b), _p(r))
    else:
        nr = lib().or_residual(n, _p(rp), _p(ci), _p(v), 0, None, None, None, None, _p(x),
                               _p(b), _p(r))
    return r, nr


def relres(sys_, x):
    _, nr = residual(sys_.row_ptr, sys_.col, sys_.val, x, sys_.b, sys_.lowrank)
    return nr / float(np.linalg.norm(sys_.b))


def filter_correct(rp, ci, v, block_ptr, mode=FILTER_NONE, tau=0.0, flags=0, delta=0.0, n_int=None):
    """Filtered + corrected block-diagonal matrix P_hat.  Returns
    (p_rp, p_ci, p_v, dropsum)."""
    rp, ci, v = _csr(rp, ci, v)
    bp = np.ascontiguousarray(block_ptr, dtype=np.int32)
    n_int = int(bp[-1]) if n_int is None else n_int
    nnz = int(rp[n_int])
    orp = np.zeros(n_int + 1, dtype=np.int64)
    oci = np.empty(max(nnz, 1), dtype=np.int32)
    ov = np.empty(max(nnz, 1), dtype=np.float64)
    ds = np.empty(max(n_int, 1), dtype=np.float64)
    kept = lib().or_filter(n_int, _p(rp), _p(ci), _p(v), bp.shape[0] - 1, _p(bp), mode, tau, flags,
                           delta, _p(orp), _p(oci), _p(ov), _p(ds))
    if kept < 0:
        raise ValueError("row without a stored diagonal")
    return orp, oci[:kept].copy(), ov[:kept].copy(), ds[:n_int].copy()


def ilu0(rp, ci, v, spd=False, pivot_fix=False):
    """In-place IKJ ILU(0) on a copy.  Returns (values, diag_pos, status,
    pivot fixes, bad row)."""
    rp, ci, v = _csr(rp, ci, v)
    v = v.copy()
    n = rp.shape[0] - 1
    dp = np.empty(max(n, 1), dtype=np.int64)
    nfix = C.c_int32(0)
    bad = C.c_int64(-1)
    st = lib().or_ilu0(n, _p(rp), _p(ci), _p(v), int(spd), int(pivot_fix), _p(dp), C.byref(nfix),
                       C.byref(bad))
    return v, dp[:n].copy(), st, nfix.value, bad.value


def lu_solve(rp, ci, v, dp, r):
    rp, ci, v = _csr(rp, ci, v)
    n = rp.shape[0] - 1
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(n)
    dp = np.ascontiguousarray(dp, dtype=np.int64)
    lib().or_bj_apply(n, _p(rp), _p(ci), _p(v), _p(dp), _p(r), _p(z))
    return z


class BJ:
    """Block-Jacobi preconditioner of paper Sec. 2.3 with the filter and
    correction of Sec. 3.2-3.3: filtered, corrected, ILU(0)-factored blocks.
    ``policy`` handles ILU(0) breakdown (fail / replace the pivot / shift the
    block's diagonal by a relative amount starting at ``shift0``)."""

    def __init__(self, sys_, mode=FILTER_NONE, tau=0.0, flags=0, delta=0.0, spd=True,
                 policy=PIVOT_SHIFT, shift0=1e-2, border=False, complete=False):
        self.rp, self.ci, v0, self.dropsum = filter_correct(sys_.row_ptr, sys_.col, sys_.val,
                                                            sys_.block_ptr, mode, tau, flags, delta)
        n = self.rp.shape[0] - 1
        bp = np.ascontiguousarray(sys_.block_ptr, dtype=np.int32)
        if complete:
            # complete LU without pivoting of each block (Sec. 3.1, Alg. 2):
            # the same elimination over the block's full (dense) pattern
            self.rp, self.ci, v0 = _dense_blocks(self.rp, self.ci, v0, bp)
        self.corrected = v0
        self.bp, self.nb = bp, bp.shape[0] - 1
        self.v = np.empty_like(v0)
        self.dp = np.empty(max(n, 1), dtype=np.int64)
        self.shifts = np.zeros(bp.shape[0] - 1)
        nfix = C.c_int32(0)
        bad = C.c_int64(-1)
        self.status = lib().or_bj_factor(n, _p(self.rp), _p(self.ci), _p(v0), bp.shape[0] - 1, _p(bp),
                                         int(spd), policy, shift0, _p(self.v), _p(self.dp),
                                         _p(self.shifts), C.byref(nfix), C.byref(bad))
        self.dp = self.dp[:n]
        self.nfix, self.bad_row = nfix.value, bad.value
        self.border = None
        if border and sys_.lowrank is not None and self.status == OK:
            U, c = sys_.lowrank
            self._bk = _csr(U.indptr, U.indices, U.data) + (np.ascontiguousarray(c, dtype=np.float64),)
            urp, uci, uv, cc = self._bk
            st = C.c_int32(0)
            self.border = lib().or_border_setup(n, _p(self.rp), _p(self.ci), _p(self.v), _p(self.dp), self.nb,
                                                _p(self.bp), U.shape[1], _p(urp), _p(uci), _p(uv), _p(cc),
                                                C.byref(st))
            self.border_status = st.value

    def apply(self, r):
        if self.border:
            r = np.ascontiguousarray(r, dtype=np.float64)
            z = np.empty(r.shape[0])
            lib().or_border_apply(self.border, _p(r), _p(z))
            return z
        return lu_solve(self.rp, self.ci, self.v, self.dp, r)

    def __del__(self):
        try:
            if getattr(self, "border", None):
                lib().or_border_free(self.border)
                self.border = None
        except Exception:
            pass  # interpreter shutdown


def _dense_blocks(rp, ci, v, bp):
    """Every block of a block-diagonal CSR matrix stored densely (all
    columns of the block in every row, zeros where the matrix has none)."""
    n = rp.shape[0] - 1
    sizes = np.zeros(n, dtype=np.int64)
    for b in range(bp.shape[0] - 1):
        sizes[bp[b]:bp[b + 1]] = bp[b + 1] - bp[b]
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum(sizes)
    ci2 = np.empty(int(rp2[-1]), dtype=np.int32)
    v2 = np.zeros(int(rp2[-1]))
    for b in range(bp.shape[0] - 1):
        lo, hi = int(bp[b]), int(bp[b + 1])
        for i in range(lo, hi):
            ci2[rp2[i]:rp2[i + 1]] = np.arange(lo, hi, dtype=np.int32)
            q = slice(int(rp[i]), int(rp[i + 1]))
            v2[rp2[i] + ci[q].astype(np.int64) - lo] = v[q]
    return rp2, ci2, v2


def _lr_args(lowrank):
    if lowrank is None:
        return 0, None, None, None, None, ()
    U, c = lowrank
    urp, uci, uv = _csr(U.indptr, U.indices, U.data)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return U.shape[1], urp, uci, uv, c, (urp, uci, uv, c)


def pcg_bj(sys_, P: BJ, tol=1e-8, maxit=10_000, hist=False):
    """PCG with the block-Jacobi preconditioner.  Returns (x, iters, relres,
    status, history)."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    k, urp, uci, uv, c, _keep = _lr_args(sys_.lowrank)
    x = np.zeros(n)
    its = C.c_int32(0)
    rr = C.c_double(0.0)
    h = np.zeros(maxit) if hist else None
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    st = lib().or_pcg_bj(n, _p(rp), _p(ci), _p(v), k, _p(urp), _p(uci), _p(uv), _p(c), _p(P.rp),
                         _p(P.ci), _p(P.v), _p(P.dp), P.nb, _p(P.bp), P.border, _p(b), _p(x), tol, maxit, C.byref(its),
                         C.byref(rr), _p(h))
    return x, its.value, rr.value, st, (h[:its.value] if hist else None)


# refinement decisions of the FP32 modes (or_refine_decide)
RF_DONE, RF_CONTINUE, RF_FALLBACK, RF_REVERT, RF_FAIL = range(5)
RF_NAMES = ["done", "continue", "fallback", "revert", "fail"]
HIST_CAP = 256


def refine_decide(mode, nr, prev, tol_nb, breakdown, slow):
    """One refinement-point decision: returns (action, new slow count).
    mode 0 = mixed recurrence, 1 = classical refinement."""
    s = C.c_int32(slow)
    act = lib().or_refine_decide(mode, nr, prev, tol_nb, int(breakdown), C.byref(s))
    return act, s.value


def fallback_decide(nr, tol_nb, st64, nsolves):
    """Decision after an FP64 solve of the residual equation."""
    return lib().or_fallback_decide(nr, tol_nb, st64, nsolves)


def refine_constants():
    """(weak ratio, weak points of the mixed mode, weak steps of classical
    refinement, max fallback solves, fallback tolerance fraction)."""
    out = np.zeros(5)
    lib().or_refine_constants(_p(out))
    return tuple(out)


def _hist_arrays():
    return (np.zeros(HIST_CAP, dtype=np.int32), np.zeros(HIST_CAP), np.zeros(HIST_CAP, dtype=np.int32),
            np.zeros(HIST_CAP, dtype=np.int32))


def _hist_list(n, h):
    it, nr, act, flag = h
    return [dict(it=int(it[e]), nr=float(nr[e]), act=int(act[e]), breakdown=bool(flag[e] & 1),
                 after_fallback=bool(flag[e] & 2)) for e in range(min(n, HIST_CAP))]


def replay_refine(hist, mode, nb, tol, maxit):
    """Re-derive every decision of an FP32-mode history (a list of dicts with
    it, nr, act, breakdown, after_fallback) with the rule alone; raises
    AssertionError at the first decision the rule does not give."""
    slow, prev, nsolves = 0, nb, 0
    for e, h in enumerate(hist):
        if h["after_fallback"]:
            nsolves += 1
            want = fallback_decide(h["nr"], tol * nb, OK, nsolves)
            if h["it"] >= maxit and h["nr"] > tol * nb:
                want = RF_FAIL
            # a FAIL also follows an FP64 solve that did not converge
            assert h["act"] == want or (h["act"] == RF_FAIL and want == RF_FALLBACK), (e, h, want)
            continue
        want, slow = refine_decide(mode, h["nr"], prev, tol * nb, h["breakdown"], slow)
        assert h["act"] == want, (e, h, want)
        prev = h["nr"]


def bicgstab_bj(sys_, P: BJ, tol=1e-8, maxit=10_000, hist=False):
    """Right-preconditioned BiCGSTAB with the block-Jacobi preconditioner.
    Returns (x, iterations, relres, status, history)."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    k, urp, uci, uv, c, _keep = _lr_args(sys_.lowrank)
    x = np.zeros(n)
    its = C.c_int32(0)
    rr = C.c_double(0.0)
    h = np.zeros(maxit) if hist else None
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    st = lib().or_bicgstab_bj(n, _p(rp), _p(ci), _p(v), k, _p(urp), _p(uci), _p(uv), _p(c), _p(P.rp), _p(P.ci),
                              _p(P.v), _p(P.dp), P.nb, _p(P.bp), P.border, _p(b), _p(x), tol, maxit,
                              C.byref(its), C.byref(rr), _p(h))
    return x, its.value, rr.value, st, (h[:its.value] if hist else None)


def gcr_bj(sys_, P: BJ, tol=1e-8, m=30, maxit=10_000, hist=False):
    """Right-preconditioned restarted GCR(m) with the block-Jacobi
    preconditioner.  Returns (x, iterations, relres, status, history)."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    k, urp, uci, uv, c, _keep = _lr_args(sys_.lowrank)
    x = np.zeros(n)
    its = C.c_int32(0)
    rr = C.c_double(0.0)
    h = np.zeros(maxit) if hist else None
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    st = lib().or_gcr_bj(n, _p(rp), _p(ci), _p(v), k, _p(urp), _p(uci), _p(uv), _p(c), _p(P.rp), _p(P.ci),
                         _p(P.v), _p(P.dp), P.nb, _p(P.bp), P.border, _p(b), _p(x), tol, m, maxit,
                         C.byref(its), C.byref(rr), _p(h))
    return x, its.value, rr.value, st, (h[:its.value] if hist else None)


def ir_pcg_bj(sys_, P: BJ, tol=1e-8, inner_tol=1e-4, max_outer=30, maxit=10_000, every=500, with_history=False):
    """FP32-inner PCG inside FP64 iterative refinement (each inner solve to
    inner_tol or for at most `every` iterations).  Returns (x, outer, inner
    total, fp64 fallbacks, relres, status) and, with_history, the list of
    decisions taken."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    k, urp, uci, uv, c, _keep = _lr_args(sys_.lowrank)
    x = np.zeros(n)
    out = np.zeros(4, dtype=np.int32)
    rr = C.c_double(0.0)
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    h = _hist_arrays()
    st = lib().or_ir_pcg_bj(n, _p(rp), _p(ci), _p(v), k, _p(urp), _p(uci), _p(uv), _p(c), _p(P.rp),
                            _p(P.ci), _p(P.v), _p(P.dp), P.nb, _p(P.bp), P.border, _p(b), _p(x), tol, inner_tol, max_outer,
                            every, maxit, _p(out), C.byref(rr), HIST_CAP, *[_p(a) for a in h])
    res = (x, int(out[0]), int(out[1]), int(out[2]), rr.value, st)
    return res + (_hist_list(int(out[3]), h),) if with_history else res


def mx_pcg_bj(sys_, P: BJ, tol=1e-8, delta=0.1, every=500, maxit=100_000, with_history=False):
    """PCG with FP32 SpMV / preconditioner apply inside FP64 refinement.
    Returns (x, refinement points, iterations, fp64 fallbacks, relres,
    status) and, with_history, the list of decisions taken."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    k, urp, uci, uv, c, _keep = _lr_args(sys_.lowrank)
    x = np.zeros(n)
    out = np.zeros(4, dtype=np.int32)
    rr = C.c_double(0.0)
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    h = _hist_arrays()
    st = lib().or_mx_pcg_bj(n, _p(rp), _p(ci), _p(v), k, _p(urp), _p(uci), _p(uv), _p(c), _p(P.rp),
                            _p(P.ci), _p(P.v), _p(P.dp), P.nb, _p(P.bp), P.border, _p(b), _p(x), tol, delta, every, maxit,
                            _p(out), C.byref(rr), HIST_CAP, *[_p(a) for a in h])
    res = (x, int(out[0]), int(out[1]), int(out[2]), rr.value, st)
    return res + (_hist_list(int(out[3]), h),) if with_history else res


def gmres_bj(sys_, P: BJ, tol=1e-8, m=30, maxit=10_000, hist=False):
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    x = np.zeros(n)
    its = C.c_int32(0)
    rr = C.c_double(0.0)
    h = np.zeros(maxit) if hist else None
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    st = lib().or_gmres_bj(n, _p(rp), _p(ci), _p(v), _p(P.rp), _p(P.ci), _p(P.v), _p(P.dp), P.nb, _p(P.bp),
                           _p(b), _p(x), tol, m, maxit, C.byref(its), C.byref(rr), _p(h))
    return x, its.value, rr.value, st, (h[:its.value] if hist else None)


class BBD:
    """Bordered-block-diagonal preconditioner of paper Sec. 2.4."""

    def __init__(self, sys_, mode=FILTER_NONE, tau=0.0, flags=0, delta=0.0, pivot_fix=False, complete=False):
        self.rp, self.ci, self.v = _csr(sys_.row_ptr, sys_.col, sys_.val)
        self.bp = np.ascontiguousarray(sys_.block_ptr, dtype=np.int32)
        self.n = sys_.n
        self.n_border = sys_.n_border
        st = C.c_int32(0)
        info = np.zeros(3, dtype=np.int64)
        self.ctx = lib().or_bbd_setup(self.n, _p(self.rp), _p(self.ci), _p(self.v),
                                      self.bp.shape[0] - 1, _p(self.bp), self.n_border, mode, tau,
                                      flags, delta, int(pivot_fix), int(complete), C.byref(st), _p(info))
        self.status = st.value
        self.kept, self.nfix, self.bad_row = (int(t) for t in info)

    def apply(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty(self.n)
        lib().or_bbd_apply(self.ctx, _p(r), _p(z))
        return z

    def parts(self):
        nb = self.bp.shape[0] - 1
        n_int = self.n - self.n_border
        tail = np.empty(nb, dtype=np.int64)
        lrp = np.empty(n_int + 1, dtype=np.int64)
        lib().or_bbd_get(self.ctx, _p(tail), _p(lrp), None, None, None, None)
        lci = np.empty(int(lrp[-1]), dtype=np.int32)
        lv = np.empty(int(lrp[-1]))
        S = np.empty((self.n_border, self.n_border))
        piv = np.empty(self.n_border, dtype=np.int32)
        lib().or_bbd_get(self.ctx, None, None, _p(lci), _p(lv), _p(S), _p(piv))
        return dict(tail=tail, lrp=lrp, lci=lci, lv=lv, S=S, piv=piv)

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().or_bbd_free(self.ctx)
                self.ctx = None
        except Exception:
            pass  # interpreter shutdown


def gmres_bbd(sys_, P: BBD, tol=1e-8, m=30, maxit=10_000, hist=False):
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    x = np.zeros(n)
    its = C.c_int32(0)
    rr = C.c_double(0.0)
    h = np.zeros(maxit) if hist else None
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    st = lib().or_gmres_bbd(n, _p(rp), _p(ci), _p(v), P.ctx, _p(b), _p(x), tol, m, maxit,
                            C.byref(its), C.byref(rr), _p(h))
    return x, its.value, rr.value, st, (h[:its.value] if hist else None)


def gcr_bbd(sys_, P: BBD, tol=1e-8, m=30, maxit=10_000, hist=False):
    """Right-preconditioned restarted GCR(m) with the BBD preconditioner."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    x = np.zeros(n)
    its = C.c_int32(0)
    rr = C.c_double(0.0)
    h = np.zeros(maxit) if hist else None
    b = np.ascontiguousarray(sys_.b, dtype=np.float64)
    st = lib().or_gcr_bbd(n, _p(rp), _p(ci), _p(v), P.ctx, _p(b), _p(x), tol, m, maxit,
                          C.byref(its), C.byref(rr), _p(h))
    return x, its.value, rr.value, st, (h[:its.value] if hist else None)


def dense_lu(a):
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    n = a.shape[0]
    piv = np.empty(n, dtype=np.int32)
    st = lib().or_dense_lu(n, _p(a), _p(piv))
    return a, piv, st


def dense_lu_solve(lu, piv, b):
    b = np.ascontiguousarray(b, dtype=np.float64).copy()
    lib().or_dense_lu_solve(lu.shape[0], _p(np.ascontiguousarray(lu)), _p(piv), _p(b))
    return b


def mc64(sys_):
    """MC64 maximum-product matching and scaling (Sec. 3.3, Alg. 3 step 1).
    Returns (match, dr, dc, status): row i is matched to column match[i];
    |dr_i a_ij dc_j| <= 1 with equality on the matching."""
    rp, ci, v = _csr(sys_.row_ptr, sys_.col, sys_.val)
    n = sys_.n
    match = np.empty(n, dtype=np.int32)
    dr = np.empty(n)
    dc = np.empty(n)
    st = lib().or_mc64(n, _p(rp), _p(ci), _p(v), _p(match), _p(dr), _p(dc))
    return match, dr, dc, st


def mc64_transform(sys_, match, dr, dc, spd=False):
    """The system Alg. 3 hands to the preconditioner and the Krylov method:
    A' = Q Dr A Dc, row i moved to position match[i], with right-hand side
    b' = Q Dr b and x = Dc y.  spd: the symmetric form S A S with
    s = sqrt(dr dc) (the matching of a symmetric positive definite matrix is
    the identity), b' = S b and x = S y.  Returns (System A', x_of_y)."""
    import scipy.sparse as sp
    M = sp.csr_matrix((np.asarray(sys_.val, dtype=np.float64), np.asarray(sys_.col),
                       np.asarray(sys_.row_ptr)), shape=(sys_.n, sys_.n))
    b = np.asarray(sys_.b, dtype=np.float64)
    if spd:
        if not np.array_equal(match, np.arange(sys_.n)):
            raise ValueError("a symmetric positive definite matrix matches every row to its own column")
        s = np.sqrt(dr * dc)
        A2 = (sp.diags(s) @ M @ sp.diags(s)).tocsr()
        b2 = s * b
        x_of = (lambda y, s=s: s * np.asarray(y))
    else:
        Q = sp.csr_matrix((np.ones(sys_.n), (match, np.arange(sys_.n))), shape=(sys_.n, sys_.n))
        A2 = (Q @ sp.diags(dr) @ M @ sp.diags(dc)).tocsr()
        b2 = np.empty(sys_.n)
        b2[match] = dr * b
        x_of = (lambda y, dc=dc: dc * np.asarray(y))
    A2.sort_indices()
    out = type(sys_)(sys_.name + "-mc64", A2.indptr.astype(np.int64), A2.indices.astype(np.int32), A2.data, b2,
                     sys_.block_ptr, n_border=getattr(sys_, "n_border", 0))
    return out, x_of

