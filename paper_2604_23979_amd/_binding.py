"""ctypes binding of libsdsl.so (the C ABI declared in include/sdsl.h).

Argument marshalling only: every numerical step runs in the library's gfx950
kernels.  Device memory and streams come from PyTorch.  There is no fallback:
if the library is missing, importing the solver raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import dataclasses
import os
import weakref
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdsl.so")

OK, E_INVALID, E_STRUCTURE, E_NOMEM, E_BREAKDOWN, E_NOT_CONVERGED, E_DEVICE, E_STATE = range(8)
STATUS_NAMES = ["OK", "E_INVALID", "E_STRUCTURE", "E_NOMEM", "E_BREAKDOWN", "E_NOT_CONVERGED", "E_DEVICE",
                "E_STATE"]
BJ, BBD = 0, 1
FILTER_NONE, FILTER_MIN, FILTER_GEOMEAN = 0, 1, 2
DIAG_DELTA, DIAG_DROPSUM = 1, 2
PIVOT_FAIL, PIVOT_REPLACE, PIVOT_SHIFT = 0, 1, 2
PCG, GMRES, BICGSTAB, GCR = 0, 1, 2, 3
FACT_ILU0, FACT_COMPLETE = 0, 1
FP64, FP32_IR, FP32_IR_RESTART = 0, 1, 2
MEM_DEVICE, MEM_HOST = 0, 1


class SdslError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


class CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("mem", C.c_int)]


class Partition(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("block_ptr", C.c_void_p), ("n_border", C.c_int32)]


class LowRank(C.Structure):
    _fields_ = [("k", C.c_int32), ("U", CSR), ("c", C.c_void_p)]


class COptions(C.Structure):
    _fields_ = [("method", C.c_int), ("filter", C.c_int), ("tau", C.c_double), ("diag_flags", C.c_uint32),
                ("delta", C.c_double), ("pivot", C.c_int), ("shift0", C.c_double), ("spd", C.c_int32),
                ("krylov", C.c_int), ("restart", C.c_int32), ("max_iter", C.c_int32), ("precision", C.c_int),
                ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("check_every", C.c_int32),
                ("kernel_timing", C.c_int32), ("border", C.c_int32), ("refine_delta", C.c_double),
                ("refine_every", C.c_int32), ("mc64", C.c_int32), ("factor", C.c_int), ("graphs", C.c_int32)]


class CInfo(C.Structure):
    _fields_ = [("nnz_kept", C.c_int64), ("nnz_dropped", C.c_int64), ("pivot_fixes", C.c_int32),
                ("shifted_blocks", C.c_int32), ("max_shift", C.c_double), ("outer_iters", C.c_int32),
                ("inner_iters", C.c_int32), ("fp64_fallbacks", C.c_int32), ("restarts", C.c_int32),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("relres", C.c_double),
                ("bytes_per_iter", C.c_int64), ("device_bytes", C.c_int64), ("spmv_ms", C.c_double * 2),
                ("spmv_launches", C.c_int64 * 2), ("bj_ms", C.c_double * 2), ("bj_launches", C.c_int64 * 2),
                ("spmv_bytes", C.c_int64 * 2), ("bj_bytes", C.c_int64 * 2), ("rf_count", C.c_int32),
                ("rf_it", C.c_int32 * 64), ("rf_nr", C.c_double * 64), ("rf_act", C.c_int32 * 64),
                ("rf_flag", C.c_int32 * 64), ("rf_nb", C.c_double), ("mc64_moved", C.c_int32),
                ("sweep_levels_max", C.c_int32), ("sweep_levels_mean", C.c_double)]


class Allocator(C.Structure):
    pass


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
Allocator._fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None


def _torch_free(ptr, nbytes, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass  # interpreter shutdown: the process returns the memory


_TORCH_ALLOC = None
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_solvers():
    """Handles still open at exit are destroyed while PyTorch (which may own
    their memory) is still alive."""
    for s in list(_LIVE):
        try:
            s.close()
        except Exception:
            pass


def torch_allocator() -> Allocator:
    """The sdsl_allocator that serves handles from PyTorch's caching
    allocator (kept alive for the life of the process)."""
    global _TORCH_ALLOC
    if _TORCH_ALLOC is None:
        _TORCH_ALLOC = Allocator(ALLOC_FN(_torch_alloc), FREE_FN(_torch_free), None)
    return _TORCH_ALLOC


class CGroupStats(C.Structure):
    _fields_ = [("flushes", C.c_int64), ("slot_issues", C.c_int64), ("launches", C.c_int64),
                ("graph_launches", C.c_int64), ("captures", C.c_int64)]


# every symbol the header declares, with its ctypes signature
H = C.c_void_p
P = C.c_void_p
SIGNATURES = {
    "sdsl_default_options": (None, [C.POINTER(COptions)]),
    "sdsl_footprint_bytes": (C.c_size_t, [C.POINTER(CSR), C.POINTER(Partition), C.POINTER(COptions),
                                          C.POINTER(LowRank)]),
    "sdsl_setup": (C.c_int, [C.POINTER(CSR), C.POINTER(Partition), C.POINTER(COptions), C.POINTER(LowRank),
                             C.POINTER(Allocator), P, C.POINTER(H)]),
    "sdsl_refactor": (C.c_int, [H, P]),
    "sdsl_update_values": (C.c_int, [H, P]),
    "sdsl_set_max_iter": (C.c_int, [H, C.c_int32]),
    "sdsl_solve": (C.c_int, [H, P, P, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "sdsl_solve_batch": (C.c_int, [C.c_int32, P, P, P, C.c_double, P, P]),
    "sdsl_get_info": (C.c_int, [H, C.POINTER(CInfo)]),
    "sdsl_last_error": (C.c_char_p, [H]),
    "sdsl_destroy": (None, [H]),
    "sdsl_spmv": (C.c_int, [H, C.c_int32, P, P]),
    "sdsl_precond_apply": (C.c_int, [H, C.c_int32, P, P]),
    "sdsl_residual": (C.c_int, [H, P, P, P, C.POINTER(C.c_double)]),
    "sdsl_residual_noalloc": (C.c_int, [H, P, P, P, C.POINTER(C.c_double)]),
    "sdsl_get_factors": (C.c_int, [H, P, P, P, P, P]),
    "sdsl_get_schur": (C.c_int, [H, P, P, P]),
    "sdsl_get_mc64": (C.c_int, [H, P, P, P]),
    "sdsl_solve_begin": (C.c_int, [H, P, P, C.c_double]),
    "sdsl_solve_step": (C.c_int, [H, P]),
    "sdsl_solve_end": (C.c_int, [H, P, P]),
    "sdsl_group_create": (C.c_int, [P, C.c_int32, C.POINTER(Allocator), C.POINTER(H)]),
    "sdsl_group_begin": (C.c_int, [H, H, P, P, C.c_double]),
    "sdsl_group_step": (C.c_int, [H, C.c_int32, P, P]),
    "sdsl_group_get_stats": (C.c_int, [H, C.POINTER(CGroupStats)]),
    "sdsl_group_destroy": (None, [H]),
}

_lib = None


def lib():
    """Load libsdsl.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2604_23979_amd.build` first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


@dataclasses.dataclass
class Options:
    method: int = BJ
    filter: int = FILTER_NONE
    tau: float = 0.0
    diag_flags: int = 0
    delta: float = 0.0
    pivot: int = PIVOT_SHIFT
    shift0: float = 1e-2
    spd: bool = True
    krylov: int = PCG
    restart: int = 30
    max_iter: int = 100000
    precision: int = FP64
    inner_tol: float = 1e-4
    max_outer: int = 30
    check_every: int = 16
    kernel_timing: int = 0
    border: bool = True
    refine_delta: float = 0.1
    refine_every: int = 500
    mc64: bool = False
    factor: int = 0  # FACT_ILU0 or FACT_COMPLETE
    graphs: bool = False

    def c(self) -> COptions:
        o = COptions()
        for f in dataclasses.fields(self):
            setattr(o, f.name, int(getattr(self, f.name)) if isinstance(getattr(self, f.name), bool)
                    else getattr(self, f.name))
        return o


def _check(h, st):
    if st != OK:
        msg = lib().sdsl_last_error(h)
        raise SdslError(st, msg.decode() if msg else "")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


class Solver:
    """A resident preconditioned solver for one sparsity pattern.

    ``row_ptr``/``col``/``val`` are numpy arrays (copied from host memory) or
    torch CUDA tensors (int64 / int32 / float64, copied device to device).
    ``block_ptr`` is a host int array of contiguous row blocks.  With
    ``torch_memory`` the handle's device memory comes from PyTorch's caching
    allocator (sdsl_allocator), otherwise from hipMalloc."""

    def __init__(self, row_ptr, col, val, block_ptr, n_border: int = 0, lowrank=None,
                 options: Optional[Options] = None, stream=None, torch_memory: bool = True):
        import torch
        self.options = options or Options()
        self._keep = []
        on_dev = isinstance(val, torch.Tensor)
        if on_dev:
            row_ptr = row_ptr.to(torch.int64).contiguous()
            col = col.to(torch.int32).contiguous()
            val = val.to(torch.float64).contiguous()
            ptrs = [C.c_void_p(t.data_ptr()) for t in (row_ptr, col, val)]
            n = row_ptr.numel() - 1
            nnz = col.numel()
            self._keep += [row_ptr, col, val]
        else:
            row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            val = np.ascontiguousarray(val, dtype=np.float64)
            ptrs = [a.ctypes.data_as(C.c_void_p) for a in (row_ptr, col, val)]
            n = row_ptr.shape[0] - 1
            nnz = col.shape[0]
            self._keep += [row_ptr, col, val]
        A = CSR(n, nnz, ptrs[0], ptrs[1], ptrs[2], MEM_DEVICE if on_dev else MEM_HOST)
        bp = np.ascontiguousarray(block_ptr, dtype=np.int32)
        self._keep.append(bp)
        part = Partition(bp.shape[0] - 1, bp.ctypes.data_as(C.c_void_p), int(n_border))
        lrp = None
        if lowrank is not None:
            U, cvec = lowrank
            urp = np.ascontiguousarray(U.indptr, dtype=np.int64)
            uci = np.ascontiguousarray(U.indices, dtype=np.int32)
            uv = np.ascontiguousarray(U.data, dtype=np.float64)
            cc = np.ascontiguousarray(cvec, dtype=np.float64)
            self._keep += [urp, uci, uv, cc]
            lrp = LowRank(U.shape[1], CSR(n, uv.shape[0], urp.ctypes.data_as(C.c_void_p),
                                          uci.ctypes.data_as(C.c_void_p), uv.ctypes.data_as(C.c_void_p),
                                          MEM_HOST), cc.ctypes.data_as(C.c_void_p))
        self.n, self.nnz, self.nblocks, self.n_border = n, nnz, bp.shape[0] - 1, int(n_border)
        self.stream = stream
        self._opts = self.options.c()
        h = C.c_void_p()
        self._alloc = torch_allocator() if torch_memory else None
        st = lib().sdsl_setup(C.byref(A), C.byref(part), C.byref(self._opts),
                              C.byref(lrp) if lrp is not None else None,
                              C.byref(self._alloc) if self._alloc is not None else None, _stream_ptr(stream),
                              C.byref(h))
        self._keep = []
        if st != OK:
            msg = lib().sdsl_last_error(None)
            raise SdslError(st, msg.decode() if msg else "")
        self.h = h
        _LIVE.add(self)

    # -- solves
    def solve(self, b, x=None, tol: float = 1e-8, check: bool = True, log=None, extra: Optional[dict] = None):
        """Solve M x = b (b: CUDA float64 tensor).  Returns (x, iters, relres, status).
        With ``log`` (a solvelog.JsonlLog) one record of the solve is written,
        with ``extra`` fields added."""
        import torch
        assert b.is_cuda and b.dtype == torch.float64 and b.numel() == self.n
        b = b.contiguous()
        self._order()
        if x is None:
            x = torch.empty_like(b)
        its = C.c_int32(0)
        rr = C.c_double(0.0)
        st = lib().sdsl_solve(self.h, _dptr(b), _dptr(x), tol, C.byref(its), C.byref(rr))
        if check and st not in (OK, E_NOT_CONVERGED, E_BREAKDOWN):
            _check(self.h, st)
        if log is not None:
            from .solvelog import record
            log.write(record(self, st, dict(extra or {}, tol=tol)))
        return x, its.value, rr.value, st

    # -- asynchronous solve (serving loops)
    def solve_begin(self, b, x, tol: float = 1e-8):
        """Start M x = b without waiting; b and x (CUDA float64) must stay
        alive until solve_end."""
        import torch
        assert b.is_cuda and b.dtype == torch.float64 and b.numel() == self.n and x.numel() == self.n
        self._order()
        self._async = (b, x)
        _check(self.h, lib().sdsl_solve_begin(self.h, _dptr(b), _dptr(x), tol))

    def solve_step(self) -> bool:
        """Advance the running solve if its stream is idle; True once done."""
        done = C.c_int32(0)
        _check(self.h, lib().sdsl_solve_step(self.h, C.byref(done)))
        return bool(done.value)

    def solve_end(self):
        """(x, iters, relres, status) of the finished solve."""
        its = C.c_int32(0)
        rr = C.c_double(0.0)
        st = lib().sdsl_solve_end(self.h, C.byref(its), C.byref(rr))
        if st not in (OK, E_NOT_CONVERGED, E_BREAKDOWN):
            _check(self.h, st)
        x = self._async[1]
        self._async = None
        return x, its.value, rr.value, st

    def _order(self):
        """Work on torch's current stream must be finished before a handle
        on another stream reads it."""
        if self.stream is not None:
            import torch
            torch.cuda.current_stream().synchronize()

    def refactor(self, vals):
        self._order()
        _check(self.h, lib().sdsl_refactor(self.h, _dptr(vals.contiguous())))

    def update_values(self, vals):
        self._order()
        _check(self.h, lib().sdsl_update_values(self.h, _dptr(vals.contiguous())))

    def set_max_iter(self, max_iter: int):
        _check(self.h, lib().sdsl_set_max_iter(self.h, int(max_iter)))

    # -- single steps
    def spmv(self, x, fp32: bool = False):
        import torch
        y = torch.empty_like(x)
        _check(self.h, lib().sdsl_spmv(self.h, FP32_IR if fp32 else FP64, _dptr(x), _dptr(y)))
        return y

    def precond_apply(self, r, fp32: bool = False):
        import torch
        z = torch.empty_like(r)
        _check(self.h, lib().sdsl_precond_apply(self.h, FP32_IR if fp32 else FP64, _dptr(r), _dptr(z)))
        return z

    def residual(self, b, x):
        import torch
        r = torch.empty_like(b)
        nr = C.c_double(0.0)
        _check(self.h, lib().sdsl_residual(self.h, _dptr(b), _dptr(x), _dptr(r), C.byref(nr)))
        return r, nr.value

    def residual_noalloc(self, b, x, r):
        """sdsl_residual_noalloc: r = b - M x into the caller's r (the library
        allocates nothing); returns ||r||."""
        nr = C.c_double(0.0)
        _check(self.h, lib().sdsl_residual_noalloc(self.h, _dptr(b), _dptr(x), _dptr(r), C.byref(nr)))
        return nr.value

    def factors(self):
        info = self.info()
        kept = int(info["nnz_kept"])
        rp = np.zeros(self.n + 1, dtype=np.int64)   # the first n - n_border + 1 are filled
        ci = np.zeros(max(kept, 1), dtype=np.int32)
        corr = np.zeros(max(kept, 1))
        lu = np.zeros(max(kept, 1))
        sh = np.zeros(self.nblocks)
        _check(self.h, lib().sdsl_get_factors(self.h, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                                              corr.ctypes.data_as(C.c_void_p), lu.ctypes.data_as(C.c_void_p),
                                              sh.ctypes.data_as(C.c_void_p)))
        return dict(row_ptr=rp, col=ci[:kept], corrected=corr[:kept], lu=lu[:kept], shifts=sh)

    def schur(self):
        """BBD handles: the border Schur complement's LU (row-major), pivot
        rows and inverse, as numpy arrays."""
        m = self.n_border
        lu = np.zeros((m, m))
        piv = np.zeros(m, dtype=np.int32)
        inv = np.zeros((m, m))
        _check(self.h, lib().sdsl_get_schur(self.h, lu.ctypes.data_as(C.c_void_p), piv.ctypes.data_as(C.c_void_p),
                                            inv.ctypes.data_as(C.c_void_p)))
        return lu, piv, inv

    def mc64(self):
        """(row_of, row_scale, col_scale) of a handle set up with mc64: row k
        of A' is row row_of[k] of A, scaled by row_scale of that row; column
        j is scaled by col_scale[j]."""
        row_of = np.empty(self.n, dtype=np.int32)
        dr = np.empty(self.n)
        dc = np.empty(self.n)
        _check(self.h, lib().sdsl_get_mc64(self.h, row_of.ctypes.data_as(C.c_void_p), dr.ctypes.data_as(C.c_void_p),
                                           dc.ctypes.data_as(C.c_void_p)))
        return row_of, dr, dc

    def info(self) -> dict:
        inf = CInfo()
        _check(self.h, lib().sdsl_get_info(self.h, C.byref(inf)))
        out = {}
        for f, _ in CInfo._fields_:
            v = getattr(inf, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out

    def rf_history(self) -> list:
        """Decisions of the last FP32-mode solve: dicts with it, nr, act,
        breakdown, after_fallback (see sdsl_info.rf_*)."""
        inf = CInfo()
        _check(self.h, lib().sdsl_get_info(self.h, C.byref(inf)))
        return [dict(it=int(inf.rf_it[e]), nr=float(inf.rf_nr[e]), act=int(inf.rf_act[e]),
                     breakdown=bool(inf.rf_flag[e] & 1), after_fallback=bool(inf.rf_flag[e] & 2))
                for e in range(min(int(inf.rf_count), 64))]

    def close(self):
        if getattr(self, "h", None):
            lib().sdsl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Shared launches for the running solves of several Solvers set up on
    one stream (sdsl_group_*): each PCG iteration of all of them is one
    launch per kernel, optionally replayed from a HIP graph.  Each solve's
    result is bitwise the one Solver.solve gives."""

    def __init__(self, stream=None, graphs: bool = True, torch_memory: bool = True):
        self.stream = stream
        self._alloc = torch_allocator() if torch_memory else None
        g = C.c_void_p()
        st = lib().sdsl_group_create(_stream_ptr(stream), int(graphs),
                                     C.byref(self._alloc) if self._alloc is not None else None, C.byref(g))
        if st != OK:
            msg = lib().sdsl_last_error(None)
            raise SdslError(st, msg.decode() if msg else "")
        self.g = g
        _LIVE.add(self)

    def begin(self, solver: "Solver", b, x, tol: float = 1e-8):
        """Start M x = b on solver; its first iterations go out with the next
        step.  b and x (CUDA float64) must stay alive until solve_end."""
        import torch
        assert b.is_cuda and b.dtype == torch.float64 and b.numel() == solver.n and x.numel() == solver.n
        solver._order()
        solver._async = (b, x)
        _check(solver.h, lib().sdsl_group_begin(self.g, solver.h, _dptr(b), _dptr(x), tol))

    def step(self, solvers) -> list:
        """Advance every listed solve once (waiting for its last iterations)
        and launch the collected iterations together; True where done."""
        k = len(solvers)
        hs = (C.c_void_p * max(k, 1))(*[s.h for s in solvers])
        done = np.zeros(max(k, 1), dtype=np.int32)
        st = lib().sdsl_group_step(self.g, k, hs, done.ctypes.data_as(C.c_void_p))
        if st != OK:
            for s in solvers:
                msg = lib().sdsl_last_error(s.h)
                if msg:
                    raise SdslError(st, msg.decode())
            _check(None, st)
        return [bool(d) for d in done[:k]]

    def stats(self) -> dict:
        s = CGroupStats()
        _check(None, lib().sdsl_group_get_stats(self.g, C.byref(s)))
        return {f: int(getattr(s, f)) for f, _ in CGroupStats._fields_}

    def close(self):
        if getattr(self, "g", None):
            lib().sdsl_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers, bs, xs, tol: float = 1e-8):
    """Solve several systems with interleaved launches (one per solver)."""
    k = len(solvers)
    hs = (C.c_void_p * k)(*[s.h for s in solvers])
    bp = (C.c_void_p * k)(*[b.data_ptr() for b in bs])
    xp = (C.c_void_p * k)(*[x.data_ptr() for x in xs])
    its = np.zeros(k, dtype=np.int32)
    rr = np.zeros(k)
    st = lib().sdsl_solve_batch(k, hs, bp, xp, tol, its.ctypes.data_as(C.c_void_p), rr.ctypes.data_as(C.c_void_p))
    return its, rr, st
