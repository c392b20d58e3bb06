"""Serving loop: IPM solve requests arriving over time share the GPU.

Continuous batching: a request is admitted as soon as it has arrived, a slot
is free and its predicted device footprint (``sdsl_footprint_bytes``) fits
the free HBM (or an artificial budget); every admitted request gets a
resident preconditioner, and new requests join while others are still
iterating.  A finished request releases its slot and memory at once.

Shared mode (the default): every request's handle lives on one stream and a
``Group`` advances them together, so each PCG iteration of all running
requests is one launch per kernel (replayed from a HIP graph once a shape
repeats); each result is bitwise the one a solve alone gives.  Stream mode:
one stream per request, advanced with the non-blocking ``sdsl_solve_step``,
so the requests' kernels overlap only as far as the hardware queues allow.
Latency counts from arrival to completion (queueing, setup and solve)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import time
from collections import deque
from typing import Optional

import numpy as np

from . import _binding as B


@dataclasses.dataclass
class Request:
    system: object               # row_ptr, col, val, block_ptr, b (, n_border, lowrank)
    arrival: float = 0.0         # seconds after the start of the run
    tag: object = None
    # filled in by the server
    x: object = None
    iters: int = 0
    relres: float = float("nan")
    status: int = -1
    admitted: float = float("nan")
    finished: float = float("nan")

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint(system, options: B.Options) -> int:
    """Device bytes a handle for this system is predicted to hold."""
    rp = np.ascontiguousarray(system.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(system.col, dtype=np.int32)   # read for BBD (tail factors)
    A = B.CSR(rp.shape[0] - 1, int(rp[-1]), rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p), None,
              B.MEM_HOST)
    bp = np.ascontiguousarray(system.block_ptr, dtype=np.int32)
    part = B.Partition(bp.shape[0] - 1, bp.ctypes.data_as(C.c_void_p), int(getattr(system, "n_border", 0)))
    o = options.c()
    lr = None
    low = getattr(system, "lowrank", None)
    if low is not None:
        # only the sizes are read: k, nnz(U), n
        U = low[0]
        urp = np.ascontiguousarray(U.indptr, dtype=np.int64)
        lr = B.LowRank(U.shape[1], B.CSR(rp.shape[0] - 1, int(U.nnz), urp.ctypes.data_as(C.c_void_p), None, None,
                                         B.MEM_HOST), None)
    return int(B.lib().sdsl_footprint_bytes(C.byref(A), C.byref(part), C.byref(o),
                                            C.byref(lr) if lr is not None else None))


class Server:
    """Runs a list of requests to completion; ``stats()`` summarises."""

    def __init__(self, options: Optional[B.Options] = None, tol: float = 1e-8, max_active: int = 8,
                 budget_bytes: Optional[int] = None, reserve_bytes: int = 1 << 30, shared: bool = True,
                 graphs: bool = True, on_done=None, log=None):
        self.options = options or B.Options(precision=B.FP32_IR)
        self.tol = tol
        self.max_active = max_active
        self.shared = shared
        self.graphs = graphs
        self.on_done = on_done      # called with each finished Request
        self.log = log              # solvelog.JsonlLog: one record per finished request
        self.group_stats = None
        self.budget = budget_bytes
        self.reserve = reserve_bytes
        self.done: list[Request] = []
        self.t_start = 0.0
        self.t_end = 0.0
        self.max_concurrency = 0
        self.waited_for_memory = 0

    def _free_bytes(self, used: int) -> int:
        import torch
        free, _ = torch.cuda.mem_get_info()
        # handles come from torch's caching allocator: blocks it has cached
        # but not handed out are free for the next handle too
        free += torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
        avail = free - self.reserve
        if self.budget is not None:
            avail = min(avail, self.budget - used)
        return avail

    def _log(self, req: Request, solver) -> None:
        if self.log is None:
            return
        from .solvelog import record
        self.log.write(record(solver, req.status, {"request": req.tag, "arrival_s": req.arrival,
                                                   "admitted_s": req.admitted, "finished_s": req.finished,
                                                   "latency_s": req.latency, "tol": self.tol,
                                                   "shared_launches": self.shared}))

    def run(self, requests: list[Request]) -> list[Request]:
        if self.shared:
            return self._run_shared(requests)
        return self._run_streams(requests)

    def _admit(self, pending, active, used, now):
        """Requests that may start now (arrived, a slot and memory free)."""
        out = []
        while pending and pending[0].arrival <= now and len(active) + len(out) < self.max_active:
            req = pending[0]
            need = footprint(req.system, self.options)
            if need > self._free_bytes(used):
                if active or out:
                    self.waited_for_memory += 1
                    break          # wait until a running request frees memory
                raise MemoryError(f"request {req.tag} needs {need} bytes, more than the device can give")
            pending.popleft()
            out.append((req, need))
            used += need
        return out, used

    def _run_shared(self, requests: list[Request]) -> list[Request]:
        import torch
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        stream = torch.cuda.Stream()
        group = B.Group(stream, graphs=self.graphs)
        active = []      # (request, solver, b, bytes)
        used = 0
        self.t_start = time.perf_counter()
        try:
            while pending or active:
                now = time.perf_counter() - self.t_start
                admit, used = self._admit(pending, active, used, now)
                for req, need in admit:
                    with torch.cuda.stream(stream):
                        b = torch.as_tensor(np.ascontiguousarray(req.system.b), device="cuda:0")
                        x = torch.empty_like(b)
                    solver = B.Solver(req.system.row_ptr, req.system.col, req.system.val, req.system.block_ptr,
                                      n_border=getattr(req.system, "n_border", 0),
                                      lowrank=getattr(req.system, "lowrank", None), options=self.options,
                                      stream=stream)
                    group.begin(solver, b, x, self.tol)
                    req.admitted = time.perf_counter() - self.t_start
                    active.append((req, solver, b, need))
                    self.max_concurrency = max(self.max_concurrency, len(active))
                if active:
                    done = group.step([a[1] for a in active])
                    still = []
                    for item, d in zip(active, done):
                        req, solver, b, need = item
                        if d:
                            req.x, req.iters, req.relres, req.status = solver.solve_end()
                            req.finished = time.perf_counter() - self.t_start
                            self._log(req, solver)
                            solver.close()
                            used -= need
                            self.done.append(req)
                            if self.on_done:
                                self.on_done(req)
                        else:
                            still.append(item)
                    active = still
                elif pending and pending[0].arrival > now:
                    time.sleep(min(0.001, pending[0].arrival - now))
            stream.synchronize()
        finally:
            self.group_stats = group.stats()
            group.close()
        self.t_end = time.perf_counter() - self.t_start
        return self.done

    def _run_streams(self, requests: list[Request]) -> list[Request]:
        import torch
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        active = []      # (request, solver, stream, b, bytes)
        used = 0
        self.t_start = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - self.t_start
            # admission: arrived, a free slot, and memory for it
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                req = pending[0]
                need = footprint(req.system, self.options)
                if need > self._free_bytes(used):
                    if active:
                        self.waited_for_memory += 1
                        break          # wait until a running request frees memory
                    raise MemoryError(f"request {req.tag} needs {need} bytes, more than the device can give")
                pending.popleft()
                stream = torch.cuda.Stream()
                with torch.cuda.stream(stream):
                    b = torch.as_tensor(np.ascontiguousarray(req.system.b), device="cuda:0")
                    x = torch.empty_like(b)
                solver = B.Solver(req.system.row_ptr, req.system.col, req.system.val, req.system.block_ptr,
                                  n_border=getattr(req.system, "n_border", 0),
                                  lowrank=getattr(req.system, "lowrank", None), options=self.options,
                                  stream=stream)
                stream.synchronize()
                solver.solve_begin(b, x, self.tol)
                req.admitted = time.perf_counter() - self.t_start
                active.append((req, solver, stream, b, need))
                used += need
                self.max_concurrency = max(self.max_concurrency, len(active))
            # advance every running solve that is ready for its next step
            still = []
            for item in active:
                req, solver, stream, b, need = item
                if solver.solve_step():
                    req.x, req.iters, req.relres, req.status = solver.solve_end()
                    stream.synchronize()
                    req.finished = time.perf_counter() - self.t_start
                    self._log(req, solver)
                    solver.close()
                    used -= need
                    self.done.append(req)
                    if self.on_done:
                        self.on_done(req)
                else:
                    still.append(item)
            active = still
            if not active and pending and pending[0].arrival > now:
                time.sleep(min(0.001, pending[0].arrival - now))
        self.t_end = time.perf_counter() - self.t_start
        return self.done

    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.done]) * 1e3
        ok = sum(1 for r in self.done if r.status == B.OK)
        return {"requests": len(self.done), "ok": ok, "makespan_s": self.t_end,
                "solves_per_s": len(self.done) / self.t_end if self.t_end > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
                "max_concurrency": self.max_concurrency, "waited_for_memory": self.waited_for_memory,
                "shared_launches": self.shared, "graphs": self.shared and self.graphs,
                "group": self.group_stats}
