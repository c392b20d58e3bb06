"""Linear solves along an interior-point sequence (one sparsity pattern,
new values at every step).

The preconditioner is reused across steps (Sec. 3.4): after a fresh
factorisation the following steps only copy in the new operator values, for
at most ``reuse_every - 1`` steps, and a reused step is capped at
``degrade`` times the iterations of the last fresh one; a capped step that
does not converge is taken as convergence degradation (the end of a reuse
period in Sec. 3.4) and is solved again after a refactorisation.  A step
that fails with fresh factors switches the sequence from block Jacobi to the
BBD preconditioner for good (Alg. 1) when BBD options are given and the
system has a bordered form; otherwise the failure is reported.

``tau_schedule`` changes the filter threshold along the sequence (Sec.
4.3.3: 1e-3 for the early steps, 1e-2 later); a change builds the
preconditioner anew.  ``degrade = inf`` keeps the fixed schedule only.  ``make_solver(system,
options)`` builds a solver (``from_system`` for the
GPU library); the solver needs ``solve``, ``refactor``, ``update_values``,
``set_max_iter`` and ``close``."""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import Any, Callable, Optional

from ._binding import E_STRUCTURE, OK, SdslError


@dataclass
class StepRecord:
    k: int
    kind: str                 # setup, reuse, refactor (+refresh, +bbd)
    iterations: int = 0       # all Krylov iterations spent on the step
    status: int = OK
    relres: float = 1.0
    method: str = "BJ"
    events: list = field(default_factory=list)


class SequenceSolver:
    def __init__(self, make_solver: Callable[[Any, Any], Any], options, reuse_every: int = 5,
                 degrade: float = 1.5, min_cap: int = 50, bbd_options=None, tau_schedule=None):
        self.make_solver = make_solver
        self.options = options
        # [(first step, tau), ...] ascending: the filter threshold from that
        # step on (Sec. 4.3.3 runs tau = 1e-3 and later 1e-2); a change builds
        # the preconditioner anew with the new threshold
        self.tau_schedule = sorted(tau_schedule) if tau_schedule else None
        self.reuse_every = max(1, int(reuse_every))
        self.degrade = float(degrade)
        self.min_cap = int(min_cap)
        self.bbd_options = bbd_options
        self.max_iter = int(getattr(options, "max_iter", 100_000))
        self.sv = None
        self.method = "BJ"
        self.switched = False
        self.ref_its: Optional[int] = None   # iterations of the last fresh solve
        self.since = 0                       # steps since the last fresh factorisation

    def _tau_at(self, k: int):
        if not self.tau_schedule:
            return None
        tau = None
        for k0, t in self.tau_schedule:
            if k >= k0:
                tau = t
        return tau

    def _fresh_solve(self, b, tol):
        self.sv.set_max_iter(self.max_iter)
        return self.sv.solve(b, tol=tol)

    def step(self, k: int, system, vals, b, tol: float = 1e-8):
        """Solve step k: ``system`` (for a first setup or a switch), ``vals``
        its operator values on the device, ``b`` its right-hand side.
        Returns (x, StepRecord)."""
        rec = StepRecord(k=k, kind="", method=self.method)
        fresh = True
        want = self._tau_at(k)
        if self.sv is not None and want is not None and self.method == "BJ" and want != self.options.tau:
            self.sv.close()
            self.sv = None
            rec.events.append(f"tau {self.options.tau:g} -> {want:g}")
        if want is not None and self.method == "BJ":
            self.options = dataclasses.replace(self.options, tau=want)
        if self.sv is None:
            self.sv = self.make_solver(system, self.options)
            rec.kind = "setup"
        elif self.since + 1 >= self.reuse_every:
            self.sv.refactor(vals)
            rec.kind = "refactor"
        else:
            self.sv.update_values(vals)
            rec.kind = "reuse"
            fresh = False
        if fresh:
            x, its, rr, st = self._fresh_solve(b, tol)
        else:
            cap = self.max_iter if self.ref_its is None or not math.isfinite(self.degrade) else \
                min(self.max_iter, max(self.min_cap, int(self.degrade * self.ref_its)))
            self.sv.set_max_iter(cap)
            x, its, rr, st = self.sv.solve(b, tol=tol)
        rec.iterations += its
        if st != OK and not fresh:
            # convergence degradation: refresh the factors, solve again
            rec.events.append(f"degraded after {its} iterations")
            self.sv.refactor(vals)
            rec.kind += "+refresh"
            fresh = True
            x, its, rr, st = self._fresh_solve(b, tol)
            rec.iterations += its
        if st != OK and fresh and not self.switched and self.bbd_options is not None:
            # Alg. 1: block Jacobi failed with fresh factors; BBD from now on
            self.switched = True
            try:
                bbd = self.make_solver(system, self.bbd_options)
            except SdslError as e:
                if e.status != E_STRUCTURE:
                    raise
                rec.events.append("no bordered form: BBD unavailable")
            else:
                self.sv.close()
                self.sv, self.method, self.options = bbd, "BBD", self.bbd_options
                self.max_iter = int(getattr(self.bbd_options, "max_iter", self.max_iter))
                rec.kind += "+bbd"
                rec.method = "BBD"
                x, its, rr, st = self._fresh_solve(b, tol)
                rec.iterations += its
        if fresh:
            self.since = 0
            if st == OK:
                self.ref_its = max(1, its)
        else:
            self.since += 1
        rec.status, rec.relres = st, rr
        return x, rec

    def close(self):
        if self.sv is not None:
            self.sv.close()
            self.sv = None
