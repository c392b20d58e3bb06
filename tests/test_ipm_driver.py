"""Host logic of the interior-point sequence driver (preconditioner reuse with
a refresh on convergence degradation, Sec. 3.4; block Jacobi -> BBD switch on
failure, Alg. 1), checked with scripted stand-in solvers on the CPU."""

from paper_2604_23979_amd._binding import E_NOT_CONVERGED, E_STRUCTURE, OK, Options, SdslError, BBD
from paper_2604_23979_amd.ipm import SequenceSolver


class FakeSolver:
    """Iterations needed at step k: need(k, age), age = steps since the
    factors were built; a solve stops at max_iter with E_NOT_CONVERGED."""

    def __init__(self, need, log, method="BJ"):
        self.need, self.log, self.method = need, log, method
        self.k = 0
        self.built_at = 0
        self.max_iter = 10 ** 9
        self.closed = False

    def set_max_iter(self, m):
        self.max_iter = m

    def refactor(self, vals):
        self.k = vals
        self.built_at = vals
        self.log.append(("refactor", vals))

    def update_values(self, vals):
        self.k = vals
        self.log.append(("update", vals))

    def solve(self, b, tol=1e-8):
        n = self.need(self.k, self.k - self.built_at, self.method)
        if n is None or n > self.max_iter:
            return None, self.max_iter, 1.0, E_NOT_CONVERGED
        return None, n, 0.5 * tol, OK

    def close(self):
        self.closed = True


def make_factory(need, log, bbd_ok=True):
    def make(system, options):
        method = "BBD" if options.method == BBD else "BJ"
        if method == "BBD" and not bbd_ok:
            raise SdslError(E_STRUCTURE, "no border")
        s = FakeSolver(need, log, method)
        s.k = s.built_at = system
        log.append(("setup", method, system))
        return s
    return make


def run(seq, steps):
    return [seq.step(k, k, k, None)[1] for k in range(steps)]


def test_fixed_schedule_refactors_every_five_steps():
    log = []
    seq = SequenceSolver(make_factory(lambda k, age, m: 100 + 10 * age, log), Options(max_iter=1000))
    recs = run(seq, 11)
    assert [r.kind for r in recs] == ["setup", "reuse", "reuse", "reuse", "reuse", "refactor",
                                      "reuse", "reuse", "reuse", "reuse", "refactor"]
    assert all(r.status == OK for r in recs)
    assert [r.iterations for r in recs[:5]] == [100, 110, 120, 130, 140]


def test_degraded_reuse_is_refreshed_and_solved_again():
    log = []
    # a reused factor needs 3x the fresh count from age 2 on
    need = lambda k, age, m: 100 if age < 2 else 300
    seq = SequenceSolver(make_factory(need, log), Options(max_iter=1000), degrade=1.5)
    recs = run(seq, 4)
    assert [r.kind for r in recs] == ["setup", "reuse", "reuse+refresh", "reuse"]
    # the capped attempt (1.5 x 100) plus the fresh solve
    assert recs[2].iterations == 150 + 100 and recs[2].status == OK
    assert ("refactor", 2) in log
    # the refresh restarts the reuse period
    assert seq.since == 1


def test_failure_with_fresh_factors_switches_to_bbd_for_good():
    log = []
    need = lambda k, age, m: 5 if m == "BBD" else (None if k >= 2 else 100)
    seq = SequenceSolver(make_factory(need, log), Options(max_iter=1000),
                         bbd_options=Options(method=BBD, max_iter=500))
    recs = run(seq, 5)
    assert recs[2].kind.endswith("+bbd") and recs[2].method == "BBD" and recs[2].status == OK
    assert all(r.method == "BBD" and r.status == OK for r in recs[3:])
    assert seq.switched and seq.max_iter == 500
    assert sum(1 for e in log if e[:2] == ("setup", "BBD")) == 1


def test_switch_unavailable_reports_the_failure():
    log = []
    need = lambda k, age, m: None if k >= 1 else 100
    seq = SequenceSolver(make_factory(need, log, bbd_ok=False), Options(max_iter=400),
                         bbd_options=Options(method=BBD))
    recs = run(seq, 2)
    assert recs[1].status == E_NOT_CONVERGED
    assert any("BBD unavailable" in e for e in recs[1].events)
    assert recs[1].kind == "reuse+refresh"


def test_infinite_degrade_keeps_the_fixed_schedule():
    log = []
    need = lambda k, age, m: 100 if age < 2 else 300
    seq = SequenceSolver(make_factory(need, log), Options(max_iter=1000), degrade=float("inf"))
    recs = run(seq, 4)
    assert [r.kind for r in recs] == ["setup", "reuse", "reuse", "reuse"]
    assert [r.iterations for r in recs] == [100, 100, 300, 300]


def test_two_phase_tau_schedule_rebuilds_the_preconditioner():
    """Sec. 4.3.3 filters with tau = 1e-3 for the early IPM steps and 1e-2
    later: the driver builds the preconditioner anew with the new threshold
    at the step where the schedule changes, then reuses it as before."""
    log, taus = [], []

    def make(system, options):
        taus.append((system, options.tau))
        return make_factory(lambda k, age, m: 100, log)(system, options)
    seq = SequenceSolver(make, Options(max_iter=1000, tau=1e-3), tau_schedule=[(0, 1e-3), (24, 1e-2)])
    recs = run(seq, 27)
    assert taus == [(0, 1e-3), (24, 1e-2)]
    assert recs[24].kind == "setup" and any("tau 0.001 -> 0.01" in e for e in recs[24].events)
    assert [r.kind for r in recs[20:27]] == ["refactor", "reuse", "reuse", "reuse", "setup", "reuse", "reuse"]
    assert seq.options.tau == 1e-2
