"""Serving loop scheduling on the CPU with a fake device backend: admission
by bytes and slots, continuous joining, rejection and failure paths, latency
and throughput accounting."""
import math

import pytest

from paper_2507_11542_amd import inputs
from paper_2507_11542_amd.serve import Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += s


class FakeBackend:
    """A macro-iteration of a family costs `cost(key)` of fake time (1 ms
    unless given); a request needs ceil(tf / 0.1) steps."""

    def __init__(self, clock, fail_names=(), cost=None):
        self.clock = clock
        self.fail_names = set(fail_names)
        self.cost = cost or (lambda key: 0.001)
        self.live = 0
        self.max_live = 0
        self.released = []
        self.busy_until = {}
        self.launches = []

    def bytes_needed(self, j):
        return j.problem.points * 16

    def admit(self, j):
        if j.problem.name in self.fail_names:
            raise MemoryError("injected")
        j.dev = {"left": int(math.ceil(j.problem.tf / 0.1))}
        j.dev_finished = j.dev["left"] == 0
        self.live += 1
        self.max_live = max(self.max_live, self.live)

    def advance(self, key, group, k):
        assert self.ready(key), "relaunched a family still in flight"
        self.launches.append((key, len(group), k))
        for j in group:
            n = min(k, j.dev["left"])
            j.dev["left"] -= n
            j.steps_done += n
            j.dev_finished = j.dev["left"] == 0
        self.busy_until[key] = self.clock.t + self.cost(key)

    def ready(self, key):
        return self.clock.t >= self.busy_until.get(key, 0.0) - 1e-12

    def idle(self, key):
        pass

    def result(self, j):
        return None

    def release(self, j):
        self.live -= 1
        self.released.append(j.rid)


def _req(arrival, n, tf, name="p", dyn="rel_dubins"):
    p = inputs.rel_dubins_3d(n=(n, n, n), tf=tf).with_(name=name)
    return inputs.Request(arrival, p)


def test_all_complete_and_account():
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = [_req(0.0005 * k, 11, 0.35 + 0.1 * (k % 3)) for k in range(12)]
    rep, jobs = Server(be, hbm_budget=10 ** 9, macro_steps=2, clock=clk, sleep=clk.sleep).run(reqs)
    assert rep.completed == 12 and rep.rejected == 0
    assert all(j.state == "done" and j.latency > 0 for j in jobs)
    steps = sum(math.ceil(r.problem.tf / 0.1) for r in reqs)
    assert rep.updates == pytest.approx(11 ** 3 * steps)
    assert be.live == 0 and sorted(be.released) == list(range(12))
    assert rep.p99_s >= rep.p50_s > 0


def test_budget_limits_concurrency_and_late_requests_join():
    clk = FakeClock()
    be = FakeBackend(clk)
    per = 11 ** 3 * 16
    reqs = [_req(0.0, 11, 1.0) for _ in range(3)] + [_req(0.0025, 11, 0.2)]
    rep, jobs = Server(be, hbm_budget=2 * per, macro_steps=1, clock=clk, sleep=clk.sleep).run(reqs)
    assert rep.completed == 4
    assert be.max_live == 2 and rep.max_active == 2 and rep.peak_bytes == 2 * per
    # the third request waits for memory, then joins while another still runs
    first_done = min(j.finished_at for j in jobs[:2])
    assert jobs[2].admitted_at >= first_done
    assert any(j.finished_at > jobs[2].admitted_at for j in jobs[:2] if j.rid != 2) or \
        jobs[3].admitted_at < jobs[2].finished_at


def test_slot_limit():
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = [_req(0.0, 11, 0.3) for _ in range(5)]
    rep, _ = Server(be, hbm_budget=10 ** 9, max_active=2, macro_steps=1, clock=clk,
                    sleep=clk.sleep).run(reqs)
    assert rep.completed == 5 and be.max_live == 2


def test_over_budget_and_failed_allocation_are_rejected():
    clk = FakeClock()
    be = FakeBackend(clk, fail_names={"boom"})
    reqs = [_req(0.0, 11, 0.3), _req(0.0, 41, 0.3, name="huge"), _req(0.0, 11, 0.3, name="boom"),
            _req(0.001, 11, 0.2)]
    rep, jobs = Server(be, hbm_budget=2 * 11 ** 3 * 16, macro_steps=1, clock=clk,
                       sleep=clk.sleep).run(reqs)
    assert rep.rejected == 2 and rep.completed == 2
    assert "budget" in jobs[1].reason and "allocation failed" in jobs[2].reason
    assert be.live == 0


def test_idle_waits_for_arrivals():
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = [_req(0.5, 11, 0.2), _req(1.25, 11, 0.2)]
    rep, jobs = Server(be, hbm_budget=10 ** 9, macro_steps=4, clock=clk, sleep=clk.sleep).run(reqs)
    assert rep.completed == 2
    assert jobs[0].admitted_at >= 0.5 and jobs[1].admitted_at >= 1.25
    assert rep.makespan_s >= 1.25


def _req_dyn(arrival, tf, dyn):
    if dyn == "d4":
        p = inputs.dubins4d(n=(9, 9, 9, 9), tf=tf)
    else:
        p = inputs.double_integrator_2d(n=21, tf=tf)
    return inputs.Request(arrival, p)


def test_families_progress_independently():
    """A slow family (4-D, 20 ms per macro-iteration) and a fast one (2-D,
    1 ms): the 2-D requests finish long before the first 4-D macro-iteration
    ends, instead of waiting for it at every iteration."""
    clk = FakeClock()
    be = FakeBackend(clk, cost=lambda key: 0.020 if key[0] == 4 else 0.001)
    reqs = [_req_dyn(0.0, 0.9, "d4")] + [_req_dyn(0.0, 0.3, "di") for _ in range(3)]
    rep, jobs = Server(be, hbm_budget=10 ** 9, macro_steps=2, clock=clk, sleep=clk.sleep).run(reqs)
    assert rep.completed == 4
    # di: 3 steps at 2 per iteration = 2 iterations of 1 ms
    assert all(j.finished_at <= 0.0025 for j in jobs[1:])
    # d4: 9 steps = 5 iterations of 20 ms
    assert jobs[0].finished_at == pytest.approx(0.100, abs=1e-3)


def test_joiners_wait_for_the_family_in_flight():
    """A request arriving while its family is in flight joins at the family's
    next launch, not before; and macro_updates sizes the step count by the
    family's total nodes."""
    clk = FakeClock()
    be = FakeBackend(clk, cost=lambda key: 0.010)
    reqs = [_req(0.0, 11, 2.0), _req(0.003, 11, 0.2)]
    srv = Server(be, hbm_budget=10 ** 9, macro_steps=8, macro_updates=4 * 11 ** 3, clock=clk,
                 sleep=clk.sleep)
    rep, jobs = srv.run(reqs)
    assert rep.completed == 2
    assert be.launches[0] == (jobs[0].key, 1, 4)   # 4 steps for one 11^3 grid
    assert be.launches[1] == (jobs[0].key, 2, 2)   # joined at 10 ms: 2 steps each
    assert jobs[1].finished_at == pytest.approx(0.020, abs=1e-3)


def test_cancel_waiting_request_is_never_admitted():
    """A request withdrawn while it waits for memory leaves the queue: it is
    never admitted, and the request behind it takes the memory instead."""
    clk = FakeClock()
    be = FakeBackend(clk)
    per = 11 ** 3 * 16
    reqs = [_req(0.0, 11, 1.0), _req(0.0, 11, 0.5), _req(0.0, 11, 0.2)]
    rep, jobs = Server(be, hbm_budget=per, macro_steps=1, clock=clk,
                       sleep=clk.sleep).run(reqs, cancels={1: 0.0005})
    assert rep.completed == 2 and rep.cancelled == 1
    assert jobs[1].state == "cancelled" and jobs[1].admitted_at is None
    assert 1 not in be.released and be.live == 0
    assert jobs[2].admitted_at >= jobs[0].finished_at


def test_cancel_resident_request_frees_slot_and_bytes():
    """A resident request withdrawn mid-solve is released once its family has
    nothing in flight: its slot and bytes return at once, so a request that
    did not fit is admitted long before the withdrawn solve would have
    ended; its steps so far count as work, the others are unaffected."""
    clk = FakeClock()
    be = FakeBackend(clk)
    per = 11 ** 3 * 16
    # request 0 needs 30 steps of 1 ms; it is withdrawn after ~5 ms
    reqs = [_req(0.0, 11, 3.0), _req(0.001, 11, 0.3)]
    rep, jobs = Server(be, hbm_budget=per, macro_steps=1, clock=clk,
                       sleep=clk.sleep).run(reqs, cancels={0: 0.005})
    assert jobs[0].state == "cancelled" and 0 in be.released
    assert 0 < jobs[0].steps_done < 30
    assert jobs[0].finished_at == pytest.approx(0.005, abs=0.002)
    assert jobs[1].state == "done" and jobs[1].admitted_at < 0.008
    assert rep.completed == 1 and rep.cancelled == 1 and be.live == 0
    assert rep.updates == pytest.approx(11 ** 3 * (jobs[0].steps_done + 3))


def test_cancel_after_finish_has_no_effect():
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = [_req(0.0, 11, 0.2), _req(0.0, 11, 0.3)]
    rep, jobs = Server(be, hbm_budget=10 ** 9, macro_steps=1, clock=clk,
                       sleep=clk.sleep).run(reqs, cancels={0: 1.0})
    assert rep.completed == 2 and rep.cancelled == 0
    assert all(j.state == "done" for j in jobs)
