"""Continuous-batching request server for level-set solves on one GPU.

Requests (a Problem: grid, dynamics, scheme, horizon, V0 recipe) arrive over
time.  The server admits a request when it has arrived, a slot is free and
its device bytes fit the HBM budget, and keeps every admitted solve resident
on the device until it finishes.  Admitted requests are grouped by kernel
family (ndim, dynamics, scheme, RK order, precision); a macro-iteration of a
family advances every instance in it by up to `macro_steps` RK steps with one
batched launch sequence (hj_step_batch, replayed from one captured graph).
The families run on their own streams, so their work overlaps on the device,
and progress independently: when a family's macro-iteration completes, its
finished requests retire (their memory returns to the budget), waiting
requests are admitted as slots and memory free up, and the family is
relaunched with the requests that joined it.

Scheduling is separate from the device: `Server` drives a backend with
`bytes_needed / admit / advance / ready / release`; `GpuBackend` implements it
with libhj through its C ABI (torch for device memory and streams).  The
per-request results equal those of a request solved alone (the batched kernels
run the same per-node arithmetic with the same FP64 step sizes).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import inputs


@dataclasses.dataclass
class Job:
    rid: int
    problem: inputs.Problem
    arrival: float
    t: float = 0.0
    state: str = "pending"       # pending | active | done | rejected | cancelled
    cancel_at: Optional[float] = None  # the client withdraws the request at this time
    reason: str = ""
    admitted_at: Optional[float] = None
    finished_at: Optional[float] = None
    nbytes: int = 0
    steps_done: int = 0
    dev_finished: bool = False   # set by the backend after each advance
    result: Optional[np.ndarray] = None
    dev: object = None           # backend state

    @property
    def key(self) -> Tuple:
        p = self.problem
        return (p.ndim, p.dynamics, p.scheme, p.order)

    @property
    def latency(self) -> Optional[float]:
        if self.finished_at is None:
            return None
        return self.finished_at - self.arrival


@dataclasses.dataclass
class ServeReport:
    requests: int
    completed: int
    rejected: int
    cancelled: int
    makespan_s: float
    updates: float
    updates_per_s: float
    p50_s: float
    p99_s: float
    mean_s: float
    max_active: int
    peak_bytes: int
    macro_iterations: int

    def as_dict(self):
        return dataclasses.asdict(self)


def percentile(xs: Sequence[float], q: float) -> float:
    if not xs:
        return float("nan")
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def report(jobs: List[Job], makespan: float, max_active: int, peak: int, iters: int,
           updates: float) -> ServeReport:
    lat = [j.latency for j in jobs if j.state == "done"]
    return ServeReport(len(jobs), len(lat), sum(j.state == "rejected" for j in jobs),
                       sum(j.state == "cancelled" for j in jobs), makespan,
                       updates, updates / makespan if makespan > 0 else 0.0,
                       percentile(lat, 50), percentile(lat, 99),
                       float(np.mean(lat)) if lat else float("nan"), max_active, peak, iters)


class Server:
    """Admission by device bytes and slots, continuous batching by family.

    Families progress independently: each has at most one macro-iteration in
    flight on its own stream, and the loop polls them, so a family of small
    grids is never held back by a family of large ones; when a family's
    macro-iteration completes its finished requests retire at once and the
    family is relaunched with whoever has joined it meanwhile.

    macro_steps caps the RK steps per instance in one macro-iteration; with
    macro_updates set, a family takes ceil(macro_updates / its total nodes)
    steps (at least 1, at most macro_steps), rounded down to a power of two
    (few distinct step counts, so few distinct captured launch graphs), so a
    macro-iteration costs about the same device time whatever the family's
    size.
    """

    def __init__(self, backend, hbm_budget: int, max_active: int = 256, macro_steps: int = 32,
                 macro_updates: Optional[float] = None, poll_s: float = 2e-4,
                 clock=time.perf_counter, sleep=time.sleep):
        self.backend = backend
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.macro_steps = int(macro_steps)
        self.macro_updates = macro_updates
        self.poll_s = float(poll_s)
        self.clock = clock
        self.sleep = sleep

    def steps_for(self, group: List[Job]) -> int:
        if not self.macro_updates:
            return self.macro_steps
        pts = sum(j.problem.points for j in group)
        k = max(1, min(self.macro_steps, int(math.ceil(self.macro_updates / max(pts, 1)))))
        return 1 << (k.bit_length() - 1)

    def run(self, requests: Sequence[inputs.Request], keep_results: bool = False,
            cancels: Optional[Dict[int, float]] = None) -> Tuple[ServeReport, List[Job]]:
        """Serve `requests` (arrival times relative to the start); cancels maps
        a request's index to the time its client withdraws it.  A withdrawn
        request leaves the queue if it is still waiting; if it is resident it
        is released as soon as its family has no work in flight (at once if
        none is), which returns its slot and bytes to the budget; a finished
        request is not affected."""
        jobs = [Job(k, r.problem, r.arrival, t=r.problem.t0) for k, r in enumerate(requests)]
        for k, t in (cancels or {}).items():
            jobs[k].cancel_at = float(t)
        pending = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.rid)))
        active: Dict[Tuple, List[Job]] = collections.OrderedDict()
        inflight = set()
        used = 0
        n_active = 0
        max_active = peak = iters = 0
        updates = 0.0
        start = self.clock()
        while pending or n_active:
            now = self.clock() - start
            # withdrawn while waiting: never admitted
            if any(j.cancel_at is not None and j.cancel_at <= now for j in pending):
                keep_q = collections.deque()
                for j in pending:
                    if j.cancel_at is not None and j.cancel_at <= now:
                        j.state, j.reason = "cancelled", "withdrawn before admission"
                        j.finished_at = now
                    else:
                        keep_q.append(j)
                pending = keep_q
            # admission: arrived, slot free, bytes fit (arrival order)
            while pending and pending[0].arrival <= now:
                j = pending[0]
                need = self.backend.bytes_needed(j)
                if need > self.hbm_budget:
                    pending.popleft()
                    j.state, j.reason = "rejected", "needs %d bytes > budget" % need
                    continue
                if used + need > self.hbm_budget or n_active >= self.max_active:
                    break
                pending.popleft()
                try:
                    self.backend.admit(j)
                except MemoryError as e:
                    j.state, j.reason = "rejected", "allocation failed: %s" % e
                    continue
                j.nbytes = need
                j.state = "active"
                j.admitted_at = now
                used += need
                n_active += 1
                active.setdefault(j.key, []).append(j)
            max_active = max(max_active, n_active)
            peak = max(peak, used)
            # families with nothing in flight: retire, then relaunch
            for key in list(active):
                if key in inflight:
                    continue
                group = active[key]
                keep = []
                now = self.clock() - start
                for j in group:
                    if j.cancel_at is not None and j.cancel_at <= now and not j.dev_finished:
                        # withdrawn while resident: its work so far counts, its
                        # memory and slot return now
                        updates += float(j.problem.points) * j.steps_done
                        self.backend.release(j)
                        j.state, j.reason = "cancelled", "withdrawn after admission"
                        j.finished_at = now
                        used -= j.nbytes
                        n_active -= 1
                    elif j.dev_finished:
                        if keep_results:
                            j.result = self.backend.result(j)
                        updates += float(j.problem.points) * j.steps_done
                        self.backend.release(j)
                        j.state = "done"
                        j.finished_at = self.clock() - start
                        used -= j.nbytes
                        n_active -= 1
                    else:
                        keep.append(j)
                if not keep:
                    del active[key]
                    self.backend.idle(key)
                    continue
                active[key] = keep
                self.backend.advance(key, keep, self.steps_for(keep))
                inflight.add(key)
            if not inflight:
                if pending and not n_active:
                    wait = pending[0].arrival - (self.clock() - start)
                    if wait > 0:
                        self.sleep(min(wait, 0.05))
                continue
            done = [k for k in inflight if self.backend.ready(k)]
            if not done:
                self.sleep(self.poll_s)
                continue
            for k in done:
                inflight.discard(k)
                iters += 1
        makespan = self.clock() - start
        return report(jobs, makespan, max_active, peak, iters, updates), jobs


class GpuBackend:
    """libhj through its C ABI; torch supplies device memory and streams.

    Every family has its own stream and engine; uploads of admitted requests
    go through a separate stream, so admitting never waits for a family's
    work in flight, and a family's next launch waits on the uploads of the
    requests that joined it (stream-ordered events, no host wait).

    fp64_finish (FP32 only): each request also keeps its V0 in FP64, the FP32
    working V0 is that rounded once, and a finished request's result is
    widened to FP64 with the tube minimum retaken in FP64 near the zero level
    set (hj_tube_finish), as hj_solve_mixed does for a single solve.

    solo_points: a request with at least this many nodes fills the chip with
    its own launches, so its family advances it with its own hj_step calls
    (the single-solve stage kernel) after the batched launch of the family's
    smaller requests, on the same stream; None batches every request."""

    def __init__(self, prec: str = "fp32", tile_nodes: int = 256, workgroups: int = 0,
                 use_graph: bool = True, v0_cache: Optional[Dict[int, np.ndarray]] = None,
                 device_v0: bool = False, fp64_finish: bool = False,
                 solo_points: Optional[int] = 2_000_000):
        import torch

        from . import hj

        self.torch = torch
        self.hj = hj
        self.prec = prec
        self.dtype = torch.float32 if prec == "fp32" else torch.float64
        self.elem = 4 if prec == "fp32" else 8
        self.cfg = (tile_nodes, workgroups, use_graph)
        self.v0_cache = v0_cache if v0_cache is not None else {}
        self.device_v0 = device_v0  # build V0 from the problem's shape recipe on the GPU
        if fp64_finish and prec != "fp32":
            raise ValueError("fp64_finish needs prec='fp32'")
        self.fp64_finish = fp64_finish
        self.solo_points = solo_points
        self.engines: Dict[Tuple, object] = {}
        self.streams: Dict[Tuple, object] = {}
        self.events: Dict[Tuple, object] = {}
        self.device = torch.device("cuda")
        self.upload = torch.cuda.Stream(device=self.device)

    def bytes_needed(self, j: Job) -> int:
        # V0, V and two stage buffers, plus the coordinate tables (FP64 and FP32);
        # with the FP64 finish also the FP64 V0 and result
        p = j.problem
        extra = 16 * p.points if self.fp64_finish else 0
        return 4 * p.points * self.elem + extra + sum(p.n) * 3 * (8 + 4) + 4096

    def _engine(self, key):
        if key not in self.engines:
            self.engines[key] = self.hj.Batch(*self.cfg)
            self.streams[key] = self.torch.cuda.Stream(device=self.device)
        return self.engines[key], self.streams[key]

    def admit(self, j: Job):
        torch = self.torch
        p = j.problem
        g = self.hj.Grid.from_problem(p, self.prec)
        extra = {}
        try:
            with torch.cuda.stream(self.upload):
                if self.device_v0:
                    v0 = torch.empty(tuple(p.n), dtype=self.dtype, device=self.device)
                    g.init_shapes(v0, p.shapes(), self.upload)
                    if self.fp64_finish:  # the same recipe evaluated in FP64
                        extra["v0_64"], extra["grid64"] = _device_v0_f64(self.hj, torch, p,
                                                                         self.upload)
                else:
                    v0h = self.v0_cache.get(j.rid)
                    if v0h is None:
                        v0h = p.v0()
                    host = torch.from_numpy(np.ascontiguousarray(v0h))
                    v0 = host.to(self.device, self.dtype, non_blocking=False)
                    if self.fp64_finish:
                        extra["v0_64"] = host.to(self.device, torch.float64)
                if self.fp64_finish:
                    extra["out64"] = torch.empty_like(extra["v0_64"])
                v = v0.clone()
                a = torch.empty_like(v0)
                b = torch.empty_like(v0)
                if self.fp64_finish and p.tf <= p.t0:  # nothing to solve: finish V0
                    g.tube_finish(v, extra["v0_64"], extra["out64"], p.mode, -1.0,
                                  self.upload)
                ready = torch.cuda.Event()
                ready.record(self.upload)
        except RuntimeError as e:  # torch reports device OOM as RuntimeError
            g.close()
            if "grid64" in extra:
                extra["grid64"].close()
            raise MemoryError(str(e))
        g.set_workspace(a, b)
        if self._solo(j):  # its step count (and alpha, cached in the handle)
            extra["steps"] = g.schedule(p.t0, p.tf, self.upload)[2]
        j.dev = {"grid": g, "v0": v0, "v": v, "a": a, "b": b, "ready": ready, **extra}
        j.t = p.t0
        j.dev_finished = p.tf <= p.t0

    def _solo(self, j: Job) -> bool:
        return self.solo_points is not None and j.problem.points >= self.solo_points

    def advance(self, key, group: List[Job], max_steps: int):
        eng, stream = self._engine(key)
        todo = [j for j in group if not j.dev_finished]
        for j in todo:
            ev = j.dev.pop("ready", None)
            if ev is not None:  # first launch of a joined request: wait for its upload
                stream.wait_event(ev)
                for name in ("v0", "v", "a", "b", "v0_64", "out64"):
                    if name in j.dev:
                        j.dev[name].record_stream(stream)
        batched = [j for j in todo if not self._solo(j)]
        if batched:
            ts, taken, fin = eng.step([j.dev["grid"] for j in batched],
                                      [j.dev["v0"] for j in batched],
                                      [j.dev["v"] for j in batched],
                                      [j.problem.t0 for j in batched], [j.t for j in batched],
                                      [j.problem.tf for j in batched],
                                      [j.problem.mode for j in batched], max_steps, stream)
            for j, t, k, f in zip(batched, ts, taken, fin):
                j.t = t
                j.steps_done += k
                j.dev_finished = f
        for j in todo:
            if not self._solo(j):
                continue
            # the same steps as hj_solve: its step count, each of
            # min(dt, tf - t), t accumulated in FP64 on the host
            k = min(max_steps, j.dev["steps"] - j.steps_done)
            g, t = j.dev["grid"], j.t
            for _ in range(k):
                t, _ = g.step(j.dev["v"], j.dev["v0"], t, j.problem.tf, j.problem.mode, stream)
            j.t = t
            j.steps_done += k
            j.dev_finished = j.steps_done >= j.dev["steps"]
        if self.fp64_finish:
            for j in todo:
                if j.dev_finished:
                    j.dev["grid"].tube_finish(j.dev["v"], j.dev["v0_64"], j.dev["out64"],
                                              j.problem.mode, -1.0, stream)
        ev = self.torch.cuda.Event()
        ev.record(stream)
        self.events[key] = ev

    def ready(self, key) -> bool:
        ev = self.events.get(key)
        return ev is None or ev.query()

    def sync(self, key):
        ev = self.events.get(key)
        if ev is not None:
            ev.synchronize()

    def idle(self, key):
        pass

    @staticmethod
    def _settle(j: Job):
        # a request that never reached a family launch (empty horizon) still
        # has its upload-stream work pending: wait for it before reading or
        # freeing its buffers
        ev = j.dev.get("ready")
        if ev is not None:
            ev.synchronize()

    def result(self, j: Job) -> np.ndarray:
        self._settle(j)
        if self.fp64_finish:
            return j.dev["out64"].cpu().numpy()
        return j.dev["v"].double().cpu().numpy()

    def release(self, j: Job):
        self._settle(j)
        j.dev["grid"].close()
        if "grid64" in j.dev:
            j.dev["grid64"].close()
        j.dev = None

    def close(self):
        for key in list(self.events):
            self.sync(key)
        for e in self.engines.values():
            e.close()
        self.engines.clear()


def _device_v0_f64(hj, torch, p, stream):
    """V0 of problem p built on the device in FP64 from its shape recipe, and
    the FP64 grid handle whose coordinate tables the kernel reads (to be
    closed once the stream has passed it)."""
    g64 = hj.Grid(p.n, p.lo, p.hi, p.periodic, "fp64")
    try:
        v0 = torch.empty(tuple(p.n), dtype=torch.float64, device="cuda")
        g64.init_shapes(v0, p.shapes(), stream)
    except BaseException:
        g64.close()
        raise
    return v0, g64


def run_plain(requests: Sequence[inputs.Request], prec: str = "fp32",
              v0_cache: Optional[Dict[int, np.ndarray]] = None, keep_results: bool = False,
              device_v0: bool = False, clock=time.perf_counter, sleep=time.sleep,
              fp64_finish: bool = False) -> Tuple[ServeReport, List[Job]]:
    """The same requests one at a time through hj_solve (no batching, no
    graph): each starts when it has arrived and the previous one finished.
    device_v0 builds V0 on the GPU from the problem's shape recipe, as the
    serving backend can; fp64_finish solves through hj_solve_mixed (FP64 V0
    and result, FP32 bulk), the single-solve form of the backend's option."""
    import torch

    from . import hj

    dtype = torch.float32 if prec == "fp32" else torch.float64
    jobs = [Job(k, r.problem, r.arrival, t=r.problem.t0) for k, r in enumerate(requests)]
    order = sorted(jobs, key=lambda j: (j.arrival, j.rid))
    stream = torch.cuda.current_stream()
    updates = 0.0
    start = clock()
    for j in order:
        wait = j.arrival - (clock() - start)
        while wait > 0:
            sleep(min(wait, 0.05))
            wait = j.arrival - (clock() - start)
        p = j.problem
        g = hj.Grid.from_problem(p, prec)
        vdtype = torch.float64 if fp64_finish else dtype
        g64 = None
        if device_v0:
            if fp64_finish:
                v0, g64 = _device_v0_f64(hj, torch, p, stream)
            else:
                v0 = torch.empty(tuple(p.n), dtype=dtype, device="cuda")
                g.init_shapes(v0, p.shapes(), stream)
        else:
            v0h = (v0_cache or {}).get(j.rid)
            v0 = torch.from_numpy(np.ascontiguousarray(v0h if v0h is not None else p.v0())).to(
                "cuda", vdtype)
        out = torch.empty_like(v0)
        _, _, steps = g.schedule(p.t0, p.tf, stream)
        if fp64_finish:
            g.solve_mixed(v0, out, p.t0, p.tf, p.mode, -1.0, stream)
        else:
            g.solve(v0, out, p.t0, p.tf, p.mode, stream)
        stream.synchronize()
        if keep_results:
            j.result = out.double().cpu().numpy()
        g.close()
        if g64 is not None:
            g64.close()
        j.state = "done"
        j.steps_done = steps
        j.finished_at = clock() - start
        updates += float(p.points) * steps
    makespan = clock() - start
    return report(jobs, makespan, 1, 0, len(jobs), updates), jobs
