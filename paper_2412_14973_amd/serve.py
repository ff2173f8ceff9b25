"""Continuous-batching server for per-frequency TLR-MDD solves.

Each request is one frequency's solve (the paper solves every frequency
independently, Theory section, eq. standard_solver) with its own layout,
sizes and iteration count. The scheduler admits requests in arrival order
(FIFO, no overtaking) as soon as a slot and enough of the HBM budget are free;
an admitted solve keeps its inputs, factors and optimiser state resident and
runs on its own HIP stream, so solves admitted at different times overlap on
the device. A request's footprint counts everything it holds on the device
while admitted: the solve workspace, theta in and out, the f-history, its
inputs D and U and, when its inputs are produced at admission, the
transient memory that takes. A request whose footprint exceeds the whole
budget is rejected.

The policy is independent of the device: `Server` drives a backend with
`footprint(req)`, `start(req)`, `done(handle)`, `finish(handle)` and a clock.
`GpuBackend` runs the HIP library; tests drive the same policy with a
simulated device on a virtual clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional


@dataclasses.dataclass
class Job:
    rid: int
    arrival: float                  # seconds on the server clock
    payload: Any                    # backend-specific request data
    admitted: Optional[float] = None
    finished: Optional[float] = None
    rejected: bool = False
    footprint: int = 0
    result: Any = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class Server:
    """FIFO admission under an HBM budget and a slot limit; overlapping execution."""

    def __init__(self, backend, hbm_budget: int, max_active: int = 4):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.in_use = 0
        self.peak_in_use = 0
        self.log: List[tuple] = []   # (time, event, rid); "wait_memory": the head waits for memory, not a slot

    def run(self, jobs: List[Job], poll_interval: float = 2e-4,
            on_done: Optional[Callable[[Job], None]] = None) -> List[Job]:
        clock = self.backend.clock
        pending = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.rid)))
        active: Dict[int, tuple] = {}
        while pending or active:
            now = clock.now()
            # completions first: they free memory and slots for the next admissions
            for rid in list(active):
                job, handle = active[rid]
                if self.backend.done(handle):
                    job.result = self.backend.finish(handle)
                    job.finished = clock.now()
                    self.in_use -= job.footprint
                    del active[rid]
                    self.log.append((job.finished, "done", rid))
                    if on_done is not None:
                        on_done(job)
            # admissions in arrival order; the head waits if it does not fit yet
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                job = pending[0]
                job.footprint = int(self.backend.footprint(job.payload))
                if job.footprint > self.budget:
                    pending.popleft()
                    job.rejected = True
                    job.finished = now
                    self.log.append((now, "reject", job.rid))
                    continue
                if self.in_use + job.footprint > self.budget:
                    if not self.log or self.log[-1][1:] != ("wait_memory", job.rid):
                        self.log.append((now, "wait_memory", job.rid))
                    break
                pending.popleft()
                self.in_use += job.footprint
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                job.admitted = clock.now()
                active[job.rid] = (job, self.backend.start(job.payload))
                self.log.append((job.admitted, "admit", job.rid))
            if not active and pending and pending[0].arrival > now:
                clock.sleep_until(pending[0].arrival)
            elif active:
                clock.sleep(poll_interval)
        return jobs


def percentile(values: List[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]


def summarize(jobs: List[Job]) -> dict:
    done = [j for j in jobs if j.finished is not None and not j.rejected]
    lat = [j.latency for j in done]
    if not done:
        return {"completed": 0}
    t_first = min(j.arrival for j in jobs)
    t_last = max(j.finished for j in done)
    return {"completed": len(done), "rejected": sum(j.rejected for j in jobs),
            "solves_per_s": len(done) / (t_last - t_first),
            "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
            "mean_latency_s": sum(lat) / len(lat), "makespan_s": t_last - t_first}


# ---------------------------------------------------------------------------
# clocks
# ---------------------------------------------------------------------------
class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep(self, dt: float) -> None:
        time.sleep(dt)

    def sleep_until(self, t: float) -> None:
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


class VirtualClock:
    """Deterministic clock for simulated backends: sleeping advances time."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep(self, dt: float) -> None:
        self.t += dt

    def sleep_until(self, t: float) -> None:
        self.t = max(self.t, t)


# ---------------------------------------------------------------------------
# GPU backend (HIP library)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class SolveRequest:
    plan: Any          # paper_2412_14973_amd.Plan
    D: Any             # device complex64 ns x nr (Hilbert order), or None: made at admission
    U: Any
    theta0: Any
    iters: int
    precision: int = 0
    lbfgs_m: int = 5
    line_products: int = 0    # LINE_DENSE, LINE_TILE or LINE_TILE_GRAD
    # inputs produced at admission, on the request's stream: make_inputs() -> (D, U, theta0) as above;
    # make_bytes: the device memory that takes beyond D, U and theta0 themselves (transients)
    make_inputs: Optional[Callable[[], tuple]] = None
    make_bytes: int = 0


class GpuBackend:
    """Runs each admitted solve on its own stream from a fixed pool (default priority)."""

    def __init__(self, n_streams: int = 4, clock=None):
        import torch

        from . import make_opts
        self.torch = torch
        self.make_opts = make_opts
        self.clock = clock or WallClock()
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))

    def footprint(self, req: SolveRequest) -> int:
        """Device bytes a solve holds while admitted: the solve workspace, theta in and out, the
        f-history, the inputs D and U, and the transients of making them at admission."""
        from . import _lib
        opts = self.make_opts(req.iters, lbfgs_m=req.lbfgs_m, precision=req.precision,
                              line_products=req.line_products)
        ws = req.plan.workspace_bytes(_lib.OP_SOLVE, opts)
        inputs = 2 * 8 * req.plan.ns * req.plan.nr
        return ws + 2 * 8 * req.plan.theta_size + 8 * (req.iters + 1) + inputs + int(req.make_bytes)

    def start(self, req: SolveRequest):
        from . import solve
        torch = self.torch
        sidx = self.free_streams.pop(0)
        stream = self.streams[sidx]
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            D, U, th0 = (req.D, req.U, req.theta0) if req.make_inputs is None else req.make_inputs()
            theta, fh = solve(req.plan, D, U, th0, req.iters, lbfgs_m=req.lbfgs_m,
                              precision=req.precision, line_products=req.line_products)
            ev = torch.cuda.Event()
            ev.record(stream)
        # the inputs stay referenced until the solve is finished (made ones are freed then)
        return {"event": ev, "stream": sidx, "theta": theta, "fhist": fh, "inputs": (D, U, th0)}

    def done(self, handle) -> bool:
        return handle["event"].query()

    def finish(self, handle):
        handle["event"].synchronize()
        self.free_streams.append(handle["stream"])
        return {"theta": handle["theta"], "fhist": handle["fhist"]}


# ---------------------------------------------------------------------------
# simulated backend (CPU tests of the policy)
# ---------------------------------------------------------------------------
class SimBackend:
    """Simulated device: request payload = dict(bytes=..., service=...); a job's
    service time stretches by the number of jobs sharing the device (processor
    sharing with `width` solves at full speed)."""

    def __init__(self, width: int = 1, fail: Callable[[Any], bool] = lambda p: False):
        self.clock = VirtualClock()
        self.width = width
        self.fail = fail
        self.running: Dict[int, dict] = {}
        self.next_id = 0
        self.t_last = 0.0

    def _advance(self):
        now = self.clock.now()
        dt = now - self.t_last
        if dt > 0 and self.running:
            share = min(1.0, self.width / len(self.running))
            for h in self.running.values():
                h["left"] -= dt * share
        self.t_last = now

    def footprint(self, payload) -> int:
        return int(payload["bytes"])

    def start(self, payload):
        self._advance()
        h = {"id": self.next_id, "left": float(payload["service"]), "payload": payload}
        self.next_id += 1
        self.running[h["id"]] = h
        return h

    def done(self, h) -> bool:
        self._advance()
        return h["left"] <= 1e-12

    def finish(self, h):
        del self.running[h["id"]]
        p = h["payload"]
        return {"ok": not self.fail(p), "value": p.get("value")}
