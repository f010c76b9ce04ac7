"""Continuous-batching server for nonnegative CP / Tucker decomposition requests.

Requests arrive over time, each a dense 3-way tensor with its own shape, model
(CP rank or Tucker core size) and beta.  The server keeps every admitted
request's tensor, parameters and workspace on the device and advances all of
them together: one batched J-CoMM outer iteration per step
(``comm_jcomm_outer_batched``), then one read of all their objectives.  A
request leaves when its objective changes by less than ``tol`` (relative)
between two outer iterations, or after ``max_iters``; requests that arrived
meanwhile are admitted first-come first-served as soon as a slot and enough
device memory are free (admission by footprint: tensor + parameters +
workspace bytes).  A request's iterates do not depend on what else is in the
batch, so it converges in the same number of iterations, to the same factors,
alone or in the mix.

The scheduler (:class:`Server`) is host logic and talks to an *executor*:

* ``footprint(payload) -> int``   device bytes of its own data while resident
* ``workspace(payload) -> int``   (optional) library workspace bytes it needs; the
                                   executor's ``ws_growth`` says how the library
                                   sizes the shared workspace (a factor over the
                                   active requests' sum, never shrunk)
* ``load(payload) -> handle``     put the request on the device
* ``step(handles) -> [float]``    one outer iteration for each handle, returns
                                   the objective at each reference point
* ``unload(handle) -> result``    take the result off the device, free it

:class:`BatchedExecutor` runs the batch through the library (graph replay while
the batch is unchanged); :class:`SingleExecutor` is the plain per-request loop
(one ``comm_jcomm_outer`` call and one objective read per iteration).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class ServeRequest:
    rid: int
    arrival: float        # seconds after the start of the stream
    payload: Any          # what the executor loads


@dataclasses.dataclass
class Completion:
    rid: int
    arrival: float
    admitted: float
    finished: float
    iters: int
    objective: float      # objective at the last reference point
    status: str           # "converged", "max_iters" or "rejected"
    result: Any = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Active:
    req: ServeRequest
    handle: Any
    footprint: int
    workspace: int
    admitted: float
    iters: int = 0
    prev: Optional[float] = None


class Server:
    """First-come first-served continuous batching under a slot and a memory budget."""

    def __init__(self, executor, hbm_budget: int, max_slots: int, tol: float = 1e-4, max_iters: int = 1000,
                 clock: Callable[[], float] = time.perf_counter, wait: Optional[Callable[[float], None]] = None):
        if max_slots < 1:
            raise ValueError("max_slots must be >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.tol = float(tol)
        self.max_iters = int(max_iters)
        self.clock = clock
        self.wait = wait or (lambda dt: time.sleep(max(dt, 0.0)))
        self.peak_bytes = 0
        self.peak_slots = 0
        self.steps = 0
        self.mem_waits = 0        # admissions held back for memory (head of the queue)
        self.ws_reserved = 0      # workspace the library keeps (it grows, never shrinks)
        self._ws = getattr(executor, "workspace", None)
        self._growth = float(getattr(executor, "ws_growth", 1.0))

    def run(self, requests: Sequence[ServeRequest]) -> List[Completion]:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        active: List[_Active] = []
        done: List[Completion] = []
        used = 0       # the active requests' own data
        ws_active = 0  # the active requests' workspace needs
        held = None    # rid of the head last held back for memory
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission: FIFO; the head waits for room rather than being overtaken
            while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                r = pending[0]
                fp = int(self.ex.footprint(r.payload))
                ws = int(self._ws(r.payload)) if self._ws else 0
                reserve = max(self.ws_reserved, math.ceil(self._growth * (ws_active + ws)))
                alone = max(self.ws_reserved, math.ceil(self._growth * ws))
                if fp + math.ceil(self._growth * ws) > self.budget or (not active and fp + alone > self.budget):
                    # can never fit (or cannot fit even alone, next to the workspace
                    # the library already holds)
                    pending.popleft()
                    done.append(Completion(r.rid, r.arrival, now, now, 0, float("nan"), "rejected"))
                    continue
                if used + fp + reserve > self.budget:
                    if held != r.rid:
                        self.mem_waits += 1
                        held = r.rid
                    break
                pending.popleft()
                active.append(_Active(r, self.ex.load(r.payload), fp, ws, now))
                used += fp
                ws_active += ws
                self.ws_reserved = reserve
                self.peak_bytes = max(self.peak_bytes, used + self.ws_reserved)
            self.peak_slots = max(self.peak_slots, len(active))
            if not active:
                if pending:
                    self.wait(pending[0].arrival - (self.clock() - t0))
                continue
            objs = self.ex.step([a.handle for a in active])
            self.steps += 1
            now = self.clock() - t0
            keep = []
            for a, f in zip(active, objs):
                a.iters += 1
                f = float(f)
                converged = a.prev is not None and abs(a.prev - f) <= self.tol * abs(a.prev)
                a.prev = f
                if converged or a.iters >= self.max_iters:
                    res = self.ex.unload(a.handle)
                    used -= a.footprint
                    ws_active -= a.workspace
                    done.append(Completion(a.req.rid, a.req.arrival, a.admitted, now, a.iters, f,
                                           "converged" if converged else "max_iters", res))
                else:
                    keep.append(a)
            active = keep
        return done


def summarize(done: Sequence[Completion]) -> dict:
    """Solves/s over the span from the first arrival to the last completion,
    and latency percentiles (ms) over the served requests."""
    served = [c for c in done if c.status != "rejected"]
    if not served:
        return {"served": 0, "rejected": len(done), "solves_per_s": 0.0}
    lat = np.array([c.latency for c in served]) * 1e3
    queue = np.array([c.admitted - c.arrival for c in served]) * 1e3
    span = max(c.finished for c in served) - min(c.arrival for c in served)
    return {"served": len(served), "rejected": len(done) - len(served),
            "converged": sum(c.status == "converged" for c in served),
            "solves_per_s": len(served) / span if span > 0 else float("inf"),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "queue_p50_ms": float(np.percentile(queue, 50)), "queue_p99_ms": float(np.percentile(queue, 99)),
            "mean_iters": float(np.mean([c.iters for c in served])), "span_s": span}


# ----------------------------------------------------------------------------------------------- executors

@dataclasses.dataclass
class Decomposition:
    """A request's tensor, model and options on the host (float32)."""
    X: np.ndarray
    factors: List[np.ndarray]
    core: Optional[np.ndarray] = None
    beta: float = 1.0
    L: int = 1
    eps: float = 1e-12
    precision: str = "fp32"
    tag: Any = None       # the caller's label, returned with the result


def from_workload(req, precision: str = "fp32") -> Decomposition:
    """A :class:`Decomposition` from a generated serving request (``workloads.Request``)."""
    s = req.spec
    if s.model == "cp":
        return Decomposition(req.X.astype(np.float32), [a.astype(np.float32) for a in req.init], None, s.beta,
                             precision=precision)
    return Decomposition(req.X.astype(np.float32), [a.astype(np.float32) for a in req.init[1:]],
                         req.init[0].astype(np.float32), s.beta, precision=precision)


class _DeviceBase:
    # the library sizes a grown workspace at 1.25 x the need and keeps it
    ws_growth = 1.25

    def __init__(self, ctx, max_slots: int):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.objs = torch.zeros(max_slots, dtype=torch.float64, device="cuda")
        self.free = list(range(max_slots))[::-1]

    def footprint(self, d: Decomposition) -> int:
        params = sum(a.size for a in d.factors) + (d.core.size if d.core is not None else 0)
        return 4 * (d.X.size + params)

    def workspace(self, d: Decomposition) -> int:
        ws = self.ctx.workspace_bytes(d.X.shape, rank=d.factors[0].shape[1],
                                      core_dims=None if d.core is None else d.core.shape, beta=d.beta, L=d.L)
        return ((ws + 255) // 256) * 256

    def load(self, d: Decomposition) -> dict:
        torch = self.torch
        slot = self.free.pop()
        h = {"slot": slot, "X": torch.from_numpy(d.X).cuda(),
             "factors": [torch.from_numpy(a).cuda() for a in d.factors],
             "core": torch.from_numpy(d.core).cuda() if d.core is not None else None,
             "beta": d.beta, "L": d.L, "eps": d.eps, "precision": d.precision,
             "obj_out": self.objs[slot:slot + 1], "tag": d.tag}
        return h

    def unload(self, h: dict) -> dict:
        out = {"factors": [a.cpu().numpy() for a in h["factors"]],
               "core": h["core"].cpu().numpy() if h["core"] is not None else None, "tag": h["tag"]}
        self.free.append(h["slot"])
        return out


class BatchedExecutor(_DeviceBase):
    """All active requests advance in one ``comm_jcomm_outer_batched`` call; the
    problem list is marshalled once per change of the batch, and with
    ``graph=True`` the library replays a captured HIP graph until it changes;
    ``grouped=True`` has it launch each kernel once for all requests."""

    def __init__(self, ctx, max_slots: int, graph: bool = True, grouped: bool = False):
        super().__init__(ctx, max_slots)
        self.graph = graph
        self.grouped = grouped
        self._ids = None
        self._batch = None

    def step(self, handles: Sequence[dict]) -> List[float]:
        from . import Batch
        ids = [id(h) for h in handles]
        if ids != self._ids:
            self._batch = Batch(handles)
            self._ids = ids
        self.ctx.jcomm_outer_batched(self._batch, graph=self.graph, grouped=self.grouped)
        host = self.objs.cpu().numpy()
        return [float(host[h["slot"]]) for h in handles]

    def unload(self, h: dict) -> dict:
        self._ids = None
        return super().unload(h)


class SingleExecutor(_DeviceBase):
    """The plain per-request loop: one ``comm_jcomm_outer`` call and one
    objective read per outer iteration (run it with ``max_slots = 1``)."""

    def step(self, handles: Sequence[dict]) -> List[float]:
        out = []
        for h in handles:
            self.ctx.jcomm_outer(h["X"], h["factors"], core=h["core"], beta=h["beta"], L=h["L"], eps=h["eps"],
                                 obj_out=h["obj_out"], precision=h["precision"])
            out.append(float(h["obj_out"].item()))
        return out
