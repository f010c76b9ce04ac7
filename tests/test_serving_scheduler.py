"""Host logic of the continuous-batching server, with a fake executor on the CPU.

The fake executor replays a scripted objective sequence per request, charges
one virtual second per batched step and checks the slot and memory budgets on
every load, so these tests pin admission order, budgets, continuous admission,
the stopping rule and the latency bookkeeping without a GPU."""
import math

import numpy as np
import pytest

from paper_2602_14683_amd.serving import Completion, ServeRequest, Server, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor:
    def __init__(self, clock, budget, max_slots, step_cost=1.0):
        self.clock = clock
        self.budget = budget
        self.max_slots = max_slots
        self.step_cost = step_cost
        self.resident = {}
        self.log = []

    def footprint(self, p):
        return p["fp"]

    def load(self, p):
        assert len(self.resident) < self.max_slots
        h = {"p": p, "t": 0}
        self.resident[id(h)] = p["fp"]
        assert sum(self.resident.values()) <= self.budget
        self.log.append(("load", p["name"], self.clock()))
        return h

    def step(self, handles):
        self.clock.t += self.step_cost
        out = []
        for h in handles:
            seq = h["p"]["objs"]
            out.append(seq[min(h["t"], len(seq) - 1)])
            h["t"] += 1
        return out

    def unload(self, h):
        del self.resident[id(h)]
        self.log.append(("unload", h["p"]["name"], self.clock()))
        return h["p"]["name"]


def geometric(n_big, tol=1e-4):
    """Objective sequence whose relative change first drops to <= tol at
    iteration n_big + 1 (1-based): large steps, then a constant."""
    seq = [100.0 * (1.0 + 0.5 ** k) for k in range(n_big)]
    seq += [seq[-1]] * 3
    return seq


def expected_iters(seq, tol=1e-4, max_iters=1000):
    prev = None
    for t, f in enumerate(seq + [seq[-1]] * max_iters, start=1):
        if prev is not None and abs(prev - f) <= tol * abs(prev):
            return t
        if t >= max_iters:
            return t
        prev = f


def req(rid, arrival, fp, n_big, name=None):
    return ServeRequest(rid, arrival, {"fp": fp, "objs": geometric(n_big), "name": name or f"r{rid}"})


def run(reqs, budget=100, slots=4, **kw):
    clk = Clock()
    ex = FakeExecutor(clk, budget, slots)
    srv = Server(ex, budget, slots, clock=clk, wait=clk.wait, **kw)
    done = srv.run(reqs)
    return {c.rid: c for c in done}, ex, srv


def test_every_request_finishes_with_its_own_iteration_count():
    reqs = [req(k, 0.3 * k, 10, n_big=3 + (k * 7) % 11) for k in range(20)]
    done, ex, srv = run(reqs, budget=45, slots=3)
    assert set(done) == set(range(20))
    for r in reqs:
        assert done[r.rid].status == "converged"
        assert done[r.rid].iters == expected_iters(r.payload["objs"])
    assert ex.resident == {}
    assert srv.peak_slots <= 3 and srv.peak_bytes <= 45


def test_memory_budget_limits_concurrency():
    # four requests of 40 bytes under an 100-byte budget: at most two resident
    reqs = [req(k, 0.0, 40, n_big=5) for k in range(4)]
    done, ex, srv = run(reqs, budget=100, slots=8)
    assert srv.peak_bytes == 80 and srv.peak_slots == 2
    loads = [t for kind, _, t in ex.log if kind == "load"]
    assert loads[:2] == [0.0, 0.0] and min(loads[2:]) > 0.0


def test_continuous_admission_joins_a_running_batch():
    # A runs long, B short; C arrives while both are on the device and takes
    # B's slot as soon as B leaves, while A is still running
    a = req(0, 0.0, 10, n_big=12, name="A")
    b = req(1, 0.0, 10, n_big=1, name="B")
    c = req(2, 0.5, 10, n_big=2, name="C")
    done, ex, _ = run([a, b, c], slots=2)
    assert done[1].finished == pytest.approx(2.0)      # B: converges at its 2nd iteration
    assert done[2].admitted == pytest.approx(2.0)      # C admitted right then ...
    assert done[0].finished > done[2].admitted         # ... while A is still running
    assert done[2].latency == pytest.approx(done[2].finished - 0.5)


def test_fifo_head_waits_for_room_and_is_not_overtaken():
    big = req(1, 0.1, 90, n_big=2, name="big")
    small = req(2, 0.2, 5, n_big=2, name="small")
    first = req(0, 0.0, 20, n_big=6, name="first")
    done, ex, _ = run([first, big, small], budget=100, slots=4)
    order = [n for kind, n, _ in ex.log if kind == "load"]
    assert order == ["first", "big", "small"]
    assert done[1].admitted >= done[0].finished


def test_oversized_request_is_rejected_without_blocking():
    reqs = [req(0, 0.0, 500, n_big=2), req(1, 0.0, 10, n_big=2)]
    done, _, _ = run(reqs, budget=100)
    assert done[0].status == "rejected" and done[0].iters == 0
    assert done[1].status == "converged"


def test_max_iters_stops_a_request():
    done, _, _ = run([req(0, 0.0, 10, n_big=50)], max_iters=7)
    assert done[0].status == "max_iters" and done[0].iters == 7


def test_idle_server_waits_for_the_next_arrival():
    done, ex, _ = run([req(0, 5.0, 10, n_big=1)])
    assert done[0].admitted == pytest.approx(5.0)
    assert done[0].finished == pytest.approx(7.0)


def test_same_iterations_alone_and_in_the_mix():
    reqs = [req(k, 0.25 * k, 10, n_big=2 + k % 5) for k in range(12)]
    mixed, _, _ = run(reqs, budget=1000, slots=6)
    for r in reqs:
        alone, _, _ = run([ServeRequest(r.rid, 0.0, r.payload)], slots=1)
        assert alone[r.rid].iters == mixed[r.rid].iters
        assert alone[r.rid].objective == mixed[r.rid].objective


def test_summary_statistics():
    done = [Completion(k, float(k), float(k), float(k) + 1.0 + k, 3, 1.0, "converged") for k in range(100)]
    done.append(Completion(100, 0.0, 0.0, 0.0, 0, math.nan, "rejected"))
    s = summarize(done)
    lat = np.array([1.0 + k for k in range(100)]) * 1e3
    assert s["served"] == 100 and s["rejected"] == 1
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert s["solves_per_s"] == pytest.approx(100 / (99.0 + 1.0 + 99.0))


def test_server_rejects_bad_slot_count():
    with pytest.raises(ValueError):
        Server(None, 10, 0)


class WorkspaceExecutor(FakeExecutor):
    """A fake library whose shared workspace grows to ws_growth x the active
    requests' sum and never shrinks (as the batched path sizes it); every load
    checks data + that workspace against the budget."""
    ws_growth = 1.25

    def __init__(self, clock, budget, max_slots):
        super().__init__(clock, budget, max_slots)
        self.ws_held = 0
        self.ws_need = {}

    def footprint(self, p):
        return p["fp"]

    def workspace(self, p):
        return p["ws"]

    def load(self, p):
        h = {"p": p, "t": 0}
        self.resident[id(h)] = p["fp"]
        self.ws_need[id(h)] = p["ws"]
        self.ws_held = max(self.ws_held, math.ceil(1.25 * sum(self.ws_need.values())))
        assert len(self.resident) <= self.max_slots
        assert sum(self.resident.values()) + self.ws_held <= self.budget
        self.log.append(("load", p["name"], self.clock()))
        return h

    def unload(self, h):
        del self.ws_need[id(h)]
        return super().unload(h)


def wreq(rid, arrival, fp, ws, n_big):
    return ServeRequest(rid, arrival, {"fp": fp, "ws": ws, "objs": geometric(n_big), "name": f"r{rid}"})


def test_admission_counts_the_library_workspace_it_keeps():
    # data 10 + workspace 20 each: two together need 20 + 1.25 * 40 = 70; a
    # third would need 30 + 75 = 105 > 100, so it waits; after both leave the
    # library still holds 50 bytes of workspace, which later admissions count
    clk = Clock()
    ex = WorkspaceExecutor(clk, 100, 8)
    srv = Server(ex, 100, 8, clock=clk, wait=clk.wait)
    reqs = [wreq(0, 0.0, 10, 20, 4), wreq(1, 0.0, 10, 20, 4), wreq(2, 0.0, 10, 20, 2), wreq(3, 20.0, 45, 8, 2)]
    done = {c.rid: c for c in srv.run(reqs)}
    assert all(c.status == "converged" for c in done.values())
    assert done[2].admitted >= min(done[0].finished, done[1].finished)
    assert srv.mem_waits >= 1
    assert srv.ws_reserved == 50 and srv.peak_bytes <= 100


def test_request_that_cannot_fit_beside_the_held_workspace_is_rejected():
    # the first request leaves 1.25 * 60 = 75 bytes of workspace behind; a later
    # one with 30 bytes of data can never fit beside it and must not wait forever
    clk = Clock()
    ex = WorkspaceExecutor(clk, 100, 4)
    srv = Server(ex, 100, 4, clock=clk, wait=clk.wait)
    done = {c.rid: c for c in srv.run([wreq(0, 0.0, 10, 60, 2), wreq(1, 10.0, 30, 4, 2)])}
    assert done[0].status == "converged"
    assert done[1].status == "rejected"
