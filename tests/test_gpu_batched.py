"""Batched J-CoMM (comm_jcomm_outer_batched) and the serving loop on the GPU.

* A mixed batch (CP and Tucker, ragged shapes, ranks, core sizes, beta, L,
  cached and recomputed P~/Q~) gives, problem by problem, bitwise the result
  of comm_jcomm_outer on that problem alone, eagerly and through graph
  replays; every replay is checked, with eager work and synchronisations in
  between, and the batch is changed mid-way so the graph is captured anew.
* One batched iteration matches the FP64 oracle per problem (1e-4 relative on
  parameters after an outer iteration, 1e-5 on the objective).
* Served requests give the same iteration count and bitwise the same factors
  alone and in the mix.
"""
import numpy as np
import pytest

import workloads
from oracle import cp as ocp
from oracle import tucker as otk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from paper_2602_14683_amd import serving  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

# (kind, dims, rank or core dims, beta, L, cache_pq)
MIX = [
    ("cp", (20, 33, 47), 5, 1.0, 2, False),
    ("tucker", (37, 21, 30), (4, 6, 5), 0.0, 1, False),
    ("cp", (64, 48, 70), 32, 0.5, 1, True),
    ("tucker", (16, 40, 33), (8, 8, 8), 1.5, 2, True),
    ("cp", (17, 16, 129), 8, 0.0, 1, False),
    ("tucker", (50, 45, 24), (16, 3, 7), 1.0, 1, False),
    ("cp", (33, 90, 31), 16, 1.5, 2, False),
    ("cp", (40, 40, 40), 4, 0.7, 1, False),
]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _problem(k, spec):
    kind, dims, r, beta, L, cache = spec
    rng = np.random.default_rng(100 + k)
    if kind == "cp":
        fac = [rng.uniform(0.0, 1.0, size=(d, r)) for d in dims]
        X = rng.poisson(ocp.rebuild(fac) * 2.0).astype(np.float64)
        init = [f32(rng.uniform(0.1, 1.0, size=(d, r))) for d in dims]
        core = None
    else:
        core0 = rng.uniform(0.0, 1.0, size=r)
        fac = [rng.uniform(0.0, 1.0, size=(d, j)) for d, j in zip(dims, r)]
        X = rng.poisson(otk.rebuild(core0, fac)).astype(np.float64)
        init = [f32(rng.uniform(0.1, 1.0, size=(d, j))) for d, j in zip(dims, r)]
        core = f32(rng.uniform(0.1, 1.0, size=r))
    if beta == 0.0:
        X = np.maximum(X, 1e-12)
    return {"X64": X, "init": init, "core0": core, "beta": beta, "L": L, "cache": cache}


def _device(p, obj):
    return {"X": dev(p["X64"]), "factors": [dev(a) for a in p["init"]],
            "core": dev(p["core0"]) if p["core0"] is not None else None,
            "beta": p["beta"], "L": p["L"], "cache_pq": p["cache"], "obj_out": obj}


def _state(d):
    out = [host64(a) for a in d["factors"]]
    if d["core"] is not None:
        out.append(host64(d["core"]))
    return out


@pytest.fixture(scope="module")
def problems():
    return [_problem(k, s) for k, s in enumerate(MIX)]


def _alone_step(ctx, d):
    ctx.jcomm_outer(d["X"], d["factors"], core=d["core"], beta=d["beta"], L=d["L"], cache_pq=d["cache_pq"],
                    obj_out=d["obj_out"])


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("grouped", [False, True])
def test_batched_equals_alone_bitwise(ctx, problems, graph, grouped):
    n = len(problems)
    ob_batch = torch.zeros(n, dtype=torch.float64, device="cuda")
    ob_alone = torch.zeros(n, dtype=torch.float64, device="cuda")
    bat = [_device(p, ob_batch[k:k + 1]) for k, p in enumerate(problems)]
    alo = [_device(p, ob_alone[k:k + 1]) for k, p in enumerate(problems)]
    batch = comm.Batch(bat)
    for it in range(4):
        ctx.jcomm_outer_batched(batch, graph=graph, grouped=grouped)
        for d in alo:
            _alone_step(ctx, d)
        torch.cuda.synchronize()
        assert torch.equal(ob_batch, ob_alone), f"objectives differ at iteration {it}"
        for k in range(n):
            for a, b in zip(_state(bat[k]), _state(alo[k])):
                assert np.array_equal(a, b), f"problem {k} differs at iteration {it}"
    # change the batch (drop two problems, reorder): recaptured, still exact
    sub = [bat[5], bat[0], bat[3], bat[7], bat[1], bat[6]]
    sub_alone = [alo[5], alo[0], alo[3], alo[7], alo[1], alo[6]]
    batch2 = comm.Batch(sub)
    for it in range(3):
        ctx.jcomm_outer_batched(batch2, graph=graph, grouped=grouped)
        for d in sub_alone:
            _alone_step(ctx, d)
        torch.cuda.synchronize()
        for d, e in zip(sub, sub_alone):
            for a, b in zip(_state(d), _state(e)):
                assert np.array_equal(a, b), f"changed batch differs at iteration {it}"


# repeats of each shape so that grouped launches hold several problems; bf16
# tiles, ranks on both tile widths, both models, every beta class
GROUP_MIX = [
    ("cp", (40, 36, 50), 8, 1.0, 1, False, "fp32"),
    ("cp", (40, 36, 50), 8, 1.0, 1, False, "fp32"),
    ("cp", (33, 70, 41), 32, 0.5, 1, True, "fp32"),
    ("cp", (33, 70, 41), 32, 0.5, 1, True, "fp32"),
    ("cp", (33, 70, 41), 32, 0.5, 1, False, "bf16"),
    ("cp", (19, 23, 90), 16, 0.0, 2, False, "fp32"),
    ("cp", (19, 23, 90), 12, 1.5, 1, True, "fp32"),
    ("tucker", (30, 28, 26), (6, 5, 4), 1.0, 1, False, "fp32"),
    ("tucker", (30, 28, 26), (6, 5, 4), 1.0, 1, False, "fp32"),
    ("tucker", (44, 20, 36), (8, 8, 8), 0.0, 1, True, "fp32"),
    ("tucker", (44, 20, 36), (8, 8, 8), 1.5, 2, False, "bf16"),
    ("cp", (256, 17, 33), 4, 0.7, 1, False, "fp32"),
]


@pytest.mark.parametrize("graph", [False, True])
def test_grouped_repeats_and_precisions_bitwise(ctx, graph):
    """Grouped launches over repeated shapes, bf16 and float32 tiles: every
    problem bitwise equal to its single call, over several replays."""
    probs = [_problem(200 + k, spec[:6]) for k, spec in enumerate(GROUP_MIX)]
    n = len(probs)
    ob_b = torch.zeros(n, dtype=torch.float64, device="cuda")
    ob_a = torch.zeros(n, dtype=torch.float64, device="cuda")
    bat = [dict(_device(p, ob_b[k:k + 1]), precision=GROUP_MIX[k][6]) for k, p in enumerate(probs)]
    alo = [dict(_device(p, ob_a[k:k + 1]), precision=GROUP_MIX[k][6]) for k, p in enumerate(probs)]
    batch = comm.Batch(bat)
    for it in range(3):
        ctx.jcomm_outer_batched(batch, graph=graph, grouped=True)
        for d in alo:
            ctx.jcomm_outer(d["X"], d["factors"], core=d["core"], beta=d["beta"], L=d["L"], cache_pq=d["cache_pq"],
                            obj_out=d["obj_out"], precision=d["precision"])
        torch.cuda.synchronize()
        assert torch.equal(ob_b, ob_a), f"objectives differ at iteration {it}"
        for k in range(n):
            for a, b in zip(_state(bat[k]), _state(alo[k])):
                assert np.array_equal(a, b), f"problem {k} differs at iteration {it}"


def test_grouped_batch_with_order4_runs_ungrouped(ctx, problems):
    """A batch holding an order-4 problem runs ungrouped, still exact."""
    rng = np.random.default_rng(7)
    dims4, R = (6, 7, 8, 9), 3
    X4 = rng.poisson(ocp.rebuild([rng.uniform(0, 1, size=(d, R)) for d in dims4]) * 3.0).astype(np.float64)
    init4 = [f32(rng.uniform(0.1, 1.0, size=(d, R))) for d in dims4]
    obj = torch.zeros(2, dtype=torch.float64, device="cuda")
    d3 = _device(problems[0], obj[0:1])
    d4 = {"X": dev(X4), "factors": [dev(a) for a in init4], "core": None, "beta": 1.0, "L": 1, "cache_pq": False,
          "obj_out": obj[1:2]}
    e3 = _device(problems[0], torch.zeros(1, dtype=torch.float64, device="cuda"))
    e4 = dict(d4, factors=[dev(a) for a in init4], obj_out=torch.zeros(1, dtype=torch.float64, device="cuda"))
    ctx.jcomm_outer_batched(comm.Batch([d3, d4]), grouped=True)
    for d in (e3, e4):
        _alone_step(ctx, d)
    torch.cuda.synchronize()
    for x, y in ((d3, e3), (d4, e4)):
        for a, b in zip(_state(x), _state(y)):
            assert np.array_equal(a, b)


def test_batched_matches_oracle(ctx, problems):
    n = len(problems)
    obj = torch.zeros(n, dtype=torch.float64, device="cuda")
    bat = [_device(p, obj[k:k + 1]) for k, p in enumerate(problems)]
    ctx.jcomm_outer_batched(comm.Batch(bat), graph=True)
    torch.cuda.synchronize()
    got_obj = obj.cpu().numpy()
    for k, p in enumerate(problems):
        if p["core0"] is None:
            want, fref = ocp.jcomm_outer(p["X64"], p["init"], p["beta"], L=p["L"], return_ref_obj=True)
            got = _state(bat[k])
        else:
            wc, wf, fref = otk.jcomm_outer(p["X64"], p["core0"], p["init"], p["beta"], L=p["L"],
                                           return_ref_obj=True)
            want = list(wf) + [wc]
            got = _state(bat[k])
        for a, b in zip(got, want):
            assert max_rel(a, b) < 1e-4, f"problem {k}"
        assert abs(got_obj[k] - fref) / fref < 1e-5, f"problem {k}"


def test_batched_rejects_bad_problem_before_launching(ctx, problems):
    obj = torch.zeros(2, dtype=torch.float64, device="cuda")
    good = _device(problems[0], obj[0:1])
    bad = _device(problems[2], obj[1:2])
    before = _state(good)
    bad["beta"] = 2.5
    with pytest.raises(comm.CommError) as e:
        ctx.jcomm_outer_batched(comm.Batch([good, bad]))
    assert e.value.code == comm.COMM_EINVAL and "problem 1" in str(e.value)
    torch.cuda.synchronize()
    for a, b in zip(_state(good), before):
        assert np.array_equal(a, b)


def test_batched_workspace_limit(problems):
    small = comm.Context(0, workspace_limit=1 << 16)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    d = _device(problems[2], obj)
    with pytest.raises(comm.CommError) as e:
        small.jcomm_outer_batched(comm.Batch([d]))
    assert e.value.code == comm.COMM_ENOMEM
    small.close()


def test_empty_batch_is_a_no_op(ctx):
    ctx.jcomm_outer_batched(comm.Batch([]), graph=True)
    torch.cuda.synchronize()


class StepClock:
    """Virtual time: one unit per batched step, so admission is reproducible."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 0.0)


class CountingExecutor(serving.BatchedExecutor):
    def __init__(self, clock, *a, **k):
        super().__init__(*a, **k)
        self.clock = clock

    def step(self, handles):
        self.clock.t += 1.0
        return super().step(handles)


def test_served_results_same_alone_and_in_the_mix(ctx):
    specs = workloads.serving_specs(seed=3, count=8, rate=2.0, dim_range=(16, 48))
    decs = [serving.from_workload(workloads.materialize(s)) for s in specs]
    reqs = [serving.ServeRequest(s.rid, s.arrival, d) for s, d in zip(specs, decs)]
    clk = StepClock()
    ex = CountingExecutor(clk, ctx, max_slots=4, graph=True)
    srv = serving.Server(ex, hbm_budget=1 << 30, max_slots=4, tol=1e-4, max_iters=60, clock=clk, wait=clk.wait)
    mixed = {c.rid: c for c in srv.run(reqs)}
    assert srv.peak_slots > 1  # the requests really overlapped
    for r in reqs:
        clk1 = StepClock()
        ex1 = serving.SingleExecutor(ctx, max_slots=1)
        alone = serving.Server(ex1, 1 << 30, 1, tol=1e-4, max_iters=60, clock=clk1, wait=clk1.wait)
        c = alone.run([serving.ServeRequest(r.rid, 0.0, r.payload)])[0]
        m = mixed[r.rid]
        assert c.iters == m.iters and c.status == m.status
        assert c.objective == m.objective
        for a, b in zip(c.result["factors"], m.result["factors"]):
            assert np.array_equal(a, b)
        if c.result["core"] is not None:
            assert np.array_equal(c.result["core"], m.result["core"])
