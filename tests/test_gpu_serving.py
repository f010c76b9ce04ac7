"""Served requests against the float64 oracle (the reading of "bf16 at <= 1e-3
relative objective error against FP64": solution quality).  A short Poisson
stream of small CP and Tucker requests goes through the continuous-batching
server with bf16 tiles; each request runs to a relative objective change of
1e-4.  The oracle runs the same J-CoMM from the same initial parameters with
the same stopping rule in float64, and the two final objectives (at the last
reference point) must agree to 1e-3.  The float32 batched path is held to the
same bar."""
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
from tests.gpu_util import f32  # noqa: E402

TOL, MAX_ITERS = 1e-4, 300


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _oracle_final(m):
    """F at the last reference point of an FP64 J-CoMM run with the server's stopping rule."""
    s = m.spec
    X = m.X
    if s.model == "cp":
        cur = [f32(a) for a in m.init]
    else:
        core, cur = f32(m.init[0]), [f32(a) for a in m.init[1:]]
    prev = None
    for _ in range(MAX_ITERS):
        if s.model == "cp":
            cur, f = ocp.jcomm_outer(X, cur, s.beta, L=1, return_ref_obj=True)
        else:
            core, cur, f = otk.jcomm_outer(X, core, cur, s.beta, L=1, return_ref_obj=True)
        if prev is not None and abs(prev - f) <= TOL * abs(prev):
            return f
        prev = f
    return f


@pytest.fixture(scope="module")
def stream():
    specs = workloads.serving_specs(seed=5, count=8, rate=200.0, dim_range=(16, 36), ranks=(4, 8))
    mats = [workloads.materialize(s) for s in specs]
    return specs, mats, {m.spec.rid: _oracle_final(m) for m in mats}


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_served_objective_matches_fp64_oracle(ctx, stream, prec):
    specs, mats, want = stream
    reqs = [serving.ServeRequest(s.rid, s.arrival, serving.from_workload(m, prec)) for s, m in zip(specs, mats)]
    srv = serving.Server(serving.BatchedExecutor(ctx, 4, graph=True), 8 << 30, 4, tol=TOL, max_iters=MAX_ITERS)
    done = {c.rid: c for c in srv.run(reqs)}
    assert set(done) == {s.rid for s in specs}
    for rid, c in done.items():
        assert c.status == "converged", (rid, c.status)
        assert abs(c.objective - want[rid]) / want[rid] < 1e-3, (rid, c.objective, want[rid])
