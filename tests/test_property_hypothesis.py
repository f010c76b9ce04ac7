"""Property-based tests (Hypothesis) of host logic and the oracle, on the CPU.

* The continuous-batching scheduler, driven by randomly drawn request streams
  against a fake library that checks slots and memory on every load: each
  request ends exactly once, oversized requests are rejected, admission is
  first-come first-served, and the slot and memory budgets always hold.
* The oracle's updates keep the majorisation-minimisation guarantee (Sec. 4
  for block updates, Sec. 5 for J-CoMM): on random small CP and Tucker
  problems and random beta in [0, 2), the objective does not increase.  A
  wrong exponent, a swapped numerator and denominator or a missing anchor in
  the update breaks this on some draw.
* The beta-divergence is nonnegative, zero on the diagonal and homogeneous of
  degree beta (Sec. 3.2) at random points."""
import math

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from oracle import cp as ocp  # noqa: E402
from oracle import tucker as otk  # noqa: E402
from oracle.divergence import beta_divergence, objective  # noqa: E402
from paper_2602_14683_amd.serving import Server  # noqa: E402
from tests.test_serving_scheduler import Clock, WorkspaceExecutor, wreq  # noqa: E402

SETTINGS = settings(max_examples=60, deadline=None, derandomize=True)

requests = st.lists(st.tuples(st.floats(0.0, 40.0), st.integers(1, 70), st.integers(0, 40), st.integers(1, 5)),
                    min_size=1, max_size=14)


@SETTINGS
@given(reqs=requests, budget=st.integers(40, 200), slots=st.integers(1, 5))
def test_scheduler_invariants(reqs, budget, slots):
    clk = Clock()
    ex = WorkspaceExecutor(clk, budget, slots)  # asserts slots and memory on every load
    srv = Server(ex, budget, slots, clock=clk, wait=clk.wait, max_iters=50)
    stream = [wreq(k, t, fp, ws, n) for k, (t, fp, ws, n) in enumerate(reqs)]
    done = srv.run(stream)
    by_rid = {c.rid: c for c in done}
    assert len(done) == len(stream) == len(by_rid)
    for r in stream:
        c = by_rid[r.rid]
        fp, ws = r.payload["fp"], r.payload["ws"]
        if fp + math.ceil(1.25 * ws) > budget:
            assert c.status == "rejected"
        assert c.admitted >= r.arrival - 1e-12 and c.finished >= c.admitted
    served = sorted((c for c in done if c.status != "rejected"), key=lambda c: (c.arrival, c.rid))
    assert all(a.admitted <= b.admitted for a, b in zip(served, served[1:]))  # FIFO
    assert srv.peak_slots <= slots and srv.peak_bytes <= budget
    assert not ex.resident


betas = st.one_of(st.sampled_from([0.0, 0.5, 1.0, 1.5]), st.floats(0.05, 1.95))


def _cp_problem(seed, dims, R):
    rng = np.random.default_rng(seed)
    planted = [rng.uniform(0.1, 1.0, size=(d, R)) for d in dims]
    X = rng.poisson(ocp.rebuild(planted) * 3.0).astype(np.float64) + rng.uniform(0.0, 0.5, size=dims)
    init = [rng.uniform(0.1, 1.0, size=(d, R)) for d in dims]
    return X, init


@SETTINGS
@given(seed=st.integers(0, 10_000), dims=st.tuples(*[st.integers(2, 5)] * 3), R=st.integers(1, 3), beta=betas,
       n=st.integers(0, 2))
def test_cp_block_update_does_not_increase_the_objective(seed, dims, R, beta, n):
    X, init = _cp_problem(seed, dims, R)
    before = objective(X, ocp.rebuild(init), beta)
    new = list(init)
    new[n] = ocp.block_update(X, init, n, beta)
    after = objective(X, ocp.rebuild(new), beta)
    assert after <= before * (1 + 1e-12) + 1e-12


@SETTINGS
@given(seed=st.integers(0, 10_000), dims=st.tuples(*[st.integers(2, 5)] * 3), R=st.integers(1, 3), beta=betas,
       L=st.integers(1, 3))
def test_cp_jcomm_outer_does_not_increase_the_objective(seed, dims, R, beta, L):
    X, init = _cp_problem(seed, dims, R)
    cur, fref = ocp.jcomm_outer(X, init, beta, L=L, return_ref_obj=True)
    after = objective(X, ocp.rebuild(cur), beta)
    assert after <= fref * (1 + 1e-12) + 1e-12


@SETTINGS
@given(seed=st.integers(0, 10_000), dims=st.tuples(*[st.integers(2, 4)] * 3),
       J=st.tuples(*[st.integers(1, 2)] * 3), beta=betas, L=st.integers(1, 2))
def test_tucker_jcomm_outer_does_not_increase_the_objective(seed, dims, J, beta, L):
    rng = np.random.default_rng(seed)
    core = rng.uniform(0.1, 1.0, size=J)
    fac = [rng.uniform(0.1, 1.0, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(otk.rebuild(core, fac) * 3.0).astype(np.float64) + rng.uniform(0.0, 0.5, size=dims)
    c0 = rng.uniform(0.1, 1.0, size=J)
    f0 = [rng.uniform(0.1, 1.0, size=(d, j)) for d, j in zip(dims, J)]
    core1, fac1, fref = otk.jcomm_outer(X, c0, f0, beta, L=L, return_ref_obj=True)
    after = objective(X, otk.rebuild(core1, fac1), beta)
    assert after <= fref * (1 + 1e-12) + 1e-12


@SETTINGS
@given(x=st.floats(1e-3, 1e3), y=st.floats(1e-3, 1e3), c=st.floats(1e-2, 1e2), beta=betas)
def test_divergence_properties(x, y, c, beta):
    d = float(beta_divergence(x, y, beta))
    assert d >= -1e-12 * max(1.0, abs(x) ** max(beta, 1e-9), abs(y) ** max(beta, 1e-9))
    assert abs(float(beta_divergence(x, x, beta))) <= 1e-12 * max(1.0, x ** beta)
    scaled = float(beta_divergence(c * x, c * y, beta))
    assert math.isclose(scaled, c ** beta * d, rel_tol=1e-7, abs_tol=1e-9 * max(1.0, c ** beta * (x + y) ** beta))
