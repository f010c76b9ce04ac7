"""Extrapolated B-CoMM and J-CoMM (comm_bcomm_sweep_extrap,
comm_jcomm_outer_extrap) against oracle/extrapolation.py, over several chained
outer iterations so that the previous-iterate bookkeeping is exercised.

Bars: the weight alpha_t to 1e-6 relative (float64 norm, stored as float32);
parameters to 1e-4 relative after up to four chained outer iterations (the
per-update bar is 1e-5; the chain compounds it), the objective at the
reference to 1e-5."""
import numpy as np
import pytest

from oracle import cp as ocp
from oracle import extrapolation as ox
from oracle import tucker as otk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

ITERS = 4
C, DELTA = 0.5, 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _cp(seed, dims=(30, 41, 50), R=6):
    rng = np.random.default_rng(seed)
    X = np.maximum(rng.poisson(ocp.rebuild([rng.uniform(0, 1, (d, R)) for d in dims]) * 3).astype(np.float64), 1e-12)
    cur = [f32(rng.uniform(0.1, 1.0, (d, R))) for d in dims]
    prev = [f32(a * rng.uniform(0.5, 1.2, a.shape)) for a in cur]
    return X, cur, prev


def _tk(seed, dims=(30, 41, 50), J=(4, 5, 3)):
    rng = np.random.default_rng(seed)
    X = np.maximum(rng.poisson(otk.rebuild(rng.uniform(0, 1, J), [rng.uniform(0, 1, (d, j))
                                                                  for d, j in zip(dims, J)]) * 2).astype(np.float64),
                   1e-12)
    core = f32(rng.uniform(0.1, 1.0, J))
    cur = [f32(rng.uniform(0.1, 1.0, (d, j))) for d, j in zip(dims, J)]
    pcore = f32(core * rng.uniform(0.5, 1.2, J))
    prev = [f32(a * rng.uniform(0.5, 1.2, a.shape)) for a in cur]
    return X, core, cur, pcore, prev


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5])
def test_cp_extrapolated_bcomm(ctx, beta):
    X, cur, prev = _cp(1)
    Xd = dev(X)
    F, P = [dev(a) for a in cur], [dev(a) for a in prev]
    alpha = torch.zeros(1, dtype=torch.float32, device="cuda")
    wc, wp = cur, prev
    for t in range(1, ITERS + 1):
        an = ox.nesterov_weight(t + 1)
        w_alpha = ox.weight(wc, wp, an, C, DELTA)
        want, want_prev = ox.cp_bcomm_sweep(X, wc, wp, beta, w_alpha)
        ctx.bcomm_sweep_extrap(Xd, F, P, beta=beta, alpha_nes=an, c=C, delta=DELTA, alpha_out=alpha)
        torch.cuda.synchronize()
        assert abs(alpha.item() - w_alpha) <= 1e-6 * max(w_alpha, 1e-30)
        for a, b in zip(F, want):
            assert max_rel(host64(a), b) < 1e-4
        for a, b in zip(P, want_prev):
            assert np.array_equal(host64(a), b)
        # the next step starts from the GPU's own state
        wc, wp = [host64(a) for a in F], [host64(a) for a in P]


@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5])
def test_tucker_extrapolated_bcomm(ctx, beta):
    X, core, cur, pcore, prev = _tk(2)
    Xd = dev(X)
    G, F, PG, P = dev(core), [dev(a) for a in cur], dev(pcore), [dev(a) for a in prev]
    gc, gf, pc, pf = core, cur, pcore, prev
    for t in range(1, ITERS + 1):
        an = ox.nesterov_weight(t + 1)
        w_alpha = ox.weight([gc] + gf, [pc] + pf, an, C, DELTA)
        wg, wf, wpg, wpf = ox.tucker_bcomm_sweep(X, gc, gf, pc, pf, beta, w_alpha)
        ctx.bcomm_sweep_extrap(Xd, F, P, core=G, prev_core=PG, beta=beta, alpha_nes=an, c=C, delta=DELTA)
        torch.cuda.synchronize()
        assert max_rel(host64(G), wg) < 1e-4
        for a, b in zip(F, wf):
            assert max_rel(host64(a), b) < 1e-4
        assert np.array_equal(host64(PG), wpg)
        gc, gf, pc, pf = host64(G), [host64(a) for a in F], host64(PG), [host64(a) for a in P]


@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_cp_extrapolated_jcomm(ctx, beta):
    X, cur, prev = _cp(3)
    Xd = dev(X)
    F, P = [dev(a) for a in cur], [dev(a) for a in prev]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    wc, wp = cur, prev
    for t in range(1, ITERS + 1):
        an = ox.nesterov_weight(t + 1)
        w_alpha = ox.weight(wc, wp, an, C, DELTA)
        want, want_prev, fref = ox.cp_jcomm_outer(X, wc, wp, beta, w_alpha, L=2, return_ref_obj=True)
        ctx.jcomm_outer_extrap(Xd, F, P, beta=beta, L=2, alpha_nes=an, c=C, delta=DELTA, obj_out=obj)
        torch.cuda.synchronize()
        for a, b in zip(F, want):
            assert max_rel(host64(a), b) < 1e-4
        for a, b in zip(P, want_prev):
            assert np.array_equal(host64(a), b)
        assert abs(obj.item() - fref) / fref < 1e-5
        wc, wp = [host64(a) for a in F], [host64(a) for a in P]


@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_tucker_extrapolated_jcomm(ctx, beta):
    X, core, cur, pcore, prev = _tk(4)
    Xd = dev(X)
    G, F, PG, P = dev(core), [dev(a) for a in cur], dev(pcore), [dev(a) for a in prev]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    an = 0.6
    w_alpha = ox.weight([core] + cur, [pcore] + prev, an, C, DELTA)
    wg, wf, wpg, wpf, fref = ox.tucker_jcomm_outer(X, core, cur, pcore, prev, beta, w_alpha, return_ref_obj=True)
    ctx.jcomm_outer_extrap(Xd, F, P, core=G, prev_core=PG, beta=beta, alpha_nes=an, c=C, delta=DELTA, obj_out=obj)
    torch.cuda.synchronize()
    assert max_rel(host64(G), wg) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4
    assert abs(obj.item() - fref) / fref < 1e-5


def test_extrap_rejects_aliased_prev(ctx):
    X, cur, _ = _cp(5)
    F = [dev(a) for a in cur]
    with pytest.raises(comm.CommError) as e:
        ctx.bcomm_sweep_extrap(dev(X), F, F, beta=1.0, alpha_nes=0.5)
    assert e.value.code == comm.COMM_EINVAL


def test_extrapolation_accelerates_kl_bcomm(ctx):
    """Not a guarantee of the method, a check that the inertial step is wired
    as intended: on this planted KL problem, 40 extrapolated sweeps reach a
    lower objective than 40 plain ones from the same start (the FP64 oracle
    gives 6.680e4 against 6.726e4 here, a 0.7% gap far above float32 noise)."""
    rng = np.random.default_rng(7)
    dims, R = (60, 50, 40), 5
    X = rng.poisson(ocp.rebuild([rng.uniform(0, 1, (d, R)) for d in dims]) * 4).astype(np.float64)
    init = [f32(rng.uniform(0.1, 1.0, (d, R))) for d in dims]
    Xd = dev(X)
    Fp = [dev(a) for a in init]
    for _ in range(40):
        ctx.cp_update(Xd, Fp, block=-1, beta=1.0)
    Fe, Pe = [dev(a) for a in init], [dev(a) for a in init]
    for t in range(1, 41):
        ctx.bcomm_sweep_extrap(Xd, Fe, Pe, beta=1.0, alpha_nes=ox.nesterov_weight(t), c=1e3, delta=1e-12)
    plain = ctx.beta_objective(Xd, Fp, beta=1.0).item()
    extrap = ctx.beta_objective(Xd, Fe, beta=1.0).item()
    assert extrap < plain
