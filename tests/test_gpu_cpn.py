"""GPU parity of dense CP of order 4 and 5 against the FP64 oracle (which is
written for any order), through the C ABI.

The library runs these orders through a 3-way view of the same memory (modes
1..N-2 fused, their factor the Khatri-Rao product) and folds the fused mode's
numerator back into each grouped mode's; the oracle contracts the order-N
tensor directly (Sec. 6.1), so a mistake in the grouping, the product or the
fold shows up here.  Bars as for order 3: 1e-5 relative per factor entry after
one block update, 3e-5 after a sweep or two inner sweeps, 1e-5 on the
objective; bf16 tiles as in the order-3 bf16 tests (8e-3 per entry)."""
import numpy as np
import pytest

from oracle import cp as ocp
from oracle import extrapolation as ox
from oracle.divergence import objective as oobjective

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

TOL = 1e-5
# ragged in every mode; the fused mode spans several 16-row tiles; order 5
# fuses three modes; a grouped mode of extent 1; rank 32 fills the tile
SHAPES = [((12, 9, 40, 70), 5), ((6, 5, 7, 30, 40), 4), ((1, 23, 33, 65), 6), ((7, 11, 17, 19), 32)]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _problem(dims, R, seed, scale=4.0):
    rng = np.random.default_rng(seed)
    planted = [rng.uniform(0.0, 1.0, size=(d, R)) for d in dims]
    X = rng.poisson(ocp.rebuild(planted) * scale).astype(np.float64)
    init = [f32(rng.uniform(0.1, 1.0, size=(d, R))) for d in dims]
    return X, init


def _xf(X, beta):
    return np.maximum(X, 1e-12) if beta == 0.0 else X


@pytest.mark.parametrize("dims,R", SHAPES)
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5])
def test_block_update_every_mode(ctx, dims, R, beta):
    X, init = _problem(dims, R, 1)
    Xd = dev(X)
    for n in range(len(dims)):
        fac = [dev(a) for a in init]
        ctx.cp_update(Xd, fac, block=n, beta=beta)
        torch.cuda.synchronize()
        assert max_rel(host64(fac[n]), ocp.block_update(X, init, n, beta)) < TOL, f"mode {n}"
        for m in range(len(dims)):
            if m != n:
                assert np.array_equal(host64(fac[m]), init[m])


@pytest.mark.parametrize("dims,R", SHAPES[:2])
@pytest.mark.parametrize("beta", [0.0, 1.0, 1.3])
def test_bcomm_sweep(ctx, dims, R, beta):
    X, init = _problem(dims, R, 2)
    fac = [dev(a) for a in init]
    ctx.cp_update(dev(X), fac, block=-1, beta=beta)
    torch.cuda.synchronize()
    for a, b in zip(fac, ocp.bcomm_sweep(X, init, beta)):
        assert max_rel(host64(a), b) < 3 * TOL


@pytest.mark.parametrize("dims,R", SHAPES)
@pytest.mark.parametrize("beta,cache", [(0.0, False), (0.5, True), (1.0, False), (1.5, False), (1.5, True)])
def test_jcomm_outer(ctx, dims, R, beta, cache):
    X, init = _problem(dims, R, 3)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(X), fac, beta=beta, L=2, obj_out=obj, cache_pq=cache)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(X, init, beta, L=2, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3 * TOL
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("dims,R", SHAPES[:2])
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5])
def test_objective(ctx, dims, R, beta):
    X, init = _problem(dims, R, 4)
    out = ctx.beta_objective(dev(X), [dev(a) for a in init], beta=beta)
    want = oobjective(_xf(X, beta), ocp.rebuild(init), beta)
    assert abs(out.item() - want) / want < 1e-5


@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_paper_shape_80x70x60x50_r10(ctx, beta):
    """The synthetic CP shape of the paper's experiments (order 4,
    80 x 70 x 60 x 50, R = 10): one J-CoMM outer iteration (L = 2) and one
    B-CoMM sweep against the oracle on the same inputs."""
    X, init = _problem((80, 70, 60, 50), 10, 5, scale=2.0)
    Xd = dev(X)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(Xd, fac, beta=beta, L=2, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(X, init, beta, L=2, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3 * TOL
    assert abs(obj.item() - fref) / fref < 1e-5
    fac = [dev(a) for a in init]
    ctx.cp_update(Xd, fac, block=-1, beta=beta)
    torch.cuda.synchronize()
    for a, b in zip(fac, ocp.bcomm_sweep(X, init, beta)):
        assert max_rel(host64(a), b) < 3 * TOL


def test_objective_trace_decreases_like_oracle(ctx):
    """Ten J-CoMM outer iterations at beta = 1.5 on an order-4 problem: the
    objective at each reference matches the oracle's trace to 1e-4 and
    decreases."""
    X, init = _problem((10, 8, 30, 40), 6, 6)
    Xd = dev(X)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    got = []
    for _ in range(10):
        ctx.jcomm_outer(Xd, fac, beta=1.5, L=1, obj_out=obj)
        got.append(obj.item())
    _, trace = ocp.run(X, init, 1.5, 10, method="jcomm", L=1)
    assert max_rel(got, trace[:10]) < 1e-4
    assert all(b <= a * (1 + 1e-6) for a, b in zip(got, got[1:]))


def test_deterministic_bitwise(ctx):
    X, init = _problem((12, 9, 40, 70), 5, 7)
    Xd = dev(X)
    outs = []
    for _ in range(2):
        fac = [dev(a) for a in init]
        ctx.jcomm_outer(Xd, fac, beta=0.5, L=2)
        ctx.cp_update(Xd, fac, block=-1, beta=1.0)
        torch.cuda.synchronize()
        outs.append([host64(a) for a in fac])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_bf16_block_update(ctx):
    X, init = _problem((12, 9, 40, 70), 8, 8)
    Xd = dev(X)
    for n in (0, 1, 3):
        fac = [dev(a) for a in init]
        ctx.cp_update(Xd, fac, block=n, beta=1.5, precision="bf16")
        torch.cuda.synchronize()
        assert max_rel(host64(fac[n]), ocp.block_update(X, init, n, 1.5)) < 8e-3


@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_extrapolated_variants(ctx, beta):
    X, cur = _problem((10, 8, 30, 40), 5, 9)
    prev = [f32(a * np.random.default_rng(10).uniform(0.5, 1.2, a.shape)) for a in cur]
    Xd = dev(X)
    an, c, delta = 0.6, 0.5, 1e-12
    alpha = ox.weight(cur, prev, an, c, delta)
    F, P = [dev(a) for a in cur], [dev(a) for a in prev]
    ctx.bcomm_sweep_extrap(Xd, F, P, beta=beta, alpha_nes=an, c=c, delta=delta)
    torch.cuda.synchronize()
    want, want_prev = ox.cp_bcomm_sweep(X, cur, prev, beta, alpha)
    for a, b in zip(F, want):
        assert max_rel(host64(a), b) < 1e-4
    for a, b in zip(P, want_prev):
        assert np.array_equal(host64(a), b)
    F, P = [dev(a) for a in cur], [dev(a) for a in prev]
    ctx.jcomm_outer_extrap(Xd, F, P, beta=beta, L=2, alpha_nes=an, c=c, delta=delta)
    torch.cuda.synchronize()
    want, _ = ox.cp_jcomm_outer(X, cur, prev, beta, alpha, L=2)
    for a, b in zip(F, want):
        assert max_rel(host64(a), b) < 1e-4


def test_batched_mix_of_orders_is_bitwise_single(ctx):
    """Orders 3, 4 and 5 in one batch: each problem's result is bitwise that of
    a single call on it."""
    probs = [(_problem((20, 30, 40), 5, 11), 1.0), (_problem((12, 9, 40, 70), 5, 12), 1.5),
             (_problem((6, 5, 7, 30, 40), 4, 13), 1.0)]
    # the same arguments as the batch, objective output included (the pass that
    # also sums the objective is another kernel instantiation)
    singles, single_objs = [], []
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    for (X, init), beta in probs:
        fac = [dev(a) for a in init]
        ctx.jcomm_outer(dev(X), fac, beta=beta, L=2, obj_out=one)
        torch.cuda.synchronize()
        singles.append([host64(a) for a in fac])
        single_objs.append(one.item())
    objs = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    handles = []
    for k, ((X, init), beta) in enumerate(probs):
        handles.append({"X": dev(X), "factors": [dev(a) for a in init], "core": None, "beta": beta, "L": 2,
                        "eps": 1e-12, "precision": "fp32", "obj_out": objs[k:k + 1]})
    ctx.jcomm_outer_batched(comm.Batch(handles), graph=False)
    torch.cuda.synchronize()
    for h, want in zip(handles, singles):
        for a, b in zip(h["factors"], want):
            assert np.array_equal(host64(a), b)
    assert objs.cpu().tolist() == single_objs


def test_unsupported_and_invalid(ctx):
    X, init = _problem((6, 5, 7, 30), 4, 14)
    Xd = dev(X)
    fac = [dev(a) for a in init]
    with pytest.raises(comm.CommError) as e:
        ctx.cp_update(Xd, fac, block=4, beta=1.0)
    assert e.value.code == comm.COMM_EINVAL
    torch.cuda.synchronize()
    for a, b in zip(fac, init):
        assert np.array_equal(host64(a), b)
