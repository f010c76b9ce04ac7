"""GPU parity of dense Tucker of order 4 and 5 against the FP64 oracle (written
for any order), through the C ABI.

The library runs these orders through the (I_1 ... I_{N-1}) x I_N view of X
with the fused order-3 passes and mode-product GEMM chains; the oracle
contracts the order-N tensor directly (App. C), so a mistake in a chain's
strides or in the view shows up here.  Bars as for order 3: 1e-5 relative per block entry after one
block update, 3e-5 after a sweep or two inner sweeps, 1e-5 on the objective."""
import numpy as np
import pytest

from oracle import extrapolation as ox
from oracle import tucker as otk
from oracle.divergence import objective as oobjective

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

TOL = 1e-5
# ragged everywhere; I4 a multiple of 4 (vector fibre loads); a core size of
# 32 in the fibre mode; a mode of extent 1
SHAPES = [((9, 7, 11, 40), (3, 4, 2, 5)), ((12, 10, 8, 33), (5, 4, 3, 6)), ((5, 6, 7, 64), (2, 2, 2, 32)),
          ((1, 13, 6, 21), (1, 3, 4, 2)), ((5, 4, 3, 6, 37), (2, 3, 2, 2, 3)), ((3, 7, 2, 5, 16), (3, 2, 2, 4, 5))]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _problem(dims, J, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    X = rng.poisson(otk.rebuild(rng.uniform(0, 1, J), [rng.uniform(0, 1, (d, j)) for d, j in zip(dims, J)])
                    * scale / np.prod(J) ** 0.5).astype(np.float64)
    core = f32(rng.uniform(0.1, 1.0, J))
    fac = [f32(rng.uniform(0.1, 1.0, (d, j))) for d, j in zip(dims, J)]
    return X, core, fac


def _xf(X, beta):
    return np.maximum(X, 1e-12) if beta == 0.0 else X


@pytest.mark.parametrize("dims,J", SHAPES)
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5])
def test_block_update_every_block(ctx, dims, J, beta):
    X, core, fac = _problem(dims, J, 1)
    Xd = dev(X)
    for blk in range(-1, len(dims)):
        G, F = dev(core), [dev(a) for a in fac]
        ctx.tucker_update(Xd, G, F, block=blk, beta=beta)
        torch.cuda.synchronize()
        if blk == -1:
            assert max_rel(host64(G), otk.block_update_core(X, core, fac, beta)) < TOL, "core"
            for a, b in zip(F, fac):
                assert np.array_equal(host64(a), b)
        else:
            want = otk.block_update_factor(X, core, fac, blk, beta)
            assert max_rel(host64(F[blk]), want) < TOL, f"mode {blk}"
            assert np.array_equal(host64(G), core)


@pytest.mark.parametrize("dims,J", SHAPES[:2] + SHAPES[4:5])
@pytest.mark.parametrize("beta", [0.0, 1.0, 1.3])
def test_bcomm_sweep(ctx, dims, J, beta):
    X, core, fac = _problem(dims, J, 2)
    G, F = dev(core), [dev(a) for a in fac]
    ctx.tucker_update(dev(X), G, F, block=-2, beta=beta)
    torch.cuda.synchronize()
    wg, wf = otk.bcomm_sweep(X, core, fac, beta)
    assert max_rel(host64(G), wg) < 3 * TOL
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3 * TOL


@pytest.mark.parametrize("dims,J", SHAPES)
@pytest.mark.parametrize("beta,cache", [(0.0, False), (0.5, True), (1.0, False), (1.5, False), (1.5, True)])
def test_jcomm_outer(ctx, dims, J, beta, cache):
    X, core, fac = _problem(dims, J, 3)
    G, F = dev(core), [dev(a) for a in fac]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(X), F, core=G, beta=beta, L=2, obj_out=obj, cache_pq=cache)
    torch.cuda.synchronize()
    wg, wf, fref = otk.jcomm_outer(X, core, fac, beta, L=2, return_ref_obj=True)
    assert max_rel(host64(G), wg) < 3 * TOL
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3 * TOL
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5])
def test_objective(ctx, beta):
    X, core, fac = _problem((12, 10, 8, 33), (5, 4, 3, 6), 4)
    out = ctx.beta_objective(dev(X), [dev(a) for a in fac], core=dev(core), beta=beta)
    want = oobjective(_xf(X, beta), otk.rebuild(core, fac), beta)
    assert abs(out.item() - want) / want < 1e-5


@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_paper_shape_80x70x60x50_core_10x9x8x7(ctx, beta):
    """The synthetic Tucker shape of the paper's experiments (order 4,
    80 x 70 x 60 x 50, core 10 x 9 x 8 x 7): one J-CoMM outer iteration
    (L = 2) and one B-CoMM sweep against the oracle on the same inputs."""
    X, core, fac = _problem((80, 70, 60, 50), (10, 9, 8, 7), 5, scale=1.0)
    Xd = dev(X)
    G, F = dev(core), [dev(a) for a in fac]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(Xd, F, core=G, beta=beta, L=2, obj_out=obj)
    torch.cuda.synchronize()
    wg, wf, fref = otk.jcomm_outer(X, core, fac, beta, L=2, return_ref_obj=True)
    assert max_rel(host64(G), wg) < 3 * TOL
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3 * TOL
    assert abs(obj.item() - fref) / fref < 1e-5
    G, F = dev(core), [dev(a) for a in fac]
    ctx.tucker_update(Xd, G, F, block=-2, beta=beta)
    torch.cuda.synchronize()
    wg, wf = otk.bcomm_sweep(X, core, fac, beta)
    assert max_rel(host64(G), wg) < 3 * TOL
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3 * TOL


@pytest.mark.parametrize("beta", [1.0, 1.5])
def test_uber_shaped_order5_27x24x7x100x100_ranks_10_10_5_10_10(ctx, beta):
    """The shape and ranks of the paper's 5-way count-tensor experiment (run
    there with dense contractions), on synthetic Poisson counts: one J-CoMM
    outer iteration (L = 1) against the oracle, and the core and mode-3 block
    updates."""
    dims, J = (27, 24, 7, 100, 100), (10, 10, 5, 10, 10)
    rng = np.random.default_rng(14)
    X = rng.poisson(0.5, size=dims).astype(np.float64)
    core = f32(rng.uniform(0.1, 1.0, J))
    fac = [f32(rng.uniform(0.1, 1.0, (d, j))) for d, j in zip(dims, J)]
    Xd = dev(X)
    G, F = dev(core), [dev(a) for a in fac]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(Xd, F, core=G, beta=beta, L=1, obj_out=obj)
    torch.cuda.synchronize()
    wg, wf, fref = otk.jcomm_outer(X, core, fac, beta, L=1, return_ref_obj=True)
    assert max_rel(host64(G), wg) < 3 * TOL
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3 * TOL
    assert abs(obj.item() - fref) / fref < 1e-5
    for blk in (-1, 2):
        G, F = dev(core), [dev(a) for a in fac]
        ctx.tucker_update(Xd, G, F, block=blk, beta=beta)
        torch.cuda.synchronize()
        got = host64(G) if blk == -1 else host64(F[blk])
        want = (otk.block_update_core(X, core, fac, beta) if blk == -1
                else otk.block_update_factor(X, core, fac, blk, beta))
        assert max_rel(got, want) < TOL


def test_objective_trace_like_oracle(ctx):
    X, core, fac = _problem((9, 7, 11, 40), (3, 4, 2, 5), 6)
    Xd = dev(X)
    G, F = dev(core), [dev(a) for a in fac]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    got = []
    for _ in range(8):
        ctx.jcomm_outer(Xd, F, core=G, beta=0.5, L=1, obj_out=obj)
        got.append(obj.item())
    _, _, trace = otk.run(X, core, fac, 0.5, 8, method="jcomm", L=1)
    assert max_rel(got, trace[:8]) < 1e-4
    assert all(b <= a * (1 + 1e-6) for a, b in zip(got, got[1:]))


def test_deterministic_bitwise(ctx):
    X, core, fac = _problem((12, 10, 8, 33), (5, 4, 3, 6), 7)
    Xd = dev(X)
    outs = []
    for _ in range(2):
        G, F = dev(core), [dev(a) for a in fac]
        ctx.jcomm_outer(Xd, F, core=G, beta=1.5, L=2)
        ctx.tucker_update(Xd, G, F, block=-2, beta=1.0)
        torch.cuda.synchronize()
        outs.append([host64(G)] + [host64(a) for a in F])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_bf16_block_update(ctx):
    X, core, fac = _problem((12, 10, 8, 33), (5, 4, 3, 6), 8)
    Xd = dev(X)
    for blk in (-1, 1, 3):
        G, F = dev(core), [dev(a) for a in fac]
        ctx.tucker_update(Xd, G, F, block=blk, beta=1.5, precision="bf16")
        torch.cuda.synchronize()
        got = host64(G) if blk == -1 else host64(F[blk])
        want = (otk.block_update_core(X, core, fac, 1.5) if blk == -1
                else otk.block_update_factor(X, core, fac, blk, 1.5))
        assert max_rel(got, want) < 8e-3


@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_extrapolated_variants(ctx, beta):
    X, core, fac = _problem((9, 7, 11, 40), (3, 4, 2, 5), 9)
    rng = np.random.default_rng(10)
    pcore = f32(core * rng.uniform(0.5, 1.2, core.shape))
    prev = [f32(a * rng.uniform(0.5, 1.2, a.shape)) for a in fac]
    Xd = dev(X)
    an, c, delta = 0.6, 0.5, 1e-12
    alpha = ox.weight([core] + fac, [pcore] + prev, an, c, delta)
    G, F, PG, P = dev(core), [dev(a) for a in fac], dev(pcore), [dev(a) for a in prev]
    ctx.bcomm_sweep_extrap(Xd, F, P, core=G, prev_core=PG, beta=beta, alpha_nes=an, c=c, delta=delta)
    torch.cuda.synchronize()
    wg, wf, wpg, wpf = ox.tucker_bcomm_sweep(X, core, fac, pcore, prev, beta, alpha)
    assert max_rel(host64(G), wg) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4
    assert np.array_equal(host64(PG), wpg)
    G, F, PG, P = dev(core), [dev(a) for a in fac], dev(pcore), [dev(a) for a in prev]
    ctx.jcomm_outer_extrap(Xd, F, P, core=G, prev_core=PG, beta=beta, L=2, alpha_nes=an, c=c, delta=delta)
    torch.cuda.synchronize()
    wg, wf, _, _ = ox.tucker_jcomm_outer(X, core, fac, pcore, prev, beta, alpha, L=2)
    assert max_rel(host64(G), wg) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4


def test_batched_order3_and_order4_tucker_is_bitwise_single(ctx):
    probs = [(_problem((20, 30, 40), (4, 5, 3), 11), 1.5), (_problem((9, 7, 11, 40), (3, 4, 2, 5), 12), 1.0),
             (_problem((12, 10, 8, 33), (5, 4, 3, 6), 13), 0.5)]
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    singles, single_objs = [], []
    for (X, core, fac), beta in probs:
        G, F = dev(core), [dev(a) for a in fac]
        ctx.jcomm_outer(dev(X), F, core=G, beta=beta, L=2, obj_out=one)
        torch.cuda.synchronize()
        singles.append([host64(G)] + [host64(a) for a in F])
        single_objs.append(one.item())
    objs = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    handles = []
    for k, ((X, core, fac), beta) in enumerate(probs):
        handles.append({"X": dev(X), "factors": [dev(a) for a in fac], "core": dev(core), "beta": beta, "L": 2,
                        "obj_out": objs[k:k + 1]})
    ctx.jcomm_outer_batched(comm.Batch(handles), graph=True)
    torch.cuda.synchronize()
    for h, want in zip(handles, singles):
        got = [host64(h["core"])] + [host64(a) for a in h["factors"]]
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
    assert objs.cpu().tolist() == single_objs


def test_batched_order5_graph_replays(ctx):
    """An order-5 problem in a graph-captured batch beside an order-3 one,
    replayed twice: bitwise the single calls, iteration by iteration."""
    probs = [(_problem((20, 30, 40), (4, 5, 3), 15), 1.0), (_problem((5, 4, 3, 6, 37), (2, 3, 2, 2, 3), 16), 1.5)]
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    singles = []
    for (X, core, fac), beta in probs:
        G, F = dev(core), [dev(a) for a in fac]
        Xd = dev(X)
        for _ in range(2):
            ctx.jcomm_outer(Xd, F, core=G, beta=beta, L=1, obj_out=one)
        torch.cuda.synchronize()
        singles.append([host64(G)] + [host64(a) for a in F])
    objs = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    handles = [{"X": dev(X), "factors": [dev(a) for a in fac], "core": dev(core), "beta": beta, "L": 1,
                "obj_out": objs[k:k + 1]} for k, ((X, core, fac), beta) in enumerate(probs)]
    batch = comm.Batch(handles)
    for _ in range(2):
        ctx.jcomm_outer_batched(batch, graph=True)
    torch.cuda.synchronize()
    for h, want in zip(handles, singles):
        got = [host64(h["core"])] + [host64(a) for a in h["factors"]]
        for a, b in zip(got, want):
            assert np.array_equal(a, b)


def test_unsupported_orders(ctx):
    # the ABI holds at most five modes: the binding refuses a sixth
    with pytest.raises(ValueError):
        ctx.tucker_update(dev(np.ones((2, 2, 2, 2, 2, 2))), dev(np.ones((1, 1, 1, 1, 1, 1))),
                          [dev(np.ones((2, 1))) for _ in range(6)], block=-2, beta=1.0)
    # a core size beyond the 32-wide tile
    X = dev(np.ones((3, 4, 5, 40)))
    with pytest.raises(comm.CommError) as e:
        ctx.tucker_update(X, dev(np.ones((2, 2, 2, 33))), [dev(np.ones((d, j))) for d, j in
                                                           zip((3, 4, 5, 40), (2, 2, 2, 33))], block=-2, beta=1.0)
    assert e.value.code == comm.COMM_EUNSUPPORTED
