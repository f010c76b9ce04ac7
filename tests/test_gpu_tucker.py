"""GPU parity of the dense Tucker path against the FP64 oracle, through the C ABI.

Float32 inputs on the GPU; the oracle runs in float64 on the same values.
Bars: 1e-5 relative per parameter entry after one block update (1e-4 after a
full sweep or outer iteration, which chains four block updates), 1e-5 on the
float64 objective."""
import numpy as np
import pytest

import workloads
from oracle import tucker as otk
from oracle.divergence import objective as oobjective

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

BETAS = [0.0, 0.5, 1.0, 1.5, 0.7]
# ragged tails in every mode; K = 96 takes the vector fibre loads throughout and
# 100 x 90 pairs split the mode-3 pass over several pair tiles per wave
SHAPES = [((20, 24, 28), (3, 4, 5)), ((37, 45, 70), (8, 6, 5)), ((64, 48, 40), (16, 16, 16)),
          ((100, 90, 96), (5, 7, 9))]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _problem(dims, J, seed):
    rng = np.random.default_rng(seed)
    core = rng.uniform(0.0, 1.0, size=J)
    fac = [rng.uniform(0.0, 1.0, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(otk.rebuild(core, fac) * 2.0).astype(np.float64)
    icore = f32(rng.uniform(0.1, 1.0, size=J))
    ifac = [f32(rng.uniform(0.1, 1.0, size=(d, j))) for d, j in zip(dims, J)]
    return X, icore, ifac


def _dev_model(core, fac):
    return dev(core), [dev(a) for a in fac]


@pytest.mark.parametrize("dims,J", SHAPES)
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("block", [-1, 0, 1, 2])
def test_tucker_block_update_matches_oracle(ctx, dims, J, beta, block):
    X, core, fac = _problem(dims, J, 1)
    G, F = _dev_model(core, fac)
    ctx.tucker_update(dev(X), G, F, block=block, beta=beta)
    torch.cuda.synchronize()
    if block == -1:
        want = otk.block_update_core(X, core, fac, beta)
        assert max_rel(host64(G), want) < 1e-5
        for a, b in zip(F, fac):
            assert np.array_equal(host64(a), b)
    else:
        want = otk.block_update_factor(X, core, fac, block, beta)
        assert max_rel(host64(F[block]), want) < 1e-5
        assert np.array_equal(host64(G), core)


@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5])
def test_tucker_bcomm_sweep_matches_oracle(ctx, beta):
    X, core, fac = _problem((37, 45, 70), (8, 6, 5), 2)
    G, F = _dev_model(core, fac)
    ctx.tucker_update(dev(X), G, F, block=-2, beta=beta)
    torch.cuda.synchronize()
    wc, wf = otk.bcomm_sweep(X, core, fac, beta)
    assert max_rel(host64(G), wc) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4


@pytest.mark.parametrize("dims,J", SHAPES)
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("L", [1, 2])
@pytest.mark.parametrize("cache", [False, True])
def test_tucker_jcomm_outer_matches_oracle(ctx, dims, J, beta, L, cache):
    if cache and beta == 1.0:
        pytest.skip("beta = 1 never caches P~ / Q~")
    X, core, fac = _problem(dims, J, 3)
    G, F = _dev_model(core, fac)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(X), F, core=G, beta=beta, L=L, cache_pq=cache, obj_out=obj)
    torch.cuda.synchronize()
    wc, wf, fref = otk.jcomm_outer(X, core, fac, beta, L=L, return_ref_obj=True)
    assert max_rel(host64(G), wc) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("beta", BETAS)
def test_tucker_objective_matches_oracle(ctx, beta):
    X, core, fac = _problem((37, 45, 70), (8, 6, 5), 4)
    G, F = _dev_model(core, fac)
    out = ctx.beta_objective(dev(X), F, core=G, beta=beta)
    torch.cuda.synchronize()
    want = oobjective(X, otk.rebuild(core, fac), beta)
    assert abs(out.item() - want) / want < 1e-5


def test_tucker_trace_jcomm(ctx):
    d = workloads.tucker_dense(0, dims=(40, 36, 44), core_dims=(6, 5, 4))
    core, fac = f32(d.init_core), [f32(a) for a in d.init_factors]
    _, _, want = otk.run(d.X, core, fac, 1.5, 15, method="jcomm", L=1)
    Xd = dev(d.X)
    G, F = _dev_model(core, fac)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    got = []
    for _ in range(15):
        ctx.jcomm_outer(Xd, F, core=G, beta=1.5, L=1, obj_out=obj)
        got.append(obj.item())
    got.append(ctx.beta_objective(Xd, F, core=G, beta=1.5).item())
    assert max_rel(got, want) < 1e-4
    assert all(b <= a * (1 + 1e-6) for a, b in zip(got, got[1:]))


@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_full_size_tucker_jcomm(ctx, beta):
    """200^3 Gamma-perturbed Tucker tensor with a 16^3 core (the measured
    Tucker workload): one J-CoMM outer iteration against the oracle."""
    d = workloads.tucker_dense(0)
    core, fac = f32(d.init_core), [f32(a) for a in d.init_factors]
    G, F = _dev_model(core, fac)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(d.X), F, core=G, beta=beta, L=1, obj_out=obj)
    torch.cuda.synchronize()
    wc, wf, fref = otk.jcomm_outer(d.X, core, fac, beta, L=1, return_ref_obj=True)
    assert max_rel(host64(G), wc) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4
    assert abs(obj.item() - fref) / fref < 1e-5


def test_tucker_deterministic(ctx):
    X, core, fac = _problem((37, 45, 70), (8, 6, 5), 5)
    outs = []
    for _ in range(2):
        G, F = _dev_model(core, fac)
        ctx.jcomm_outer(dev(X), F, core=G, beta=0.5, L=1)
        outs.append([host64(G)] + [host64(a) for a in F])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_tucker_unaligned_tensor(ctx):
    """X whose base address is 4 bytes past a 16-byte boundary takes the scalar
    fibre loads (K = 64 would otherwise use vector loads)."""
    X, core, fac = _problem((30, 20, 64), (5, 4, 6), 6)
    buf = torch.zeros(X.size + 1, dtype=torch.float32, device="cuda")
    Xd = buf[1:].view(X.shape)
    Xd.copy_(torch.tensor(X, dtype=torch.float32))
    G, F = _dev_model(core, fac)
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(Xd, F, core=G, beta=0.5, L=1, obj_out=obj)
    torch.cuda.synchronize()
    wc, wf, fref = otk.jcomm_outer(X, core, fac, 0.5, L=1, return_ref_obj=True)
    assert max_rel(host64(G), wc) < 1e-4
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-4
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("beta", BETAS)
def test_tucker_objective_at_exact_fit(ctx, beta):
    """Data equal to the Tucker model (rounded to float32): the objective is
    of the order of 1e-14 of sum(x^beta) when every term is evaluated without
    cancellation (about 1e-10 or more otherwise)."""
    rng = np.random.default_rng(22)
    dims, J = (37, 45, 70), (8, 6, 5)
    core = f32(rng.uniform(0.1, 1.0, size=J))
    fac = [f32(rng.uniform(0.1, 1.0, size=(d, j))) for d, j in zip(dims, J)]
    X = f32(otk.rebuild(core, fac))
    G, F = _dev_model(core, fac)
    out = ctx.beta_objective(dev(X), F, core=G, beta=beta)
    torch.cuda.synchronize()
    scale = float(np.sum(X.astype(np.float64) ** beta))
    assert 0.0 <= out.item() < 1e-11 * scale
