"""GPU parity of Tucker on sparse COO data (orders 3 to 5, beta in (0, 2)),
and of order-5 CP on sparse data, against the FP64 oracle on the densified
tensor.

The sparse Tucker path scatters the nonzeros into the rows of the
(I_1 ... I_{N-1}) x I_N view (the numerators' contraction along the last mode)
and gathers the rebuild table for the last mode's numerator; the other
contractions are the dense order-N path's.  Float atomics: reproducible to
rounding only; the bars are the dense path's (1e-5 per entry after one block
update or a J-CoMM outer iteration with L = 1, 3e-5 after a sweep or L = 2,
1e-5 on the objective)."""
import numpy as np
import pytest

import workloads
from oracle import cp as ocp
from oracle import tucker as otk
from oracle.divergence import objective as oobjective

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

CASES = [((13, 17, 9), 0.1, (3, 4, 2)), ((9, 7, 11, 40), 0.03, (3, 4, 2, 5)),
         ((5, 4, 3, 6, 37), 0.05, (2, 3, 2, 2, 3)), ((12, 10, 8, 33), 0.02, (5, 4, 3, 32))]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _problem(dims, density, J, seed):
    s = workloads.sparse_small(seed, dims=dims, density=density, rank=2)
    rng = np.random.default_rng(seed + 100)
    core = f32(rng.uniform(0.1, 1.0, J))
    fac = [f32(rng.uniform(0.1, 1.0, (d, j))) for d, j in zip(dims, J)]
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(len(dims))]
    return workloads.densify(s), idx, dev(s.val), core, fac


@pytest.mark.parametrize("dims,density,J", CASES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_block_update_every_block(ctx, dims, density, J, beta):
    X, idx, val, core, fac = _problem(dims, density, J, 1)
    for blk in range(-1, len(dims)):
        G, F = dev(core), [dev(a) for a in fac]
        ctx.tucker_update_coo(idx, val, dims, G, F, block=blk, beta=beta)
        torch.cuda.synchronize()
        if blk == -1:
            assert max_rel(host64(G), otk.block_update_core(X, core, fac, beta)) < 1e-5, "core"
        else:
            assert max_rel(host64(F[blk]), otk.block_update_factor(X, core, fac, blk, beta)) < 1e-5, f"mode {blk}"


@pytest.mark.parametrize("dims,density,J", CASES[:3])
@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_bcomm_sweep(ctx, dims, density, J, beta):
    X, idx, val, core, fac = _problem(dims, density, J, 2)
    G, F = dev(core), [dev(a) for a in fac]
    ctx.tucker_update_coo(idx, val, dims, G, F, block=-2, beta=beta)
    torch.cuda.synchronize()
    wg, wf = otk.bcomm_sweep(X, core, fac, beta)
    assert max_rel(host64(G), wg) < 3e-5
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3e-5


@pytest.mark.parametrize("dims,density,J", CASES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_jcomm_outer(ctx, dims, density, J, beta):
    X, idx, val, core, fac = _problem(dims, density, J, 3)
    G, F = dev(core), [dev(a) for a in fac]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.tucker_jcomm_outer_coo(idx, val, dims, G, F, beta=beta, L=2, obj_out=obj)
    torch.cuda.synchronize()
    wg, wf, fref = otk.jcomm_outer(X, core, fac, beta, L=2, return_ref_obj=True)
    assert max_rel(host64(G), wg) < 3e-5
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 3e-5
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("dims,density,J", CASES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_objective(ctx, dims, density, J, beta):
    X, idx, val, core, fac = _problem(dims, density, J, 4)
    out = ctx.beta_objective_coo(idx, val, dims, [dev(a) for a in fac], core=dev(core), beta=beta)
    want = oobjective(X, otk.rebuild(core, fac), beta)
    assert abs(out.item() - want) / want < 1e-5


@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_uber_shaped_counts_27x24x7x100x100(ctx, beta):
    """The shape, ranks and sparsity (about 0.6% nonzeros) of the paper's 5-way
    count experiment, synthetic: one J-CoMM outer iteration against the
    oracle on the densified tensor."""
    dims, J = (27, 24, 7, 100, 100), (10, 10, 5, 10, 10)
    X, idx, val, core, fac = _problem(dims, 0.006, J, 5)
    G, F = dev(core), [dev(a) for a in fac]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.tucker_jcomm_outer_coo(idx, val, dims, G, F, beta=beta, L=1, obj_out=obj)
    torch.cuda.synchronize()
    wg, wf, fref = otk.jcomm_outer(X, core, fac, beta, L=1, return_ref_obj=True)
    assert max_rel(host64(G), wg) < 1e-5
    for a, b in zip(F, wf):
        assert max_rel(host64(a), b) < 1e-5
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("beta", [0.5, 1.5])
def test_order5_cp_on_sparse_data(ctx, beta):
    dims = (6, 5, 4, 7, 8)
    s = workloads.sparse_small(6, dims=dims, density=0.05, rank=4)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(5)]
    val = dev(s.val)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo(idx, val, dims, fac, L=2, obj_out=obj, beta=beta)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(X, init, beta, L=2, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3e-5
    assert abs(obj.item() - fref) / fref < 1e-5


def test_refusals(ctx):
    X, idx, val, core, fac = _problem((13, 17, 9), 0.1, (3, 4, 2), 7)
    G, F = dev(core), [dev(a) for a in fac]
    with pytest.raises(comm.CommError) as e:
        ctx.tucker_update_coo(idx, val, (13, 17, 9), G, F, block=-2, beta=0.0)
    assert e.value.code == comm.COMM_EUNSUPPORTED
    with pytest.raises(comm.CommError) as e:
        ctx.tucker_update_coo(idx, val, (13, 17, 9), G, F, block=3, beta=1.0)
    assert e.value.code == comm.COMM_EINVAL
    with pytest.raises(comm.CommError) as e:  # a CP model on the Tucker entry
        ctx.tucker_update_coo(idx, val, (13, 17, 9), None, F, block=0, beta=1.0)
    assert e.value.code == comm.COMM_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(host64(G), core)
