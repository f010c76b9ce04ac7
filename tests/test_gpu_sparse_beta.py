"""GPU parity of the sparse COO path at beta in (0, 2) (Sec. 6.4, paragraph on
sparse tensors) against the FP64 oracle run on the densified tensor.

The updates of a sparse tensor are those of its dense form by definition; the
library accumulates the P-numerators over the nonzeros only and takes the
Q-denominators and the zero cells' objective from the dense pass over an
all-zero tensor of the same shape.  Float atomics make the nonzero sums
reproducible to rounding only (not bitwise); the bars are the dense path's:
1e-5 relative per factor entry after one block update, 3e-5 after a sweep or a
J-CoMM outer iteration with two inner sweeps, 1e-5 on the objective, 1e-4 on
an objective trace."""

import numpy as np
import pytest

import workloads
from oracle import cp as ocp
from oracle.divergence import objective as oobjective

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

# order 3 and 4; a ragged rank-32 tile; a one-percent 4-way tensor of ~200k nonzeros
CASES = [((13, 17, 9), 0.1, 5), ((40, 30, 50), 0.02, 32), ((6, 5, 7, 8), 0.05, 3), ((30, 24, 60, 70), 0.01, 8)]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _dev_coo(s):
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(s.idx.shape[1])]
    return idx, dev(s.val)


@pytest.mark.parametrize("dims,density,rank", CASES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_block_update_every_mode(ctx, dims, density, rank, beta):
    s = workloads.sparse_small(1, dims=dims, density=density, rank=rank)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    for n in range(len(dims)):
        fac = [dev(a) for a in init]
        ctx.cp_update_coo(idx, val, dims, fac, block=n, beta=beta)
        torch.cuda.synchronize()
        assert max_rel(host64(fac[n]), ocp.block_update(X, init, n, beta)) < 1e-5, f"mode {n}"
        for m in range(len(dims)):
            if m != n:
                assert np.array_equal(host64(fac[m]), init[m])


@pytest.mark.parametrize("dims,density,rank", CASES[:3])
@pytest.mark.parametrize("beta", [0.5, 1.5])
def test_bcomm_sweep(ctx, dims, density, rank, beta):
    s = workloads.sparse_small(2, dims=dims, density=density, rank=rank)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in init]
    ctx.cp_update_coo(idx, val, dims, fac, block=-1, beta=beta)
    torch.cuda.synchronize()
    for a, b in zip(fac, ocp.bcomm_sweep(X, init, beta)):
        assert max_rel(host64(a), b) < 3e-5


@pytest.mark.parametrize("dims,density,rank", CASES)
@pytest.mark.parametrize("beta", [0.5, 1.5, 1.2])
def test_jcomm_outer(ctx, dims, density, rank, beta):
    s = workloads.sparse_small(3, dims=dims, density=density, rank=rank)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo(idx, val, dims, fac, L=2, obj_out=obj, beta=beta)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(X, init, beta, L=2, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3e-5
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("dims,density,rank", CASES)
@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
def test_objective(ctx, dims, density, rank, beta):
    s = workloads.sparse_small(4, dims=dims, density=density, rank=rank)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    out = ctx.beta_objective_coo(idx, val, dims, [dev(a) for a in init], beta=beta)
    want = oobjective(X, ocp.rebuild(init), beta)
    assert abs(out.item() - want) / want < 1e-5


def test_objective_trace_decreases(ctx):
    """Six J-CoMM outer iterations at beta = 1.5 on a 4-way sparse tensor: the
    objective at each reference matches the dense oracle's trace and decreases."""
    dims = (20, 12, 30, 40)
    s = workloads.sparse_small(5, dims=dims, density=0.03, rank=6)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    got = []
    for _ in range(6):
        ctx.cp_jcomm_outer_coo(idx, val, dims, fac, L=1, obj_out=obj, beta=1.5)
        got.append(obj.item())
    _, trace = ocp.run(X, init, 1.5, 6, method="jcomm", L=1)
    assert max_rel(got, trace[:6]) < 1e-4
    assert all(b <= a * (1 + 1e-6) for a, b in zip(got, got[1:]))


def test_out_of_range_coordinates_are_skipped(ctx):
    dims = (13, 17, 9)
    s = workloads.sparse_small(6, dims=dims, density=0.1, rank=5)
    X = workloads.densify(s)
    init = [f32(a) for a in s.init]
    bad = np.array([[13, 0, 0], [0, -1, 0], [0, 0, 9]], dtype=np.int64)
    idx = [torch.tensor(np.concatenate([s.idx[:, n], bad[:, n]]).astype(np.int32), device="cuda") for n in range(3)]
    val = dev(np.concatenate([s.val, [5.0, 6.0, 7.0]]))
    fac = [dev(a) for a in init]
    ctx.cp_update_coo(idx, val, dims, fac, block=-1, beta=0.5)
    out = ctx.beta_objective_coo(idx, val, dims, [dev(a) for a in init], beta=0.5)
    torch.cuda.synchronize()
    for a, b in zip(fac, ocp.bcomm_sweep(X, init, 0.5)):
        assert max_rel(host64(a), b) < 3e-5
    want = oobjective(X, ocp.rebuild(init), 0.5)
    assert abs(out.item() - want) / want < 1e-5


def test_empty_tensor(ctx):
    """No nonzeros: every numerator is zero, so each updated block is eps; the
    objective is the sum of Xhat^beta / beta over the cells."""
    dims = (7, 6, 5)
    init = [f32(np.random.default_rng(7).uniform(0.1, 1.0, (d, 3))) for d in dims]
    idx = [torch.zeros(0, dtype=torch.int32, device="cuda") for _ in dims]
    val = torch.zeros(0, dtype=torch.float32, device="cuda")
    out = ctx.beta_objective_coo(idx, val, dims, [dev(a) for a in init], beta=1.5)
    fac = [dev(a) for a in init]
    ctx.cp_update_coo(idx, val, dims, fac, block=0, beta=1.5)
    torch.cuda.synchronize()
    X = np.zeros(dims)
    assert abs(out.item() - oobjective(X, ocp.rebuild(init), 1.5)) / oobjective(X, ocp.rebuild(init), 1.5) < 1e-5
    assert np.all(host64(fac[0]) == np.float32(1e-12))


def test_refuses_beta_zero_and_order_two(ctx):
    s = workloads.sparse_small(8, dims=(13, 17, 9), density=0.1, rank=4)
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in s.init]
    with pytest.raises(comm.CommError) as e:
        ctx.cp_update_coo(idx, val, s.dims, fac, block=0, beta=0.0)
    assert e.value.code == comm.COMM_EUNSUPPORTED
    s2 = workloads.sparse_small(9, dims=(30, 40), density=0.1, rank=4)
    idx2, val2 = _dev_coo(s2)
    with pytest.raises(comm.CommError) as e:
        ctx.cp_jcomm_outer_coo(idx2, val2, s2.dims, [dev(a) for a in s2.init], beta=0.5)
    assert e.value.code == comm.COMM_EUNSUPPORTED
    torch.cuda.synchronize()
    for a, b in zip(fac, s.init):
        assert np.array_equal(host64(a), f32(b))


@pytest.mark.parametrize("dims,density,rank", [((40, 50), 0.05, 6), ((60, 70, 80), 0.004, 32),
                                               ((9, 10, 11, 12, 30), 0.005, 5)])
def test_kl_objective_needs_no_dense_twin(dims, density, rank):
    """CP at beta = 1: zero cells contribute Xhat, so they sum in closed form
    (the model's mass minus the nonzeros' Xhat) and no dense pass runs.  The
    context's workspace limit is far below the 4 bytes per cell a dense twin
    would take; orders 2 and 5 are served too (Sec. 3.2 at beta = 1, Sec. 6.4)."""
    s = workloads.sparse_small(7, dims=dims, density=density, rank=rank)
    cells = int(np.prod(dims))
    limit = 1 << 20
    assert 4 * cells > limit or len(dims) == 2
    small = comm.Context(0, workspace_limit=limit)
    try:
        init = [f32(a) for a in s.init]
        idx, val = _dev_coo(s)
        out = small.beta_objective_coo(idx, val, dims, [dev(a) for a in init], beta=1.0)
        X = workloads.densify(s)
        want = oobjective(X, ocp.rebuild(init), 1.0)
        assert abs(out.item() - want) / want < 1e-5
    finally:
        small.close()


def test_index_space_beyond_device_is_refused(ctx):
    """Three modes of 2^24: the dense twin would need 2^72 cells.  The call is
    refused with COMM_ENOMEM before anything is allocated or launched (the
    factors are not read, so small stand-ins suffice)."""
    dims = (1 << 24, 1 << 24, 1 << 24)
    idx = [torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda") for _ in dims]
    val = dev(np.array([1.0, 2.0, 3.0]))
    fac = [dev(np.ones((4, 3))) for _ in dims]
    with pytest.raises(comm.CommError) as e:
        ctx.cp_update_coo(idx, val, dims, fac, block=0, beta=0.5)
    assert e.value.code == comm.COMM_ENOMEM
    with pytest.raises(comm.CommError) as e:
        ctx.beta_objective_coo(idx, val, dims, fac, beta=1.5)
    assert e.value.code == comm.COMM_ENOMEM
    torch.cuda.synchronize()
    assert np.array_equal(host64(fac[0]), np.ones((4, 3)))
