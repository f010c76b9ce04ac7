"""GPU parity of the sparse COO beta = 1 J-CoMM path against the FP64 oracle.

The COO path scatters with hardware float atomics, so results are reproducible
to rounding, not bitwise.  The bars are the dense path's: 1e-5 relative per
factor entry after one outer iteration with one inner sweep, 3e-5 after two or
three inner sweeps (each sweep compounds the rounding of the last)."""
import numpy as np
import pytest

import workloads
from oracle import sparse as osp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64, max_rel  # noqa: E402

TOL = 1e-5  # relative, per factor entry, after one outer iteration with L = 1


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _dev_coo(s):
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(s.idx.shape[1])]
    return idx, dev(s.val)


@pytest.mark.parametrize("dims,density,rank", [((6, 5, 7, 8), 0.05, 3), ((30, 24, 60, 70), 0.01, 8),
                                               ((40, 30, 50), 0.02, 32)])
@pytest.mark.parametrize("L", [1, 3])
def test_coo_jcomm_matches_oracle(ctx, dims, density, rank, L):
    s = workloads.sparse_small(1, dims=dims, density=density, rank=rank)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo(idx, val, dims, fac, L=L, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = osp.jcomm_outer_kl(s.idx, s.val, init, L=L, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < TOL * (1 if L == 1 else 3)
    assert abs(obj.item() - fref) / fref < 1e-5


def test_coo_day_hour_lat_lon_workload(ctx):
    """183 x 24 x 1140 x 1717 counts with 3.3M Zipf/diurnal nonzeros, rank 32:
    the objective at the reference over the full tensor, and the factors on the
    two small modes against the oracle."""
    s = workloads.sparse_counts(0)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo(idx, val, s.dims, fac, L=1, obj_out=obj)
    torch.cuda.synchronize()
    fref = osp.objective_kl(s.idx, s.val, init)
    assert abs(obj.item() - fref) / fref < 1e-5
    want = osp.jcomm_outer_kl(s.idx, s.val, init, L=1)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 1e-4


def test_coo_rejects_beta_zero(ctx):
    """Sparse data at beta = 0: d(0 | y) is infinite, so the sparse path refuses
    it (beta in (0, 2) is served; see tests/test_gpu_sparse_beta.py)."""
    s = workloads.sparse_small(2)
    idx, val = _dev_coo(s)
    fac = [dev(a) for a in s.init]
    o = comm._opts(0.0, 1e-12, None, 1)
    c = comm.Coo()
    c.ndim = 4
    for n, d in enumerate(s.dims):
        c.dims[n] = d
    c.nnz = val.numel()
    for n in range(4):
        c.idx[n] = idx[n].data_ptr()
    c.val = val.data_ptr()
    m = comm._model(fac)
    import ctypes
    rc = ctx._lib.comm_cp_jcomm_outer_coo(ctx._h, ctypes.byref(c), ctypes.byref(m), ctypes.byref(o), None, None)
    assert rc == comm.COMM_EUNSUPPORTED


# ------------------------------------------------------------------ planned (sorted copies)

def _shuffled(s, seed):
    """The same COO with its nonzeros in a random order (a plan must not rely
    on the caller's order)."""
    perm = np.random.default_rng(seed).permutation(len(s.val))
    return s.idx[perm], s.val[perm]


# orders 3 and 4 with small modes that fit the LDS take one sorted copy and
# the fused pass; (300, 260, 250) does not (two copies), nor does order 2
@pytest.mark.parametrize("dims,density,rank", [((6, 5, 7, 8), 0.05, 3), ((30, 24, 60, 70), 0.01, 8),
                                               ((40, 30, 50), 0.02, 32), ((50, 70), 0.1, 5),
                                               ((300, 260, 250), 0.0005, 4)])
@pytest.mark.parametrize("L", [1, 3])
def test_coo_plan_matches_oracle(ctx, dims, density, rank, L):
    s = workloads.sparse_small(4, dims=dims, density=density, rank=rank)
    init = [f32(a) for a in s.init]
    sidx, sval = _shuffled(s, 5)
    idx = [torch.tensor(sidx[:, n].astype(np.int32), device="cuda") for n in range(len(dims))]
    val = dev(sval)
    plan = ctx.coo_plan(idx, val, dims)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo_plan(plan, fac, L=L, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = osp.jcomm_outer_kl(s.idx, s.val, init, L=L, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < TOL * (1 if L == 1 else 3)
    assert abs(obj.item() - fref) / fref < 1e-5
    plan.close()


def test_coo_plan_skips_out_of_range_coordinates(ctx):
    s = workloads.sparse_small(6, dims=(9, 8, 7, 6), density=0.1, rank=4)
    init = [f32(a) for a in s.init]
    bad = s.idx.copy()
    bad[::7, 2] = 7          # one past the end of mode 3
    bad[3::11, 0] = -1
    idx = [torch.tensor(bad[:, n].astype(np.int32), device="cuda") for n in range(4)]
    val = dev(s.val)
    keep = (bad[:, 2] < 7) & (bad[:, 0] >= 0)
    want = osp.jcomm_outer_kl(s.idx[keep], s.val[keep], init, L=2)
    for planned in (False, True):
        fac = [dev(a) for a in init]
        if planned:
            plan = ctx.coo_plan(idx, val, s.dims)
            ctx.cp_jcomm_outer_coo_plan(plan, fac, L=2)
        else:
            ctx.cp_jcomm_outer_coo(idx, val, s.dims, fac, L=2)
        torch.cuda.synchronize()
        for a, b in zip(fac, want):
            assert max_rel(host64(a), b) < 3 * TOL


def test_coo_plan_empty_tensor(ctx):
    dims = (5, 6, 7)
    idx = [torch.zeros(0, dtype=torch.int32, device="cuda") for _ in dims]
    val = torch.zeros(0, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(0)
    init = [f32(rng.uniform(0.1, 1.0, size=(d, 3))) for d in dims]
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan = ctx.coo_plan(idx, val, dims)
    ctx.cp_jcomm_outer_coo_plan(plan, fac, L=1, obj_out=obj)
    torch.cuda.synchronize()
    empty_idx = np.zeros((0, 3), dtype=np.int64)
    want, fref = osp.jcomm_outer_kl(empty_idx, np.zeros(0), init, L=1, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 1e-5
    assert abs(obj.item() - fref) / fref < 1e-5


def test_coo_plan_day_hour_lat_lon_workload(ctx):
    """The 3.3M-nonzero workload through a plan: objective and one outer
    iteration against the oracle, and agreement with the plan-free path."""
    s = workloads.sparse_counts(0)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    plan = ctx.coo_plan(idx, val, s.dims)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo_plan(plan, fac, L=1, obj_out=obj)
    fac2 = [dev(a) for a in init]
    ctx.cp_jcomm_outer_coo(idx, val, s.dims, fac2, L=1)
    torch.cuda.synchronize()
    fref = osp.objective_kl(s.idx, s.val, init)
    assert abs(obj.item() - fref) / fref < 1e-5
    want = osp.jcomm_outer_kl(s.idx, s.val, init, L=1)
    # both float32 paths are held to the oracle; between themselves they differ
    # only in summation order over rows of up to ~6e5 nonzeros (sqrt(n) * 2^-24
    # is ~5e-5), so they are compared at the same 1e-4 bar
    for a, b, c in zip(fac, want, fac2):
        assert max_rel(host64(a), b) < 1e-4
        assert max_rel(host64(a), host64(c)) < 1e-4


def test_coo_unaligned_factors(ctx):
    """Factors whose base address is 4 bytes past a 16-byte boundary (views into
    a larger buffer) take the scalar gathers and give the same result."""
    s = workloads.sparse_small(7, dims=(20, 12, 30, 25), density=0.05, rank=8)
    init = [f32(a) for a in s.init]
    idx, val = _dev_coo(s)
    fac = []
    for a in init:
        buf = torch.zeros(a.size + 1, dtype=torch.float32, device="cuda")
        v = buf[1:].view(a.shape)
        v.copy_(torch.tensor(a, dtype=torch.float32))
        fac.append(v)
    plan = ctx.coo_plan(idx, val, s.dims)
    ctx.cp_jcomm_outer_coo_plan(plan, fac, L=2)
    torch.cuda.synchronize()
    want = osp.jcomm_outer_kl(s.idx, s.val, init, L=2)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3 * TOL


# The plan pass's edge cases: a wave with a single nonzero (its second half
# empty), odd counts (the halves differ by one), the 32-step windows and the
# 64-nonzero waves' boundaries, several waves (256 nonzeros per wave at these
# sizes; 257 leaves one nonzero to the last wave), rank 32 (the offsets that
# double as accumulator offsets) and rank 5 with an order-3 tensor (one run
# mode in the second copy).
@pytest.mark.parametrize("nnz", [1, 2, 3, 63, 64, 65, 129, 257, 1000])
@pytest.mark.parametrize("dims,rank", [((7, 6, 9, 11), 32), ((7, 6, 29), 5)])
def test_coo_plan_edge_counts(ctx, nnz, dims, rank):
    total = int(np.prod(dims))
    s = workloads.sparse_small(11, dims=dims, density=nnz / total, rank=rank)
    assert len(s.val) == nnz
    init = [f32(a) for a in s.init]
    sidx, sval = _shuffled(s, 3)
    idx = [torch.tensor(sidx[:, n].astype(np.int32), device="cuda") for n in range(len(dims))]
    plan = ctx.coo_plan(idx, dev(sval), dims)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cp_jcomm_outer_coo_plan(plan, fac, L=1, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = osp.jcomm_outer_kl(s.idx, s.val, init, L=1, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < TOL
    assert abs(obj.item() - fref) / fref < 1e-5
    plan.close()
