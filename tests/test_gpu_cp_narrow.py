"""GPU parity of the 16-wide CP pass tiles (rank <= 16, float32), through the
C ABI, against the FP64 oracle.

At rank <= 16 the dense CP passes reduce the reconstruction over 16 columns
and run the three contractions on 16x16x4 matrix-core tiles, with the weight
tile regrouped by lane swaps for mode 3 (paper Sec. 6.1 CPContr; the same
sums as the 32-wide tiles in another order).  Bars as for the 32-wide tiles:
1e-5 relative per factor entry after one block update, 3e-5 after two inner
sweeps, 1e-5 on the objective.  Shapes are ragged in every mode and span
several tiles; rank 16 fills the narrow tile, rank 1 is the degenerate case.
The 32-wide tiles (an autotune table entry) give the same results to the same
bars, and the 16-wide results are bitwise reproducible."""
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

BETAS = [0.0, 0.5, 1.0, 1.5, 0.7, 1.3]
SHAPES = [((33, 45, 70), 16), ((40, 29, 67), 10), ((17, 18, 19), 1), ((70, 9, 100), 13)]


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _problem(dims, R, seed):
    rng = np.random.default_rng(seed)
    planted = [rng.uniform(0.0, 1.0, size=(d, R)) for d in dims]
    X = rng.poisson(ocp.rebuild(planted) * 4.0).astype(np.float64)
    init = [f32(rng.uniform(0.1, 1.0, size=(d, R))) for d in dims]
    return X, init


def _xf(X, beta):
    return np.maximum(X, 1e-12) if beta == 0.0 else X


@pytest.mark.parametrize("dims,R", SHAPES)
@pytest.mark.parametrize("beta", BETAS)
def test_block_update_every_mode(ctx, dims, R, beta):
    X, init = _problem(dims, R, 1)
    Xd = dev(X)
    for n in range(3):
        fac = [dev(a) for a in init]
        ctx.cp_update(Xd, fac, block=n, beta=beta)
        torch.cuda.synchronize()
        assert max_rel(host64(fac[n]), ocp.block_update(X, init, n, beta)) < 1e-5, f"mode {n}"


@pytest.mark.parametrize("dims,R", SHAPES)
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("cache", [False, True])
def test_jcomm_outer(ctx, dims, R, beta, cache):
    if cache and beta == 1.0:
        pytest.skip("beta = 1 never caches P~ / Q~")
    X, init = _problem(dims, R, 2)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(X), fac, beta=beta, L=2, cache_pq=cache, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(X, init, beta, L=2, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3e-5
    assert abs(obj.item() - fref) / fref < 1e-5


@pytest.mark.parametrize("beta", BETAS)
def test_objective(ctx, beta):
    X, init = _problem((40, 29, 67), 10, 3)
    got = ctx.beta_objective(dev(X), [dev(a) for a in init], beta=beta).item()
    want = oobjective(_xf(X, beta), ocp.rebuild(init), beta)
    assert abs(got - want) / want < 1e-5


@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_wide_tiles_agree(beta):
    """The same J-CoMM iteration with the 32-wide tiles (table entry), on a
    fresh context: both within the bar of the oracle, and not bitwise equal
    (the entry does switch the tiles: their sums run in another order)."""
    X, init = _problem((40, 29, 67), 10, 4)
    want, fref = ocp.jcomm_outer(X, init, beta, L=2, return_ref_obj=True)
    out = {}
    for tile in (0, 32):
        c = comm.Context(0)
        try:
            Xd = dev(X)
            fac = [dev(a) for a in init]
            c.tune_set(Xd, fac, beta=beta, L=2, cp_tile=tile)
            assert c.tune_entry(Xd, fac, beta=beta, L=2)["cp_tile"] == (16 if tile == 0 else 32)
            obj = torch.zeros(1, dtype=torch.float64, device="cuda")
            c.jcomm_outer(Xd, fac, beta=beta, L=2, obj_out=obj)
            torch.cuda.synchronize()
            out[tile] = [host64(a) for a in fac]
            for a, b in zip(out[tile], want):
                assert max_rel(a, b) < 3e-5
            assert abs(obj.item() - fref) / fref < 1e-5
        finally:
            c.close()
    assert not all(np.array_equal(a, b) for a, b in zip(out[0], out[32]))


def test_bitwise_reproducible(ctx):
    X, init = _problem((70, 9, 100), 13, 5)
    runs = []
    for _ in range(2):
        fac = [dev(a) for a in init]
        obj = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.jcomm_outer(dev(X), fac, beta=0.5, L=2, obj_out=obj)
        torch.cuda.synchronize()
        runs.append(([host64(a) for a in fac], obj.item()))
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)
    assert runs[0][1] == runs[1][1]


def test_order4_rank10(ctx):
    """Order 4 at rank 10 (the paper's synthetic CP rank) through the 3-way
    view, whose passes take the 16-wide tiles."""
    X, init = _problem((12, 9, 40, 70), 10, 6)
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(X), fac, beta=1.0, L=2, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(X, init, 1.0, L=2, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3e-5
    assert abs(obj.item() - fref) / fref < 1e-5


def test_full_size_rank16_kl(ctx):
    """256^3 at rank 16, beta = 1, L = 5: every factor entry after one outer
    iteration against the oracle."""
    d = workloads.cp_dense(0, rank=16)
    init = [f32(a) for a in d.init]
    fac = [dev(a) for a in init]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.jcomm_outer(dev(d.X), fac, beta=1.0, L=5, obj_out=obj)
    torch.cuda.synchronize()
    want, fref = ocp.jcomm_outer(d.X, init, 1.0, L=5, return_ref_obj=True)
    for a, b in zip(fac, want):
        assert max_rel(host64(a), b) < 3e-5
    assert abs(obj.item() - fref) / fref < 1e-5
