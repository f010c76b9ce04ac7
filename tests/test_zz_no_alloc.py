"""GPU tests of comm_jcomm_outer_noalloc, the J-CoMM outer iteration whose
workspace is the library's fixed per-GPU array instead of the context's
allocation.  It runs the kernels and launch shapes of comm_jcomm_outer, so
every result must equal that entry point's bit for bit; two calls in a row
(the second on a smaller problem) check that nothing left in the shared array
by one call leaks into the next."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from oracle import cp as ocp  # noqa: E402
from oracle import tucker as otk  # noqa: E402
from tests.gpu_util import dev, f32  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = comm.Context(0)
    yield c
    c.close()


def _cp(seed, dims, R):
    rng = np.random.default_rng(seed)
    planted = [rng.uniform(0.0, 1.0, size=(d, R)) for d in dims]
    X = rng.poisson(ocp.rebuild(planted) * 4.0).astype(np.float64)
    init = [f32(rng.uniform(0.1, 1.0, size=(d, R))) for d in dims]
    return X, init, None


def _tucker(seed, dims, J):
    rng = np.random.default_rng(seed)
    core = rng.uniform(0.0, 1.0, size=J)
    fac = [rng.uniform(0.0, 1.0, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(otk.rebuild(core, fac) * 2.0).astype(np.float64)
    return X, [f32(rng.uniform(0.1, 1.0, size=(d, j))) for d, j in zip(dims, J)], f32(rng.uniform(0.1, 1.0, size=J))


def _both(ctx, prob, beta, L, cache_pq=False):
    X, init, core = prob
    Xd = dev(X)
    out = []
    for fn in (ctx.jcomm_outer, ctx.jcomm_outer_noalloc):
        F = [dev(a) for a in init]
        G = dev(core) if core is not None else None
        obj = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        fn(Xd, F, core=G, beta=beta, L=L, cache_pq=cache_pq, obj_out=obj)
        torch.cuda.synchronize()
        out.append(([f.cpu().numpy() for f in F], None if G is None else G.cpu().numpy(), obj.item()))
    return out


def _same(a, b):
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(x, y)
    if a[1] is not None:
        assert np.array_equal(a[1], b[1])
    assert a[2] == b[2]


# each case: a larger problem, then a smaller one in the next call
CASES = [
    (lambda: _cp(1, (96, 80, 70), 16), 0.5, 2, True, lambda: _cp(2, (40, 30, 20), 5), 1.0, 3, False),
    (lambda: _cp(3, (256, 256, 256), 32), 1.0, 5, False, lambda: _cp(4, (33, 65, 17), 32), 1.5, 1, False),
    (lambda: _tucker(5, (60, 50, 70), (8, 6, 7)), 0.0, 1, "auto", lambda: _tucker(6, (20, 25, 30), (4, 5, 3)),
     1.5, 2, False),
    (lambda: _cp(7, (30, 20, 25, 18), 6), 0.5, 1, False, lambda: _cp(8, (12, 10, 9, 8), 3), 1.0, 2, False),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_jcomm_outer_twice(ctx, case):
    big, b1, l1, c1, small, b2, l2, c2 = CASES[case]
    r1 = _both(ctx, big(), b1, l1, c1)
    _same(r1[0], r1[1])
    r2 = _both(ctx, small(), b2, l2, c2)
    _same(r2[0], r2[1])


def test_noalloc_refuses_what_does_not_fit(ctx):
    """A 512^3 rank-32 problem needs more than the fixed array: COMM_ENOMEM
    from the host check, before anything is read or launched (the tensor and
    factors are small stand-ins that are never touched), and nothing changes."""
    dims = (512, 512, 512)
    assert ctx.workspace_bytes(dims, rank=32) > comm.NOALLOC_SCRATCH_BYTES
    X = torch.zeros(4, device="cuda")
    F = [torch.ones(4, device="cuda") for _ in dims]
    d = comm.Dense()
    d.ndim = 3
    for n, v in enumerate(dims):
        d.dims[n] = v
    d.X = X.data_ptr()
    m = comm.Model()
    m.kind, m.rank = comm.COMM_CP, 32
    for n in range(3):
        m.factors[n] = F[n].data_ptr()
    o = ctx._o(1.0, 1e-12, None, 1)
    with pytest.raises(comm.CommError) as e:
        comm._check(ctx._lib.comm_jcomm_outer_noalloc(ctx._h, comm.ctypes.byref(d), comm.ctypes.byref(m),
                                                      comm.ctypes.byref(o), None, None))
    assert e.value.code == comm.COMM_ENOMEM
    torch.cuda.synchronize()
    assert all(torch.equal(f, torch.ones(4, device="cuda")) for f in F)


def test_noalloc_refuses_the_debug_check():
    c = comm.Context(0, check_inputs=True)
    try:
        X, init, _ = _cp(9, (20, 20, 20), 4)
        with pytest.raises(comm.CommError) as e:
            c.jcomm_outer_noalloc(dev(X), [dev(a) for a in init], beta=1.0)
        assert e.value.code == comm.COMM_EINVAL
    finally:
        c.close()
