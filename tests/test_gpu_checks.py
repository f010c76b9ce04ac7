"""The debug input check (comm_opts.check_inputs) and comm_check.

With the check on, data that are negative or not finite, and parameters below
eps or not finite, are refused with COMM_EINVAL before anything is launched,
so every buffer keeps its value; valid inputs give the same bits as without
the check.  comm_check reports no error after ordinary calls."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32, host64  # noqa: E402


@pytest.fixture(scope="module")
def checked():
    c = comm.Context(0, check_inputs=True)
    yield c
    c.close()


@pytest.fixture(scope="module")
def plain():
    c = comm.Context(0)
    yield c
    c.close()


def _cp(seed=0, dims=(20, 24, 28), R=6):
    d = workloads.cp_small(seed, dims=dims, rank=R)
    return f32(d.X), [f32(a) for a in d.init]


def _refused(fn):
    with pytest.raises(comm.CommError) as e:
        fn()
    assert e.value.code == comm.COMM_EINVAL
    assert "check_inputs" in str(e.value)


@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5])
def test_valid_inputs_same_bits(checked, plain, beta):
    X, init = _cp(1)
    a = [dev(f) for f in init]
    b = [dev(f) for f in init]
    oa = torch.zeros(1, dtype=torch.float64, device="cuda")
    ob = torch.zeros(1, dtype=torch.float64, device="cuda")
    checked.jcomm_outer(dev(X), a, beta=beta, L=2, obj_out=oa)
    plain.jcomm_outer(dev(X), b, beta=beta, L=2, obj_out=ob)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    assert oa.item() == ob.item()
    checked.check()


@pytest.mark.parametrize("bad", ["negative", "nan", "inf"])
def test_bad_data_refused(checked, bad):
    X, init = _cp(2)
    X[3, 4, 5] = {"negative": -1.0, "nan": np.nan, "inf": np.inf}[bad]
    fac = [dev(f) for f in init]
    Xd = dev(X)
    _refused(lambda: checked.cp_update(Xd, fac, block=-1, beta=1.0))
    _refused(lambda: checked.jcomm_outer(Xd, fac, beta=0.5, L=1))
    _refused(lambda: checked.beta_objective(Xd, fac, beta=1.5))
    torch.cuda.synchronize()
    for f, g in zip(fac, init):
        assert np.array_equal(host64(f), g)


@pytest.mark.parametrize("bad", ["below_eps", "zero", "nan"])
def test_bad_parameter_refused(checked, bad):
    X, init = _cp(3)
    init[1][7, 2] = {"below_eps": 1e-20, "zero": 0.0, "nan": np.nan}[bad]
    init[1] = f32(init[1])  # the value the device holds
    fac = [dev(f) for f in init]
    _refused(lambda: checked.cp_update(dev(X), fac, block=0, beta=1.0, eps=1e-12))
    torch.cuda.synchronize()
    for f, g in zip(fac, init):
        assert np.array_equal(host64(f), g, equal_nan=True)


def test_tucker_core_checked(checked):
    d = workloads.tucker_dense(0, dims=(12, 10, 8), core_dims=(3, 4, 2))
    core = f32(d.init_core)
    core[1, 2, 1] = -0.5
    fac = [dev(f32(a)) for a in d.init_factors]
    G = dev(core)
    _refused(lambda: checked.tucker_update(dev(f32(d.X)), G, fac, block=-2, beta=1.0))
    torch.cuda.synchronize()
    assert np.array_equal(host64(G), core)


def test_coo_values_checked(checked):
    s = workloads.sparse_small(4, dims=(13, 17, 9), density=0.1, rank=4)
    val = s.val.copy()
    val[5] = -2.0
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(3)]
    fac = [dev(f32(a)) for a in s.init]
    _refused(lambda: checked.cp_jcomm_outer_coo(idx, dev(val), s.dims, fac, L=1))
    _refused(lambda: checked.cp_update_coo(idx, dev(val), s.dims, fac, block=0, beta=0.5))
    torch.cuda.synchronize()
    for f, g in zip(fac, s.init):
        assert np.array_equal(host64(f), f32(g))


def test_batched_problem_checked(plain):
    X, init = _cp(5)
    good = [dev(f) for f in init]
    bad_init = [f.copy() for f in init]
    bad_init[2][0, 0] = -1.0
    bad = [dev(f) for f in bad_init]
    batch = comm.Batch([{"X": dev(X), "factors": good, "beta": 1.0, "check_inputs": True},
                        {"X": dev(X), "factors": bad, "beta": 0.5, "check_inputs": True}])
    with pytest.raises(comm.CommError) as e:
        plain.jcomm_outer_batched(batch)
    assert e.value.code == comm.COMM_EINVAL and "problem 1" in str(e.value)
    torch.cuda.synchronize()
    for f, g in zip(good, init):
        assert np.array_equal(host64(f), g)


def test_comm_check_after_calls(plain):
    X, init = _cp(6)
    fac = [dev(f) for f in init]
    plain.jcomm_outer(dev(X), fac, beta=1.0, L=1)
    plain.check()
