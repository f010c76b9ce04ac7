"""The C-ABI J-CoMM call captured into a HIP graph by the caller
(torch.cuda.graph) and replayed: every replay, with eager work and
synchronisations in between, bitwise equal to the same call made eagerly on
a twin problem.  The workspace is grown by an eager call before the capture
(a call that would have to grow it cannot be captured)."""
import numpy as np
import pytest

from oracle import cp as ocp
from oracle import tucker as otk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_14683_amd as comm  # noqa: E402
from tests.gpu_util import dev, f32  # noqa: E402


def _cp(seed, dims=(40, 33, 70), R=16):
    rng = np.random.default_rng(seed)
    X = rng.poisson(ocp.rebuild([rng.uniform(0, 1, size=(d, R)) for d in dims]) * 3.0).astype(np.float64)
    return X, [f32(rng.uniform(0.1, 1.0, size=(d, R))) for d in dims], None


def _tucker(seed, dims=(30, 36, 40), J=(6, 5, 4)):
    rng = np.random.default_rng(seed)
    X = rng.poisson(otk.rebuild(rng.uniform(0, 1, size=J), [rng.uniform(0, 1, size=(d, j)) for d, j in zip(dims, J)])
                    * 2.0).astype(np.float64)
    return X, [f32(rng.uniform(0.1, 1.0, size=(d, j))) for d, j in zip(dims, J)], f32(rng.uniform(0.1, 1.0, size=J))


@pytest.mark.parametrize("make,beta,cache,R", [(_cp, 1.0, False, 16), (_cp, 1.0, False, 32), (_cp, 0.5, True, 32),
                                               (_cp, 1.5, False, 8), (_tucker, 0.0, False, None),
                                               (_tucker, 1.0, False, None)])
def test_captured_call_replays_bitwise(make, beta, cache, R):
    X, init, core = make(3) if R is None else make(3, R=R)
    ctx = comm.Context(0)
    try:
        Xd = dev(X)
        F, Fe = [dev(a) for a in init], [dev(a) for a in init]
        G = dev(core) if core is not None else None
        Ge = dev(core) if core is not None else None
        ob, oe = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2))
        call = lambda f, g, o: ctx.jcomm_outer(Xd, f, core=g, beta=beta, L=2, cache_pq=cache, obj_out=o)  # noqa: E731
        call(F, G, ob)  # grows the workspace; the captured twin advances by the same call
        call(Fe, Ge, oe)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            call(F, G, ob)
        for it in range(4):
            graph.replay()
            call(Fe, Ge, oe)
            torch.cuda.synchronize()
            for a, b in zip(F + ([G] if G is not None else []), Fe + ([Ge] if Ge is not None else [])):
                assert torch.equal(a, b), f"replay {it}"
            assert ob.item() == oe.item(), f"replay {it}"
    finally:
        ctx.close()
