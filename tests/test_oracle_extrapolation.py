"""Pins of the extrapolated variants in oracle/extrapolation.py (Sec. "Going
beyond: Majorization-Minimization with Extrapolation") against special cases
that reduce to the already pinned methods, and hand-computed values."""
import numpy as np
import pytest

from oracle import cp as ocp
from oracle import extrapolation as ox
from oracle import tucker as otk

BETAS = [0.0, 0.5, 1.0, 1.5]


def _cp(seed, dims=(6, 7, 8), R=3):
    rng = np.random.default_rng(seed)
    X = rng.poisson(ocp.rebuild([rng.uniform(0, 1, (d, R)) for d in dims]) * 3) + 0.5
    cur = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
    prev = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
    return X, cur, prev


def _tk(seed, dims=(6, 7, 8), J=(2, 3, 2)):
    rng = np.random.default_rng(seed)
    X = rng.poisson(otk.rebuild(rng.uniform(0, 1, J), [rng.uniform(0, 1, (d, j)) for d, j in zip(dims, J)]) * 3) + 0.5
    core = rng.uniform(0.1, 1.0, J)
    cur = [rng.uniform(0.1, 1.0, (d, j)) for d, j in zip(dims, J)]
    pcore = rng.uniform(0.1, 1.0, J)
    prev = [rng.uniform(0.1, 1.0, (d, j)) for d, j in zip(dims, J)]
    return X, core, cur, pcore, prev


def test_extrapolate_hand_values():
    # [2, 1] with previous [1, 3]: the first entry grew by 1 (extrapolated by
    # alpha * 1), the second shrank (positive part 0, unchanged); an entry that
    # would fall below eps is clipped
    a = np.array([[2.0, 1.0, 1e-13]])
    p = np.array([[1.0, 3.0, 1e-13]])
    got = ox.extrapolate(a, p, 0.5, eps=1e-12)
    assert np.array_equal(got, np.array([[2.5, 1.0, 1e-12]]))


def test_weight_cap_and_nesterov():
    a = [np.array([[3.0, 0.0]]), np.array([[4.0]])]
    p = [np.array([[0.0, 1.0]]), np.array([[0.0]])]
    # ||[a - p]_+|| = ||(3, 0, 4)|| = 5
    assert ox.positive_part_norm(a, p) == pytest.approx(5.0)
    assert ox.weight(a, p, 0.9, 1.0, 0.0) == pytest.approx(0.2)      # cap: 1 / 5
    assert ox.weight(a, p, 0.1, 1.0, 0.0) == pytest.approx(0.1)      # Nesterov weight below the cap
    assert ox.weight(p, p, 0.7, 1.0, 1e-3) == pytest.approx(0.7)     # no displacement: no cap
    assert [ox.nesterov_weight(t) for t in (1, 2, 4)] == pytest.approx([0.0, 0.25, 0.5])


@pytest.mark.parametrize("beta", BETAS)
def test_alpha_zero_is_plain_bcomm(beta):
    X, cur, prev = _cp(1)
    got, _ = ox.cp_bcomm_sweep(X, cur, prev, beta, 0.0)
    want = ocp.bcomm_sweep(X, cur, beta)
    for a, b in zip(got, want):
        assert np.allclose(a, b, rtol=1e-13, atol=0)
    X, core, fac, pcore, pfac = _tk(2)
    G, F, _, _ = ox.tucker_bcomm_sweep(X, core, fac, pcore, pfac, beta, 0.0)
    wg, wf = otk.bcomm_sweep(X, core, fac, beta)
    assert np.allclose(G, wg, rtol=1e-13, atol=0)
    for a, b in zip(F, wf):
        assert np.allclose(a, b, rtol=1e-13, atol=0)


@pytest.mark.parametrize("beta", BETAS)
def test_no_displacement_is_plain_method(beta):
    X, cur, _ = _cp(3)
    got, prev2 = ox.cp_bcomm_sweep(X, cur, [a.copy() for a in cur], beta, 0.8)
    want = ocp.bcomm_sweep(X, cur, beta)
    for a, b in zip(got, want):
        assert np.allclose(a, b, rtol=1e-13, atol=0)
    for a, b in zip(prev2, cur):
        assert np.array_equal(a, b)
    got, _ = ox.cp_jcomm_outer(X, cur, [a.copy() for a in cur], beta, 0.8, L=2)
    want = ocp.jcomm_outer(X, cur, beta, L=2)
    for a, b in zip(got, want):
        assert np.allclose(a, b, rtol=1e-13, atol=0)


@pytest.mark.parametrize("beta", BETAS)
def test_shrinking_iterates_are_not_extrapolated(beta):
    # every entry decreased since the previous iterate: the positive part is 0
    X, core, fac, _, _ = _tk(4)
    pcore = core * 1.5
    pfac = [a + 0.2 for a in fac]
    G, F, _, _ = ox.tucker_jcomm_outer(X, core, fac, pcore, pfac, beta, 0.9)
    wg, wf = otk.jcomm_outer(X, core, fac, beta)
    assert np.allclose(G, wg, rtol=1e-13, atol=0)
    for a, b in zip(F, wf):
        assert np.allclose(a, b, rtol=1e-13, atol=0)


@pytest.mark.parametrize("beta", [0.5, 1.0])
def test_extrapolated_block_is_anchor_and_reconstruction_point(beta):
    """With a positive displacement the block is moved before its update, and
    that moved block, not the current one, is what the MM step starts from:
    the result differs from the plain sweep and equals the plain block update
    taken at the moved point."""
    X, cur, _ = _cp(5)
    # every entry grew since the previous iterate, by different ratios (a
    # uniform rescaling of the block would leave the beta = 1 update unchanged)
    shrink = np.random.default_rng(6).uniform(0.3, 0.9, size=cur[0].shape)
    prev = [cur[0] * shrink] + [a.copy() for a in cur[1:]]
    alpha = 0.6
    got, _ = ox.cp_bcomm_sweep(X, cur, prev, beta, alpha)
    plain = ocp.bcomm_sweep(X, cur, beta)
    assert not np.allclose(got[0], plain[0])
    moved = [a.copy() for a in cur]
    moved[0] = cur[0] + alpha * (cur[0] - prev[0])
    first = ocp.block_update(X, moved, 0, beta)
    assert np.allclose(got[0], first, rtol=1e-12, atol=0)
