"""Pins of the joint surrogate (tightness, majorisation, blockwise minimality),
the scalar subproblems (brute force) and the sparse beta = 1 path (equal to the
dense path on the densified tensor).  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import cp, sparse, surrogate, tucker
from oracle.divergence import objective, powers

BETAS = [0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.9]


def _tiny(seed, dims=(4, 3, 5), R=3):
    rng = np.random.default_rng(seed)
    fac = [rng.uniform(0.2, 1.5, size=(d, R)) for d in dims]
    X = rng.poisson(2.0, size=dims).astype(float) + rng.uniform(0.05, 0.5, size=dims)
    return X, fac, rng


@pytest.mark.parametrize("beta", BETAS)
def test_surrogate_tight_and_majorising_cp(beta):
    X, ref, rng = _tiny(1)
    F = objective(X, cp.rebuild(ref), beta)
    assert surrogate.surrogate_cp(X, ref, ref, beta) == pytest.approx(F, rel=1e-13)
    for _ in range(20):
        th = [a * np.exp(rng.normal(0, 0.5, size=a.shape)) for a in ref]
        assert surrogate.surrogate_cp(X, th, ref, beta) >= objective(X, cp.rebuild(th), beta) * (1 - 1e-13)


@pytest.mark.parametrize("beta", BETAS)
def test_surrogate_tight_and_majorising_tucker(beta):
    rng = np.random.default_rng(2)
    dims, J = (3, 4, 3), (2, 2, 2)
    core = rng.uniform(0.3, 1.2, size=J)
    ref = [rng.uniform(0.3, 1.2, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(2.0, size=dims).astype(float) + 0.1
    F = objective(X, tucker.rebuild(core, ref), beta)
    assert surrogate.surrogate_tucker(X, core, ref, core, ref, beta) == pytest.approx(F, rel=1e-13)
    for _ in range(10):
        c2 = core * np.exp(rng.normal(0, 0.4, size=J))
        t2 = [a * np.exp(rng.normal(0, 0.4, size=a.shape)) for a in ref]
        assert (surrogate.surrogate_tucker(X, c2, t2, core, ref, beta)
                >= objective(X, tucker.rebuild(c2, t2), beta) * (1 - 1e-13))


@pytest.mark.parametrize("beta", BETAS)
def test_inner_update_is_block_minimiser_and_decreases_G(beta):
    X, ref, rng = _tiny(3)
    Pt, Qt = powers(X, cp.rebuild(ref), beta)
    cur = [a * np.exp(rng.normal(0, 0.2, size=a.shape)) for a in ref]
    g_prev = surrogate.surrogate_cp(X, cur, ref, beta)
    for n in range(3):
        new = cp.jcomm_inner_update(Pt, Qt, cur, ref, n, beta)
        cur = cur[:n] + [new] + cur[n + 1:]
        g_new = surrogate.surrogate_cp(X, cur, ref, beta)
        assert g_new <= g_prev * (1 + 1e-13)
        g_prev = g_new
        for _ in range(8):
            pert = cur[:n] + [new * np.exp(rng.normal(0, 0.05, size=new.shape))] + cur[n + 1:]
            assert surrogate.surrogate_cp(X, pert, ref, beta) >= g_new * (1 - 1e-13)


@pytest.mark.parametrize("beta", BETAS)
def test_tucker_inner_updates_decrease_G(beta):
    rng = np.random.default_rng(4)
    dims, J = (3, 4, 3), (2, 2, 2)
    core = rng.uniform(0.3, 1.2, size=J)
    ref = [rng.uniform(0.3, 1.2, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(2.0, size=dims).astype(float) + 0.1
    g0 = surrogate.surrogate_tucker(X, core, ref, core, ref, beta)
    G, fac = tucker.jcomm_outer(X, core, ref, beta, L=2)
    g1 = surrogate.surrogate_tucker(X, G, fac, core, ref, beta)
    assert g1 <= g0 * (1 + 1e-13)
    assert objective(X, tucker.rebuild(G, fac), beta) <= g1 * (1 + 1e-13)
    # the core block (updated first, while the factors still equal the reference)
    # is the block minimiser of G(. | ref)
    G1, _ = tucker.jcomm_outer(X, core, ref, beta, L=1)
    g_core = surrogate.surrogate_tucker(X, G1, ref, core, ref, beta)
    for _ in range(8):
        Gp = G1 * np.exp(rng.normal(0, 0.05, size=J))
        assert surrogate.surrogate_tucker(X, Gp, ref, core, ref, beta) >= g_core * (1 - 1e-13)


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("L", [1, 2])
def test_tucker_every_inner_block_is_block_minimiser(beta, L):
    """Each block of a Tucker J-CoMM sweep (the core, then every factor, in
    every inner sweep) is the minimiser of G(. | ref) over that block with the
    other blocks at their current inner values (Sec. 5.3; App. C.3): random
    log-perturbations of the freshly updated block never lower G, and G does
    not increase from one block to the next."""
    rng = np.random.default_rng(6)
    dims, J = (4, 3, 5), (2, 3, 2)
    Gref = rng.uniform(0.3, 1.2, size=J)
    ref = [rng.uniform(0.3, 1.2, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(2.0, size=dims).astype(float) + 0.1
    Pt, Qt = powers(X, tucker.rebuild(Gref, ref), beta)
    G, cur = Gref.copy(), [a.copy() for a in ref]
    g_prev = surrogate.surrogate_tucker(X, G, cur, Gref, ref, beta)

    def check_minimal(G, cur, g_new, block):
        for _ in range(6):
            if block < 0:
                Gp, cp_ = G * np.exp(rng.normal(0, 0.05, size=G.shape)), cur
            else:
                Gp = G
                cp_ = [a * np.exp(rng.normal(0, 0.05, size=a.shape)) if m == block else a
                       for m, a in enumerate(cur)]
            assert surrogate.surrogate_tucker(X, Gp, cp_, Gref, ref, beta) >= g_new * (1 - 1e-13), block

    for _ in range(L):
        G = tucker.jcomm_inner_update_core(Pt, Qt, cur, ref, Gref, beta)
        g_new = surrogate.surrogate_tucker(X, G, cur, Gref, ref, beta)
        assert g_new <= g_prev * (1 + 1e-13)
        check_minimal(G, cur, g_new, -1)
        g_prev = g_new
        for n in range(3):
            cur[n] = tucker.jcomm_inner_update_factor(Pt, Qt, G, Gref, cur, ref, n, beta)
            g_new = surrogate.surrogate_tucker(X, G, cur, Gref, ref, beta)
            assert g_new <= g_prev * (1 + 1e-13), n
            check_minimal(G, cur, g_new, n)
            g_prev = g_new
    # the step-by-step sweep is the oracle's outer iteration
    G2, cur2 = tucker.jcomm_outer(X, Gref, ref, beta, L=L)
    np.testing.assert_array_equal(G, G2)
    for a, b in zip(cur, cur2):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("beta", BETAS)
def test_scalar_minimiser_brute_force(beta):
    rng = np.random.default_rng(5)
    for _ in range(5):
        num, den = rng.uniform(0.1, 5.0, size=2)
        u_star = surrogate.scalar_minimiser(num, den, beta)
        grid = np.exp(np.linspace(np.log(u_star) - 3, np.log(u_star) + 3, 200001))
        g = surrogate.scalar_surrogate(grid, num, den, beta)
        assert grid[np.argmin(g)] == pytest.approx(u_star, rel=1e-4)


def test_sparse_kl_equals_dense_on_densified_tensor():
    s = workloads.sparse_small(0, dims=(5, 4, 6, 7), density=0.08, rank=3)
    X = workloads.densify(s)
    for L in (1, 2):
        got, fobj = sparse.jcomm_outer_kl(s.idx, s.val, s.init, L=L, return_ref_obj=True)
        want, wobj = cp.jcomm_outer(X, s.init, 1.0, L=L, return_ref_obj=True)
        for a, b in zip(got, want):
            np.testing.assert_allclose(a, b, rtol=1e-12)
        assert fobj == pytest.approx(wobj, rel=1e-13)
