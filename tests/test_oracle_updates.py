"""Pins of the oracle's reconstructions, contractions and B-CoMM / J-CoMM updates
(CPU only).  Each check holds the oracle to something other than itself: an
independent computation route (explicit loops, unfoldings with Khatri-Rao /
Kronecker products), a textbook special case (N = 2 beta-NMF), a planted exact
factorisation that must be a fixed point, an invariant (mass conservation at
beta = 1, equivariances) or a proved descent property."""
import numpy as np
import pytest

import workloads
from oracle import cp, loops, tucker, unfolding
from oracle.divergence import gamma, objective, powers

BETAS = [0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.9]


def _tiny_cp(seed=0, dims=(4, 5, 3), R=3):
    rng = np.random.default_rng(seed)
    fac = [rng.uniform(0.2, 1.5, size=(d, R)) for d in dims]
    X = rng.poisson(2.0, size=dims).astype(float) + rng.uniform(0.0, 0.5, size=dims)
    return X, fac


def _tiny_tucker(seed=0, dims=(4, 3, 5), J=(2, 3, 2)):
    rng = np.random.default_rng(seed)
    core = rng.uniform(0.2, 1.5, size=J)
    fac = [rng.uniform(0.2, 1.5, size=(d, j)) for d, j in zip(dims, J)]
    X = rng.poisson(2.0, size=dims).astype(float) + rng.uniform(0.0, 0.5, size=dims)
    return X, core, fac


# ---------------------------------------------------------------- routes agree

def test_cp_rebuild_three_routes():
    X, fac = _tiny_cp()
    a = cp.rebuild(fac)
    np.testing.assert_allclose(a, loops.cp_rebuild(fac), rtol=1e-13)
    np.testing.assert_allclose(a, unfolding.cp_rebuild(fac), rtol=1e-13)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_cp_contraction_three_routes(n):
    X, fac = _tiny_cp(1)
    others = [fac[m] for m in range(3) if m != n]
    a = cp.cp_contr(X, others, n)
    np.testing.assert_allclose(a, loops.cp_contr(X, others, n), rtol=1e-13)
    np.testing.assert_allclose(a, unfolding.mttkrp(X, fac, n), rtol=1e-13)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_cp_contraction_order4_vs_mttkrp(n):
    rng = np.random.default_rng(2)
    dims = (3, 4, 2, 5)
    fac = [rng.uniform(0.1, 1.0, size=(d, 3)) for d in dims]
    T = rng.uniform(0.0, 2.0, size=dims)
    np.testing.assert_allclose(cp.cp_contr(T, [fac[m] for m in range(4) if m != n], n),
                               unfolding.mttkrp(T, fac, n), rtol=1e-13)


def test_tucker_rebuild_three_routes():
    X, core, fac = _tiny_tucker()
    a = tucker.rebuild(core, fac)
    np.testing.assert_allclose(a, loops.tucker_rebuild(core, fac), rtol=1e-13)
    np.testing.assert_allclose(a, unfolding.tucker_rebuild(core, fac), rtol=1e-13)


def test_tucker_core_contraction_three_routes():
    X, core, fac = _tiny_tucker(1)
    a = tucker.core_contr(X, fac)
    np.testing.assert_allclose(a, loops.tucker_core_contr(X, fac), rtol=1e-13)
    np.testing.assert_allclose(a, unfolding.tucker_core(X, fac), rtol=1e-13)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_tucker_factor_contraction_four_routes(n):
    X, core, fac = _tiny_tucker(2)
    others = [fac[m] for m in range(3) if m != n]
    a = tucker.factor_contr(X, core, others, n)
    np.testing.assert_allclose(a, loops.tucker_factor_contr(X, core, others, n), rtol=1e-13)
    np.testing.assert_allclose(a, unfolding.tucker_factor(X, core, fac, n), rtol=1e-13)
    # two-step route through the partial tensor B^(n) (App. C eq. block_Bn)
    B = tucker.partial_tensor(core, fac, n)
    Xn = np.moveaxis(X, n, 0).reshape(X.shape[n], -1)
    np.testing.assert_allclose(a, Xn @ B.reshape(B.shape[0], -1).T, rtol=1e-13)
    # Xhat is linear in A^(n) through B^(n)
    Xh = np.einsum("ia,a...->i...", fac[n], B)
    np.testing.assert_allclose(np.moveaxis(Xh, 0, n), tucker.rebuild(core, fac), rtol=1e-13)


# ------------------------------------------------------- textbook special case

@pytest.mark.parametrize("beta", BETAS)
def test_order2_cp_is_matrix_beta_nmf_mu(beta):
    """N = 2: X ~ W H with W = A^(1), H = A^(2)^T; the mode-2 block update is the
    Fevotte-Idier MU H <- H * [W^T (V (WH)^(b-2))] / [W^T (WH)^(b-1)] ^ gamma."""
    rng = np.random.default_rng(7)
    V = rng.uniform(0.5, 3.0, size=(6, 7))
    W = rng.uniform(0.2, 1.0, size=(6, 3))
    H = rng.uniform(0.2, 1.0, size=(3, 7))
    WH = W @ H
    H_mu = H * ((W.T @ (V * WH ** (beta - 2))) / (W.T @ WH ** (beta - 1))) ** gamma(beta)
    W_mu = W * (((V * WH ** (beta - 2)) @ H.T) / (WH ** (beta - 1) @ H.T)) ** gamma(beta)
    got_h = cp.block_update(V, [W, H.T], 1, beta)
    got_w = cp.block_update(V, [W, H.T], 0, beta)
    np.testing.assert_allclose(got_h, H_mu.T, rtol=1e-12)
    np.testing.assert_allclose(got_w, W_mu, rtol=1e-12)


# ---------------------------------------------------------- planted fixed point

@pytest.mark.parametrize("beta", BETAS)
def test_planted_cp_is_fixed_point(beta):
    d = workloads.planted_exact_cp(5, (5, 6, 4), 3)
    out = cp.bcomm_sweep(d.X, d.init, beta)
    for a, b in zip(out, d.init):
        np.testing.assert_allclose(a, b, rtol=1e-12)
    for L in (1, 2):
        out = cp.jcomm_outer(d.X, d.init, beta, L=L)
        for a, b in zip(out, d.init):
            np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("beta", BETAS)
def test_planted_tucker_is_fixed_point(beta):
    d = workloads.planted_exact_tucker(6, (5, 4, 6), (2, 3, 2))
    G, fac = tucker.bcomm_sweep(d.X, d.init_core, d.init_factors, beta)
    np.testing.assert_allclose(G, d.init_core, rtol=1e-12)
    for a, b in zip(fac, d.init_factors):
        np.testing.assert_allclose(a, b, rtol=1e-12)
    G, fac = tucker.jcomm_outer(d.X, d.init_core, d.init_factors, beta, L=2)
    np.testing.assert_allclose(G, d.init_core, rtol=1e-12)
    for a, b in zip(fac, d.init_factors):
        np.testing.assert_allclose(a, b, rtol=1e-12)


# --------------------------------------------------------------- descent

@pytest.mark.parametrize("beta", BETAS)
def test_cp_block_updates_decrease_objective(beta):
    X, fac = _tiny_cp(3, dims=(6, 5, 7), R=3)
    cur = [a.copy() for a in fac]
    f = objective(X, cp.rebuild(cur), beta)
    for sweep in range(4):
        for n in range(3):
            cur[n] = cp.block_update(X, cur, n, beta)
            f_new = objective(X, cp.rebuild(cur), beta)
            assert f_new <= f * (1 + 1e-13)
            f = f_new


@pytest.mark.parametrize("beta", BETAS)
def test_tucker_block_updates_decrease_objective(beta):
    X, core, fac = _tiny_tucker(4, dims=(6, 5, 4), J=(2, 3, 2))
    G = core.copy()
    cur = [a.copy() for a in fac]
    f = objective(X, tucker.rebuild(G, cur), beta)
    for sweep in range(3):
        G = tucker.block_update_core(X, G, cur, beta)
        f_new = objective(X, tucker.rebuild(G, cur), beta)
        assert f_new <= f * (1 + 1e-13)
        f = f_new
        for n in range(3):
            cur[n] = tucker.block_update_factor(X, G, cur, n, beta)
            f_new = objective(X, tucker.rebuild(G, cur), beta)
            assert f_new <= f * (1 + 1e-13)
            f = f_new


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("L", [1, 3])
def test_jcomm_outer_iterations_decrease_objective(beta, L):
    X, fac = _tiny_cp(8, dims=(6, 7, 5), R=4)
    _, trace = cp.run(X, fac, beta, 6, method="jcomm", L=L)
    assert all(b <= a * (1 + 1e-13) for a, b in zip(trace, trace[1:]))
    X, core, tf = _tiny_tucker(9, dims=(5, 6, 4), J=(2, 2, 3))
    _, _, trace = tucker.run(X, core, tf, beta, 5, method="jcomm", L=L)
    assert all(b <= a * (1 + 1e-13) for a, b in zip(trace, trace[1:]))


# ---------------------------------------------- J-CoMM relative to B-CoMM

@pytest.mark.parametrize("beta", BETAS)
def test_jcomm_first_block_equals_block_update(beta):
    """chi(Z, Z) = Z, so the first inner block of J-CoMM is the block-MM update."""
    X, fac = _tiny_cp(10)
    ref = [a.copy() for a in fac]
    Pt, Qt = powers(X, cp.rebuild(ref), beta)
    got = cp.jcomm_inner_update(Pt, Qt, ref, ref, 0, beta)
    np.testing.assert_allclose(got, cp.block_update(X, fac, 0, beta), rtol=1e-13)
    X, core, tf = _tiny_tucker(11)
    G_j, _ = tucker.jcomm_outer(X, core, tf, beta, L=1)
    np.testing.assert_allclose(G_j, tucker.block_update_core(X, core, tf, beta), rtol=1e-13)


# ------------------------------------------------------------ beta = 1 structure

def _mass(X, fac):
    return cp.rebuild(fac).sum(), X.sum()


def test_kl_mass_conservation_cp():
    X, fac = _tiny_cp(12, dims=(5, 6, 7), R=3)
    cur = [a.copy() for a in fac]
    for n in range(3):
        cur[n] = cp.block_update(X, cur, n, 1.0)
        np.testing.assert_allclose(cp.rebuild(cur).sum(), X.sum(), rtol=1e-13)
    ref = [a.copy() for a in fac]
    Pt, Qt = powers(X, cp.rebuild(ref), 1.0)
    cur = [a.copy() for a in fac]
    for _ in range(2):
        for n in range(3):
            cur[n] = cp.jcomm_inner_update(Pt, Qt, cur, ref, n, 1.0)
            np.testing.assert_allclose(cp.rebuild(cur).sum(), X.sum(), rtol=1e-13)


def test_kl_mass_conservation_tucker():
    X, core, fac = _tiny_tucker(13)
    G, cur = tucker.bcomm_sweep(X, core, fac, 1.0)
    np.testing.assert_allclose(tucker.rebuild(G, cur).sum(), X.sum(), rtol=1e-13)
    G, cur = tucker.jcomm_outer(X, core, fac, 1.0, L=2)
    np.testing.assert_allclose(tucker.rebuild(G, cur).sum(), X.sum(), rtol=1e-13)


def test_kl_denominator_is_product_of_column_sums():
    X, fac = _tiny_cp(14)
    ones = np.ones_like(X)
    den = cp.cp_contr(ones, [fac[1], fac[2]], 0)
    np.testing.assert_allclose(den, np.tile(fac[1].sum(0) * fac[2].sum(0), (X.shape[0], 1)), rtol=1e-13)


# ---------------------------------------------------------------- equivariance

@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5])
def test_component_permutation_equivariance(beta):
    X, fac = _tiny_cp(15, R=4)
    perm = np.array([2, 0, 3, 1])
    a = cp.jcomm_outer(X, fac, beta, L=2)
    b = cp.jcomm_outer(X, [f[:, perm] for f in fac], beta, L=2)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x[:, perm], y, rtol=1e-12)


@pytest.mark.parametrize("beta", BETAS)
def test_scaling_equivariance(beta):
    """d_beta(cx|cy) = c^beta d_beta(x|y): scaling X and A^(1) by c scales the new
    A^(1) by c and leaves the other factors unchanged."""
    X, fac = _tiny_cp(16)
    c = 5.0
    a = cp.bcomm_sweep(X, fac, beta)
    b = cp.bcomm_sweep(c * X, [c * fac[0], fac[1], fac[2]], beta)
    np.testing.assert_allclose(b[0], c * a[0], rtol=1e-11)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-11)
    np.testing.assert_allclose(b[2], a[2], rtol=1e-11)
    a = cp.jcomm_outer(X, fac, beta, L=2)
    b = cp.jcomm_outer(c * X, [c * fac[0], fac[1], fac[2]], beta, L=2)
    np.testing.assert_allclose(b[0], c * a[0], rtol=1e-11)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-11)
    assert objective(c * X, c * cp.rebuild(fac), beta) == pytest.approx(
        c ** beta * objective(X, cp.rebuild(fac), beta), rel=1e-11)


def test_eps_clip_binds_on_zero_numerator():
    """A row of X that is all zero gives Num = 0 (beta > 0): the block minimiser on
    the eps-constrained set is eps."""
    X, fac = _tiny_cp(17)
    X[1] = 0.0
    out = cp.block_update(X, fac, 0, 1.0, eps=1e-9)
    assert np.all(out[1] == 1e-9)
    assert np.all(out[0] > 1e-9)


# ------------------------------------------------------------ order 4 (the paper's CP shape class)

@pytest.mark.parametrize("beta", BETAS)
def test_planted_order4_cp_is_fixed_point(beta):
    d = workloads.planted_exact_cp(13, (5, 4, 3, 6), 3)
    for out in (cp.bcomm_sweep(d.X, d.init, beta), cp.jcomm_outer(d.X, d.init, beta, L=2)):
        for a, b in zip(out, d.init):
            np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("beta", BETAS)
def test_order4_cp_updates_decrease_objective(beta):
    rng = np.random.default_rng(14)
    dims, R = (5, 4, 3, 6), 3
    X = rng.poisson(cp.rebuild([rng.uniform(0, 1, (d, R)) for d in dims]) * 4) + 0.5
    fac = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
    for method in ("bcomm", "jcomm"):
        _, trace = cp.run(X, fac, beta, 5, method=method, L=2)
        assert all(b <= a * (1 + 1e-13) for a, b in zip(trace, trace[1:]))


# ------------------------------------------------------- order-4 Tucker

@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_order4_tucker_contractions_vs_unfolding(n):
    """The einsum contractions of the order-4 Tucker oracle equal the
    unfolding / Kronecker identities (Kolda-Bader), a route that shares no code
    with them."""
    rng = np.random.default_rng(21)
    dims, J = (4, 3, 5, 3), (2, 3, 2, 2)
    T = rng.uniform(0.0, 2.0, size=dims)
    core = rng.uniform(0.1, 1.0, size=J)
    fac = [rng.uniform(0.1, 1.0, size=(d, j)) for d, j in zip(dims, J)]
    others = [fac[m] for m in range(4) if m != n]
    np.testing.assert_allclose(tucker.factor_contr(T, core, others, n),
                               unfolding.tucker_factor(T, core, fac, n), rtol=1e-13)
    np.testing.assert_allclose(tucker.core_contr(T, fac), unfolding.tucker_core(T, fac), rtol=1e-13)
    np.testing.assert_allclose(tucker.rebuild(core, fac), unfolding.tucker_rebuild(core, fac), rtol=1e-13)


@pytest.mark.parametrize("beta", BETAS)
def test_planted_order4_tucker_is_fixed_point(beta):
    d = workloads.planted_exact_tucker(22, (5, 4, 3, 6), (2, 3, 2, 2))
    for G, fac in (tucker.bcomm_sweep(d.X, d.init_core, d.init_factors, beta),
                   tucker.jcomm_outer(d.X, d.init_core, d.init_factors, beta, L=2)):
        np.testing.assert_allclose(G, d.init_core, rtol=1e-12)
        for a, b in zip(fac, d.init_factors):
            np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("beta", BETAS)
def test_order4_tucker_updates_decrease_objective(beta):
    rng = np.random.default_rng(23)
    dims, J = (5, 4, 3, 6), (2, 3, 2, 2)
    X = rng.poisson(tucker.rebuild(rng.uniform(0, 1, J), [rng.uniform(0, 1, (d, j)) for d, j in zip(dims, J)])
                    * 4) + 0.5
    core = rng.uniform(0.1, 1.0, J)
    fac = [rng.uniform(0.1, 1.0, (d, j)) for d, j in zip(dims, J)]
    for method in ("bcomm", "jcomm"):
        _, _, trace = tucker.run(X, core, fac, beta, 5, method=method, L=2)
        assert all(b <= a * (1 + 1e-13) for a, b in zip(trace, trace[1:]))


def test_kl_mass_conservation_order4_tucker():
    rng = np.random.default_rng(24)
    dims, J = (5, 4, 3, 6), (2, 3, 2, 2)
    X = rng.poisson(3.0, size=dims) + 0.5
    core = rng.uniform(0.1, 1.0, J)
    fac = [rng.uniform(0.1, 1.0, (d, j)) for d, j in zip(dims, J)]
    G, cur = tucker.bcomm_sweep(X, core, fac, 1.0)
    np.testing.assert_allclose(tucker.rebuild(G, cur).sum(), X.sum(), rtol=1e-13)
    G, cur = tucker.jcomm_outer(X, core, fac, 1.0, L=2)
    np.testing.assert_allclose(tucker.rebuild(G, cur).sum(), X.sum(), rtol=1e-13)


# ------------------------------------------------------- order-5 Tucker

@pytest.mark.parametrize("n", [0, 2, 4])
def test_order5_tucker_contractions_vs_unfolding(n):
    rng = np.random.default_rng(31)
    dims, J = (3, 4, 2, 3, 4), (2, 2, 1, 2, 3)
    T = rng.uniform(0.0, 2.0, size=dims)
    core = rng.uniform(0.1, 1.0, size=J)
    fac = [rng.uniform(0.1, 1.0, size=(d, j)) for d, j in zip(dims, J)]
    others = [fac[m] for m in range(5) if m != n]
    np.testing.assert_allclose(tucker.factor_contr(T, core, others, n),
                               unfolding.tucker_factor(T, core, fac, n), rtol=1e-13)
    np.testing.assert_allclose(tucker.core_contr(T, fac), unfolding.tucker_core(T, fac), rtol=1e-13)


@pytest.mark.parametrize("beta", BETAS)
def test_planted_order5_tucker_is_fixed_point(beta):
    d = workloads.planted_exact_tucker(32, (4, 3, 2, 3, 5), (2, 2, 1, 2, 2))
    for G, fac in (tucker.bcomm_sweep(d.X, d.init_core, d.init_factors, beta),
                   tucker.jcomm_outer(d.X, d.init_core, d.init_factors, beta, L=2)):
        np.testing.assert_allclose(G, d.init_core, rtol=1e-12)
        for a, b in zip(fac, d.init_factors):
            np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5])
def test_order5_tucker_updates_decrease_objective(beta):
    rng = np.random.default_rng(33)
    dims, J = (4, 3, 2, 3, 5), (2, 2, 1, 2, 2)
    X = rng.poisson(tucker.rebuild(rng.uniform(0, 1, J), [rng.uniform(0, 1, (d, j)) for d, j in zip(dims, J)])
                    * 4) + 0.5
    core = rng.uniform(0.1, 1.0, J)
    fac = [rng.uniform(0.1, 1.0, (d, j)) for d, j in zip(dims, J)]
    for method in ("bcomm", "jcomm"):
        _, _, trace = tucker.run(X, core, fac, beta, 4, method=method, L=2)
        assert all(b <= a * (1 + 1e-13) for a, b in zip(trace, trace[1:]))
