"""Pins of the oracle's beta-divergence, objective, gamma and transforms against
closed forms, a library routine and mathematical identities (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special

import oracle
from oracle.divergence import beta_divergence, chi1, chi2, gamma, objective, powers

BETAS = [0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.9]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid():
    rng = np.random.default_rng(11)
    x = rng.uniform(0.05, 5.0, size=400)
    y = rng.uniform(0.05, 5.0, size=400)
    return x, y


@pytest.mark.parametrize("beta", BETAS)
def test_divergence_zero_on_diagonal_and_nonnegative(beta):
    x, y = _grid()
    assert np.max(np.abs(beta_divergence(x, x, beta))) < 1e-14
    assert np.all(beta_divergence(x, y, beta) >= -1e-15)


def test_kl_matches_scipy_kl_div():
    x, y = _grid()
    x = np.concatenate([x, [0.0, 0.0]])
    y = np.concatenate([y, [0.3, 2.0]])
    np.testing.assert_allclose(beta_divergence(x, y, 1.0), scipy.special.kl_div(x, y), rtol=1e-13, atol=1e-15)


def test_general_branch_at_beta_two_is_half_squared_error():
    x, y = _grid()
    np.testing.assert_allclose(beta_divergence(x, y, 2.0), 0.5 * (x - y) ** 2, rtol=1e-12, atol=1e-14)


def test_itakura_saito_closed_form_and_limit():
    x, y = _grid()
    np.testing.assert_allclose(beta_divergence(x, y, 0.0), x / y - np.log(x / y) - 1.0, rtol=1e-14)
    # the general branch tends to the beta = 0 and beta = 1 branches
    np.testing.assert_allclose(beta_divergence(x, y, 1e-6), beta_divergence(x, y, 0.0), rtol=2e-4, atol=1e-7)
    np.testing.assert_allclose(beta_divergence(x, y, 1.0 + 1e-6), beta_divergence(x, y, 1.0), rtol=2e-4, atol=1e-7)


@pytest.mark.parametrize("beta", BETAS)
def test_homogeneity(beta):
    x, y = _grid()
    c = 3.7
    np.testing.assert_allclose(beta_divergence(c * x, c * y, beta), c ** beta * beta_divergence(x, y, beta),
                               rtol=1e-11, atol=1e-13)


def test_golden_scalar_values():
    with open(os.path.join(GOLDEN, "beta_divergence_values.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        got = float(beta_divergence(c["x"], c["y"], c["beta"]))
        assert math.isclose(got, c["value"], rel_tol=1e-13, abs_tol=1e-15), c


def test_gamma_values():
    assert gamma(0.0) == 0.5
    assert gamma(0.5) == pytest.approx(1.0 / 1.5)
    assert gamma(1.0) == 1.0 and gamma(1.5) == 1.0
    with pytest.raises(ValueError):
        gamma(2.0)


@pytest.mark.parametrize("beta", BETAS)
def test_chi_transforms_are_identity_at_reference(beta):
    rng = np.random.default_rng(3)
    Z = rng.uniform(0.1, 2.0, size=(5, 4))
    np.testing.assert_allclose(chi1(Z, Z, beta), Z, rtol=1e-14)
    np.testing.assert_allclose(chi2(Z, Z, beta), Z, rtol=1e-14)


def test_chi_transforms_ratio_forms():
    # chi_1 = Z~ (Z/Z~)^(beta-1); chi_2 = Z~ (Z/Z~)^beta for beta >= 1 (App. B.5)
    rng = np.random.default_rng(4)
    Z, Zt = rng.uniform(0.1, 2.0, size=(2, 6, 3))
    for beta in BETAS:
        np.testing.assert_allclose(chi1(Z, Zt, beta), Zt * (Z / Zt) ** (beta - 1.0), rtol=1e-13)
        want = Z if beta < 1.0 else Zt * (Z / Zt) ** beta
        np.testing.assert_allclose(chi2(Z, Zt, beta), want, rtol=1e-13)


def test_objective_conventions():
    X = np.array([0.0, 1.0, 2.0, 0.0])
    Xh = np.array([0.5, 1.0, 1.5, 2.0])
    # beta = 1: zero entries contribute y (0 log 0 = 0)
    want = 0.5 + 0.0 + (2 * math.log(2 / 1.5) - 2 + 1.5) + 2.0
    assert objective(X, Xh, 1.0) == pytest.approx(want, rel=1e-15)
    # beta = 0: data floored at eps_x
    eps_x = 1e-3
    Xf = np.maximum(X, eps_x)
    want0 = sum(a / b - math.log(a / b) - 1 for a, b in zip(Xf, Xh))
    assert objective(X, Xh, 0.0, eps_x=eps_x) == pytest.approx(want0, rel=1e-14)
    # model clipped at eps where it enters
    assert objective(np.array([1.0]), np.array([0.0]), 1.0, eps=1e-3) == pytest.approx(
        math.log(1 / 1e-3) - 1 + 1e-3, rel=1e-14)


def test_objective_sum_matches_pairwise_sum():
    rng = np.random.default_rng(5)
    X = rng.poisson(3.0, size=(20, 30, 40)).astype(float)
    Xh = rng.uniform(0.5, 6.0, size=X.shape)
    for beta in BETAS:
        ref = np.sum(beta_divergence(oracle.divergence.data_floor(X, beta, 1e-12), Xh, beta))
        assert objective(X, Xh, beta) == pytest.approx(ref, rel=1e-12)


def test_powers_definition_points():
    X = np.array([2.0, 0.0, 3.0])
    Xh = np.array([4.0, 1.0, 1e-20])
    P, Q = powers(X, Xh, 0.5, eps=1e-12)
    np.testing.assert_allclose(P, [2.0 * 4.0 ** -1.5, 0.0, 3.0 * (1e-12) ** -1.5], rtol=1e-14)
    np.testing.assert_allclose(Q, [4.0 ** -0.5, 1.0, (1e-12) ** -0.5], rtol=1e-14)
    P1, Q1 = powers(X, Xh[:2].tolist() + [2.0], 1.0)
    np.testing.assert_allclose(P1, [0.5, 0.0, 1.5])
    np.testing.assert_allclose(Q1, [1.0, 1.0, 1.0])
