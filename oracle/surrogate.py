"""Explicit joint surrogate G(Theta | Theta~) with all constants, for tiny tensors.

Test infrastructure only (see the package docstring).

The model is written as a sum of nonnegative contributions z_{i,rho}(Theta)
(Sec. 5.2, step 1): CP uses rho = r with z = prod_n A^(n)_{i_n r}; Tucker uses
the multi-index rho = j with z = G_j prod_n A^(n)_{i_n j_n}.  Reference weights
lambda~_{i,rho} = z_{i,rho}(Theta~) / X~_i (step 2).

* 1 <= beta < 2: Jensen on the convex map y -> d_beta(x|y) (App. B.2,
  eq. app_jensen_beta_ge_1):
  G_i = sum_rho lambda~ d_beta(X_i | z_rho / lambda~).
* 0 < beta < 1: split d_beta(x|y) = y^beta/beta + x y^(beta-1)/(1-beta)
  + x^beta/(beta(beta-1)) (App. A.1, eq. dbeta_split); tangent bound on the
  concave first term at X~_i, Jensen on the convex second term (App. A.3-A.4,
  eq. surrogate_beta_lt_1).
* beta = 0: d_0(x|y) = x/y + log y - log x - 1; tangent bound on log y at X~_i,
  Jensen on x/y.
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence

import numpy as np

from .divergence import beta_divergence, data_floor


def contributions_cp(factors: Sequence[np.ndarray]) -> np.ndarray:
    """z[i..., r] = prod_n A^(n)_{i_n r}; shape I_1 x ... x I_N x R."""
    N = len(factors)
    z = np.ones(tuple(A.shape[0] for A in factors) + (factors[0].shape[1],))
    for n, A in enumerate(factors):
        shape = [1] * N + [A.shape[1]]
        shape[n] = A.shape[0]
        z = z * A.reshape(shape)
    return z


def contributions_tucker(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """z[i..., j...] = G_j prod_n A^(n)_{i_n j_n}, flattened over j; shape I... x prod(J)."""
    N = len(factors)
    I = tuple(A.shape[0] for A in factors)
    J = core.shape
    z = np.zeros(I + (int(np.prod(J)),))
    for flat, j in enumerate(itertools.product(*[range(x) for x in J])):
        t = np.full(I, core[j])
        for n, A in enumerate(factors):
            shape = [1] * N
            shape[n] = A.shape[0]
            t = t * A[:, j[n]].reshape(shape)
        z[..., flat] = t
    return z


def joint_surrogate(X: np.ndarray, z: np.ndarray, zref: np.ndarray, beta: float,
                    eps_x: float = 1e-12) -> float:
    """G(Theta | Theta~) summed over all entries, from contributions z (at Theta)
    and zref (at Theta~), both with the component axis last."""
    Xf = data_floor(np.asarray(X, dtype=np.float64), beta, eps_x)
    Xt = zref.sum(axis=-1)
    lam = zref / Xt[..., None]
    Xhat = z.sum(axis=-1)
    x = Xf[..., None]
    if beta >= 1.0:
        G = (lam * beta_divergence(np.broadcast_to(x, z.shape), z / lam, beta)).sum(axis=-1)
    elif beta > 0.0:
        const = np.power(Xf, beta) / (beta * (beta - 1.0))
        tangent = np.power(Xt, beta) / beta + np.power(Xt, beta - 1.0) * (Xhat - Xt)
        jensen = (lam * x / (1.0 - beta) * np.power(z / lam, beta - 1.0)).sum(axis=-1)
        G = const + tangent + jensen
    else:
        G = -np.log(Xf) - 1.0 + np.log(Xt) + (Xhat - Xt) / Xt + (x * lam * lam / z).sum(axis=-1)
    return math.fsum(G.ravel())


def surrogate_cp(X, factors, ref, beta, eps_x=1e-12) -> float:
    return joint_surrogate(X, contributions_cp(factors), contributions_cp(ref), beta, eps_x)


def surrogate_tucker(X, core, factors, core_ref, ref, beta, eps_x=1e-12) -> float:
    return joint_surrogate(X, contributions_tucker(core, factors),
                           contributions_tucker(core_ref, ref), beta, eps_x)


def scalar_surrogate(u, num: float, den: float, beta: float):
    """Scalar subproblem g(u) in the ratio variable u (Lemma on the CP scalar form,
    App. B.5), up to its additive constant:
    1 < beta < 2: den/beta u^beta - num/(beta-1) u^(beta-1);
    beta = 1:     den u - num log u;
    beta < 1:     den u + num/(1-beta) u^(beta-1)."""
    u = np.asarray(u, dtype=np.float64)
    if beta > 1.0:
        return den / beta * u ** beta - num / (beta - 1.0) * u ** (beta - 1.0)
    if beta == 1.0:
        return den * u - num * np.log(u)
    return den * u + num / (1.0 - beta) * u ** (beta - 1.0)


def scalar_minimiser(num: float, den: float, beta: float) -> float:
    """Closed-form minimiser u* = (num/den)^gamma(beta) of :func:`scalar_surrogate`."""
    g = 1.0 / (2.0 - beta) if beta < 1.0 else 1.0
    return (num / den) ** g
