"""beta-divergence, objective, weight tensors, gamma and the chi transforms (FP64).

Test infrastructure only (see the package docstring)."""
from __future__ import annotations

import math

import numpy as np

#: Lower bound on every model parameter (Assumption "positivity safeguard").  The
#: paper only asks for a small eps > 0; 1e-12 is the value this library uses.
EPS_DEFAULT = 1e-12


def _check_beta(beta: float) -> None:
    if not (0.0 <= beta < 2.0):
        raise ValueError("beta must lie in [0, 2)")


def beta_divergence(x, y, beta: float) -> np.ndarray:
    """Entrywise d_beta(x | y), Sec. 3.2 (Definition of the beta-divergence).

    beta not in {0, 1}: (x^b + (b-1) y^b - b x y^(b-1)) / (b (b-1));
    beta = 1: x log(x/y) - x + y, with 0 log 0 taken as 0 (its limit);
    beta = 0: x/y - log(x/y) - 1 (needs x > 0).
    For beta > 0, 0^beta is 0.  Requires y > 0.
    Any beta (also >= 2) is accepted here so that tests can probe the
    general branch."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if beta == 1.0:
        xlogx = np.where(x > 0, x * np.log(np.where(x > 0, x, 1.0) / y), 0.0)
        return xlogx - x + y
    if beta == 0.0:
        r = x / y
        return r - np.log(r) - 1.0
    return (np.power(x, beta) + (beta - 1.0) * np.power(y, beta)
            - beta * x * np.power(y, beta - 1.0)) / (beta * (beta - 1.0))


def data_floor(X: np.ndarray, beta: float, eps_x: float) -> np.ndarray:
    """X used by the objective and by P: max(X, eps_x) at beta = 0 (Remark on
    beta = 0, which allows evaluating on a floored copy of the data), X otherwise."""
    return np.maximum(X, eps_x) if beta == 0.0 else X


def objective(X: np.ndarray, Xhat: np.ndarray, beta: float, eps: float = EPS_DEFAULT,
              eps_x: float | None = None) -> float:
    """D_beta(X, Xhat) = sum_i d_beta(X_i | Xhat_i), summed exactly with math.fsum.

    The reconstruction enters through max(Xhat, eps) (the clip the positivity
    safeguard allows where powers, logs or divisions of Xhat are taken); at
    beta = 0 the data enter as max(X, eps_x) with eps_x = eps unless given."""
    _check_beta(beta)
    eps_x = eps if eps_x is None else eps_x
    Xf = data_floor(np.asarray(X, dtype=np.float64), beta, eps_x)
    Xc = np.maximum(np.asarray(Xhat, dtype=np.float64), eps)
    return math.fsum(beta_divergence(Xf, Xc, beta).ravel())


def gamma(beta: float) -> float:
    """Multiplicative exponent (Remark on gamma(beta)): 1/(2-beta) for beta < 1,
    1 for 1 <= beta < 2.  beta = 0 gives 1/2, beta = 1 gives 1."""
    _check_beta(beta)
    return 1.0 / (2.0 - beta) if beta < 1.0 else 1.0


def powers(X: np.ndarray, Xhat: np.ndarray, beta: float, eps: float = EPS_DEFAULT,
           eps_x: float | None = None):
    """Weight tensors of Sec. 4.1: P = X * Xhat^(beta-2), Q = Xhat^(beta-1).

    Same safeguards as :func:`objective`: Xhat enters as max(Xhat, eps) and, at
    beta = 0, X as max(X, eps_x).  Used both for the block weights P, Q and for
    the reference-powered tensors P~, Q~ of J-CoMM (Sec. 5.3)."""
    _check_beta(beta)
    eps_x = eps if eps_x is None else eps_x
    Xf = data_floor(np.asarray(X, dtype=np.float64), beta, eps_x)
    Xc = np.maximum(np.asarray(Xhat, dtype=np.float64), eps)
    P = Xf * np.power(Xc, beta - 2.0)
    Q = np.power(Xc, beta - 1.0)
    return P, Q


def chi1(Z: np.ndarray, Zref: np.ndarray, beta: float) -> np.ndarray:
    """chi_{1,beta}(Z, Z~) = Z~^(2-beta) * Z^(beta-1) (Sec. 5.3, "Two transforms")."""
    return np.power(Zref, 2.0 - beta) * np.power(Z, beta - 1.0)


def chi2(Z: np.ndarray, Zref: np.ndarray, beta: float) -> np.ndarray:
    """chi_{2,beta}(Z, Z~) = Z for beta < 1, Z^beta * Z~^(1-beta) for 1 <= beta < 2."""
    if beta < 1.0:
        return np.array(Z, dtype=np.float64, copy=True)
    return np.power(Z, beta) * np.power(Zref, 1.0 - beta)
