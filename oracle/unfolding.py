"""Classical unfolding / Khatri-Rao / Kronecker form of the same MU numerators
and denominators (Sec. 7, "unfolding-based MU" baseline).

Test infrastructure only (see the package docstring).  This route forms the
mode-n unfolding X_(n) (Kolda-Bader ordering: the remaining indices vary with
the lowest mode fastest) and the Khatri-Rao product of the other factors, so it
shares no contraction code with :mod:`oracle.cp` / :mod:`oracle.tucker`.  The
paper states the contraction-only updates are algebraically identical to these
classical rules; the tests hold the two routes to each other on tiny tensors."""
from __future__ import annotations

from typing import Sequence

import numpy as np


def unfold(T: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding X_(n) of shape I_n x prod_{m != n} I_m, column index
    sum_{m != n} i_m prod_{k < m, k != n} I_k."""
    return np.reshape(np.moveaxis(T, n, 0), (T.shape[n], -1), order="F")


def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Column-wise Kronecker product mats[0] (.) mats[1] (.) ...; the row index of
    the last matrix varies fastest."""
    out = mats[0]
    for M in mats[1:]:
        R = out.shape[1]
        out = (out[:, None, :] * M[None, :, :]).reshape(-1, R)
    return out


def kron_all(mats: Sequence[np.ndarray]) -> np.ndarray:
    out = mats[0]
    for M in mats[1:]:
        out = np.kron(out, M)
    return out


def mttkrp(T: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """X_(n) (A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1)): MTTKRP."""
    N = T.ndim
    order = [m for m in reversed(range(N)) if m != n]
    return unfold(T, n) @ khatri_rao([factors[m] for m in order])


def tucker_factor(T: np.ndarray, core: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """T_(n) (A^(N) kron ... kron A^(n+1) kron A^(n-1) kron ... kron A^(1)) G_(n)^T."""
    N = T.ndim
    order = [m for m in reversed(range(N)) if m != n]
    return unfold(T, n) @ kron_all([factors[m] for m in order]) @ unfold(core, n).T


def tucker_core(T: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """vec(T x_1 A^(1)T ... x_N A^(N)T) = (A^(N) kron ... kron A^(1))^T vec(T),
    with the column-major vec of the Kolda-Bader convention."""
    N = T.ndim
    K = kron_all([factors[m] for m in reversed(range(N))])
    vec = K.T @ np.reshape(T, -1, order="F")
    return np.reshape(vec, tuple(A.shape[1] for A in factors), order="F")


def cp_rebuild(factors: Sequence[np.ndarray]) -> np.ndarray:
    """X = A^(1) (A^(N) (.) ... (.) A^(2))^T folded back (mode-1 unfolding identity)."""
    N = len(factors)
    X1 = factors[0] @ khatri_rao([factors[m] for m in reversed(range(1, N))]).T
    return np.reshape(X1, tuple(A.shape[0] for A in factors), order="F")


def tucker_rebuild(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """X_(1) = A^(1) G_(1) (A^(N) kron ... kron A^(2))^T folded back."""
    N = len(factors)
    X1 = factors[0] @ unfold(core, 0) @ kron_all([factors[m] for m in reversed(range(1, N))]).T
    shape = tuple(A.shape[0] for A in factors)
    return np.reshape(X1, shape, order="F")
