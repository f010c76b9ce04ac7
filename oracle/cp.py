"""Nonnegative CP: reconstruction, CPContr, block update, B-CoMM and J-CoMM (FP64).

Test infrastructure only (see the package docstring).  Factors are float64
arrays A^(n) of shape I_n x R; every function works for any order N >= 2."""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .divergence import EPS_DEFAULT, chi1, chi2, gamma, objective, powers

_IDX = "abcdefgh"


def rebuild(factors: Sequence[np.ndarray]) -> np.ndarray:
    """Xhat_i = sum_r prod_n A^(n)_{i_n r} (Sec. 3.3, nonnegative CP)."""
    n = len(factors)
    spec = ",".join(f"{_IDX[m]}z" for m in range(n)) + "->" + _IDX[:n]
    return np.einsum(spec, *factors, optimize=True)


def cp_contr(T: np.ndarray, others: Sequence[np.ndarray], n: int) -> np.ndarray:
    """CPContr^(n)(T; {B^(m)}_{m != n}) (Sec. 6.1): the I_n x R matrix
    sum_{i_-n} T_i prod_{m != n} B^(m)_{i_m r}.

    ``others`` lists the N-1 matrices B^(m) in increasing m, skipping n.  For
    N = 3 this is the App. E recipe 'ijk,jr,kr->ir' and its permutations."""
    N = T.ndim
    modes = [m for m in range(N) if m != n]
    assert len(others) == len(modes)
    spec = _IDX[:N] + "," + ",".join(f"{_IDX[m]}z" for m in modes) + "->" + _IDX[n] + "z"
    return np.einsum(spec, T, *others, optimize=True)


def block_update(X: np.ndarray, factors: List[np.ndarray], n: int, beta: float,
                 eps: float = EPS_DEFAULT, eps_x: float | None = None) -> np.ndarray:
    """One CP block update of mode n (Theorem "CP block multiplicative update").

    Rebuilds Xhat from the current factors, forms P and Q (Sec. 4.1), contracts
    both against the other factors, and returns
    max(A^(n) * (Num/Den)^gamma, eps).  ``factors`` is not modified."""
    Xhat = rebuild(factors)
    P, Q = powers(X, Xhat, beta, eps, eps_x)
    others = [factors[m] for m in range(len(factors)) if m != n]
    num = cp_contr(P, others, n)
    den = cp_contr(Q, others, n)
    return np.maximum(factors[n] * np.power(num / den, gamma(beta)), eps)


def bcomm_sweep(X: np.ndarray, factors: Sequence[np.ndarray], beta: float,
                eps: float = EPS_DEFAULT, eps_x: float | None = None) -> List[np.ndarray]:
    """One outer iteration of B-CoMM (Algorithm B-CoMM): modes 1..N in order, each
    block update seeing the blocks already updated in this sweep."""
    cur = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    for n in range(len(cur)):
        cur[n] = block_update(X, cur, n, beta, eps, eps_x)
    return cur


def jcomm_inner_update(Pt: np.ndarray, Qt: np.ndarray, cur: Sequence[np.ndarray],
                       ref: Sequence[np.ndarray], n: int, beta: float,
                       eps: float = EPS_DEFAULT) -> np.ndarray:
    """CP inner update of J-CoMM for mode n (Sec. 5.3, "CP inner update").

    Num_J = CPContr^(n)(P~; chi_1(A^(m), A~^(m))), Den_J = CPContr^(n)(Q~;
    chi_2(A^(m), A~^(m))) over m != n, with the current inner iterate A^(m);
    the update is anchored at the reference block: max(A~^(n) (Num_J/Den_J)^gamma, eps)."""
    N = len(cur)
    b1 = [chi1(cur[m], ref[m], beta) for m in range(N) if m != n]
    b2 = [chi2(cur[m], ref[m], beta) for m in range(N) if m != n]
    num = cp_contr(Pt, b1, n)
    den = cp_contr(Qt, b2, n)
    return np.maximum(ref[n] * np.power(num / den, gamma(beta)), eps)


def jcomm_outer(X: np.ndarray, factors: Sequence[np.ndarray], beta: float, L: int = 1,
                eps: float = EPS_DEFAULT, eps_x: float | None = None, return_ref_obj: bool = False):
    """One outer iteration of J-CoMM for CP (Algorithm J-CoMM).

    Reference Theta~ = current factors; X~ = rebuild(Theta~); P~, Q~ formed once
    and kept for the whole inner loop; L inner sweeps over modes 1..N, eps
    enforced after every block.  With ``return_ref_obj`` also returns
    F(Theta~) = D_beta(X, X~), the objective at the reference."""
    if L < 1:
        raise ValueError("L must be >= 1")
    ref = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    Xt = rebuild(ref)
    Pt, Qt = powers(X, Xt, beta, eps, eps_x)
    cur = [a.copy() for a in ref]
    for _ in range(L):
        for n in range(len(cur)):
            cur[n] = jcomm_inner_update(Pt, Qt, cur, ref, n, beta, eps)
    if return_ref_obj:
        return cur, objective(X, Xt, beta, eps, eps_x)
    return cur


def run(X: np.ndarray, factors: Sequence[np.ndarray], beta: float, iters: int,
        method: str = "jcomm", L: int = 1, eps: float = EPS_DEFAULT,
        eps_x: float | None = None):
    """Run ``iters`` outer iterations; returns (factors, trace) with
    trace[t] = F(Theta^(t)) for t = 0..iters (iters + 1 values)."""
    cur = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    trace = [objective(X, rebuild(cur), beta, eps, eps_x)]
    for _ in range(iters):
        if method == "jcomm":
            cur = jcomm_outer(X, cur, beta, L, eps, eps_x)
        elif method == "bcomm":
            cur = bcomm_sweep(X, cur, beta, eps, eps_x)
        else:
            raise ValueError(method)
        trace.append(objective(X, rebuild(cur), beta, eps, eps_x))
    return cur, trace
