"""Nonnegative Tucker: reconstruction, block and joint contractions, B-CoMM and
J-CoMM (FP64).  Test infrastructure only (see the package docstring).

The core G has shape J_1 x ... x J_N and the factors A^(n) are I_n x J_n.
Block order (the paper lists Theta = {G, A^(1), ..., A^(N)} and presents the
core first; it does not fix the order): the core, then modes 1..N."""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .divergence import EPS_DEFAULT, chi1, chi2, gamma, objective, powers

_DATA = "abcdefgh"
_CORE = "ABCDEFGH"


def rebuild(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """Xhat_i = sum_j G_j prod_n A^(n)_{i_n j_n} (App. C, eq. tucker_entry);
    the App. E recipe 'abc,ia,jb,kc->ijk' for N = 3."""
    N = len(factors)
    spec = (_CORE[:N] + "," + ",".join(f"{_DATA[m]}{_CORE[m]}" for m in range(N))
            + "->" + _DATA[:N])
    return np.einsum(spec, core, *factors, optimize=True)


def core_contr(T: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """T x_1 B^(1)T ... x_N B^(N)T, i.e. sum_i T_i prod_n B^(n)_{i_n j_n}
    (App. C, eqs. block_core_num_den / block_core_den and jmm_core_num / jmm_core_den)."""
    N = T.ndim
    spec = (_DATA[:N] + "," + ",".join(f"{_DATA[m]}{_CORE[m]}" for m in range(N))
            + "->" + _CORE[:N])
    return np.einsum(spec, T, *factors, optimize=True)


def factor_contr(T: np.ndarray, core: np.ndarray, others: Sequence[np.ndarray], n: int) -> np.ndarray:
    """Direct factor contraction without forming the partial tensor B^(n)
    (App. C, eqs. block_factor_num / block_factor_den, jmm_factor_num /
    jmm_factor_den; App. E 'ijk,abc,jb,kc->ia'):
    sum_{i_-n} sum_{j_-n} T_i G_{j} prod_{m != n} B^(m)_{i_m j_m}, shape I_n x J_n.

    ``others`` lists the N-1 matrices B^(m) in increasing m, skipping n."""
    N = T.ndim
    modes = [m for m in range(N) if m != n]
    assert len(others) == len(modes)
    spec = (_DATA[:N] + "," + _CORE[:N] + ","
            + ",".join(f"{_DATA[m]}{_CORE[m]}" for m in modes)
            + "->" + _DATA[n] + _CORE[n])
    return np.einsum(spec, T, core, *others, optimize=True)


def partial_tensor(core: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """B^(n) = G x_{m != n} A^(m) with j_n kept as the first index (App. C, eq. block_Bn).

    Only used to check the direct form against the two-step form."""
    N = core.ndim
    modes = [m for m in range(N) if m != n]
    spec = (_CORE[:N] + "," + ",".join(f"{_DATA[m]}{_CORE[m]}" for m in modes)
            + "->" + _CORE[n] + "".join(_DATA[m] for m in modes))
    return np.einsum(spec, core, *[factors[m] for m in modes], optimize=True)


def block_update_core(X, core, factors, beta, eps=EPS_DEFAULT, eps_x=None) -> np.ndarray:
    """Block-MM core update (Sec. 4.3 core update; Theorem "Tucker block
    multiplicative updates"): max(G * (P_core/Q_core)^gamma, eps)."""
    Xhat = rebuild(core, factors)
    P, Q = powers(X, Xhat, beta, eps, eps_x)
    num = core_contr(P, factors)
    den = core_contr(Q, factors)
    return np.maximum(core * np.power(num / den, gamma(beta)), eps)


def block_update_factor(X, core, factors, n, beta, eps=EPS_DEFAULT, eps_x=None) -> np.ndarray:
    """Block-MM factor update of mode n (Sec. 4.3 factor update):
    max(A^(n) * (Num^(n)/Den^(n))^gamma, eps)."""
    Xhat = rebuild(core, factors)
    P, Q = powers(X, Xhat, beta, eps, eps_x)
    others = [factors[m] for m in range(len(factors)) if m != n]
    num = factor_contr(P, core, others, n)
    den = factor_contr(Q, core, others, n)
    return np.maximum(factors[n] * np.power(num / den, gamma(beta)), eps)


def bcomm_sweep(X, core, factors, beta, eps=EPS_DEFAULT, eps_x=None) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Tucker B-CoMM sweep: Algorithm B-CoMM with blocks {G, A^(1), ..., A^(N)}
    (the paper says the Tucker variant is analogous), rebuilding Xhat before
    every block."""
    G = np.array(core, dtype=np.float64, copy=True)
    cur = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    G = block_update_core(X, G, cur, beta, eps, eps_x)
    for n in range(len(cur)):
        cur[n] = block_update_factor(X, G, cur, n, beta, eps, eps_x)
    return G, cur


def jcomm_inner_update_core(Pt, Qt, cur, ref, Gref, beta, eps=EPS_DEFAULT) -> np.ndarray:
    """Tucker core inner update of J-CoMM (Sec. 5.3; App. C.3, eqs. jmm_core_num,
    jmm_core_den): P~ contracted against chi_1(A^(n), A~^(n)) and Q~ against
    chi_2(A^(n), A~^(n)) for every n, with the current inner factors; anchored at
    the reference core: max(G~ (Num_J / Den_J)^gamma, eps)."""
    N = len(cur)
    a1 = [chi1(cur[m], ref[m], beta) for m in range(N)]
    a2 = [chi2(cur[m], ref[m], beta) for m in range(N)]
    num = core_contr(Pt, a1)
    den = core_contr(Qt, a2)
    return np.maximum(Gref * np.power(num / den, gamma(beta)), eps)


def jcomm_inner_update_factor(Pt, Qt, G, Gref, cur, ref, n, beta, eps=EPS_DEFAULT) -> np.ndarray:
    """Tucker factor inner update of J-CoMM for mode n (App. C.3, eqs.
    jmm_factor_num, jmm_factor_den): Num_J / Den_J contract P~ / Q~ with
    chi_1 / chi_2 of the current core against G~ and of the other current
    factors against their references; anchored at A~^(n)."""
    N = len(cur)
    g1 = chi1(G, Gref, beta)
    g2 = chi2(G, Gref, beta)
    o1 = [chi1(cur[m], ref[m], beta) for m in range(N) if m != n]
    o2 = [chi2(cur[m], ref[m], beta) for m in range(N) if m != n]
    num = factor_contr(Pt, g1, o1, n)
    den = factor_contr(Qt, g2, o2, n)
    return np.maximum(ref[n] * np.power(num / den, gamma(beta)), eps)


def jcomm_outer(X, core, factors, beta, L=1, eps=EPS_DEFAULT, eps_x=None, return_ref_obj=False):
    """One outer iteration of J-CoMM for Tucker (Algorithm J-CoMM with the Tucker
    inner updates of Sec. 5.3 and App. C.3): the reference Theta~ = (G~, A~),
    P~ and Q~ formed once from X~ = rebuild(Theta~), then L sweeps of the core
    update followed by the factor updates of modes 1..N.  The transforms always
    use the current inner values, so the factor updates see the new core."""
    if L < 1:
        raise ValueError("L must be >= 1")
    Gref = np.array(core, dtype=np.float64, copy=True)
    ref = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    Xt = rebuild(Gref, ref)
    Pt, Qt = powers(X, Xt, beta, eps, eps_x)
    G = Gref.copy()
    cur = [a.copy() for a in ref]
    for _ in range(L):
        G = jcomm_inner_update_core(Pt, Qt, cur, ref, Gref, beta, eps)
        for n in range(len(cur)):
            cur[n] = jcomm_inner_update_factor(Pt, Qt, G, Gref, cur, ref, n, beta, eps)
    if return_ref_obj:
        return G, cur, objective(X, Xt, beta, eps, eps_x)
    return G, cur


def run(X, core, factors, beta, iters, method="jcomm", L=1, eps=EPS_DEFAULT, eps_x=None):
    """``iters`` outer iterations; returns (core, factors, trace) with iters+1 objective values."""
    G = np.array(core, dtype=np.float64, copy=True)
    cur = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    trace = [objective(X, rebuild(G, cur), beta, eps, eps_x)]
    for _ in range(iters):
        if method == "jcomm":
            G, cur = jcomm_outer(X, G, cur, beta, L, eps, eps_x)
        elif method == "bcomm":
            G, cur = bcomm_sweep(X, G, cur, beta, eps, eps_x)
        else:
            raise ValueError(method)
        trace.append(objective(X, rebuild(G, cur), beta, eps, eps_x))
    return G, cur, trace
