"""J-CoMM for CP at beta = 1 on sparse COO count data (FP64).

Test infrastructure only (see the package docstring).

Sec. 6.4 (paragraph on sparse tensors): numerators built from P = X * Xhat^(beta-2)
are accumulated over the nonzeros only; the denominators use Q = Xhat^(beta-1),
which is identically one at beta = 1, so Den_J^(n)(i_n, r) = sum_{i_-n}
prod_{m != n} chi_2(A^(m), A~^(m))_{i_m r} = prod_{m != n} sum_i A^(m)_{i r}
(chi_2(Z, Z~) = Z at beta = 1) and does not depend on i_n.  At beta = 1,
chi_1(Z, Z~) = Z~, so Num_J^(n) only involves the reference factors.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from .divergence import EPS_DEFAULT


def reference_values(idx: np.ndarray, ref: Sequence[np.ndarray], eps: float = EPS_DEFAULT,
                     chunk: int = 1 << 18) -> np.ndarray:
    """X~ at the nonzero coordinates, clipped at eps: sum_r prod_n A~^(n)_{i_n r}."""
    nnz = idx.shape[0]
    out = np.empty(nnz, dtype=np.float64)
    for s in range(0, nnz, chunk):
        e = min(nnz, s + chunk)
        z = np.ones((e - s, ref[0].shape[1]), dtype=np.float64)
        for m, A in enumerate(ref):
            z *= A[idx[s:e, m]]
        out[s:e] = z.sum(axis=1)
    return np.maximum(out, eps)


def numerators(idx: np.ndarray, val: np.ndarray, ref: Sequence[np.ndarray], xt: np.ndarray,
               chunk: int = 1 << 18) -> List[np.ndarray]:
    """Num_J^(n)(i_n, r) = sum over nonzeros of P~_i prod_{m != n} A~^(m)_{i_m r},
    with P~_i = X_i / X~_i, for every mode n."""
    N = len(ref)
    R = ref[0].shape[1]
    nums = [np.zeros_like(A) for A in ref]
    pt = val / xt
    for s in range(0, idx.shape[0], chunk):
        e = min(idx.shape[0], s + chunk)
        rows = [A[idx[s:e, m]] for m, A in enumerate(ref)]
        for n in range(N):
            w = np.repeat(pt[s:e, None], R, axis=1)
            for m in range(N):
                if m != n:
                    w = w * rows[m]
            np.add.at(nums[n], idx[s:e, n], w)
    return nums


def objective_kl(idx, val, ref, eps: float = EPS_DEFAULT) -> float:
    """D_1(X, X~) for sparse X: nonzeros give x log(x/X~) - x + X~, zeros give X~.

    Summing X~ over all cells in closed form, sum_i X~_i = sum_r prod_n
    colsum(A~^(n))_r, the objective is sum_nnz (x log(x/X~) - x) + that sum.
    (Reading: the zero cells use the unclipped model value.)"""
    xt = reference_values(idx, ref, eps)
    terms = val * np.log(val / xt) - val
    total_model = np.prod(np.stack([A.sum(axis=0) for A in ref]), axis=0).sum()
    return math.fsum(np.concatenate([terms, [total_model]]))


def jcomm_outer_kl(idx: np.ndarray, val: np.ndarray, factors: Sequence[np.ndarray], L: int = 1,
                   eps: float = EPS_DEFAULT, return_ref_obj: bool = False):
    """One J-CoMM outer iteration at beta = 1 from COO data (Algorithm J-CoMM,
    with the sparse accumulation of Sec. 6.4)."""
    ref = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    xt = reference_values(idx, ref, eps)
    nums = numerators(idx, val, ref, xt)
    cur = [a.copy() for a in ref]
    N = len(cur)
    for _ in range(L):
        for n in range(N):
            den = np.ones(ref[0].shape[1])
            for m in range(N):
                if m != n:
                    den = den * cur[m].sum(axis=0)
            cur[n] = np.maximum(ref[n] * nums[n] / den[None, :], eps)
    if return_ref_obj:
        return cur, objective_kl(idx, val, ref, eps)
    return cur
