"""Explicit-loop forms (pure Python) of the reconstructions and contractions, for
tensors with a few entries per mode.  Test infrastructure only.

They spell out the indexed sums of Sec. 3.3 (CP model), Sec. 6.1 (CPContr) and
App. C (eqs. tucker_entry, block_core_num_den, block_factor_num)."""
from __future__ import annotations

import itertools
from typing import Sequence

import numpy as np


def cp_rebuild(factors: Sequence[np.ndarray]) -> np.ndarray:
    dims = tuple(A.shape[0] for A in factors)
    R = factors[0].shape[1]
    out = np.zeros(dims)
    for i in itertools.product(*[range(d) for d in dims]):
        s = 0.0
        for r in range(R):
            p = 1.0
            for n, A in enumerate(factors):
                p *= A[i[n], r]
            s += p
        out[i] = s
    return out


def cp_contr(T: np.ndarray, others: Sequence[np.ndarray], n: int) -> np.ndarray:
    N = T.ndim
    modes = [m for m in range(N) if m != n]
    R = others[0].shape[1]
    out = np.zeros((T.shape[n], R))
    for i in itertools.product(*[range(d) for d in T.shape]):
        for r in range(R):
            p = T[i]
            for B, m in zip(others, modes):
                p *= B[i[m], r]
            out[i[n], r] += p
    return out


def tucker_rebuild(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    dims = tuple(A.shape[0] for A in factors)
    out = np.zeros(dims)
    for i in itertools.product(*[range(d) for d in dims]):
        s = 0.0
        for j in itertools.product(*[range(d) for d in core.shape]):
            p = core[j]
            for n, A in enumerate(factors):
                p *= A[i[n], j[n]]
            s += p
        out[i] = s
    return out


def tucker_core_contr(T: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    J = tuple(A.shape[1] for A in factors)
    out = np.zeros(J)
    for j in itertools.product(*[range(d) for d in J]):
        s = 0.0
        for i in itertools.product(*[range(d) for d in T.shape]):
            p = T[i]
            for n, A in enumerate(factors):
                p *= A[i[n], j[n]]
            s += p
        out[j] = s
    return out


def tucker_factor_contr(T: np.ndarray, core: np.ndarray, others: Sequence[np.ndarray], n: int) -> np.ndarray:
    N = T.ndim
    modes = [m for m in range(N) if m != n]
    out = np.zeros((T.shape[n], core.shape[n]))
    for i in itertools.product(*[range(d) for d in T.shape]):
        for j in itertools.product(*[range(d) for d in core.shape]):
            p = T[i] * core[j]
            for B, m in zip(others, modes):
                p *= B[i[m], j[m]]
            out[i[n], j[n]] += p
    return out
