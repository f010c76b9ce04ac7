"""Extrapolated variants of the contraction-only updates (Sec. "Going beyond:
Majorization-Minimization with Extrapolation"), FP64.  Test infrastructure
only (see the package docstring).

The section adapts BMMe: before a block is updated, it is moved to an inertial
point built from the two most recent iterates, using only the positive part of
the displacement, and the same MM step is then taken with the surrogate built
at, and the multiplicative update anchored at, that point.

Readings of the passage (the paper leaves these open):
* The weight: one scalar for all blocks,
  alpha_t = min(alpha_nes, c / (||[Theta^(t) - Theta^(t-1)]_+|| + delta)), with
  the norm taken over every block of the model (Frobenius over all entries);
  alpha_nes, c and delta are inputs (the paper fixes none of them).
  nesterov_weight gives the usual (t - 1) / (t + 2) sequence as a default.
* The previous iterate: the text sets A_prev <- A "at the end of the outer
  iteration", which taken literally would make the displacement zero at every
  later step.  Read here as: A_prev of a block holds the value the block had
  when the previous outer iteration reached it (before its update there), so
  the displacement is the change made by that update.
* Block-MM: a block is extrapolated just before its own update; blocks after it
  in the sweep keep their current values in its reconstruction.
* J-CoMM: the whole reference is extrapolated at the start of the outer
  iteration and the inner iterate starts at that reference."""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from . import cp, tucker
from .divergence import EPS_DEFAULT


def nesterov_weight(t: int) -> float:
    """(t - 1) / (t + 2) for outer iteration t >= 1 (0 at t = 1)."""
    return max(0.0, (t - 1.0) / (t + 2.0))


def positive_part_norm(blocks: Sequence[np.ndarray], prev: Sequence[np.ndarray]) -> float:
    """|| [Theta - Theta_prev]_+ || over all blocks."""
    return math.sqrt(math.fsum(float(np.sum(np.maximum(a - b, 0.0) ** 2)) for a, b in zip(blocks, prev)))


def weight(blocks, prev, alpha_nes: float, c: float, delta: float) -> float:
    """alpha_t = min(alpha_nes, c / (||P(Delta)|| + delta))."""
    return min(alpha_nes, c / (positive_part_norm(blocks, prev) + delta))


def extrapolate(a: np.ndarray, a_prev: np.ndarray, alpha: float, eps: float = EPS_DEFAULT) -> np.ndarray:
    """max(A + alpha [A - A_prev]_+, eps)."""
    return np.maximum(a + alpha * np.maximum(a - a_prev, 0.0), eps)


def cp_bcomm_sweep(X, factors, prev, beta, alpha, eps=EPS_DEFAULT, eps_x=None) -> Tuple[List, List]:
    """Extrapolated B-CoMM sweep for CP (item (i) of the section).  Returns the
    new factors and the new previous iterates (each block's value before its
    update in this sweep)."""
    cur = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    new_prev = []
    for n in range(len(cur)):
        new_prev.append(cur[n].copy())
        cur[n] = extrapolate(cur[n], prev[n], alpha, eps)
        cur[n] = cp.block_update(X, cur, n, beta, eps, eps_x)
    return cur, new_prev


def tucker_bcomm_sweep(X, core, factors, prev_core, prev, beta, alpha, eps=EPS_DEFAULT, eps_x=None):
    """Extrapolated B-CoMM sweep for Tucker (item (ii)): the core, then modes
    1..N, each extrapolated just before its update.  Returns
    (core, factors, previous core, previous factors)."""
    G = np.array(core, dtype=np.float64, copy=True)
    cur = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    new_prev_core = G.copy()
    G = extrapolate(G, prev_core, alpha, eps)
    G = tucker.block_update_core(X, G, cur, beta, eps, eps_x)
    new_prev = []
    for n in range(len(cur)):
        new_prev.append(cur[n].copy())
        cur[n] = extrapolate(cur[n], prev[n], alpha, eps)
        cur[n] = tucker.block_update_factor(X, G, cur, n, beta, eps, eps_x)
    return G, cur, new_prev_core, new_prev


def cp_jcomm_outer(X, factors, prev, beta, alpha, L=1, eps=EPS_DEFAULT, eps_x=None, return_ref_obj=False):
    """Outer-reference extrapolation for CP J-CoMM (item (iii)): the reference
    is max(Theta + alpha [Theta - Theta_prev]_+, eps), then one J-CoMM outer
    iteration from it.  Returns (factors, previous factors[, F(reference)])."""
    new_prev = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    ref = [extrapolate(a, b, alpha, eps) for a, b in zip(new_prev, prev)]
    out = cp.jcomm_outer(X, ref, beta, L, eps, eps_x, return_ref_obj=return_ref_obj)
    if return_ref_obj:
        return out[0], new_prev, out[1]
    return out, new_prev


def tucker_jcomm_outer(X, core, factors, prev_core, prev, beta, alpha, L=1, eps=EPS_DEFAULT, eps_x=None,
                       return_ref_obj=False):
    """Outer-reference extrapolation for Tucker J-CoMM (item (iii))."""
    new_prev_core = np.array(core, dtype=np.float64, copy=True)
    new_prev = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    G = extrapolate(new_prev_core, prev_core, alpha, eps)
    ref = [extrapolate(a, b, alpha, eps) for a, b in zip(new_prev, prev)]
    out = tucker.jcomm_outer(X, G, ref, beta, L, eps, eps_x, return_ref_obj=return_ref_obj)
    if return_ref_obj:
        return out[0], out[1], new_prev_core, new_prev, out[2]
    return out[0], out[1], new_prev_core, new_prev
