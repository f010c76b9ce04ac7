"""Seeded synthetic workloads shared by the tests, the oracle checks and the benchmark.

This module only draws random numbers and assembles planted data sets.  It holds
none of the update arithmetic of the method: neither the oracle nor the HIP path
lives here, and both consume what it returns.

Every generator takes an integer ``seed`` and derives two independent streams
with ``numpy.random.SeedSequence(seed).spawn(2)``: stream 0 draws the data
(planted model and noise), stream 1 draws the initial parameters.  The same seed
therefore gives the same data whatever initialisation is asked for.

Shapes and distributions follow the five workloads the library is measured on:

* ``cp_small``   – 30x40x50 Poisson counts from a rank-5 CP model with U(0,1)
                   factors; rank-5 U(0.1,1) init (plain block-MM, beta=1).
* ``cp_dense``   – IxJxK (256^3 by default) Poisson counts from a rank-R CP model
                   with Gamma(1,1) factors; U(0.1,1) init.
* ``tucker_dense`` – 200^3 tensor, Gamma(shape 10, scale Xtrue/10) noise around
                   a Tucker model with a 16^3 U(0,1) core and U(0,1) factors.
* ``sparse_counts`` – 4-way 183x24x1140x1717 day x hour x lat x lon count tensor
                   with ~3.3M unique nonzeros: uniform day, diurnal hour profile,
                   Zipf(1.1) latitude / longitude over seeded permutations,
                   values Poisson(2)+1, COO sorted lexicographically.
* ``serving_specs`` – a stream of small CP / Tucker problems with ragged
                   dims, ranks and beta, arriving as a Poisson process.

The planted tensors are formed with a NumPy ``einsum`` of the planted
parameters; this is data synthesis only (the planted model is never an input
of either implementation).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np


def streams(seed: int) -> Tuple[np.random.Generator, np.random.Generator]:
    """(data_rng, init_rng) for ``seed``: two independent child streams."""
    data_ss, init_ss = np.random.SeedSequence(seed).spawn(2)
    return np.random.default_rng(data_ss), np.random.default_rng(init_ss)


def _planted_cp(factors: Sequence[np.ndarray]) -> np.ndarray:
    letters = "abcdefgh"[: len(factors)]
    spec = ",".join(f"{c}z" for c in letters) + "->" + letters
    return np.einsum(spec, *factors, optimize=True)


def _planted_tucker(core: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    n = len(factors)
    core_idx = "ABCDEFGH"[:n]
    data_idx = "abcdefgh"[:n]
    spec = core_idx + "," + ",".join(f"{data_idx[m]}{core_idx[m]}" for m in range(n)) + "->" + data_idx
    return np.einsum(spec, core, *factors, optimize=True)


def init_cp(rng: np.random.Generator, dims: Sequence[int], rank: int,
            low: float = 0.1, high: float = 1.0) -> List[np.ndarray]:
    """Random nonnegative CP initialisation, every entry iid U(low, high)."""
    return [rng.uniform(low, high, size=(int(d), rank)) for d in dims]


def init_tucker(rng: np.random.Generator, dims: Sequence[int], core_dims: Sequence[int],
                low: float = 0.1, high: float = 1.0) -> Tuple[np.ndarray, List[np.ndarray]]:
    """Random nonnegative Tucker initialisation (core first, then factors), iid U(low, high)."""
    core = rng.uniform(low, high, size=tuple(int(j) for j in core_dims))
    factors = [rng.uniform(low, high, size=(int(d), int(j))) for d, j in zip(dims, core_dims)]
    return core, factors


@dataclasses.dataclass
class DenseCP:
    X: np.ndarray                 # float64, row-major, last mode fastest
    init: List[np.ndarray]        # float64 factors I_n x R
    planted: List[np.ndarray]


@dataclasses.dataclass
class DenseTucker:
    X: np.ndarray
    init_core: np.ndarray
    init_factors: List[np.ndarray]
    planted_core: np.ndarray
    planted_factors: List[np.ndarray]


def cp_small(seed: int = 0, dims=(30, 40, 50), rank: int = 5) -> DenseCP:
    """30x40x50 Poisson tensor from a rank-5 U(0,1) CP model; U(0.1,1) rank-5 init."""
    drng, irng = streams(seed)
    planted = [drng.uniform(0.0, 1.0, size=(d, rank)) for d in dims]
    X = drng.poisson(_planted_cp(planted)).astype(np.float64)
    return DenseCP(X=X, init=init_cp(irng, dims, rank), planted=planted)


def cp_dense(seed: int = 0, dims=(256, 256, 256), rank: int = 32,
             init_rank: Optional[int] = None) -> DenseCP:
    """Poisson counts around a rank-R CP model with Gamma(1,1) factors (mean entry R)."""
    drng, irng = streams(seed)
    planted = [drng.gamma(1.0, 1.0, size=(d, rank)) for d in dims]
    X = drng.poisson(_planted_cp(planted)).astype(np.float64)
    return DenseCP(X=X, init=init_cp(irng, dims, init_rank or rank), planted=planted)


def tucker_dense(seed: int = 0, dims=(200, 200, 200), core_dims=(16, 16, 16),
                 shape: float = 10.0) -> DenseTucker:
    """X ~ Gamma(shape, Xtrue/shape) around a Tucker model with U(0,1) core and factors."""
    drng, irng = streams(seed)
    core = drng.uniform(0.0, 1.0, size=tuple(core_dims))
    factors = [drng.uniform(0.0, 1.0, size=(d, j)) for d, j in zip(dims, core_dims)]
    xtrue = _planted_tucker(core, factors)
    X = drng.gamma(shape, xtrue / shape)
    icore, ifac = init_tucker(irng, dims, core_dims)
    return DenseTucker(X=X, init_core=icore, init_factors=ifac,
                       planted_core=core, planted_factors=factors)


def planted_exact_cp(seed: int, dims: Sequence[int], rank: int,
                     low: float = 0.2, high: float = 1.0) -> DenseCP:
    """Noise-free X equal to a CP model whose factors are the returned ``init``.

    Used for fixed-point checks: the parameters that generated X are also the
    starting point."""
    drng, _ = streams(seed)
    planted = [drng.uniform(low, high, size=(int(d), rank)) for d in dims]
    return DenseCP(X=_planted_cp(planted), init=[p.copy() for p in planted], planted=planted)


def planted_exact_tucker(seed: int, dims: Sequence[int], core_dims: Sequence[int],
                         low: float = 0.2, high: float = 1.0) -> DenseTucker:
    drng, _ = streams(seed)
    core = drng.uniform(low, high, size=tuple(core_dims))
    factors = [drng.uniform(low, high, size=(int(d), int(j))) for d, j in zip(dims, core_dims)]
    return DenseTucker(X=_planted_tucker(core, factors), init_core=core.copy(),
                       init_factors=[f.copy() for f in factors],
                       planted_core=core, planted_factors=factors)


# ----------------------------------------------------------------------------------------
# Sparse 4-way counts (day x hour x lat x lon)
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class SparseCOO:
    dims: Tuple[int, ...]
    idx: np.ndarray      # (nnz, ndim) int64, rows sorted lexicographically
    val: np.ndarray      # (nnz,) float64 integer counts
    init: List[np.ndarray]


def _zipf_over_perm(rng: np.random.Generator, n: int, s: float, size: int,
                    perm: np.ndarray) -> np.ndarray:
    ranks = np.arange(1, n + 1, dtype=np.float64)
    p = ranks ** (-s)
    p /= p.sum()
    return perm[rng.choice(n, size=size, p=p)]


def hour_profile(hours: int = 24) -> np.ndarray:
    """Diurnal weight 1 + 0.8 sin(2 pi (h - 10) / 24), renormalised."""
    h = np.arange(hours, dtype=np.float64)
    w = 1.0 + 0.8 * np.sin(2.0 * np.pi * (h - 10.0) / 24.0)
    return w / w.sum()


def sparse_counts(seed: int = 0, dims=(183, 24, 1140, 1717), nnz: int = 3_300_000,
                  rank: int = 32, zipf_s: float = 1.1) -> SparseCOO:
    """Unique COO coordinates with the day/hour/lat/lon marginals described above.

    Duplicated coordinates are redrawn until ``nnz`` unique ones exist."""
    drng, irng = streams(seed)
    d0, d1, d2, d3 = (int(d) for d in dims)
    perm2 = drng.permutation(d2)
    perm3 = drng.permutation(d3)
    hp = hour_profile(d1)
    strides = np.array([d1 * d2 * d3, d2 * d3, d3, 1], dtype=np.int64)
    keys = np.empty(0, dtype=np.int64)
    need = nnz
    while need > 0:
        m = int(need * 1.15) + 1024
        c0 = drng.integers(0, d0, size=m)
        c1 = drng.choice(d1, size=m, p=hp)
        c2 = _zipf_over_perm(drng, d2, zipf_s, m, perm2)
        c3 = _zipf_over_perm(drng, d3, zipf_s, m, perm3)
        new = c0 * strides[0] + c1 * strides[1] + c2 * strides[2] + c3 * strides[3]
        keys = np.unique(np.concatenate([keys, new]))
        need = nnz - keys.size
    if keys.size > nnz:
        keys = np.sort(drng.choice(keys, size=nnz, replace=False))
    idx = np.empty((nnz, 4), dtype=np.int64)
    rem = keys.copy()
    for m in range(4):
        idx[:, m] = rem // strides[m]
        rem = rem % strides[m]
    val = (drng.poisson(2.0, size=nnz) + 1).astype(np.float64)
    return SparseCOO(dims=(d0, d1, d2, d3), idx=idx, val=val, init=init_cp(irng, dims, rank))


def sparse_small(seed: int = 0, dims=(6, 5, 7, 8), density: float = 0.05, rank: int = 3) -> SparseCOO:
    """Tiny sparse tensor (a few percent dense) for checks against the densified form."""
    drng, irng = streams(seed)
    total = int(np.prod(dims))
    nnz = max(1, int(round(density * total)))
    keys = np.sort(drng.choice(total, size=nnz, replace=False))
    idx = np.stack(np.unravel_index(keys, dims), axis=1).astype(np.int64)
    val = (drng.poisson(2.0, size=nnz) + 1).astype(np.float64)
    return SparseCOO(dims=tuple(int(d) for d in dims), idx=idx, val=val,
                     init=init_cp(irng, dims, rank))


def densify(coo: SparseCOO) -> np.ndarray:
    X = np.zeros(coo.dims, dtype=np.float64)
    X[tuple(coo.idx.T)] = coo.val
    return X


# ----------------------------------------------------------------------------------------
# Serving stream
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class RequestSpec:
    rid: int
    arrival: float            # seconds since the stream started
    model: str                # "cp" or "tucker"
    dims: Tuple[int, int, int]
    rank: int                 # CP rank, or Tucker core size per mode (clamped to the dim)
    beta: float
    seed: int                 # seed of this request's own data / init streams


@dataclasses.dataclass
class Request:
    spec: RequestSpec
    X: np.ndarray
    init: List[np.ndarray]    # CP: factors; Tucker: [core, A1, A2, A3]


def serving_specs(seed: int = 0, count: int = 2000, rate: float = 100.0,
                  dim_range=(16, 256), ranks=(4, 8, 16, 32),
                  betas=(0.0, 0.5, 1.0, 1.5)) -> List[RequestSpec]:
    """Poisson arrivals (rate per second) of CP/Tucker requests on dense 3-way tensors.

    model ~ {cp, tucker} with p = 1/2, dims iid U{dim_range}, rank ~ U(ranks),
    beta ~ U(betas).  The tensors themselves are drawn lazily by
    :func:`materialize` from the per-request seed, so a long stream costs no
    memory until a request is admitted."""
    drng, _ = streams(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += drng.exponential(1.0 / rate)
        model = "cp" if drng.random() < 0.5 else "tucker"
        dims = tuple(int(d) for d in drng.integers(dim_range[0], dim_range[1] + 1, size=3))
        rank = int(ranks[drng.integers(0, len(ranks))])
        beta = float(betas[drng.integers(0, len(betas))])
        out.append(RequestSpec(rid=rid, arrival=t, model=model, dims=dims, rank=rank,
                               beta=beta, seed=int(drng.integers(0, 2**62))))
    return out


def materialize(spec: RequestSpec, eps_x: float = 1e-12) -> Request:
    """Planted U(0,1) parameters; X = Poisson(planted model), floored at eps_x when
    beta = 0; init U(0.1, 1)."""
    drng, irng = streams(spec.seed)
    dims, rank = spec.dims, spec.rank
    if spec.model == "cp":
        planted = [drng.uniform(0.0, 1.0, size=(d, rank)) for d in dims]
        xtrue = _planted_cp(planted)
        init = init_cp(irng, dims, rank)
    else:
        cd = tuple(min(rank, d) for d in dims)
        core = drng.uniform(0.0, 1.0, size=cd)
        planted = [drng.uniform(0.0, 1.0, size=(d, j)) for d, j in zip(dims, cd)]
        xtrue = _planted_tucker(core, planted)
        c0, f0 = init_tucker(irng, dims, cd)
        init = [c0] + f0
    X = drng.poisson(xtrue).astype(np.float64)
    if spec.beta == 0.0:
        X = np.maximum(X, eps_x)
    return Request(spec=spec, X=X, init=init)
