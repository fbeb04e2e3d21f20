"""Seeded synthetic inputs shaped like the msRep evaluation workloads.

This module only draws random structure and values; it holds none of the
method's arithmetic (no products, no partitioning, no conversion).  The same
arrays are handed, byte for byte, to the GPU library and to the CPU oracle.

Recipes (all generators use numpy's PCG64 and draw in the fixed order
structure -> values in canonical CSR order -> x):

* ``uniform_csr``  -- every row holds ``per_row`` distinct columns drawn
  uniformly (with duplicate columns re-drawn until none are left), columns
  sorted within the row; values and x ~ U(-1, 1).
* ``rmat_csr``     -- R-MAT (Chakrabarti et al. 2004) with quadrant
  probabilities a, b, c, d, ``edge_factor * 2**scale`` draws, ``scale`` levels,
  no noise and no vertex permutation; self loops kept, duplicates merged,
  directed.  Stands in for the paper's power-law SuiteSparse matrices (its
  Table of input matrices), which are not available here.
* ``stencil7_csr`` -- 3-D 7-point Laplacian on a g^3 grid in lexicographic
  order (x fastest), Dirichlet boundary (no wrap): diagonal 6, neighbours -1.
* ``batched_set``  -- many square matrices with log-uniform row counts, even
  ones uniform (4..64 distinct columns per row), odd ones R-MAT-like (scale
  ceil(log2 m), 16*m draws, out-of-range draws rejected, duplicates merged);
  matrix k is seeded by SeedSequence(seed).spawn(count)[k].
* ``serving_trace`` -- Poisson arrivals, each request a pool matrix and a
  count of SpMVs drawn uniformly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Csr:
    """A canonical CSR matrix (columns strictly increasing within a row)."""

    m: int
    n: int
    ptr: np.ndarray  # int32, m + 1
    col: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.ptr[-1])


def rng_for(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def _ptr_from_counts(counts: np.ndarray) -> np.ndarray:
    ptr = np.zeros(len(counts) + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    if ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return ptr.astype(np.int32)


def _distinct_sorted_cols(rng, n: int, deg: np.ndarray):
    """Row-sorted (row, col) pairs with deg[r] distinct uniform columns per row."""
    deg = np.asarray(deg, np.int64)
    if np.any(deg > n):
        raise ValueError("more distinct columns requested than the matrix has")
    rows = np.repeat(np.arange(len(deg), dtype=np.int64), deg)
    cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    while True:
        key = np.sort(rows * n + cols)
        rows, cols = key // n, key % n
        dup = np.zeros(key.size, bool)
        dup[1:] = key[1:] == key[:-1]
        k = int(dup.sum())
        if k == 0:
            return rows, cols
        cols[dup] = rng.integers(0, n, size=k, dtype=np.int64)


def uniform_csr(m: int, n: int, per_row, seed=0, rng=None):
    """Uniform-random matrix; ``per_row`` is an int or an array of row degrees.
    Returns (Csr, x)."""
    rng = rng if rng is not None else rng_for(seed)
    deg = np.full(m, per_row, np.int64) if np.isscalar(per_row) else np.asarray(per_row)
    rows, cols = _distinct_sorted_cols(rng, n, deg)
    ptr = _ptr_from_counts(np.bincount(rows, minlength=m))
    val = rng.uniform(-1.0, 1.0, size=cols.size)
    x = rng.uniform(-1.0, 1.0, size=n)
    return Csr(m, n, ptr, cols.astype(np.int32), val, name="uniform"), x


def rmat_pairs(rng, scale: int, ndraws: int, a=0.57, b=0.19, c=0.19, d=0.05):
    """Raw R-MAT (row, col) draws, ``scale`` recursion levels each."""
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("quadrant probabilities must sum to 1")
    rows = np.zeros(ndraws, np.int64)
    cols = np.zeros(ndraws, np.int64)
    for _ in range(scale):
        u = rng.random(ndraws)
        rbit = u >= a + b                             # quadrants c, d: lower half
        cbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)  # quadrants b, d: right half
        rows = 2 * rows + rbit
        cols = 2 * cols + cbit
    return rows, cols


def _csr_from_pairs(rng, m, n, rows, cols, name):
    key = np.unique(rows * n + cols)  # sorted row-major, duplicates merged
    rows, cols = key // n, key % n
    ptr = _ptr_from_counts(np.bincount(rows, minlength=m))
    val = rng.uniform(-1.0, 1.0, size=cols.size)
    x = rng.uniform(-1.0, 1.0, size=n)
    return Csr(m, n, ptr, cols.astype(np.int32), val, name=name), x


def rmat_csr(scale=20, edge_factor=16, a=0.57, b=0.19, c=0.19, d=0.05, seed=0, rng=None):
    """R-MAT power-law matrix of 2**scale rows.  Returns (Csr, x)."""
    rng = rng if rng is not None else rng_for(seed)
    m = 1 << scale
    rows, cols = rmat_pairs(rng, scale, edge_factor * m, a, b, c, d)
    A, x = _csr_from_pairs(rng, m, m, rows, cols, "rmat%d" % scale)
    A.meta.update(scale=scale, edge_factor=edge_factor, abcd=(a, b, c, d))
    return A, x


def stencil7_csr(g=256, seed=0, rng=None):
    """3-D 7-point Laplacian on a g^3 grid.  Returns (Csr, x); x ~ U(-1, 1)."""
    rng = rng if rng is not None else rng_for(seed)
    m = g ** 3
    r = np.arange(m, dtype=np.int64)
    i, j, k = r % g, (r // g) % g, r // (g * g)
    # candidate columns in increasing order: -g^2, -g, -1, 0, +1, +g, +g^2
    offs = (-g * g, -g, -1, 0, 1, g, g * g)
    ok = (k > 0, j > 0, i > 0, np.ones(m, bool), i < g - 1, j < g - 1, k < g - 1)
    vals = (-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0)
    counts = np.zeros(m, np.int64)
    for o in ok:
        counts += o
    ptr = _ptr_from_counts(counts)
    nnz = int(ptr[-1])
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    pos = ptr[:-1].astype(np.int64).copy()
    for off, o, v in zip(offs, ok, vals):
        rr = r[o]
        col[pos[o]] = (rr + off).astype(np.int32)
        val[pos[o]] = v
        pos[o] += 1
    del r, i, j, k, pos
    x = rng.uniform(-1.0, 1.0, size=m)
    A = Csr(m, m, ptr, col, val, name="stencil%d" % g)
    A.meta.update(grid=g)
    return A, x


def batched_matrix(k: int, count: int, seed=0, m_lo=1_000, m_hi=200_000):
    """Matrix k of a batched set (see the module docstring).  Returns (Csr, x)."""
    ss = np.random.SeedSequence(seed).spawn(count)[k]
    rng = rng_for(ss)
    m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
    if k % 2 == 0:
        deg = rng.integers(4, 65, size=m)
        A, x = uniform_csr(m, m, np.minimum(deg, m), rng=rng)
        A.name = "batch%d-uniform" % k
    else:
        scale = max(1, math.ceil(math.log2(m)))
        rows, cols = rmat_pairs(rng, scale, 16 * m)
        keep = (rows < m) & (cols < m)
        A, x = _csr_from_pairs(rng, m, m, rows[keep], cols[keep], "batch%d-rmat" % k)
    return A, x


def batched_set(count=512, seed=0, m_lo=1_000, m_hi=200_000, indices=None):
    """The first ``count`` (or the listed) matrices of a batched set."""
    idx = range(count) if indices is None else indices
    return [batched_matrix(k, count, seed, m_lo, m_hi) for k in idx]


def dyadic(rng, size, denom=256):
    """Values k/denom with |k| <= denom: products and sums of a few thousand of
    them are exact in FP64."""
    return rng.integers(-denom, denom + 1, size=size).astype(np.float64) / denom


@dataclass
class Request:
    rid: int
    t_arrive: float   # seconds from the start of the trace
    matrix: int       # index into the pool
    steps: int        # number of SpMVs against fresh x


def serving_trace(n_req: int, rate: float, pool: int, seed=0, k_lo=10, k_hi=100):
    """Poisson arrivals at ``rate`` requests/s; matrix ~ U{0..pool-1};
    steps ~ U{k_lo..k_hi}."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    mats = rng.integers(0, pool, size=n_req)
    steps = rng.integers(k_lo, k_hi + 1, size=n_req)
    return [Request(i, float(t[i]), int(mats[i]), int(steps[i])) for i in range(n_req)]


def request_x(n: int, rid: int, step: int, seed=0):
    """The fresh x of a request's step: seeded by (seed, request id, step)."""
    rng = rng_for(np.random.SeedSequence([int(seed), int(rid), int(step)]))
    return rng.uniform(-1.0, 1.0, size=n)


def bf16_bits(v32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns with round-to-nearest-even (NaN kept
    quiet).  The host rounds stored values once, before they reach either
    side."""
    u = np.ascontiguousarray(v32, np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_SM_M1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(key: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea, Flood 2014) of uint64 keys."""
    with np.errstate(over="ignore"):
        z = np.asarray(key, np.uint64) + _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _SM_M1
        z = (z ^ (z >> np.uint64(27))) * _SM_M2
        return z ^ (z >> np.uint64(31))


def serving_x(n: int, seed: int, rid: int, step: int) -> np.ndarray:
    """Fresh x of step `step` of request `rid` in the serving loop:
    x[c] = 2u - 1, u = top 53 bits of splitmix64(key) / 2^53,
    key = seed ^ (rid << 40) ^ (step << 24) ^ c."""
    c = np.arange(n, dtype=np.uint64)
    key = (np.uint64(seed) ^ (np.uint64(rid) << np.uint64(40)) ^
           (np.uint64(step) << np.uint64(24))) ^ c
    u = (splitmix64(key) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0
