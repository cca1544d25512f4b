"""Seeded synthetic instance generators for the DOCH hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It only
draws random instances and lays them out (CSR / dense / start vectors); it
contains none of the method's arithmetic (no matvec, no update, no energy).

All randomness comes from numpy's PCG64 generator (``numpy.random.default_rng``)
keyed by an integer seed list, so every instance is reproducible bit for bit.

Workloads (the paper's benchmark families, Results "Benchmarking"; Supp. Note 9):
  * ``sk_dense``      Sherrington-Kirkpatrick: J_ij ~ N(0,1) for i<j, mirrored,
                      zero diagonal.
  * ``er_csr``        Erdos-Renyi G(n, p=d/(n-1)) with J_ij in {-1,+1}, drawn
                      over the strict lower triangle in row-major pair order
                      (the pair order of Supp. Alg. S5) by geometric skipping,
                      then mirrored.
  * ``torus_csr``     L x L periodic square lattice, 4 neighbours per site,
                      bonds in {-1,+1}, optional Gaussian field h.
  * ``uneven_batch``  a list of ER instances with n ~ U{800..20000} and mean
                      degree ~ U[3,20].
  * ``s5_csr``        sparse 9-bit integer couplings of Supp. Alg. S5.
  * ``uniform_x0``    start vectors x0 ~ U(-1,1).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

__all__ = [
    "CSR", "sk_dense", "er_csr", "torus_csr", "uniform_x0", "uneven_batch",
    "csr_from_dense", "dense_from_csr", "random_dense_int", "pm1_complete", "s5_csr",
    "circulant_csr",
    "SEEDS",
]

# Seed table of the named workloads (instance seed, start-vector seed).
SEEDS = {
    "sk1024": (1001, 2001),
    "er20000": (1002, 2002),
    "torus1e4": (1003, 2003),
    "sk4096": (1004, 2004),
    "batch512": (1005, 2005),
}


@dataclass
class CSR:
    """Symmetric coupling matrix in CSR form (both triangles stored).

    row_ptr: int32[n+1], col: int32[nnz] (ascending within a row),
    val: float32[nnz].  ``h`` is an optional float32[n] external field.
    """
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    h: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng([int(k) for k in key])


def sk_dense(n: int, seed: int) -> np.ndarray:
    """Dense SK couplings, float64 [n, n]: upper triangle drawn row-major."""
    g = _rng(seed)
    J = np.zeros((n, n), dtype=np.float64)
    iu, ju = np.triu_indices(n, 1)
    vals = g.standard_normal(iu.shape[0])
    J[iu, ju] = vals
    J[ju, iu] = vals
    return J


def pm1_complete(n: int, seed: int) -> np.ndarray:
    """Complete graph with +-1 couplings (the K_n family), float64 [n, n]."""
    g = _rng(seed)
    J = np.zeros((n, n), dtype=np.float64)
    iu, ju = np.triu_indices(n, 1)
    vals = np.where(g.integers(0, 2, iu.shape[0]) == 1, 1.0, -1.0)
    J[iu, ju] = vals
    J[ju, iu] = vals
    return J


def random_dense_int(n: int, seed: int, lo: int = -3, hi: int = 3,
                     density: float = 1.0) -> np.ndarray:
    """Small symmetric integer coupling matrix (float64 storage), zero diagonal."""
    g = _rng(seed)
    J = np.zeros((n, n), dtype=np.float64)
    iu, ju = np.triu_indices(n, 1)
    vals = g.integers(lo, hi + 1, iu.shape[0]).astype(np.float64)
    keep = g.random(iu.shape[0]) < density
    vals = vals * keep
    J[iu, ju] = vals
    J[ju, iu] = vals
    return J


def _lower_pairs_geometric(n: int, p: float, g: np.random.Generator):
    """Linear indices of kept pairs among the n(n-1)/2 strict-lower pairs.

    Pair k (0-based, row-major over i=1..n-1, j=0..i-1) is kept independently
    with probability p; the gaps between kept pairs are Geometric(p).
    """
    M = n * (n - 1) // 2
    if p <= 0.0 or M == 0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(M, dtype=np.int64)
    chunks = []
    pos = -1
    expect = int(M * p + 6.0 * np.sqrt(M * p) + 16)
    while True:
        gaps = g.geometric(p, size=max(expect, 1024)).astype(np.int64)
        idx = pos + np.cumsum(gaps)
        inside = idx[idx < M]
        chunks.append(inside)
        if inside.shape[0] < idx.shape[0]:
            break
        pos = int(idx[-1])
        expect = max(1024, expect // 4)
    return np.concatenate(chunks)


def _tri_row_col(k: np.ndarray):
    """Invert k = i(i-1)/2 + j (0 <= j < i) for int64 arrays."""
    i = np.floor((1.0 + np.sqrt(1.0 + 8.0 * k.astype(np.float64))) / 2.0).astype(np.int64)
    # fix possible off-by-one from floating sqrt
    base = i * (i - 1) // 2
    too_big = base > k
    i[too_big] -= 1
    base = i * (i - 1) // 2
    too_small = (k - base) >= i
    i[too_small] += 1
    base = i * (i - 1) // 2
    j = k - base
    return i, j


def _csr_from_lower_edges(n: int, ei: np.ndarray, ej: np.ndarray,
                          ev: np.ndarray, h: Optional[np.ndarray] = None) -> CSR:
    rows = np.concatenate([ei, ej]).astype(np.int64)
    cols = np.concatenate([ej, ei]).astype(np.int64)
    vals = np.concatenate([ev, ev]).astype(np.float32)
    order = np.argsort(rows * n + cols, kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n=n, row_ptr=row_ptr.astype(np.int32), col=cols.astype(np.int32),
               val=vals, h=h)


def er_csr(n: int, mean_degree: float, seed: int) -> CSR:
    """Erdos-Renyi G(n, d/(n-1)) with +-1 couplings (p = 1/2 each), h = 0."""
    p = float(mean_degree) / float(n - 1) if n > 1 else 0.0
    k = _lower_pairs_geometric(n, p, _rng(seed, 0))
    ei, ej = _tri_row_col(k)
    ev = np.where(_rng(seed, 1).integers(0, 2, k.shape[0]) == 1, 1.0, -1.0)
    return _csr_from_lower_edges(n, ei, ej, ev)


def s5_csr(n: int, p_percent: float, seed: int) -> CSR:
    """Sparse 9-bit integer couplings of Supp. Alg. S5.

    Every strict-lower pair (row-major order) draws z ~ U{1..N_p},
    N_p = floor(102300 / p); the pair is coupled when z < 1023, with
    J_ij = J_ji = z - 511.  The pairs are visited by geometric skipping with
    the same per-pair probability 1022 / N_p, and the value is drawn from
    U{1..1022} - 511 (the law of z given z < 1023).  A draw of z = 511 gives
    J_ij = 0 and is not stored.
    """
    Np = int(np.floor(102300.0 / float(p_percent)))
    q = min(1.0, 1022.0 / Np)
    k = _lower_pairs_geometric(n, q, _rng(seed, 0))
    z = _rng(seed, 1).integers(1, 1023, k.shape[0])
    v = (z - 511).astype(np.float64)
    keep = v != 0.0
    ei, ej = _tri_row_col(k[keep])
    return _csr_from_lower_edges(n, ei, ej, v[keep])


def torus_csr(L: int, seed: int, h_std: float = 0.0) -> CSR:
    """L x L periodic lattice, site i = r*L + c, 4 neighbours, +-1 bonds.

    Bonds are drawn site-major: for each site its "right" then its "down"
    bond.  Row i holds its up, left, right and down neighbours with columns
    sorted ascending.  With h_std > 0 the field h_i ~ N(0, h_std^2) is drawn
    (and rounded to float32, the stored precision).
    """
    if L < 3:
        raise ValueError("torus needs L >= 3 (4 distinct neighbours)")
    n = L * L
    bits = _rng(seed, 0).integers(0, 2, size=(n, 2), dtype=np.int8)
    right_bit = np.ascontiguousarray(bits[:, 0]).astype(np.int64)
    down_bit = np.ascontiguousarray(bits[:, 1]).astype(np.int64)
    del bits
    i = np.arange(n, dtype=np.int64)
    r, c = i // L, i % L
    # each entry packed as (column << 1) | (bond == +1): sorting the packed
    # keys sorts by column and carries the bond along
    up = ((r - 1) % L) * L + c
    k0 = (up << 1) | down_bit[up]
    del up
    left = r * L + (c - 1) % L
    k1 = (left << 1) | right_bit[left]
    del left
    k2 = ((r * L + (c + 1) % L) << 1) | right_bit
    k3 = ((((r + 1) % L) * L + c) << 1) | down_bit
    del r, c, i, right_bit, down_bit
    keys = [k0, k1, k2, k3]
    # 5-comparator sorting network on the 4 keys of every row
    for a, b in ((0, 1), (2, 3), (0, 2), (1, 3), (1, 2)):
        lo = np.minimum(keys[a], keys[b])
        np.maximum(keys[a], keys[b], out=keys[b])
        keys[a] = lo
    col = np.empty((n, 4), dtype=np.int32)
    val = np.empty((n, 4), dtype=np.float32)
    for q in range(4):
        col[:, q] = keys[q] >> 1
        val[:, q] = (keys[q] & 1).astype(np.float32) * 2.0 - 1.0
        keys[q] = None
    del keys
    row_ptr = (np.arange(n + 1, dtype=np.int64) * 4).astype(np.int32)
    h = None
    if h_std > 0.0:
        h = (_rng(seed, 2).standard_normal(n) * h_std).astype(np.float32)
    return CSR(n=n, row_ptr=row_ptr, col=col.reshape(-1), val=val.reshape(-1), h=h)


def uniform_x0(n: int, restarts: int, seed: int) -> np.ndarray:
    """x0 ~ U(-1,1), float64 [n, restarts] (row-major: restarts interleaved)."""
    g = _rng(seed)
    return 2.0 * g.random((n, restarts)) - 1.0


def uneven_batch(count: int = 512, seed: int = 1005, n_lo: int = 800,
                 n_hi: int = 20000, d_lo: float = 3.0, d_hi: float = 20.0) -> List[CSR]:
    """Uneven batch of ER instances: n_k ~ U{n_lo..n_hi}, d_k ~ U[d_lo, d_hi]."""
    out = []
    for k in range(count):
        g = _rng(seed, k)
        n_k = n_lo + int(np.floor((n_hi - n_lo + 1) * g.random()))
        d_k = d_lo + (d_hi - d_lo) * g.random()
        out.append(er_csr(n_k, d_k, seed * (1 << 20) + k))
    return out


def csr_from_dense(J: np.ndarray, h: Optional[np.ndarray] = None) -> CSR:
    """CSR (float32 values) of the nonzeros of a dense matrix."""
    n = J.shape[0]
    rows, cols = np.nonzero(J)
    vals = J[rows, cols].astype(np.float32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    hh = None if h is None else np.asarray(h, dtype=np.float32)
    return CSR(n=n, row_ptr=row_ptr.astype(np.int32), col=cols.astype(np.int32),
               val=vals, h=hh)


def dense_from_csr(A: CSR) -> np.ndarray:
    """Dense float64 matrix of a CSR instance (small n only)."""
    J = np.zeros((A.n, A.n), dtype=np.float64)
    rp = A.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    J[rows, A.col.astype(np.int64)] = A.val.astype(np.float64)
    return J


def circulant_csr(n: int, offsets, seed: int, h_std: float = 0.0) -> CSR:
    """Circulant graph: spin i coupled to i +- o (mod n) for every o in
    ``offsets`` (distinct, 0 < o < n/2), so every row holds exactly
    2 len(offsets) entries.  Bonds are +-1 (p = 1/2), drawn per (i, o) in
    site-major order; h ~ N(0, h_std^2) rounded to FP32 when h_std > 0."""
    offs = np.asarray(sorted(int(o) for o in offsets), dtype=np.int64)
    if offs.size == 0 or offs[0] <= 0 or 2 * offs[-1] >= n or np.unique(offs).size != offs.size:
        raise ValueError("offsets must be distinct and in (0, n/2)")
    g = _rng(seed)
    bonds = np.where(g.random((n, offs.size)) < 0.5, -1.0, 1.0)
    i = np.repeat(np.arange(n, dtype=np.int64), offs.size)
    j = (i + np.tile(offs, n)) % n
    ei, ej = np.maximum(i, j), np.minimum(i, j)
    h = None
    if h_std > 0:
        h = (_rng(seed, 2).standard_normal(n) * h_std).astype(np.float32)
    return _csr_from_lower_edges(n, ei, ej, bonds.reshape(-1), h)
