"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module builds matrix *structures and values* and seeded dense vectors.  It
holds none of the SpMV or CG arithmetic: every generator returns the stored
entries of a matrix as canonical COO triples -- rows ascending, columns
ascending within a row, no duplicates (the COO container of Section III-B,
in the sorted order that the SVE COO kernel of Section IV relies on).

Families (the paper's workloads are SuiteSparse matrices and the HPCG problem;
these synthetic families stand in for them):

* ``stencil``      -- HPCG's 27-point (or 7-point) stencil on an n^3 grid
                      (Section VII-D: Poisson on a regular 3-D grid).  Row of
                      grid point (x, y, z) is x + n*y + n*n*z.
* ``banded``       -- a few random diagonals with N(0,1) values.
* ``zipf_rows``    -- power-law row lengths, uniform random columns.
* ``block_random`` -- dense 8x8 blocks at random block columns.
* ``random_coo``   -- tiny unstructured matrices for brute-force checks.

Every random draw goes through ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Coo", "rng", "stencil", "stencil_nnz", "banded", "zipf_rows", "zipf_scale",
    "block_random", "random_coo", "shuffled", "uniform_vector", "integer_vector",
]


@dataclass
class Coo:
    """Stored entries (ai[k], aj[k], av[k]) of an nrows x ncols matrix."""

    nrows: int
    ncols: int
    ai: np.ndarray  # int32 [nnz]
    aj: np.ndarray  # int32 [nnz]
    av: np.ndarray  # float64 or float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.ai.shape[0])

    def astype(self, dtype) -> "Coo":
        return Coo(self.nrows, self.ncols, self.ai, self.aj, self.av.astype(dtype))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _from_row_major(nrows, ncols, cols2d, valid2d, values2d=None):
    """Flatten per-row candidate columns (already ascending within a row)."""
    cols = cols2d[valid2d].astype(np.int32, copy=False)
    counts = valid2d.sum(axis=1)
    ai = np.repeat(np.arange(nrows, dtype=np.int32), counts)
    av = None if values2d is None else values2d[valid2d]
    return ai, cols, av


# ---------------------------------------------------------------------------
# HPCG stencil
# ---------------------------------------------------------------------------
def stencil_nnz(n: int, points: int = 27) -> int:
    """Closed-form count of stored entries of the n^3 stencil."""
    if points == 27:
        return (3 * n - 2) ** 3
    if points == 7:
        return n ** 3 + 6 * (n - 1) * n * n
    raise ValueError("points must be 7 or 27")


def _stencil_offsets(points):
    offs = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if points == 7 and abs(dx) + abs(dy) + abs(dz) > 1:
                    continue
                offs.append((dx, dy, dz))
    return offs


def stencil(n: int, points: int = 27, diag: float | None = None, offdiag: float = -1.0,
            dtype=np.float64) -> Coo:
    """HPCG-style stencil matrix on an n x n x n grid.

    27-point: an entry for every neighbour (dx, dy, dz) in {-1,0,1}^3 inside the
    grid, ``diag`` (default 26.0) on the diagonal and ``offdiag`` elsewhere.
    7-point: the centre and its 6 face neighbours, ``diag`` default 6.0.
    """
    if points not in (7, 27):
        raise ValueError("points must be 7 or 27")
    if diag is None:
        diag = 26.0 if points == 27 else 6.0
    N = n * n * n
    if N == 0:
        z = np.zeros(0, np.int32)
        return Coo(0, 0, z, z.copy(), np.zeros(0, dtype))
    idx = np.arange(N, dtype=np.int64)
    gx = idx % n
    gy = (idx // n) % n
    gz = idx // (n * n)
    offs = _stencil_offsets(points)
    P = len(offs)
    cols = np.empty((N, P), dtype=np.int64)
    valid = np.empty((N, P), dtype=bool)
    vals = np.empty((N, P), dtype=dtype)
    for p, (dx, dy, dz) in enumerate(offs):
        ok = np.ones(N, dtype=bool)
        for g, d in ((gx, dx), (gy, dy), (gz, dz)):
            if d < 0:
                ok &= g >= 1
            elif d > 0:
                ok &= g <= n - 2
        valid[:, p] = ok
        cols[:, p] = idx + dx + n * dy + n * n * dz
        vals[:, p] = diag if (dx, dy, dz) == (0, 0, 0) else offdiag
    if n < 3:
        # Lexicographic (dz, dy, dx) order equals column order only for n >= 3;
        # re-sort the few tiny cases explicitly.
        key = np.where(valid, cols, np.iinfo(np.int64).max)
        order = np.argsort(key, axis=1, kind="stable")
        cols = np.take_along_axis(cols, order, axis=1)
        valid = np.take_along_axis(valid, order, axis=1)
        vals = np.take_along_axis(vals, order, axis=1)
    ai, aj, av = _from_row_major(N, N, cols, valid, vals)
    return Coo(N, N, ai, aj, np.ascontiguousarray(av, dtype=dtype))


# ---------------------------------------------------------------------------
# Banded: a few random diagonals
# ---------------------------------------------------------------------------
def banded(N: int, ndiag: int = 11, max_offset: int = 2000, seed: int = 3,
           dtype=np.float64) -> Coo:
    """``ndiag`` distinct offsets drawn uniformly without replacement from
    [-m, m], m = min(max_offset, N-1); every in-range slot on them is stored
    with an N(0,1) value (drawn in canonical order after the structure)."""
    g = rng(seed)
    m = min(max_offset, N - 1)
    ndiag = min(ndiag, 2 * m + 1)
    offs = np.sort(g.choice(np.arange(-m, m + 1), size=ndiag, replace=False)).astype(np.int64)
    rows = np.arange(N, dtype=np.int64)[:, None]
    cols = rows + offs[None, :]
    valid = (cols >= 0) & (cols < N)
    ai, aj, _ = _from_row_major(N, N, cols, valid)
    av = g.standard_normal(ai.shape[0]).astype(dtype)
    return Coo(N, N, ai, aj, av)


# ---------------------------------------------------------------------------
# Power-law rows
# ---------------------------------------------------------------------------
def _zipf_pmf(s, cap):
    k = np.arange(1, cap + 1, dtype=np.float64)
    w = k ** (-float(s))
    return k, w / w.sum()


def zipf_scale(s: float = 2.0, mean: float = 16.0, cap: int = 5000) -> float:
    """Scale c with E[min(cap, floor(c*k + u))] = mean for k ~ Zipf(s) on
    [1, cap] and u ~ U[0,1).  That expectation equals sum_k p_k min(c k, cap),
    which is increasing in c, so bisection finds c."""
    k, p = _zipf_pmf(s, cap)
    lo, hi = 0.0, float(cap)
    for _ in range(200):
        c = 0.5 * (lo + hi)
        if float(np.sum(p * np.minimum(c * k, cap))) < mean:
            lo = c
        else:
            hi = c
    return 0.5 * (lo + hi)


def _distinct_sorted_columns(g, ai, counts, ncols):
    """Uniform columns, distinct within a row, ascending within a row."""
    nnz = ai.shape[0]
    aj = g.integers(0, ncols, size=nnz, dtype=np.int64)
    while True:
        key = ai.astype(np.int64) * ncols + aj
        order = np.argsort(key, kind="stable")
        key = key[order]
        aj = aj[order]
        dup = np.zeros(nnz, dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            return aj.astype(np.int32)
        aj[dup] = g.integers(0, ncols, size=nd, dtype=np.int64)


def zipf_rows(N: int, s: float = 2.0, mean: float = 16.0, cap: int = 5000,
              ncols: int | None = None, seed: int = 2, dtype=np.float64) -> Coo:
    """Row lengths L = min(cap, floor(c*k + u)) with k ~ Zipf(s) truncated to
    [1, cap] (inverse CDF on the exact pmf) and c = ``zipf_scale`` so that
    E[L] = mean; columns uniform and distinct within a row; values N(0,1)."""
    ncols = N if ncols is None else ncols
    cap = min(cap, ncols)
    g = rng(seed)
    k, p = _zipf_pmf(s, cap)
    c = zipf_scale(s, mean, cap)
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    kk = k[np.searchsorted(cdf, g.random(N), side="right").clip(0, cap - 1)]
    L = np.minimum(cap, np.floor(c * kk + g.random(N))).astype(np.int64)
    L = np.maximum(L, 0)
    ai = np.repeat(np.arange(N, dtype=np.int32), L)
    aj = _distinct_sorted_columns(g, ai, L, ncols)
    av = g.standard_normal(ai.shape[0]).astype(dtype)
    return Coo(N, ncols, ai, aj, av)


# ---------------------------------------------------------------------------
# Block-random: dense 8x8 blocks
# ---------------------------------------------------------------------------
def block_random(nblockrows: int, max_blocks: int = 8, bs: int = 8, seed: int = 5,
                 dtype=np.float64) -> Coo:
    """Each block row holds U{1..max_blocks} dense bs x bs blocks at distinct
    uniformly drawn block columns; values N(0,1) in canonical order."""
    g = rng(seed)
    nbc = nblockrows
    nb = np.minimum(g.integers(1, max_blocks + 1, size=nblockrows), nbc).astype(np.int64)
    br = np.repeat(np.arange(nblockrows, dtype=np.int32), nb)
    bc = _distinct_sorted_columns(g, br, nb, nbc).astype(np.int64)
    # expand blocks: entries (br*bs + ii, bc*bs + jj)
    ii = np.arange(bs, dtype=np.int64)
    rows = (br.astype(np.int64)[:, None, None] * bs + ii[None, :, None]) + 0 * ii[None, None, :]
    cols = (bc[:, None, None] * bs + ii[None, None, :]) + 0 * ii[None, :, None]
    key = (rows * (nbc * bs) + cols).ravel()
    key.sort(kind="stable")
    ai = (key // (nbc * bs)).astype(np.int32)
    aj = (key % (nbc * bs)).astype(np.int32)
    av = g.standard_normal(ai.shape[0]).astype(dtype)
    return Coo(nblockrows * bs, nbc * bs, ai, aj, av)


# ---------------------------------------------------------------------------
# Tiny unstructured matrices and helpers
# ---------------------------------------------------------------------------
def random_coo(nrows: int, ncols: int, density: float, seed: int, integer: bool = False,
               dtype=np.float64) -> Coo:
    """Each of the nrows*ncols positions is stored with probability
    ``density``; values N(0,1) or integers in [-8, 8] without 0."""
    g = rng(seed)
    mask = g.random((nrows, ncols)) < density
    ai, aj = np.nonzero(mask)
    if integer:
        v = g.integers(1, 9, size=ai.shape[0]) * g.choice([-1, 1], size=ai.shape[0])
        av = v.astype(dtype)
    else:
        av = g.standard_normal(ai.shape[0]).astype(dtype)
    return Coo(nrows, ncols, ai.astype(np.int32), aj.astype(np.int32), av)


def shuffled(a: Coo, seed: int) -> Coo:
    """Same entries in a random order (COO carries no ordering guarantee)."""
    perm = rng(seed).permutation(a.nnz)
    return Coo(a.nrows, a.ncols, a.ai[perm].copy(), a.aj[perm].copy(), a.av[perm].copy())


def uniform_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """x ~ U[-1, 1) from ``seed``."""
    return rng(seed).uniform(-1.0, 1.0, n).astype(dtype)


def integer_vector(n: int, seed: int, lo: int = -8, hi: int = 8, dtype=np.float64) -> np.ndarray:
    """Integer-valued x in [lo, hi]: with integer matrices every partial sum is
    an exactly representable integer, so any summation order is exact."""
    return rng(seed).integers(lo, hi + 1, n).astype(dtype)


# ---------------------------------------------------------------------------
# Device-side generators (torch on the GPU) for the selector's large
# synthetic dataset.  Same families and canonical order as above; values are
# N(0,1) except the stencils.  Reproducible for a given seed and device.
# ---------------------------------------------------------------------------
def _tgen(seed, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _sorted_unique_cols(torch, g, rows, ncols, device):
    """Uniform columns, distinct within a row (duplicates redrawn), sorted by
    (row, col).  rows: int64 row id per entry (non-decreasing)."""
    n = rows.numel()
    cols = torch.randint(0, ncols, (n,), generator=g, device=device, dtype=torch.int64)
    while True:
        key = rows * ncols + cols
        key, order = torch.sort(key)
        rows = key // ncols
        cols = key % ncols
        dup = torch.zeros(n, dtype=torch.bool, device=device)
        if n > 1:
            dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            return rows, cols
        cols[dup] = torch.randint(0, ncols, (nd,), generator=g, device=device, dtype=torch.int64)


def device_stencil(n: int, points: int = 27, device="cuda", dtype=None):
    """(nrows, ncols, ai, aj, av) of the n^3 stencil as device tensors."""
    import torch
    dtype = dtype or torch.float64
    N = n ** 3
    idx = torch.arange(N, device=device, dtype=torch.int64)
    gx, gy, gz = idx % n, (idx // n) % n, idx // (n * n)
    cols, valid, vals = [], [], []
    diag = 26.0 if points == 27 else 6.0
    for (dx, dy, dz) in _stencil_offsets(points):
        ok = torch.ones(N, dtype=torch.bool, device=device)
        for gcoord, d in ((gx, dx), (gy, dy), (gz, dz)):
            if d < 0:
                ok &= gcoord >= 1
            elif d > 0:
                ok &= gcoord <= n - 2
        valid.append(ok)
        cols.append(idx + dx + n * dy + n * n * dz)
        vals.append(diag if (dx, dy, dz) == (0, 0, 0) else -1.0)
    valid = torch.stack(valid, 1)
    cols = torch.stack(cols, 1)
    vals = torch.tensor(vals, dtype=dtype, device=device).expand(N, -1)
    ai = idx[:, None].expand(-1, len(_stencil_offsets(points)))[valid]
    return N, N, ai.to(torch.int32), cols[valid].to(torch.int32), vals[valid].contiguous()


def device_banded(N: int, ndiag: int, max_offset: int, seed: int, device="cuda", dtype=None):
    import torch
    dtype = dtype or torch.float64
    g0 = rng(seed)
    m = min(max_offset, N - 1)
    ndiag = min(ndiag, 2 * m + 1)
    offs = np.sort(g0.choice(np.arange(-m, m + 1), size=ndiag, replace=False))
    o = torch.from_numpy(offs.astype(np.int64)).to(device)
    rows = torch.arange(N, device=device, dtype=torch.int64)[:, None]
    cols = rows + o[None, :]
    valid = (cols >= 0) & (cols < N)
    ai = rows.expand(-1, ndiag)[valid]
    aj = cols[valid]
    g = _tgen(seed, device)
    av = torch.randn(ai.numel(), generator=g, device=device, dtype=dtype)
    return N, N, ai.to(torch.int32), aj.to(torch.int32), av


def device_zipf_rows(N: int, seed: int, s: float = 2.0, mean: float = 16.0, cap: int = 5000,
                     device="cuda", dtype=None):
    import torch
    dtype = dtype or torch.float64
    cap = min(cap, N)
    k, p = _zipf_pmf(s, cap)
    c = zipf_scale(s, mean, cap)
    cdf = torch.from_numpy(np.cumsum(p)).to(device)
    cdf[-1] = 1.0
    g = _tgen(seed, device)
    u = torch.rand(N, generator=g, device=device, dtype=torch.float64)
    kk = torch.searchsorted(cdf, u, right=True).clamp(0, cap - 1).to(torch.float64) + 1.0
    L = torch.clamp(torch.floor(c * kk + torch.rand(N, generator=g, device=device,
                                                      dtype=torch.float64)), max=cap)
    L = L.to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(N, device=device, dtype=torch.int64), L)
    rows, cols = _sorted_unique_cols(torch, g, rows, N, device)
    av = torch.randn(rows.numel(), generator=g, device=device, dtype=dtype)
    return N, N, rows.to(torch.int32), cols.to(torch.int32), av


def device_block_random(nblockrows: int, seed: int, max_blocks: int = 8, bs: int = 8,
                        device="cuda", dtype=None):
    import torch
    dtype = dtype or torch.float64
    g = _tgen(seed, device)
    nb = torch.randint(1, max_blocks + 1, (nblockrows,), generator=g, device=device)
    nb = torch.clamp(nb, max=nblockrows)
    br = torch.repeat_interleave(torch.arange(nblockrows, device=device, dtype=torch.int64), nb)
    br, bc = _sorted_unique_cols(torch, g, br, nblockrows, device)
    ii = torch.arange(bs, device=device, dtype=torch.int64)
    rows = (br[:, None, None] * bs + ii[None, :, None]).expand(-1, bs, bs)
    cols = (bc[:, None, None] * bs + ii[None, None, :]).expand(-1, bs, bs)
    ncols = nblockrows * bs
    key, _ = torch.sort((rows * ncols + cols).reshape(-1))
    ai = (key // ncols).to(torch.int32)
    aj = (key % ncols).to(torch.int32)
    av = torch.randn(ai.numel(), generator=g, device=device, dtype=dtype)
    return nblockrows * bs, ncols, ai, aj, av


def device_banded_noise(N: int, ndiag: int, max_offset: int, noise: int, seed: int, device="cuda",
                        dtype=None):
    """The banded matrix of device_banded plus `noise` entries at uniform
    random positions (N(0,1) values; a position already on the band keeps the
    band's value), sorted by (row, column)."""
    import torch
    dtype = dtype or torch.float64
    nr, nc, ai, aj, av = device_banded(N, ndiag, max_offset, seed, device=device, dtype=dtype)
    g = _tgen(seed + 1, device)
    ni = torch.randint(0, N, (noise,), generator=g, device=device, dtype=torch.int64)
    nj = torch.randint(0, N, (noise,), generator=g, device=device, dtype=torch.int64)
    nv = torch.randn(noise, generator=g, device=device, dtype=dtype)
    key = torch.cat([ai.long() * N + aj.long(), ni * N + nj])
    val = torch.cat([av, nv])
    key, order = torch.sort(key, stable=True)
    val = val[order]
    first = torch.ones_like(key, dtype=torch.bool)
    first[1:] = key[1:] != key[:-1]
    key, val = key[first], val[first]
    return N, N, (key // N).to(torch.int32), (key % N).to(torch.int32), val.contiguous()


def device_banded_scatter(N: int, ndiag: int, max_offset: int, frac: float, concentrated: bool,
                          seed: int, device="cuda", dtype=None):
    """A banded matrix (device_banded) plus round(frac * band entries)
    entries at random positions, N(0,1) values, sorted by (row, column); a
    position already on the band keeps the band's value.  Uniform positions,
    or (concentrated) rows drawn from a random 1% of the rows: long rows over
    a short-row band."""
    import torch
    dtype = dtype or torch.float64
    nr, nc, ai, aj, av = device_banded(N, ndiag, max_offset, seed, device=device, dtype=dtype)
    noise = int(round(frac * ai.numel()))
    g = _tgen(seed + 7, device)
    if concentrated:
        pool = torch.randperm(N, generator=g, device=device)[:max(1, N // 100)]
        ni = pool[torch.randint(0, pool.numel(), (noise,), generator=g, device=device)]
    else:
        ni = torch.randint(0, N, (noise,), generator=g, device=device, dtype=torch.int64)
    nj = torch.randint(0, N, (noise,), generator=g, device=device, dtype=torch.int64)
    nv = torch.randn(noise, generator=g, device=device, dtype=dtype)
    key = torch.cat([ai.long() * N + aj.long(), ni.long() * N + nj])
    val = torch.cat([av, nv])
    key, order = torch.sort(key, stable=True)
    val = val[order]
    first = torch.ones_like(key, dtype=torch.bool)
    first[1:] = key[1:] != key[:-1]
    key, val = key[first], val[first]
    return N, N, (key // N).to(torch.int32), (key % N).to(torch.int32), val.contiguous()


def device_hypersparse(N: int, per_row: float, seed: int, device="cuda", dtype=None):
    """About per_row * N entries (fewer rows than entries' worth: most rows
    empty when per_row < 1) at distinct uniform random positions of an N x N
    matrix, N(0,1) values, sorted by (row, column)."""
    import torch
    dtype = dtype or torch.float64
    g = _tgen(seed, device)
    m = max(1, int(round(per_row * N)))
    key = torch.randint(0, N * N, (m,), generator=g, device=device, dtype=torch.int64)
    key = torch.unique(key)
    val = torch.randn(key.numel(), generator=g, device=device, dtype=dtype)
    return N, N, (key // N).to(torch.int32), (key % N).to(torch.int32), val.contiguous()


def device_windowed_rows(N: int, length: int, width: int, tail_frac: float, seed: int,
                         device="cuda", dtype=None):
    """Rows of near-equal length (length - 1 to length + 1 entries, fewer
    where columns collide) at uniform random columns within `width` of the
    diagonal, plus round(tail_frac * entries) entries at random columns in
    a random 1% of the rows (a few long rows over an ELL-friendly body);
    N(0,1) values, sorted by (row, column), distinct."""
    import torch
    dtype = dtype or torch.float64
    g = _tgen(seed, device)
    lens = length + torch.randint(-1, 2, (N,), generator=g, device=device)
    lens = lens.clamp(min=1)
    ai = torch.repeat_interleave(torch.arange(N, device=device, dtype=torch.int64), lens)
    aj = (ai + torch.randint(-width, width + 1, (ai.numel(),), generator=g, device=device)).clamp(0, N - 1)
    tail = int(round(tail_frac * ai.numel()))
    pool = torch.randperm(N, generator=g, device=device)[:max(1, N // 100)]
    ti = pool[torch.randint(0, pool.numel(), (tail,), generator=g, device=device)]
    tj = torch.randint(0, N, (tail,), generator=g, device=device, dtype=torch.int64)
    key = torch.unique(torch.cat([ai * N + aj, ti * N + tj]))
    val = torch.randn(key.numel(), generator=g, device=device, dtype=dtype)
    return N, N, (key // N).to(torch.int32), (key % N).to(torch.int32), val.contiguous()
