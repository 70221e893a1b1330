"""Shared seeded test matrices and comparison helpers (no method arithmetic)."""
import numpy as np

import workloads as wl

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(n, u):
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1 - n * u)


def stencil_kappa(n):
    """Condition number of the 27-point operator (26 / -1) on an n^3 grid
    from its closed-form spectrum: A = 27 I - T (x) T (x) T with T the n x n
    tridiagonal (1, 1, 1), whose eigenvalues are 1 + 2 cos(k pi / (n + 1))."""
    t = 1.0 + 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    lam = 27.0 - (t[None, None, :] * t[None, :, None] * t[:, None, None]).ravel()
    return float(lam.max() / lam.min())


def rel_maxnorm(y, ref):
    y = np.asarray(y, np.float64)
    ref = np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(y - ref)) / (den if den > 0 else 1.0))


def row_bound(a: wl.Coo, x, u):
    """Per-row rounding bound gamma_L * sum |a_ik x_k| for any summation order,
    doubled for the reference's own rounding."""
    mag = np.zeros(a.nrows)
    np.add.at(mag, a.ai, np.abs(a.av.astype(np.float64)) * np.abs(x.astype(np.float64)[a.aj]))
    L = np.bincount(a.ai, minlength=a.nrows) if a.nnz else np.zeros(a.nrows)
    return 2 * gamma(np.maximum(L, 1), u) * mag


def many_empty_rows(nrows=10000, live=100, seed=5):
    g = wl.rng(seed)
    rows = np.sort(g.choice(nrows, live, replace=False))
    ai, aj = [], []
    for r in rows:
        k = int(g.integers(1, 40))
        cols = np.sort(g.choice(nrows, k, replace=False))
        ai += [r] * k
        aj += list(cols)
    ai = np.array(ai, np.int32)
    aj = np.array(aj, np.int32)
    return wl.Coo(nrows, nrows, ai, aj, g.standard_normal(ai.shape[0]))


def sparse_rows(nrows=200000, live=3000, seed=7):
    """Rows of 1-3 entries about 66 rows apart: a COO tile of 1,024 entries
    meets hundreds of runs of empty rows (more than its queue of long runs
    holds), and the last live row leaves a long run to the end."""
    g = wl.rng(seed)
    rows = np.sort(g.choice(nrows - 5000, live, replace=False))
    lens = g.integers(1, 4, live)
    ai = np.repeat(rows, lens).astype(np.int32)
    aj = np.concatenate([np.sort(g.choice(nrows, k, replace=False)) for k in lens]).astype(np.int32)
    return wl.Coo(nrows, nrows, ai, aj, g.standard_normal(ai.shape[0]))


def dense_row(ncols=10000, seed=6):
    g = wl.rng(seed)
    return wl.Coo(3, ncols, np.repeat(np.array([0, 1, 2], np.int32), [ncols, 5, ncols]),
                  np.concatenate([np.arange(ncols), np.arange(5) * 7, np.arange(ncols)]).astype(np.int32),
                  g.standard_normal(2 * ncols + 5))


def single_column(nrows=10000):
    return wl.Coo(nrows, 1, np.arange(nrows, dtype=np.int32), np.zeros(nrows, np.int32),
                  np.linspace(-1, 1, nrows))


def small_cases():
    """(name, Coo) pairs that span several tiles, ragged tails and the
    degenerate shapes."""
    cases = [("stencil16", wl.stencil(16))]
    for n in (1, 2, 3, 7):
        cases.append((f"stencil{n}", wl.stencil(n)))
    cases.append(("stencil7pt_9", wl.stencil(9, points=7)))
    for (m, n, d) in [(0, 0, 0.5), (1, 1, 1.0), (5, 1, 0.6), (1, 5, 0.6), (37, 53, 0.3),
                      (300, 200, 0.05), (64, 64, 0.0)]:
        cases.append((f"random{m}x{n}", wl.random_coo(m, n, d, seed=m * 7 + n)))
    cases.append(("zipf20k", wl.zipf_rows(20000, seed=11)))
    cases.append(("banded50k", wl.banded(50000, ndiag=11, max_offset=2000, seed=12)))
    cases.append(("block3000", wl.block_random(3000, seed=13)))
    cases.append(("empty_rows", many_empty_rows()))
    cases.append(("sparse_rows", sparse_rows()))
    cases.append(("dense_rows", dense_row()))
    cases.append(("one_column", single_column()))
    return cases
