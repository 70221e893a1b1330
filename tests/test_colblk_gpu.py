"""Column blocks (COO implementation 2, CSR 4) against the CPU oracle,
through the C ABI: matrices whose x exceeds 8 MiB and whose entries mostly
lie far from the diagonal, where mxs_optimize splits the entries by column
range.

Bars as for SpMV: FP64 within 1e-12 relative max-norm of the oracle and
within the per-row rounding bound; FP32 within the FP32 bound; integer data
bit-exact; bitwise reproducible; CG with the fused p.Ap as the oracle's CG.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import U32, U64, rel_maxnorm, row_bound

pytestmark = pytest.mark.gpu
UNSUPPORTED = -10
COLBLK = {"csr": 4, "coo": 2}


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fixed_rows(nrows, ncols, k, seed, lo=0, hi=None, integer=False, dtype=np.float64):
    """k distinct uniform columns in [lo, hi) per row, values N(0,1) or
    integers in [-4, 4] without 0."""
    hi = ncols if hi is None else hi
    g = wl.rng(seed)
    L = np.full(nrows, k, np.int64)
    ai = np.repeat(np.arange(nrows, dtype=np.int32), L)
    aj = (wl._distinct_sorted_columns(g, ai, L, hi - lo) + lo).astype(np.int32)
    if integer:
        av = g.integers(1, 5, ai.size) * g.choice([-1, 1], ai.size)
    else:
        av = g.standard_normal(ai.size)
    return wl.Coo(nrows, ncols, ai, aj, av.astype(dtype))


def build(mxs, a, fmt):
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    return (A.convert("csr") if fmt == "csr" else A).optimize()


CASES = {
    # x 8.8 MB: 2 blocks; rows of 3 to 5,000 entries spread over both blocks
    "zipf_1.1M": lambda: wl.zipf_rows(1_100_000, seed=21),
    # x 12 MB: 2 blocks, 6 uniform columns per row
    "uniform_1.5M": lambda: fixed_rows(1_500_000, 1_500_000, 6, seed=22),
    # wide: 300,000 rows, x 24 MB (4 blocks)
    "wide_300k_x_3M": lambda: fixed_rows(300_000, 3_000_000, 12, seed=23),
    # x 208 MB: the block count is capped at 32 (6.5 MB of x per block)
    "very_wide_100k_x_26M": lambda: fixed_rows(100_000, 26_000_000, 8, seed=30),
    # columns only in the first half: the last of three blocks is empty
    "left_half_2M": lambda: fixed_rows(2_000_000, 2_000_000, 4, seed=24, hi=1_000_000),
    # columns only in the second half: the first block (which writes y) is empty
    "right_half_2M": lambda: fixed_rows(2_000_000, 2_000_000, 4, seed=25, lo=1_000_000),
}


@pytest.mark.parametrize("fmt", ["csr", "coo"])
@pytest.mark.parametrize("name", list(CASES))
def test_column_blocks_match_oracle(gpu, name, fmt):
    mxs = gpu
    a = CASES[name]()
    print(f"[colblk] {name} {fmt} {a.nrows}x{a.ncols} nnz={a.nnz}", flush=True)
    C = build(mxs, a, fmt)
    assert C.impl == COLBLK[fmt]     # the default where it applies
    x = wl.uniform_vector(a.ncols, seed=1)
    xd = to_dev(x)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    y = to_dev(np.full(a.nrows, np.nan))
    mxs.spmv(C, xd, y)
    y1 = y.cpu().numpy()
    assert rel_maxnorm(y1, ref) <= 1e-12
    assert np.all(np.abs(y1 - ref) <= row_bound(a, x, U64) + 1e-300)
    assert np.array_equal(mxs.spmv(C, xd).cpu().numpy(), y1)
    # every other implementation on the same handle agrees with the oracle
    for i in range(C.impl_count()):
        if i == COLBLK[fmt]:
            continue
        try:
            C.impl = i
        except mxs.MxsError as e:
            assert e.status == UNSUPPORTED
            continue
        assert rel_maxnorm(mxs.spmv(C, xd).cpu().numpy(), ref) <= 1e-12, i
    C.close()


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_column_blocks_integer_data_bit_exact(gpu, fmt):
    mxs = gpu
    a = fixed_rows(1_200_000, 1_200_000, 9, seed=26, integer=True)
    C = build(mxs, a, fmt)
    assert C.impl == COLBLK[fmt]
    x = wl.integer_vector(a.ncols, seed=3)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert np.array_equal(mxs.spmv(C, to_dev(x)).cpu().numpy(), ref)
    C.close()


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_column_blocks_fp32(gpu, fmt):
    """FP32 values and x: 2.2M columns make an 8.8 MB x again (3 blocks)."""
    mxs = gpu
    a = fixed_rows(2_200_000, 2_200_000, 5, seed=27)
    a32 = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, a.av.astype(np.float32))
    C = build(mxs, a32, fmt)
    assert C.impl == COLBLK[fmt]
    x = wl.uniform_vector(a.ncols, seed=2).astype(np.float32)
    y = mxs.spmv(C, to_dev(x)).cpu().numpy().astype(np.float64)
    a64 = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, a32.av.astype(np.float64))
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a64.av, x.astype(np.float64))
    assert np.all(np.abs(y - ref) <= row_bound(a64, x.astype(np.float64), U32) + 1e-30)
    C.close()


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_column_blocks_not_built_where_they_do_not_apply(gpu, fmt):
    """Near-diagonal entries (banded), dense 8 x 8 blocks at random block
    columns (far from the diagonal, but eight entries to a line of x), an
    x below 8 MiB, or scattered rows of two entries (x of 16 MB, but fewer
    than three entries per row): no blocks, their id refused, defaults as
    before."""
    mxs = gpu
    for a in (wl.banded(1_500_000, ndiag=11, max_offset=2000, seed=3),
              wl.block_random(200_000, seed=31),
              fixed_rows(900_000, 900_000, 6, seed=28),
              fixed_rows(2_000_000, 2_000_000, 2, seed=32)):
        C = build(mxs, a, fmt)
        assert C.impl != COLBLK[fmt]
        with pytest.raises(mxs.MxsError) as e:
            C.impl = COLBLK[fmt]
        assert e.value.status == UNSUPPORTED
        C.close()


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_column_blocks_tune(gpu, fmt):
    mxs = gpu
    a = CASES["uniform_1.5M"]()
    C = build(mxs, a, fmt)
    x = wl.uniform_vector(a.ncols, seed=4)
    y = to_dev(np.full(a.nrows, np.nan))
    best, ms = C.tune(to_dev(x), y, reps=5)
    assert len(ms) == C.impl_count() and ms[COLBLK[fmt]] is not None and ms[COLBLK[fmt]] > 0
    assert best == min((m, i) for i, m in enumerate(ms) if m is not None)[1]
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert rel_maxnorm(y.cpu().numpy(), ref) <= 1e-12
    C.close()


def scattered_spd(n, k=2, seed=29):
    """Symmetric, strictly diagonally dominant: a -1 chain plus k couplings
    per row (and their transposes) of -0.1 to columns at least n/4 away,
    diagonal 1 + the row's absolute off-diagonal sum."""
    g = wl.rng(seed)
    i = np.arange(n - 1)
    r = [i, i + 1]
    c = [i + 1, i]
    v = [np.full(n - 1, -1.0)] * 2
    fi = np.repeat(np.arange(n), k)
    fj = (fi + n // 4 + g.integers(0, n // 2, fi.size)) % n
    r += [fi, fj]
    c += [fj, fi]
    v += [np.full(fi.size, -0.1)] * 2
    r, c, v = (np.concatenate(t) for t in (r, c, v))
    key, first = np.unique(r.astype(np.int64) * n + c, return_index=True)
    r, c, v = r[first], c[first], v[first]
    d = 1.0 + np.bincount(r, weights=np.abs(v), minlength=n)
    r = np.concatenate([r, np.arange(n)])
    c = np.concatenate([c, np.arange(n)])
    v = np.concatenate([v, d])
    o = np.lexsort((c, r))
    return wl.Coo(n, n, r[o].astype(np.int32), c[o].astype(np.int32), v[o])


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_cg_with_column_blocks_matches_oracle(gpu, fmt):
    """The SpMV + p.Ap of the blocks inside CG (x 9.6 MB: 3 blocks)."""
    mxs = gpu
    a = scattered_spd(1_200_000)
    C = build(mxs, a, fmt)
    assert C.impl == COLBLK[fmt]
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, wl.uniform_vector(a.ncols, seed=5))
    st_o, x_o, it_o, _, _ = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=2000)
    st, x, res = mxs.cg_solve(C, to_dev(b), rtol=1e-10, maxit=2000)
    print(f"[colblk cg] iters={res['iters']} oracle={it_o}", flush=True)
    assert st == 0 and st_o == 0 and abs(res["iters"] - it_o) <= 2
    assert np.max(np.abs(x.cpu().numpy() - x_o)) <= 1e-8
    C.close()


@pytest.mark.parametrize("fmt", ["csr", "coo"])
def test_mixed_precision_with_column_blocks(gpu, fmt):
    """FP32 inner CG on the FP32 copy (its own column blocks: x of 4.8 MB in
    FP32 is below the threshold at 1.2M rows, so 2.4M rows are used) with
    FP64 reliable updates reaches the FP64 tolerance."""
    mxs = gpu
    a = scattered_spd(2_400_000)
    A = build(mxs, a, fmt)
    A32 = A.cast(mxs.F32).optimize()
    assert A.impl == COLBLK[fmt] and A32.impl == COLBLK[fmt]
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, wl.uniform_vector(a.ncols, seed=6))
    st, x, res = mxs.cg_solve(A, to_dev(b), rtol=1e-10, maxit=5000, mixed="ru", A32=A32)
    assert st == 0 and res["true_rel_resid"] <= 1e-10, res
    r = b - orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.5e-10
    A32.close()
    A.close()
