"""Every SpMV implementation of every format against the CPU oracle, through
the C ABI, and the run-first choice among them (mxs_tune).

Bars as for SpMV: FP64 within 1e-12 relative max-norm of the oracle and within
the per-row rounding bound; integer data bit-exact; bitwise reproducible per
implementation.  CG with each implementation matches the oracle's CG.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import U64, rel_maxnorm, row_bound, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()
IDS = [c[0] for c in CASES]
UNSUPPORTED = -10


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def build(mxs, a, fmt, opts=None):
    """The matrix in `fmt` with a plan; DIA with its row-blocked copy (an
    opt-in of the plan), so that every implementation is reachable."""
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    if fmt != "coo":
        try:
            A = A.convert(fmt)
        except mxs.MxsError as e:
            if e.status == -5:
                return None
            raise
    if opts is None:
        opts = mxs.PLAN_DIA_BLOCKED if fmt == "dia" else 0
    return A.optimize(opts)


def applicable(mxs, A):
    """Ids accepted by mxs_set_impl; the refusals must be MXS_ERR_UNSUPPORTED."""
    ok = []
    for i in range(A.impl_count()):
        try:
            A.impl = i
            ok.append(i)
        except mxs.MxsError as e:
            assert e.status == UNSUPPORTED
    return ok


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_every_impl_matches_oracle(gpu, name, a, fmt):
    mxs = gpu
    print(f"[impl] {name} {fmt} {a.nrows}x{a.ncols} nnz={a.nnz}", flush=True)
    A = build(mxs, a, fmt)
    if A is None:
        pytest.skip("DIA refused (more than 8 slots per non-zero)")
    default = A.impl
    ids = applicable(mxs, A)
    assert default in ids
    # the always-applicable fallback of each format
    assert {"coo": 1, "csr": 1, "dia": 2}[fmt] in ids
    x = wl.uniform_vector(a.ncols, seed=1)
    xd = to_dev(x)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    for i in ids:
        A.impl = i
        assert A.impl == i
        y = to_dev(np.full(a.nrows, np.nan))
        mxs.spmv(A, xd, y)
        y1 = y.cpu().numpy()
        assert rel_maxnorm(y1, ref) <= 1e-12, i
        assert np.all(np.abs(y1 - ref) <= row_bound(a, x, U64) + 1e-300), i
        assert np.array_equal(mxs.spmv(A, xd).cpu().numpy(), y1), i


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("name", ["stencil16", "gappy_long", "empty_rows"])
def test_every_impl_integer_data_bit_exact(gpu, name, fmt):
    mxs = gpu
    if name == "stencil16":
        a = wl.stencil(16)
    elif name == "empty_rows":
        a = dict(CASES)["empty_rows"]
        a = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, np.round(a.av * 4) + 1.0)
    else:
        from test_spmv_gpu import _gappy
        a = _gappy(4000, seed=2, long_rows={500, 501, 2200})
    A = build(mxs, a, fmt)
    if A is None:
        pytest.skip("DIA refused (more than 8 slots per non-zero)")
    x = wl.integer_vector(a.ncols, seed=3)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    for i in applicable(mxs, A):
        A.impl = i
        assert np.array_equal(mxs.spmv(A, to_dev(x)).cpu().numpy(), ref), i


def test_applicability_rules(gpu):
    """COO row tiles need at most 512 rows per tile; DIA id 0 needs offsets in
    runs of three, ids 0 and 1 the row-blocked copy, which only a plan asked
    for it makes; CSR id 3 needs the ELL copy, which a plan can leave out."""
    mxs = gpu
    sparse = dict(CASES)["empty_rows"]   # 10,000 rows, 100 live: one tile owns them all
    # (defaults read before applicable(), which leaves its last id active)
    A = build(mxs, sparse, "coo")
    assert A.impl == 1 and applicable(mxs, A) == [1]
    S = build(mxs, wl.stencil(16), "dia")
    assert S.impl == 0 and applicable(mxs, S) == [0, 1, 2]
    from test_spmv_gpu import _diagonals
    M = build(mxs, _diagonals(5000, [-2, -1, 0, 7, 8], seed=1), "dia")
    assert M.impl == 1 and applicable(mxs, M) == [1, 2]
    C = build(mxs, sparse, "csr")
    assert C.impl == 1 and applicable(mxs, C) == [0, 1, 2, 5]  # rows > 2 nnz: a thread per row
    assert build(mxs, wl.stencil(16), "csr").impl == 0
    # the default plan has no row-blocked DIA copy: the diagonal-major kernel
    D = build(mxs, wl.stencil(16), "dia", opts=0)
    assert D.impl == 2 and applicable(mxs, D) == [2]
    # rows of near-equal length get the ELL copy unless the plan leaves it out
    E = build(mxs, wl.stencil(48), "csr")
    assert E.impl == 3 and 3 in applicable(mxs, E)
    E2 = build(mxs, wl.stencil(48), "csr", opts=mxs.PLAN_NO_ELL)
    assert E2.impl == 0 and 3 not in applicable(mxs, E2)
    for B in (A, S):
        with pytest.raises(mxs.MxsError) as e:
            B.impl = B.impl_count()
        assert e.value.status == UNSUPPORTED
        with pytest.raises(mxs.MxsError) as e:
            B.impl = -1
        assert e.value.status == UNSUPPORTED


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
def test_tune_keeps_an_applicable_fastest_impl(gpu, fmt):
    mxs = gpu
    a = wl.stencil(24)
    A = build(mxs, a, fmt)
    x = wl.uniform_vector(a.ncols, seed=4)
    y = to_dev(np.full(a.nrows, np.nan))
    best, ms = A.tune(to_dev(x), y, reps=5)
    ids = applicable(mxs, A)
    assert len(ms) == A.impl_count()
    assert [i for i, m in enumerate(ms) if m is not None] == ids
    assert best in ids and ms[best] == min(m for m in ms if m is not None) and ms[best] > 0
    # applicable() left the last id active; tune again and the choice is kept
    best2, _ = A.tune(to_dev(x), y, reps=3)
    assert A.impl == best2
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert rel_maxnorm(y.cpu().numpy(), ref) <= 1e-12   # tune leaves y = A x
    assert rel_maxnorm(mxs.spmv(A, to_dev(x)).cpu().numpy(), ref) <= 1e-12


def test_tune_argument_checks(gpu):
    import ctypes as C
    mxs = gpu
    a = wl.stencil(6)
    A = build(mxs, a, "csr")
    x = to_dev(np.ones(a.ncols))
    lib = mxs.load()
    assert lib.mxs_tune(A.handle, mxs._ptr(x), mxs._ptr(to_dev(np.zeros(a.nrows))), 0,
                        None, None, None) == -1
    assert lib.mxs_tune(A.handle, mxs._ptr(x), mxs._ptr(x), 3, None, None, None) == -1  # aliasing
    H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).split(0.5, "csr")
    assert H.impl_count() == 0
    v = C.c_int32()
    assert lib.mxs_get_impl(H.handle, C.byref(v), None) == UNSUPPORTED
    assert lib.mxs_set_impl(H.handle, 0, None) == UNSUPPORTED
    assert lib.mxs_tune(H.handle, mxs._ptr(x), mxs._ptr(to_dev(np.zeros(a.nrows))), 3,
                        None, None, None) == UNSUPPORTED


@pytest.mark.parametrize("points,n", [(27, 12), (7, 14)])
@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
def test_cg_with_every_impl_matches_oracle(gpu, fmt, points, n):
    """The fused SpMV + p.Ap of each implementation inside CG; the 27-point
    stencil's CSR tiles take 10 entries per thread, the 7-point stencil's 8
    (more rows per tile than the LDS-staged path holds at 10)."""
    mxs = gpu
    a = wl.stencil(n, points=points)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    st_o, x_o, it_o, _, _ = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=2000)
    A = build(mxs, a, fmt)
    for i in applicable(mxs, A):
        A.impl = i
        st, x, res = mxs.cg_solve(A, to_dev(b), rtol=1e-10, maxit=2000)
        assert st == 0 and abs(res["iters"] - it_o) <= 2, (i, res["iters"], it_o)
        assert np.max(np.abs(x.cpu().numpy() - x_o)) <= 1e-8, i


def long_rows(seed, ncols=30000, integer=False, dtype=np.float64, pad_short=0):
    """Short rows (0-10 entries) around runs of long rows: 40 rows of 65
    entries (a tile then owns about 32 long rows), lengths at the wave path's
    threshold (64, 65, 66) and at the tile and extension edges of each tile
    size (2,048 and 2,560 entries, 3,072 for COO's FP32 tiles, each plus 256),
    and rows of up to 5,000 entries that span tiles.  pad_short: that many
    more rows of 0-2 entries at the end (CSR tiles then own too many rows
    for the LDS-staged path and take 8 entries per thread instead of 10)."""
    g = wl.rng(seed)
    lens = list(g.integers(0, 11, 300))
    lens += [65] * 40 + list(g.integers(0, 11, 50))
    for L in (64, 65, 66, 100, 127, 128, 129, 300, 1000, 2000, 2047, 2048, 2049,
              2303, 2304, 2305, 2500, 2559, 2560, 2561, 2815, 2816, 2817, 3071, 3072, 3073,
              3327, 3328, 3329, 4095, 4096, 4097, 4999, 5000):
        lens += [int(L)] + list(g.integers(0, 11, int(g.integers(1, 40))))
    lens += [65, 66, 64, 200] * 20 + list(g.integers(0, 11, 200))
    if pad_short:
        lens += list(g.integers(0, 3, pad_short))
    L = np.array(lens, np.int64)
    ai = np.repeat(np.arange(L.size, dtype=np.int32), L)
    aj = wl._distinct_sorted_columns(g, ai, L, ncols)
    av = (g.integers(-4, 5, ai.size).astype(np.float64) if integer
          else g.standard_normal(ai.size)).astype(dtype)
    if integer:
        av[av == 0] = 3.0
    return wl.Coo(L.size, ncols, ai, aj, av)


def wave_path_ids(mxs, fmt):
    """Implementations whose rows go through the tile reduction with the
    long-row wave path: COO row tiles; CSR entry tiles and staged gather."""
    return {"coo": [0], "csr": [0, 2]}[fmt]


@pytest.mark.parametrize("pad_short", [0, 40000])
@pytest.mark.parametrize("fmt", ["coo", "csr"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "int"])
def test_long_rows_reduced_by_waves(gpu, fmt, dtype, pad_short):
    if fmt == "coo" and pad_short:
        pytest.skip("COO's row tiles do not apply to tiles owning more than 512 rows "
                    "(the segmented tiles take them, tested with the other implementations)")
    mxs = gpu
    a = long_rows(5, integer=dtype == "int", dtype=np.float32 if dtype == "f32" else np.float64,
                  pad_short=pad_short)
    print(f"[long rows] {fmt} {dtype} {a.nrows} rows nnz={a.nnz}", flush=True)
    A = build(mxs, a, fmt)
    x = (wl.integer_vector(a.ncols, seed=3) if dtype == "int"
         else wl.uniform_vector(a.ncols, seed=3))
    if dtype == "f32":
        x = x.astype(np.float32)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av.astype(np.float64), x.astype(np.float64))
    for i in wave_path_ids(mxs, fmt):
        A.impl = i
        y = to_dev(np.full(a.nrows, np.nan, dtype=x.dtype))
        mxs.spmv(A, to_dev(x), y)
        y1 = y.cpu().numpy().astype(np.float64)
        if dtype == "int":
            assert np.array_equal(y1, ref), i
        elif dtype == "f64":
            assert rel_maxnorm(y1, ref) <= 1e-12, i
            assert np.all(np.abs(y1 - ref) <= row_bound(a, x, U64) + 1e-300), i
        else:
            from _cases import U32
            a64 = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, a.av.astype(np.float64))
            assert np.all(np.abs(y1 - ref) <= row_bound(a64, x.astype(np.float64), U32) + 1e-30), i
        assert np.array_equal(mxs.spmv(A, to_dev(x)).cpu().numpy(), y.cpu().numpy()), i


def hub_spd(n=6000, hubs=12, seed=7):
    """Symmetric, strictly diagonally dominant (hence SPD): a tridiagonal
    -1 chain plus hub rows coupled with -0.01 to 100-3,000 random columns
    (and back), diagonal 1 + the row's absolute off-diagonal sum."""
    g = wl.rng(seed)
    i = np.arange(n - 1)
    rows = [i, i + 1]
    cols = [i + 1, i]
    vals = [np.full(n - 1, -1.0)] * 2
    for h in g.choice(n, hubs, replace=False):
        c = g.choice(n, int(g.integers(100, 3001)), replace=False)
        c = c[np.abs(c - h) > 1]
        rows += [np.full(c.size, h), c]
        cols += [c, np.full(c.size, h)]
        vals += [np.full(c.size, -0.01)] * 2
    r, c, v = (np.concatenate(t) for t in (rows, cols, vals))
    key = r.astype(np.int64) * n + c
    key, first = np.unique(key, return_index=True)
    r, c, v = r[first], c[first], v[first]
    d = 1.0 + np.bincount(r, weights=np.abs(v), minlength=n)
    r = np.concatenate([r, np.arange(n)])
    c = np.concatenate([c, np.arange(n)])
    v = np.concatenate([v, d])
    o = np.lexsort((c, r))
    return wl.Coo(n, n, r[o].astype(np.int32), c[o].astype(np.int32), v[o])


@pytest.mark.parametrize("fmt", ["coo", "csr"])
def test_cg_on_long_rows_matches_oracle(gpu, fmt):
    """The fused SpMV + p.Ap of the tile kernels when hub rows take the wave path."""
    mxs = gpu
    a = hub_spd()
    assert np.bincount(a.ai).max() > 1000
    # (A 1 = 1 here, so b = A 1 would converge in one step)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, wl.uniform_vector(a.ncols, seed=2))
    st_o, x_o, it_o, _, _ = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=5000)
    assert st_o == 0
    A = build(mxs, a, fmt)
    for i in wave_path_ids(mxs, fmt):
        A.impl = i
        st, x, res = mxs.cg_solve(A, to_dev(b), rtol=1e-10, maxit=5000)
        assert st == 0 and abs(res["iters"] - it_o) <= 2, (i, res["iters"], it_o)
        assert np.max(np.abs(x.cpu().numpy() - x_o)) <= 1e-8, i


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("name", ["stencil16", "gappy_long", "random300x200", "dense_rows", "zipf20k",
                                  "banded50k"])
def test_every_impl_fp32_within_rounding_bound(gpu, name, fmt):
    """The FP32 kernels of every implementation: within the per-row FP32
    rounding bound of the oracle's FP64 product of the same FP32 values."""
    from _cases import U32
    mxs = gpu
    cases = dict(CASES)
    if name == "stencil16":
        a = wl.stencil(16)
    elif name in cases:
        a = cases[name]
    else:
        from test_spmv_gpu import _gappy
        a = _gappy(4000, seed=2, long_rows={500, 501, 2200})
    a32 = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, a.av.astype(np.float32))
    A = build(mxs, a32, fmt)
    if A is None:
        pytest.skip("DIA refused (more than 8 slots per non-zero)")
    x = wl.uniform_vector(a.ncols, seed=7).astype(np.float32)
    a64 = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, a32.av.astype(np.float64))
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a64.av, x.astype(np.float64))
    bound = row_bound(a64, x.astype(np.float64), U32) + 1e-30
    for i in applicable(mxs, A):
        A.impl = i
        y = mxs.spmv(A, to_dev(x)).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(y - ref) <= bound), (name, fmt, i)
