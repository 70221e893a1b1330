"""GPU parity of split matrices (DIA band + COO/CSR remainder) against the CPU
oracle, through the C ABI.

Bars: band offsets equal the oracle's selection; band values and remainder
arrays are the definition's, bit for bit (values are only moved); SpMV within
1e-12 of the oracle's product of the whole matrix, bit-exact on integer
data; CG on a split matrix matches the oracle's CG on the whole matrix.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import rel_maxnorm

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def merge(a, b):
    """Union of two matrices' entries; where both have (i, j), a's value."""
    ai = np.concatenate([a.ai, b.ai])
    aj = np.concatenate([a.aj, b.aj])
    av = np.concatenate([a.av, b.av])
    key = ai.astype(np.int64) * a.ncols + aj
    _, first = np.unique(key, return_index=True)
    order = first[np.lexsort((aj[first], ai[first]))]
    return wl.Coo(a.nrows, a.ncols, ai[order].copy(), aj[order].copy(), av[order].copy())


def scattered(n, density, seed):
    """About n*n*density entries at uniform random positions (duplicates
    merged), N(0,1) values; drawn without an n-by-n mask."""
    g = wl.rng(seed)
    k = int(g.binomial(n * n, density))
    ai = g.integers(0, n, k).astype(np.int32)
    aj = g.integers(0, n, k).astype(np.int32)
    return wl.Coo(n, n, ai, aj, g.standard_normal(k))


def banded_noise(n, seed, ndiag=11, width=300, density=2e-4, integer=False):
    a = wl.banded(n, ndiag=ndiag, max_offset=width, seed=seed)
    b = scattered(n, density, seed + 1)
    m = merge(a, b)
    if integer:
        g = wl.rng(seed + 2)
        m.av = g.integers(-4, 5, m.nnz).astype(np.float64)
        m.av[m.av == 0] = 3.0
    return m


def hand_built():
    M = np.zeros((6, 6))
    M[np.arange(6), np.arange(6)] = 1.0
    M[0, 1] = M[3, 4] = 2.0
    M[2, 0] = M[3, 1] = M[5, 3] = 3.0
    ai, aj = np.nonzero(M)
    return wl.Coo(6, 6, ai.astype(np.int32), aj.astype(np.int32), M[ai, aj])


CASES = [("hand6", hand_built()), ("stencil16", wl.stencil(16)),
         ("banded_noise", banded_noise(30000, seed=7)),
         ("zipf20k", wl.zipf_rows(20000, seed=11)),
         ("random", wl.random_coo(3000, 2000, 0.003, seed=9)),
         ("rect_banded", merge(wl.Coo(3000, 3500, *[np.zeros(0, np.int32)] * 2, np.zeros(0)),
                               wl.random_coo(3000, 3500, 0.001, seed=3)))]


def expected_split(a, min_fill):
    """The definition: band offsets (oracle), band DIA values of the band
    entries, the remaining entries in canonical order."""
    band = orc.split_offsets(a.nrows, a.ncols, a.ai, a.aj, min_fill)
    off = a.aj.astype(np.int64) - a.ai
    inb = np.isin(off, band)
    bd = np.zeros(band.size * a.nrows)
    pos = np.searchsorted(band, off[inb])
    bd[pos * a.nrows + a.ai[inb]] = a.av[inb]
    return band, bd, a.ai[~inb], a.aj[~inb], a.av[~inb]


@pytest.mark.parametrize("rest", ["coo", "csr"])
@pytest.mark.parametrize("min_fill", [0.5, 0.05, 1.0])
@pytest.mark.parametrize("src", ["coo", "csr"])
@pytest.mark.parametrize("name,a", CASES, ids=[c[0] for c in CASES])
def test_split_matches_definition_and_oracle(gpu, name, a, src, min_fill, rest):
    mxs = gpu
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    if src == "csr":
        A = A.convert("csr")
    band, bd, rai, raj, rav = expected_split(a, min_fill)
    assert A.split_size(min_fill) == (band.size, rai.size)
    H = A.split(min_fill, rest)
    assert H.format == mxs.HDC and H.ndiag == band.size
    doff, bvals, i0, i1, vals = [t.cpu().numpy() for t in H._keep]
    assert np.array_equal(doff, band)
    assert np.array_equal(bvals, bd)
    if rest == "coo":
        assert np.array_equal(i0, rai)
    else:
        rows_ptr = np.concatenate([[0], np.cumsum(np.bincount(rai, minlength=a.nrows))])
        assert np.array_equal(i0, rows_ptr)
    assert np.array_equal(i1, raj) and np.array_equal(vals, rav)
    x = wl.uniform_vector(a.ncols, seed=5)
    y = to_dev(np.full(a.nrows, np.nan))
    mxs.spmv(H, to_dev(x), y)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert rel_maxnorm(y.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("rest", ["coo", "csr"])
def test_split_integer_data_bit_exact(gpu, rest):
    mxs = gpu
    a = banded_noise(50000, seed=21, integer=True)
    H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).split(0.5, rest)
    assert H.ndiag == 11
    x = wl.integer_vector(a.ncols, seed=8)
    assert np.array_equal(mxs.spmv(H, to_dev(x)).cpu().numpy(),
                          orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x))


def test_split_fp32(gpu):
    mxs = gpu
    a = banded_noise(20000, seed=31)
    a32 = a.astype(np.float32)
    H = mxs.Matrix.coo(a.nrows, a.ncols, a32.ai, a32.aj, a32.av).split(0.5, "csr")
    x = wl.uniform_vector(a.ncols, seed=2).astype(np.float32)
    y = mxs.spmv(H, to_dev(x)).cpu().numpy().astype(np.float64)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a32.av.astype(np.float64), x.astype(np.float64))
    from _cases import U32, row_bound
    assert np.all(np.abs(y - ref) <= row_bound(a, x.astype(np.float64), U32) + 1e-30)


def spd_split_matrix(n):
    """27-point stencil plus symmetric long-range couplings -0.05 (at most
    two per row), still strictly diagonally dominant, hence SPD."""
    s = wl.stencil(n)
    g = wl.rng(40)
    N = s.nrows
    i = g.choice(N, N // 20, replace=False)
    j = (i + N // 3 + g.integers(0, N // 3, i.size)) % N
    keep = np.abs(j.astype(np.int64) - i) > n * n + n + 1
    i, j = i[keep], j[keep]
    extra = wl.Coo(N, N, np.concatenate([i, j]).astype(np.int32),
                   np.concatenate([j, i]).astype(np.int32), np.full(2 * i.size, -0.05))
    return merge(s, extra)


@pytest.mark.parametrize("rest", ["coo", "csr"])
def test_cg_on_split_matrix_matches_oracle(gpu, rest):
    import torch
    mxs = gpu
    a = spd_split_matrix(20)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).split(0.5, rest)
    assert H.ndiag == 27
    st, x, res = mxs.cg_solve(H, to_dev(b), rtol=1e-10, maxit=5000)
    st_o, x_o, it_o, rel_o, true_o = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=5000)
    assert st == 0 and st_o == 0 and abs(res["iters"] - it_o) <= 2
    x = x.cpu().numpy()
    assert np.max(np.abs(x - x_o)) <= 1e-7
    r = b - orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 2e-10


def test_split_unsupported_and_invalid(gpu):
    mxs = gpu
    a = banded_noise(5000, seed=3)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    H = A.split()
    for call in (lambda: H.convert("csr"), lambda: H.cast(mxs.F32), lambda: mxs.features(H),
                 lambda: H.split(),
                 lambda: mxs.Matrix.coo(*_stencil_arrays()).convert("dia").split()):
        with pytest.raises(mxs.MxsError) as e:
            call()
        assert e.value.status == -10
    with pytest.raises(mxs.MxsError) as e:
        A.split(min_fill=-1.0)
    assert e.value.status == -1
    with pytest.raises(mxs.MxsError) as e:
        A.split(rest="dia")
    assert e.value.status == -1


def _stencil_arrays():
    s = wl.stencil(5)
    return s.nrows, s.ncols, s.ai, s.aj, s.av


@pytest.mark.parametrize("rest", ["coo", "csr"])
def test_split_parts_every_impl_pair_matches_oracle(gpu, rest):
    """The parts are handles of their own; every implementation of the band
    with every implementation of the remainder gives the oracle's product."""
    mxs = gpu
    a = banded_noise(30000, seed=7)
    H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).split(0.5, rest)
    H.optimize(mxs.PLAN_DIA_BLOCKED)   # the band's row-blocked copy: every DIA implementation
    band, part = H.parts()
    assert band.format == mxs.DIA and band.ndiag == H.ndiag
    assert part.format == mxs.FORMATS[rest] and part.nnz == H._keep[3].numel()
    lib = mxs.load()
    assert lib.mxs_destroy(band.handle) == -1 and lib.mxs_destroy(part.handle) == -1
    x = wl.uniform_vector(a.ncols, seed=5)
    xd = to_dev(x)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    for bi in range(band.impl_count()):
        try:
            band.impl = bi
        except mxs.MxsError as e:
            assert e.status == -10
            continue
        for ri in range(part.impl_count()):
            try:
                part.impl = ri
            except mxs.MxsError as e:
                assert e.status == -10
                continue
            y = to_dev(np.full(a.nrows, np.nan))
            mxs.spmv(H, xd, y)
            assert rel_maxnorm(y.cpu().numpy(), ref) <= 1e-12, (bi, ri)
    with pytest.raises(mxs.MxsError) as e:
        mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).parts()
    assert e.value.status == -10


def test_split_tune_and_auto_rest(gpu):
    mxs = gpu
    a = banded_noise(30000, seed=8)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    x = wl.uniform_vector(a.ncols, seed=6)
    xd = to_dev(x)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    H = A.split(0.5, "csr")
    y = to_dev(np.full(a.nrows, np.nan))
    t = H.tune(xd, y, reps=3)
    assert rel_maxnorm(y.cpu().numpy(), ref) <= 1e-12     # tune leaves y = A x
    band, part = H.parts()
    assert band.impl == t["band"][0] and part.impl == t["rest"][0] and t["ms"] > 0
    assert rel_maxnorm(mxs.spmv(H, xd).cpu().numpy(), ref) <= 1e-12
    Hauto = A.split(0.5, "auto", x=xd, reps=3)
    assert Hauto.format == mxs.HDC and Hauto.tuning["rest_format"] in ("coo", "csr")
    assert Hauto.parts()[1].format == mxs.FORMATS[Hauto.tuning["rest_format"]]
    assert rel_maxnorm(mxs.spmv(Hauto, xd).cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("extra", [4000, 400000])
def test_split_rest_chosen_by_selector(gpu, extra):
    """rest="select": the remainder's format (COO or CSR) is the selector
    network's choice on the remainder's features; the product is the
    oracle's."""
    mxs = gpu
    from paper_2304_09511_amd import selector as S
    a = wl.banded(200000, ndiag=11, max_offset=2000, seed=12)
    g = wl.rng(13)
    rows = np.sort(g.integers(0, a.nrows, extra)).astype(np.int32)
    noise = wl.Coo(a.nrows, a.ncols, rows, g.integers(0, a.ncols, extra).astype(np.int32),
                   g.standard_normal(extra))
    m = merge(a, noise)
    A = mxs.Matrix.coo(m.nrows, m.ncols, m.ai, m.aj, m.av)
    model = S.Selector.load(str(S.MODEL_PATH))
    H = A.split(0.5, "select", model=model)
    r = H.selection["rest_format"]
    assert H.format == mxs.HDC and H.ndiag == 11 and r in ("coo", "csr")
    assert H.parts()[1].format == mxs.FORMATS[r]
    Hc = A.split(0.5, "coo")
    assert S.select_rest(model, Hc.parts()[1]) == r
    x = wl.uniform_vector(m.ncols, seed=4)
    ref = orc.coo_spmv(m.nrows, m.ai, m.aj, m.av, x)
    assert rel_maxnorm(mxs.spmv(H, to_dev(x)).cpu().numpy(), ref) <= 1e-12
