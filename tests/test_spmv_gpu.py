"""GPU parity of SpMV (Algorithms 1-3) and of the format conversions against the
CPU oracle, through the C ABI.

Bar: FP64 SpMV within 1e-12 relative max-norm of the oracle and within the
per-row rounding bound; bit-exact when every partial sum is an integer;
conversion index and value arrays bit-exact; results bitwise reproducible.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import U32, U64, rel_maxnorm, row_bound, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()
IDS = [c[0] for c in CASES]


def _torch():
    import torch
    return torch


def to_dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def build(mxs, a, fmt, dtype=np.float64):
    """Matrix in `fmt` via the device conversion from COO; None if DIA is refused."""
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av.astype(dtype))
    if fmt == "coo":
        return A
    try:
        return A.convert(fmt)
    except mxs.MxsError as e:
        if e.status == -5:
            return None
        raise


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_spmv_fp64_matches_oracle(gpu, name, a, fmt):
    print(f"[spmv] {name} {fmt} {a.nrows}x{a.ncols} nnz={a.nnz}", flush=True)
    B = build(gpu, a, fmt)
    if B is None:
        assert fmt == "dia"
        pytest.skip("DIA refused (more than 8 slots per non-zero)")
    x = wl.uniform_vector(a.ncols, seed=1)
    y = gpu.spmv(B, to_dev(x)).cpu().numpy()
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert y.shape == ref.shape
    assert rel_maxnorm(y, ref) <= 1e-12
    assert np.all(np.abs(y - ref) <= row_bound(a, x, U64) + 1e-300)


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("n", [3, 16, 33])
def test_spmv_integer_data_bit_exact(gpu, n, fmt):
    a = wl.stencil(n)
    x = wl.integer_vector(a.ncols, seed=n)
    B = build(gpu, a, fmt)
    y = gpu.spmv(B, to_dev(x)).cpu().numpy()
    assert np.array_equal(y, orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x))


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
def test_spmv_deterministic(gpu, fmt):
    a = wl.banded(60000, ndiag=7, max_offset=500, seed=21) if fmt == "dia" else wl.zipf_rows(30000, seed=21)
    B = build(gpu, a, fmt)
    x = to_dev(wl.uniform_vector(a.ncols, seed=2))
    y1 = gpu.spmv(B, x).cpu().numpy()
    y2 = gpu.spmv(B, x).cpu().numpy()
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("name,a", [c for c in CASES if c[0] in
                                    ("stencil16", "zipf20k", "banded50k", "random37x53", "empty_rows")],
                         ids=["stencil16", "random37x53", "zipf20k", "banded50k", "empty_rows"])
def test_spmv_fp32_within_rounding_bound(gpu, name, a, fmt):
    A64 = build(gpu, a, fmt)
    if A64 is None:
        pytest.skip("DIA refused")
    A32 = A64.cast(gpu.F32)
    x32 = wl.uniform_vector(a.ncols, seed=4).astype(np.float32)
    y = gpu.spmv(A32, to_dev(x32)).cpu().numpy().astype(np.float64)
    a32 = wl.Coo(a.nrows, a.ncols, a.ai, a.aj, a.av.astype(np.float32).astype(np.float64))
    ref = orc.coo_spmv(a.nrows, a32.ai, a32.aj, a32.av, x32.astype(np.float64))
    assert np.all(np.abs(y - ref) <= row_bound(a32, x32, U32) + 1e-30)


def test_spmv_y_overwritten_and_empty_rows_zero(gpu):
    torch = _torch()
    a = wl.Coo(6, 6, np.array([1, 1, 4], np.int32), np.array([0, 5, 2], np.int32),
               np.array([2.0, 3.0, 5.0]))
    x = np.arange(6, dtype=np.float64) + 1
    for fmt in ("coo", "csr", "dia"):
        B = build(gpu, a, fmt)
        y = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
        gpu.spmv(B, to_dev(x), y)
        assert y.cpu().numpy().tolist() == [0.0, 20.0, 0.0, 0.0, 15.0, 0.0]


def test_spmv_rejects_aliasing(gpu):
    A = build(gpu, wl.stencil(3), "csr")
    x = to_dev(np.ones(27))
    with pytest.raises(gpu.MxsError) as e:
        gpu.spmv(A, x, x)
    assert e.value.status == -1


# ---------------------------------------------------------------------------
# Conversions: bit-exact against the oracle's definitions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_conversions_bit_exact(gpu, name, a):
    print(f"[convert] {name}", flush=True)
    A = gpu.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    # COO -> CSR
    C = A.convert("csr")
    irp, aj, av = C.export()
    assert np.array_equal(irp, orc.coo_to_csr(a.nrows, a.ai))
    assert np.array_equal(aj, a.aj) and np.array_equal(av.view(np.uint64), a.av.view(np.uint64))
    # CSR -> COO
    ai2, aj2, av2 = C.convert("coo").export()
    assert np.array_equal(ai2, orc.csr_to_coo(irp)) and np.array_equal(ai2, a.ai)
    # COO -> DIA and CSR -> DIA
    offs = orc.dia_offsets(a.nrows, a.ncols, a.ai, a.aj)
    if offs.shape[0] * a.nrows > 8 * a.nnz:
        with pytest.raises(gpu.MxsError) as e:
            A.convert("dia")
        assert e.value.status == -5
        return
    doff_ref, avd_ref = orc.coo_to_dia(a.nrows, a.ncols, a.ai, a.aj, a.av)
    for src in (A, C):
        D = src.convert("dia")
        doff, avd = D.export()
        assert np.array_equal(doff, doff_ref)
        assert np.array_equal(avd.view(np.uint64), avd_ref.view(np.uint64))
        assert D.nnz == orc.dia_slots(a.nrows, a.ncols, doff_ref)
    # DIA -> COO and DIA -> CSR (drop stored zeros)
    bi, bj, bv = D.convert("coo").export()
    ri, rj, rv = orc.dia_to_coo(a.nrows, a.ncols, doff_ref, avd_ref)
    assert np.array_equal(bi, ri) and np.array_equal(bj, rj)
    assert np.array_equal(bv.view(np.uint64), rv.view(np.uint64))
    cirp, cj, cv = D.convert("csr").export()
    assert np.array_equal(cirp, orc.coo_to_csr(a.nrows, ri)) and np.array_equal(cj, rj)


def test_dia_round_trip_drops_stored_zeros(gpu):
    doff = np.array([-1, 0, 2], np.int32)
    avd = np.array([9.0, 0.0, -0.0, 1.0, 0.0, 2.0, 3.0, 4.0, 5.0])
    D = gpu.Matrix.dia(3, 3, doff, avd)
    ai, aj, av = D.convert("coo").export()
    ri, rj, rv = orc.dia_to_coo(3, 3, doff, avd)
    assert ai.tolist() == ri.tolist() and aj.tolist() == rj.tolist() and av.tolist() == rv.tolist()
    assert D.nnz == orc.dia_slots(3, 3, doff)


def test_cast_rounds_to_nearest(gpu):
    a = wl.zipf_rows(5000, seed=31)
    A = gpu.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    _, _, v32 = A.cast(gpu.F32).export()
    assert np.array_equal(v32, a.av.astype(np.float32))


# ---------------------------------------------------------------------------
# Problem setup on the device
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,points", [(1, 27), (2, 27), (3, 27), (16, 27), (40, 27), (2, 7), (9, 7)])
def test_device_stencil_matches_generator(gpu, n, points):
    A = gpu.stencil(n, points=points)
    ai, aj, av = A.export()
    ref = wl.stencil(n, points=points)
    assert np.array_equal(ai, ref.ai) and np.array_equal(aj, ref.aj)
    assert np.array_equal(av, ref.av)


# ---------------------------------------------------------------------------
# Validation of the containers on the device
# ---------------------------------------------------------------------------
def test_coo_validation_statuses(gpu):
    ai = np.array([0, 0, 1], np.int32)
    v = np.ones(3)
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.coo(2, 2, ai, np.array([0, 2, 1], np.int32), v)
    assert e.value.status == -2
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.coo(2, 2, ai, np.array([1, 1, 1], np.int32), v)
    assert e.value.status == -4
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.coo(2, 2, ai, np.array([1, 0, 1], np.int32), v, borrow=True)
    assert e.value.status == -3


def test_csr_and_dia_validation_statuses(gpu):
    aj = np.array([0, 2, 1], np.int32)
    v = np.ones(3)
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.csr(2, 3, np.array([0, 3, 2], np.int32), aj, v)
    assert e.value.status == -2
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.csr(2, 3, np.array([0, 2, 3], np.int32), np.array([2, 0, 1], np.int32), v)
    assert e.value.status == -3
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.csr(2, 3, np.array([0, 2, 3], np.int32), np.array([1, 1, 1], np.int32), v)
    assert e.value.status == -4
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.dia(3, 3, np.array([1, 0], np.int32), np.zeros(6))
    assert e.value.status == -3
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.dia(3, 3, np.array([0, 3], np.int32), np.zeros(6))
    assert e.value.status == -2


@pytest.mark.parametrize("name", ["stencil16", "zipf20k", "random37x53", "block3000", "one_column"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_unsorted_coo_is_sorted_on_create(gpu, name, dtype):
    """An owned COO built from shuffled entries holds the canonical (row, col)
    order: its arrays equal the sorted input bit for bit."""
    a = dict(CASES)[name]
    s = wl.shuffled(a, seed=17)
    A = gpu.Matrix.coo(s.nrows, s.ncols, s.ai, s.aj, s.av.astype(dtype))
    ai, aj, av = A.export()
    assert np.array_equal(ai, a.ai) and np.array_equal(aj, a.aj)
    assert np.array_equal(av, a.av.astype(dtype))
    x = wl.uniform_vector(a.ncols, seed=3).astype(dtype)
    y = gpu.spmv(A, to_dev(x)).cpu().numpy()
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x.astype(np.float64))
    assert rel_maxnorm(y, ref) <= (1e-12 if dtype == np.float64 else 1e-5)


def test_unsorted_coo_with_duplicate_is_refused(gpu):
    a = wl.stencil(5)
    s = wl.shuffled(a, seed=4)
    aj = s.aj.copy()
    k = int(np.flatnonzero(s.ai == s.ai[0])[1])
    aj[k] = aj[0]                                   # two entries at one (row, col)
    with pytest.raises(gpu.MxsError) as e:
        gpu.Matrix.coo(s.nrows, s.ncols, s.ai, aj, s.av)
    assert e.value.status == -4


def _diagonals(n, offsets, seed, integer=False):
    """Square matrix whose entries are every in-range slot of the given
    diagonals (values N(0,1), or small integers)."""
    g = wl.rng(seed)
    ai, aj = [], []
    for o in sorted(offsets):
        i = np.arange(max(0, -o), min(n, n - o))
        ai.append(i)
        aj.append(i + o)
    ai = np.concatenate(ai).astype(np.int32)
    aj = np.concatenate(aj).astype(np.int32)
    order = np.lexsort((aj, ai))
    ai, aj = ai[order], aj[order]
    av = g.integers(-4, 5, ai.size).astype(np.float64) if integer else g.standard_normal(ai.size)
    if integer:
        av[av == 0] = 1.0
    return wl.Coo(n, n, ai, aj, av)


@pytest.mark.parametrize("offsets", [
    [-700, -699, -698, -3, -2, -1, 40, 41, 42],            # runs of three (shared x loads)
    [-5, -4, -3, 0, 1, 2, 3, 4, 5, 9, 10, 11],              # adjacent runs
    [-2, -1, 0, 7, 8],                                      # not all runs of three
    list(range(-150, 150)),                                 # 300 diagonals (offsets not staged)
], ids=["triples", "adjacent_triples", "mixed", "ndiag300"])
@pytest.mark.parametrize("n", [1000, 70000])
def test_dia_offset_structures(gpu, offsets, n):
    """DIA paths chosen by the offset structure against the oracle: FP64 within
    1e-12, integer data bit-exact, FP32 within its rounding bound."""
    a = _diagonals(n, offsets, seed=n + len(offsets))
    A = build(gpu, a, "dia")
    assert A is not None and A.ndiag == len(offsets)
    x = wl.uniform_vector(n, seed=3)
    ref = orc.coo_spmv(n, a.ai, a.aj, a.av, x)
    y = gpu.spmv(A, to_dev(x)).cpu().numpy()
    assert rel_maxnorm(y, ref) <= 1e-12
    ai_ = _diagonals(n, offsets, seed=5, integer=True)
    B = build(gpu, ai_, "dia")
    xi = wl.integer_vector(n, seed=6)
    assert np.array_equal(gpu.spmv(B, to_dev(xi)).cpu().numpy(),
                          orc.coo_spmv(n, ai_.ai, ai_.aj, ai_.av, xi))
    A32 = A.cast(gpu.F32)
    y32 = gpu.spmv(A32, to_dev(x.astype(np.float32))).cpu().numpy().astype(np.float64)
    ref32 = orc.coo_spmv(n, a.ai, a.aj, a.av.astype(np.float32).astype(np.float64),
                         x.astype(np.float32).astype(np.float64))
    assert np.all(np.abs(y32 - ref32) <= row_bound(a, x, U32) + 1e-30)


def _gappy(nrows, seed, lead=37, trail=53, p_empty=0.3, max_len=40, long_rows=()):
    """Rows with 1..max_len entries, about p_empty of them empty, `lead` empty
    rows first and `trail` empty rows last; rows listed in long_rows get 3,000
    entries (they span tiles)."""
    g = wl.rng(seed)
    ncols = 5000
    ai, aj = [], []
    for r in range(lead, nrows - trail):
        k = 3000 if r in long_rows else (0 if g.random() < p_empty else int(g.integers(1, max_len + 1)))
        if k:
            ai.append(np.full(k, r))
            aj.append(np.sort(g.choice(ncols, k, replace=False)))
    ai = np.concatenate(ai).astype(np.int32)
    aj = np.concatenate(aj).astype(np.int32)
    av = g.integers(-3, 4, ai.size).astype(np.float64)
    av[av == 0] = 2.0
    return wl.Coo(nrows, ncols, ai, aj, av)


@pytest.mark.parametrize("long_rows", [(), (500, 501, 2200)], ids=["short", "long"])
def test_coo_empty_rows_inside_and_around_tiles(gpu, long_rows):
    """COO and CSR on rows with gaps (leading, trailing, inside tiles) and rows
    that span several tiles: integer data bit-exact, every empty row zero."""
    a = _gappy(4000, seed=len(long_rows) + 1, long_rows=set(long_rows))
    x = wl.integer_vector(a.ncols, seed=2)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    for fmt in ("coo", "csr"):
        A = build(gpu, a, fmt)
        y = to_dev(np.full(a.nrows, np.nan))
        gpu.spmv(A, to_dev(x), y)
        assert np.array_equal(y.cpu().numpy(), ref), fmt
