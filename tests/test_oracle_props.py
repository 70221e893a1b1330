"""Property tests of the oracle's containers and conversions on random
matrices (hypothesis): shapes from 0x0 to 40x40, any density, entries in any
order.  What the definitions of Section III-B fix: sorting is a permutation
into (row, col) order; CSR row pointers are the prefix sums of the row
counts; COO -> CSR -> COO, COO -> DIA -> COO, CSR -> ELL -> CSR and
CSR -> SELL -> CSR are identities; DIA offsets are the distinct j - i in
ascending order; every format's product equals the dense product exactly on
integer data (all partial sums are small integers)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle as orc

SETTINGS = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@st.composite
def matrices(draw):
    """(nrows, ncols, ai, aj, av) with distinct positions in random order and
    non-zero integer values in [-9, 9]."""
    nrows = draw(st.integers(0, 40))
    ncols = draw(st.integers(0, 40))
    cells = nrows * ncols
    nnz = draw(st.integers(0, min(cells, 200)))
    seed = draw(st.integers(0, 2 ** 32 - 1))
    g = np.random.Generator(np.random.PCG64(seed))
    pos = g.choice(cells, nnz, replace=False) if nnz else np.zeros(0, np.int64)
    ai = (pos // max(ncols, 1)).astype(np.int32)
    aj = (pos % max(ncols, 1)).astype(np.int32)
    av = g.integers(1, 10, nnz).astype(np.float64) * g.choice([-1.0, 1.0], nnz)
    return nrows, ncols, ai, aj, av


def dense(nrows, ncols, ai, aj, av):
    D = np.zeros((nrows, ncols))
    D[ai, aj] = av
    return D


@SETTINGS
@given(matrices())
def test_sort_is_a_permutation_into_row_col_order(m):
    nrows, ncols, ai, aj, av = m
    si, sj, sv = orc.coo_sort(nrows, ncols, ai, aj, av)
    key = si.astype(np.int64) * max(ncols, 1) + sj
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(dense(nrows, ncols, si, sj, sv), dense(nrows, ncols, ai, aj, av))
    assert orc.coo_check(nrows, ncols, si, sj) == 0


@SETTINGS
@given(matrices())
def test_csr_row_pointers_and_round_trip(m):
    nrows, ncols, ai, aj, av = m
    ai, aj, av = orc.coo_sort(nrows, ncols, ai, aj, av)
    irp = orc.coo_to_csr(nrows, ai)
    assert irp[0] == 0 and irp[-1] == ai.size and np.all(np.diff(irp) >= 0)
    assert np.array_equal(np.diff(irp), np.bincount(ai, minlength=nrows))
    assert np.array_equal(orc.csr_to_coo(irp), ai)
    assert orc.csr_check(nrows, ncols, irp, aj) == 0


@SETTINGS
@given(matrices())
def test_dia_offsets_and_round_trip(m):
    nrows, ncols, ai, aj, av = m
    ai, aj, av = orc.coo_sort(nrows, ncols, ai, aj, av)
    doff, av_dia = orc.coo_to_dia(nrows, ncols, ai, aj, av)
    assert np.array_equal(doff, np.unique(aj.astype(np.int64) - ai))
    bi, bj, bv = orc.dia_to_coo(nrows, ncols, doff, av_dia)
    assert np.array_equal(bi, ai) and np.array_equal(bj, aj) and np.array_equal(bv, av)
    # slots outside the matrix and not holding an entry are +0.0
    stored = dense(nrows, ncols, ai, aj, av)
    for d, o in enumerate(doff):
        for i in range(nrows):
            j = i + o
            v = av_dia[d * nrows + i]
            assert v == (stored[i, j] if 0 <= j < ncols else 0.0)


@SETTINGS
@given(matrices(), st.integers(1, 8), st.integers(1, 64))
def test_ell_and_sell_round_trips(m, C, sigma):
    nrows, ncols, ai, aj, av = m
    ai, aj, av = orc.coo_sort(nrows, ncols, ai, aj, av)
    irp = orc.coo_to_csr(nrows, ai)
    K, col, val = orc.csr_to_ell(irp, aj, av)
    assert K == (int(np.diff(irp).max()) if nrows else 0)
    e_irp, e_aj, e_av = orc.ell_to_csr(nrows, K, col, val)
    assert np.array_equal(e_irp, irp) and np.array_equal(e_aj, aj) and np.array_equal(e_av, av)
    perm, cs, scol, sval = orc.csr_to_sell(irp, aj, av, C, sigma)
    assert sorted(perm.tolist()) == list(range(nrows))
    s_irp, s_aj, s_av = orc.sell_to_csr(nrows, C, perm, cs, scol, sval)
    assert np.array_equal(s_irp, irp) and np.array_equal(s_aj, aj) and np.array_equal(s_av, av)


@SETTINGS
@given(matrices(), st.integers(0, 2 ** 32 - 1))
def test_every_format_equals_the_dense_product_on_integer_data(m, seed):
    nrows, ncols, ai, aj, av = m
    ai, aj, av = orc.coo_sort(nrows, ncols, ai, aj, av)
    x = np.random.Generator(np.random.PCG64(seed)).integers(-8, 9, ncols).astype(np.float64)
    ref = dense(nrows, ncols, ai, aj, av) @ x if nrows and ncols else np.zeros(nrows)
    irp = orc.coo_to_csr(nrows, ai)
    assert np.array_equal(orc.coo_spmv(nrows, ai, aj, av, x), ref)
    assert np.array_equal(orc.csr_spmv(irp, aj, av, x), ref)
    doff, av_dia = orc.coo_to_dia(nrows, ncols, ai, aj, av)
    assert np.array_equal(orc.dia_spmv(nrows, ncols, doff, av_dia, x), ref)
    K, col, val = orc.csr_to_ell(irp, aj, av)
    assert np.array_equal(orc.ell_spmv(nrows, K, col, val, x), ref)
