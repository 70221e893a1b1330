"""Pins of the oracle's padded formats, ELL and SELL-C-sigma (further formats
of Section IX): a hand-built layout, the two special cases that reduce
SELL-C-sigma to CSR (C = 1) and to ELL (C = nrows, sigma = 1), dense brute
force on integer data, the sort's properties, stencil closed forms and
round trips back to CSR.  Pins take the oracle module as `m` so planted
mistakes can run against a mutated copy."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl


def csr_of(a):
    return orc.coo_to_csr(a.nrows, a.ai), a.aj, a.av


def hand4():
    # rows: 0: (0,1) (0,3); 1: (1,0); 2: empty; 3: (3,0) (3,2) (3,3)
    ai = np.array([0, 0, 1, 3, 3, 3], np.int32)
    aj = np.array([1, 3, 0, 0, 2, 3], np.int32)
    av = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    return wl.Coo(4, 4, ai, aj, av)


def test_ell_hand_built_layout(m=orc):
    irp, aj, av = csr_of(hand4())
    K, col, val = m.csr_to_ell(irp, aj, av)
    assert K == 3
    # column-major: slot k of row i at k*4 + i
    assert col.tolist() == [1, 0, -1, 0,  3, -1, -1, 2,  -1, -1, -1, 3]
    assert val.tolist() == [1.0, 3.0, 0.0, 4.0,  2.0, 0.0, 0.0, 5.0,  0.0, 0.0, 0.0, 6.0]


def test_sell_hand_built_layout(m=orc):
    irp, aj, av = csr_of(hand4())
    perm, cs, col, val = m.csr_to_sell(irp, aj, av, 2, 4)
    # one window of 4 rows sorted by length, stable: rows 3 (3), 0 (2), 1 (1), 2 (0)
    assert perm.tolist() == [3, 0, 1, 2]
    # slices of 2: {3, 0} width 3, {1, 2} width 1
    assert cs.tolist() == [0, 6, 8]
    assert col.tolist() == [0, 1,  2, 3,  3, -1,   0, -1]
    assert val.tolist() == [4.0, 1.0,  5.0, 2.0,  6.0, 0.0,  3.0, 0.0]


CASES = [("stencil6", wl.stencil(6)), ("random37x53", wl.random_coo(37, 53, 0.3, seed=2)),
         ("zipf3000", wl.zipf_rows(3000, seed=4)), ("block300", wl.block_random(300, seed=5)),
         ("empty", wl.Coo(5, 7, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0)))]


@pytest.mark.parametrize("name,a", CASES, ids=[c[0] for c in CASES])
def test_sell_special_cases_reduce_to_csr_and_ell(name, a, m=orc):
    irp, aj, av = csr_of(a)
    perm, cs, col, val = m.csr_to_sell(irp, aj, av, 1, 1)
    assert np.array_equal(perm, np.arange(a.nrows)) and np.array_equal(cs, irp.astype(np.int64))
    assert np.array_equal(col, aj) and np.array_equal(val, av)
    if a.nrows:
        K, ecol, evals = m.csr_to_ell(irp, aj, av)
        perm, cs, col, val = m.csr_to_sell(irp, aj, av, a.nrows, 1)
        assert cs.tolist() == [0, K * a.nrows]
        assert np.array_equal(col, ecol) and np.array_equal(val, evals)


@pytest.mark.parametrize("C,sigma", [(1, 1), (4, 1), (4, 8), (64, 64), (64, 4096), (3, 7)])
@pytest.mark.parametrize("shape,density", [((17, 17), 0.3), ((40, 25), 0.2), ((70, 70), 0.05)])
def test_spmv_integer_bruteforce(C, sigma, shape, density, m=orc):
    g = wl.rng(shape[0] + C + sigma)
    D = (g.random(shape) < density) * g.integers(-5, 6, shape)
    ai, aj = np.nonzero(D)
    a = wl.Coo(shape[0], shape[1], ai.astype(np.int32), aj.astype(np.int32), D[ai, aj].astype(float))
    irp, aj_, av = csr_of(a)
    x = g.integers(-7, 8, shape[1]).astype(float)
    want = D @ x
    K, col, val = m.csr_to_ell(irp, aj_, av)
    assert np.array_equal(m.ell_spmv(a.nrows, K, col, val, x), want)
    perm, cs, scol, sval = m.csr_to_sell(irp, aj_, av, C, sigma)
    assert np.array_equal(m.sell_spmv(a.nrows, C, perm, cs, scol, sval, x), want)


@pytest.mark.parametrize("sigma", [1, 2, 64, 1000, 5000])
def test_sell_perm_sorts_windows_stably(sigma, m=orc):
    a = wl.zipf_rows(3000, seed=9)
    irp = orc.coo_to_csr(a.nrows, a.ai)
    lens = np.diff(irp)
    perm, cs = m.sell_layout(irp, 64, sigma)
    assert np.array_equal(np.sort(perm), np.arange(a.nrows))
    for w0 in range(0, a.nrows, sigma):
        win = perm[w0:w0 + sigma]
        assert np.array_equal(np.sort(win), np.arange(w0, min(w0 + sigma, a.nrows)))
        want = w0 + np.argsort(-lens[w0:w0 + sigma], kind="stable")
        assert np.array_equal(win, want)
    for s in range(len(cs) - 1):
        assert cs[s + 1] - cs[s] == 64 * lens[perm[s * 64:(s + 1) * 64]].max()


@pytest.mark.parametrize("n", [1, 2, 3, 8])
def test_stencil_ell_closed_form(n, m=orc):
    a = wl.stencil(n)
    irp, aj, av = csr_of(a)
    K, col, val = m.csr_to_ell(irp, aj, av)
    assert K == min(n, 3) ** 3
    assert int(np.sum(col < 0)) == K * n ** 3 - (3 * n - 2) ** 3


@pytest.mark.parametrize("name,a", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("C,sigma", [(64, 1), (64, 256), (5, 3)])
def test_round_trips_to_csr(name, a, C, sigma, m=orc):
    irp, aj, av = csr_of(a)
    if a.nrows:
        K, col, val = m.csr_to_ell(irp, aj, av)
        r = m.ell_to_csr(a.nrows, K, col, val)
        assert all(np.array_equal(u, v) for u, v in zip(r, (irp, aj, av)))
    perm, cs, col, val = m.csr_to_sell(irp, aj, av, C, sigma)
    r = m.sell_to_csr(a.nrows, C, perm, cs, col, val)
    assert all(np.array_equal(u, v) for u, v in zip(r, (irp, aj, av)))


# ------------------------------------------------------------------ HYB
def test_hyb_width_rule_hand_built(m=orc):
    # 9000 rows: 3000 with 5 entries, 3000 with 2, 3000 with 1.  need =
    # max(4096, 3000) = 4096 rows with >= k entries: k = 2 (6000 rows), not
    # k = 3 (3000 rows).
    lens = np.repeat([5, 2, 1], 3000)
    irp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    assert m.hyb_width(irp) == 2
    # fewer than 4096 rows: every row must reach k -> the shortest row
    irp_small = np.concatenate([[0], np.cumsum([4, 3, 7])]).astype(np.int32)
    assert m.hyb_width(irp_small) == 3
    assert m.hyb_width(np.zeros(6, np.int32)) == 0


@pytest.mark.parametrize("name,a", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("K", [None, 0, 1, 3, 100])
def test_hyb_partition_and_spmv(name, a, K, m=orc):
    """ELL part + COO remainder hold exactly the matrix's entries (each row's
    first K in ELL), and their products sum to the matrix's on integer
    data."""
    irp, aj, av = csr_of(a)
    K_, ecol, evals, ri, rj, rv = m.csr_to_hyb(irp, aj, av, K)
    if K is None:
        assert K_ == m.hyb_width(irp)
    lens = np.diff(irp)
    assert ri.size == int(np.maximum(lens - K_, 0).sum())
    e_irp, e_aj, e_av = orc.ell_to_csr(a.nrows, K_, ecol, evals) if a.nrows else (irp, aj, av)
    # the union, merged row by row, is the original CSR
    rows = []
    for i in range(a.nrows):
        e = list(zip(e_aj[e_irp[i]:e_irp[i + 1]], e_av[e_irp[i]:e_irp[i + 1]]))
        rsel = ri == i
        r = list(zip(rj[rsel], rv[rsel]))
        assert len(e) == min(lens[i], K_)
        rows += e + r
    if a.nrows:
        assert np.array_equal(np.array([c for c, _ in rows], np.int32), aj)
        assert np.array_equal(np.array([v for _, v in rows]), av)
    g = wl.rng(a.nrows + 7)
    x = g.integers(-6, 7, a.ncols).astype(float)
    D = np.zeros((a.nrows, a.ncols))
    D[a.ai, a.aj] = np.round(a.av * 4)
    iv = np.round(evals * 4)
    y = m.ell_spmv(a.nrows, K_, ecol, iv, x) if a.nrows else np.zeros(0)
    y = y + (orc.coo_spmv(a.nrows, ri, rj, np.round(rv * 4), x) if ri.size else 0.0)
    assert np.array_equal(y, D @ x)
