"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a brute-force
dense product, a closed form of the HPCG stencil, an invariant of the formats
of Section III-B or of CG, or a library routine on a case that reduces to it.
"""
import math

import numpy as np
import pytest

import oracle as orc
import workloads as wl

U64 = 2.0 ** -53


def dense(a: wl.Coo) -> np.ndarray:
    d = np.zeros((a.nrows, a.ncols), np.float64)
    d[a.ai, a.aj] = a.av
    return d


def gamma(n):
    return n * U64 / (1 - n * U64)


def stencil_rowcount(n):
    """c_x c_y c_z with c = 2 on a face of that axis (n > 1), 3 inside."""
    c = np.full(n, 3, np.int64)
    if n == 1:
        c[:] = 1
    else:
        c[0] = c[-1] = 2
    return (c[None, None, :] * c[None, :, None] * c[:, None, None]).ravel()


def stencil_spectrum(n):
    t = 1.0 + 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    prod = (t[None, None, :] * t[None, :, None] * t[:, None, None]).ravel()
    return 27.0 - prod


# --------------------------------------------------------------------------
# SpMV, brute force against dense products (Algorithms 1-3)
# --------------------------------------------------------------------------
SHAPES = [(0, 0), (1, 1), (1, 5), (5, 1), (7, 3), (3, 9), (17, 17), (64, 64), (40, 23)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("density", [0.0, 0.15, 0.6, 1.0])
def test_spmv_integer_bruteforce(shape, density):
    m, n = shape
    a = wl.random_coo(m, n, density, seed=m * 131 + n + int(density * 10), integer=True)
    x = wl.integer_vector(n, seed=7)
    want = dense(a) @ x  # integer data: exact in any order
    y_coo = orc.coo_spmv(m, a.ai, a.aj, a.av, x)
    assert np.array_equal(y_coo, want)
    irp = orc.coo_to_csr(m, a.ai)
    assert np.array_equal(orc.csr_spmv(irp, a.aj, a.av, x), want)
    doff, avd = orc.coo_to_dia(m, n, a.ai, a.aj, a.av)
    assert np.array_equal(orc.dia_spmv(m, n, doff, avd, x), want)


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_random_bruteforce_within_bound(shape):
    m, n = shape
    a = wl.random_coo(m, n, 0.4, seed=m + 1000 * n)
    x = wl.uniform_vector(n, seed=3)
    D = dense(a)
    want = D @ x
    mag = np.abs(D) @ np.abs(x)
    L = max(n, 1)
    for y in (orc.coo_spmv(m, a.ai, a.aj, a.av, x),
              orc.csr_spmv(orc.coo_to_csr(m, a.ai), a.aj, a.av, x),
              orc.dia_spmv(m, n, *orc.coo_to_dia(m, n, a.ai, a.aj, a.av), x)):
        assert np.all(np.abs(y - want) <= 2 * gamma(L) * mag + 1e-300)


def test_coo_spmv_overwrites_y_and_empty_rows_are_zero():
    # Algorithm 1 accumulates; the operation is y = A x: rows with no entry give 0.
    a = wl.Coo(4, 4, np.array([1, 1, 3], np.int32), np.array([0, 2, 3], np.int32),
               np.array([2.0, 3.0, 5.0]))
    y = orc.coo_spmv(4, a.ai, a.aj, a.av, np.array([1.0, 10.0, 100.0, 1000.0]))
    assert y.tolist() == [0.0, 302.0, 0.0, 5000.0]


def test_dia_bound_uses_ncols_for_rectangular():
    # Algorithm 3's bound k < N: N is the column count.  A 2x5 matrix with an
    # entry at (1, 4) lies on offset +3, which is valid only because k < ncols.
    a = wl.Coo(2, 5, np.array([0, 1], np.int32), np.array([3, 4], np.int32), np.array([1.0, 2.0]))
    doff, avd = orc.coo_to_dia(2, 5, a.ai, a.aj, a.av)
    assert doff.tolist() == [3]
    x = np.arange(5, dtype=np.float64)
    assert orc.dia_spmv(2, 5, doff, avd, x).tolist() == [3.0, 8.0]


# --------------------------------------------------------------------------
# HPCG stencil closed forms (Section VII-D problem; coefficients 26 / -1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 16])
def test_stencil_times_ones_closed_form(n):
    a = wl.stencil(n)
    assert a.nnz == (3 * n - 2) ** 3
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    want = 27.0 - stencil_rowcount(n)
    assert np.array_equal(b, want)


@pytest.mark.parametrize("n", [2, 3, 5, 6])
def test_stencil_eigenpairs(n):
    a = wl.stencil(n)
    t = np.arange(n)
    for kx, ky, kz in [(1, 1, 1), (n, 1, 2 if n > 1 else 1), (n, n, n), (2, n - 1 or 1, 1)]:
        v = (np.sin(kx * np.pi * (t + 1) / (n + 1))[None, None, :]
             * np.sin(ky * np.pi * (t + 1) / (n + 1))[None, :, None]
             * np.sin(kz * np.pi * (t + 1) / (n + 1))[:, None, None]).ravel()
        lam = 27.0 - np.prod([1 + 2 * math.cos(k * math.pi / (n + 1)) for k in (kx, ky, kz)])
        av = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, v)
        assert np.max(np.abs(av - lam * v)) <= 1e-13 * max(1.0, abs(lam)) * np.max(np.abs(v))


@pytest.mark.parametrize("n", [3, 7, 16])
def test_stencil_integer_x_all_formats_bit_identical(n):
    # Every partial sum is an integer < 2^53, so all formats and any order agree.
    a = wl.stencil(n)
    x = wl.integer_vector(a.ncols, seed=n)
    y = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    s = wl.shuffled(a, seed=1)
    assert np.array_equal(orc.coo_spmv(a.nrows, s.ai, s.aj, s.av, x), y)
    assert np.array_equal(orc.csr_spmv(orc.coo_to_csr(a.nrows, a.ai), a.aj, a.av, x), y)
    doff, avd = orc.coo_to_dia(a.nrows, a.ncols, a.ai, a.aj, a.av)
    assert np.array_equal(orc.dia_spmv(a.nrows, a.ncols, doff, avd, x), y)
    # and the dense product, exact for integers
    assert np.array_equal(dense(a) @ x, y)


# --------------------------------------------------------------------------
# Conversions (Section III-B definitions)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 4, 16])
def test_stencil_csr_and_dia_closed_forms(n):
    a = wl.stencil(n)
    N = a.nrows
    irp = orc.coo_to_csr(N, a.ai)
    assert irp[0] == 0 and irp[-1] == a.nnz
    assert np.array_equal(np.diff(irp), stencil_rowcount(n))
    doff, avd = orc.coo_to_dia(N, N, a.ai, a.aj, a.av)
    want = sorted({dx + n * dy + n * n * dz for dx in (-1, 0, 1) for dy in (-1, 0, 1)
                   for dz in (-1, 0, 1)})
    assert doff.tolist() == want
    assert len(want) == (27 if n >= 3 else 15 if n == 2 else 1)
    assert orc.dia_slots(N, N, doff) == sum(N - abs(o) for o in want)


@pytest.mark.parametrize("shape", SHAPES)
def test_conversions_against_dense_definition(shape):
    m, n = shape
    a = wl.random_coo(m, n, 0.3, seed=11 + m * 7 + n)
    D = dense(a)
    # CSR: irp[r] counts entries in rows < r; row r's columns are its non-zeros
    irp = orc.coo_to_csr(m, a.ai)
    for r in range(m):
        cols = np.nonzero(D[r])[0]
        assert irp[r + 1] - irp[r] == cols.shape[0]
        assert np.array_equal(a.aj[irp[r]:irp[r + 1]], cols)
    # DIA: av[d][i] = D[i, i+off_d] (0 outside), offsets = distinct j-i
    doff, avd = orc.coo_to_dia(m, n, a.ai, a.aj, a.av)
    offs = sorted({int(j) - int(i) for i, j in zip(*np.nonzero(D))})
    assert doff.tolist() == offs
    for d, off in enumerate(offs):
        for i in range(m):
            k = i + off
            want = D[i, k] if 0 <= k < n else 0.0
            assert avd[d * m + i] == want
    # round trips are identity
    assert np.array_equal(orc.csr_to_coo(irp), a.ai)
    bi, bj, bv = orc.dia_to_coo(m, n, doff, avd)
    assert np.array_equal(bi, a.ai) and np.array_equal(bj, a.aj) and np.array_equal(bv, a.av)


def test_dia_to_coo_drops_stored_zeros_of_both_signs():
    doff = np.array([-1, 0], np.int32)
    avd = np.array([9.0, 0.0, -0.0, 1.0, 2.0, 0.0])  # d=-1: rows 0..2; d=0: rows 0..2
    ai, aj, av = orc.dia_to_coo(3, 3, doff, avd)
    # (0,-1) out of range; (1,0)=0.0 and (2,1)=-0.0 dropped; diagonal 1,2 kept, (2,2)=0 dropped
    assert ai.tolist() == [0, 1] and aj.tolist() == [0, 1] and av.tolist() == [1.0, 2.0]


def test_coo_check_statuses():
    ai = np.array([0, 0, 1], np.int32)
    assert orc.coo_check(2, 2, ai, np.array([0, 1, 1], np.int32)) == orc.OK
    assert orc.coo_check(2, 2, ai, np.array([1, 0, 1], np.int32)) == orc.UNSORTED
    assert orc.coo_check(2, 2, ai, np.array([1, 1, 1], np.int32)) == orc.DUPLICATE
    assert orc.coo_check(2, 2, ai, np.array([0, 2, 1], np.int32)) == orc.INDEX_RANGE
    assert orc.coo_check(2, 2, np.array([0, -1, 1], np.int32), ai) == orc.INDEX_RANGE
    assert orc.coo_check(0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32)) == orc.OK


def test_csr_check_statuses():
    aj = np.array([0, 2, 1], np.int32)
    assert orc.csr_check(2, 3, np.array([0, 2, 3], np.int32), aj) == orc.OK
    assert orc.csr_check(2, 3, np.array([0, 2, 2], np.int32), aj) == orc.INDEX_RANGE
    assert orc.csr_check(2, 3, np.array([0, 3, 2], np.int32), aj) == orc.INDEX_RANGE
    assert orc.csr_check(2, 3, np.array([0, 2, 3], np.int32), np.array([2, 0, 1], np.int32)) == orc.UNSORTED
    assert orc.csr_check(2, 3, np.array([0, 2, 3], np.int32), np.array([1, 1, 1], np.int32)) == orc.DUPLICATE


@pytest.mark.parametrize("seed", range(4))
def test_coo_sort_matches_lexsort(seed):
    a = wl.random_coo(50, 37, 0.2, seed=seed)
    s = wl.shuffled(a, seed=seed + 100)
    ai, aj, av = orc.coo_sort(50, 37, s.ai, s.aj, s.av)
    order = np.lexsort((s.aj, s.ai))
    assert np.array_equal(ai, s.ai[order]) and np.array_equal(aj, s.aj[order])
    assert np.array_equal(av, s.av[order])
    assert orc.coo_check(50, 37, ai, aj) == orc.OK


# --------------------------------------------------------------------------
# CG (HPCG solver without preconditioner, Section VII-D)
# --------------------------------------------------------------------------
def spd(n, seed):
    g = wl.rng(seed)
    M = g.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    ai, aj = np.nonzero(A)
    return wl.Coo(n, n, ai.astype(np.int32), aj.astype(np.int32), A[ai, aj]), A


@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (12, 2), (30, 3)])
def test_cg_small_spd_matches_solve(n, seed):
    a, A = spd(n, seed)
    b = wl.uniform_vector(n, seed=seed + 9)
    st, x, it, rel, true_rel = orc.cg(n, a.ai, a.aj, a.av, b, tol=1e-14, maxit=500)
    assert st == orc.OK
    xs = np.linalg.solve(A, b)
    assert np.max(np.abs(x - xs)) <= 1e-12 * np.max(np.abs(xs))
    assert true_rel <= 1e-12


def test_cg_diagonal_distinct_eigenvalues_iteration_count():
    # With m distinct eigenvalues CG terminates in m steps (exact arithmetic).
    vals = np.repeat([1.0, 2.0, 4.0, 8.0], 5)
    n = vals.shape[0]
    a = wl.Coo(n, n, np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), vals)
    b = wl.uniform_vector(n, seed=1)
    st, x, it, rel, _ = orc.cg(n, a.ai, a.aj, a.av, b, tol=1e-12, maxit=50)
    assert st == orc.OK and it == 4
    assert np.max(np.abs(x - b / vals)) <= 1e-12


def test_cg_first_iterate_closed_form():
    # x1 = (b.b)/(b.Ab) b for x0 = 0.
    a, A = spd(9, 4)
    b = wl.uniform_vector(9, seed=2)
    st, x1, it, _, _ = orc.cg(9, a.ai, a.aj, a.av, b, tol=0.0, maxit=1)
    assert it == 1 and st == orc.NOT_CONVERGED
    want = (b @ b) / (b @ (A @ b)) * b
    assert np.max(np.abs(x1 - want)) <= 1e-14 * np.max(np.abs(want))


def test_cg_error_a_norm_non_increasing():
    a, A = spd(25, 5)
    b = wl.uniform_vector(25, seed=3)
    xs = np.linalg.solve(A, b)
    prev = np.inf
    for k in range(1, 26):
        _, x, _, _, _ = orc.cg(25, a.ai, a.aj, a.av, b, tol=0.0, maxit=k)
        e = x - xs
        en = math.sqrt(max(e @ A @ e, 0.0))
        assert en <= prev * (1 + 1e-10) + 1e-13
        prev = en


@pytest.mark.parametrize("n,tol", [(8, 1e-9), (16, 1e-9)])
def test_cg_stencil_recovers_ones_within_kappa_bound(n, tol):
    # HPCG's verification: b = A*1 must give x -> 1.
    a = wl.stencil(n)
    N = a.nrows
    b = 27.0 - stencil_rowcount(n).astype(np.float64)  # A*1, closed form
    st, x, it, rel, true_rel = orc.cg(N, a.ai, a.aj, a.av, b, tol=tol, maxit=10000)
    lam = stencil_spectrum(n)
    kappa = lam.max() / lam.min()
    bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2 * math.sqrt(kappa) / tol))
    assert st == orc.OK and 1 <= it <= bound
    assert rel <= tol
    assert np.max(np.abs(x - 1.0)) <= kappa * tol * 10
    # true residual measured by a library product, not by the oracle
    import scipy.sparse as sp
    A = sp.csr_matrix((a.av, (a.ai, a.aj)), shape=(N, N))
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= tol * 10


def test_cg_statuses():
    a, _ = spd(6, 1)
    z = np.zeros(6)
    st, x, it, rel, _ = orc.cg(6, a.ai, a.aj, a.av, z)
    assert st == orc.OK and it == 0 and not x.any()
    bad = z.copy()
    bad[2] = np.nan
    assert orc.cg(6, a.ai, a.aj, a.av, bad)[0] == orc.NONFINITE
    # indefinite: diag(1, -1) with b = (1, 1) gives p.Ap = 0
    ind = wl.Coo(2, 2, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    assert orc.cg(2, ind.ai, ind.aj, ind.av, np.ones(2))[0] == orc.BREAKDOWN
    st, _, it, _, _ = orc.cg(6, a.ai, a.aj, a.av, wl.uniform_vector(6, 1), tol=1e-30, maxit=2)
    assert st == orc.NOT_CONVERGED and it == 2


# --------------------------------------------------------------------------
# Mixed refinement
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 16])
def test_mixed_refinement_reaches_fp64_residual(n):
    a = wl.stencil(n)
    N = a.nrows
    b = 27.0 - stencil_rowcount(n).astype(np.float64)
    st, x, outer, inner, true_rel = orc.mixed_ir(N, a.ai, a.aj, a.av, b, tol=1e-10,
                                                 inner_rtol=1e-4)
    assert st == orc.OK
    assert 1 <= outer <= 5 and inner >= outer
    import scipy.sparse as sp
    A = sp.csr_matrix((a.av, (a.ai, a.aj)), shape=(N, N))
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-10
    assert np.max(np.abs(x - 1.0)) <= 1e-8


def test_mixed_refinement_on_spd_matches_solve():
    a, A = spd(20, 8)
    b = wl.uniform_vector(20, seed=4)
    st, x, outer, inner, true_rel = orc.mixed_ir(20, a.ai, a.aj, a.av, b, tol=1e-12,
                                                 inner_rtol=1e-3)
    assert st == orc.OK and outer >= 2  # FP32 alone cannot reach 1e-12
    xs = np.linalg.solve(A, b)
    assert np.max(np.abs(x - xs)) <= 1e-10 * np.max(np.abs(xs))


# --------------------------------------------------------------------------
# Mixed CG with reliable updates
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,delta", [(5, 0.1), (16, 0.1), (16, 1e-3), (24, 0.5)])
def test_reliable_update_reaches_fp64_residual(n, delta):
    """FP32 recurrences with FP64 residual replacement reach a residual FP32
    alone cannot, within a small multiple of the FP64 CG iteration bound."""
    a = wl.stencil(n)
    N = a.nrows
    b = 27.0 - stencil_rowcount(n).astype(np.float64)
    tol = 1e-10
    st, x, upd, it, true_rel = orc.mixed_ru(N, a.ai, a.aj, a.av, b, tol=tol, delta=delta)
    lam = stencil_spectrum(n)
    kappa = lam.max() / lam.min()
    bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2 * math.sqrt(kappa) / tol))
    assert st == orc.OK and upd >= 1 and 1 <= it <= 1.5 * bound
    import scipy.sparse as sp
    A = sp.csr_matrix((a.av, (a.ai, a.aj)), shape=(N, N))
    r = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert r <= tol and abs(r - true_rel) <= 1e-3 * tol
    assert np.max(np.abs(x - 1.0)) <= kappa * tol * 10


def test_reliable_update_on_spd_matches_solve():
    a, A = spd(20, 8)
    b = wl.uniform_vector(20, seed=4)
    st, x, upd, it, true_rel = orc.mixed_ru(20, a.ai, a.aj, a.av, b, tol=1e-12, delta=0.1)
    assert st == orc.OK and upd >= 2  # FP32 alone cannot reach 1e-12
    xs = np.linalg.solve(A, b)
    assert np.max(np.abs(x - xs)) <= 1e-10 * np.max(np.abs(xs))


def test_reliable_update_first_iterate():
    """One iteration without an update: x1 = (r.r / r.Ar) r in FP32."""
    a, A = spd(12, 5)
    b = wl.uniform_vector(12, seed=7)
    st, x, upd, it, _ = orc.mixed_ru(12, a.ai, a.aj, a.av, b, tol=1e-30, delta=1e-30, maxit=1)
    assert st == orc.NOT_CONVERGED and upd == 0 and it == 1
    x1 = (b @ b) / (b @ A @ b) * b
    assert np.max(np.abs(x - x1)) <= 1e-6 * np.max(np.abs(x1))


def test_reliable_update_statuses():
    a, A = spd(6, 1)
    z = np.zeros(6)
    st, x, upd, it, _ = orc.mixed_ru(6, a.ai, a.aj, a.av, z)
    assert st == orc.OK and it == 0 and upd == 0 and not x.any()
    bad = z.copy()
    bad[2] = np.inf
    assert orc.mixed_ru(6, a.ai, a.aj, a.av, bad)[0] == orc.NONFINITE
    ind = wl.Coo(2, 2, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    assert orc.mixed_ru(2, ind.ai, ind.aj, ind.av, np.ones(2))[0] == orc.BREAKDOWN
    b = wl.uniform_vector(6, 1)
    st, x, upd, it, true_rel = orc.mixed_ru(6, a.ai, a.aj, a.av, b, tol=1e-30, maxit=3)
    assert st == orc.NOT_CONVERGED and it == 3
    # the reported residual is that of the returned x (pending correction folded in)
    assert true_rel == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b), rel=1e-6)


# --------------------------------------------------------------------------
# Split matrices: the band of diagonals
# --------------------------------------------------------------------------
def _coo_from_dense(M):
    ai, aj = np.nonzero(M)
    return wl.Coo(M.shape[0], M.shape[1], ai.astype(np.int32), aj.astype(np.int32), M[ai, aj])


def test_split_band_hand_built():
    """6x6: main diagonal full (6 of 6 slots), offset +1 with 2 of 5, offset
    -2 with 3 of 4.  The thresholds select exactly the diagonals whose fill
    reaches them (equality included)."""
    M = np.zeros((6, 6))
    M[np.arange(6), np.arange(6)] = 1.0
    M[0, 1] = M[3, 4] = 2.0
    M[2, 0] = M[3, 1] = M[5, 3] = 3.0
    a = _coo_from_dense(M)
    band = lambda f: orc.split_offsets(6, 6, a.ai, a.aj, f).tolist()
    assert band(0.5) == [-2, 0]
    assert band(0.4) == [-2, 0, 1]
    assert band(0.8) == [0]
    assert band(1.0) == [0]
    assert band(0.0) == [-2, 0, 1]


def test_split_band_full_rectangular_and_stencil():
    """A full 3x5 matrix: every one of its 7 diagonals is full, so all are
    kept even at min_fill = 1 (this fixes the slot count of each diagonal of a
    rectangular matrix); the 27-point stencil's diagonals are all at least
    half full."""
    a = _coo_from_dense(np.arange(1.0, 16.0).reshape(3, 5))
    assert orc.split_offsets(3, 5, a.ai, a.aj, 1.0).tolist() == list(range(-2, 5))
    a = _coo_from_dense(np.arange(1.0, 16.0).reshape(5, 3))
    assert orc.split_offsets(5, 3, a.ai, a.aj, 1.0).tolist() == list(range(-4, 3))
    s = wl.stencil(16)
    assert np.array_equal(orc.split_offsets(s.nrows, s.ncols, s.ai, s.aj, 0.5),
                          orc.dia_offsets(s.nrows, s.ncols, s.ai, s.aj))


def test_split_band_random_matrix_is_empty():
    a = wl.random_coo(200, 300, 0.01, seed=4)
    assert orc.split_offsets(200, 300, a.ai, a.aj, 0.5).size == 0
    assert orc.split_offsets(200, 300, a.ai, a.aj, 0.0).size == \
        np.unique(a.aj.astype(np.int64) - a.ai).size


# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 5, 16])
def test_features_stencil_closed_form(n):
    a = wl.stencil(n)
    f = orc.features(a.nrows, a.ncols, a.ai, a.aj)
    N = n ** 3
    m = (3 * n - 2) / n
    assert f[0] == N and f[1] == (3 * n - 2) ** 3
    assert f[2] == pytest.approx(m ** 3, rel=1e-15)
    assert f[3] == pytest.approx(((9 * n - 10) / n) ** 3 - m ** 6, rel=1e-12)
    assert f[4] == 27 and f[5] == 27
    assert f[6] == pytest.approx((3 * n - 2) ** 3 / (27 * N), rel=1e-15)
    assert f[7] == pytest.approx((n * n + n + 1) / N, rel=1e-15)


def test_features_banded_closed_form():
    a = wl.banded(5000, ndiag=11, max_offset=300, seed=9)
    f = orc.features(a.nrows, a.ncols, a.ai, a.aj)
    offs = np.unique(a.aj.astype(np.int64) - a.ai)
    assert f[5] == 11
    assert f[1] == sum(5000 - abs(int(o)) for o in offs)
    assert f[6] == pytest.approx(f[1] / (11 * 5000), rel=1e-15)
    assert f[7] == pytest.approx(np.max(np.abs(offs)) / 5000, rel=1e-15)
    assert f[4] <= 11


# --------------------------------------------------------------------------
# MLP 8-64-64-7
# --------------------------------------------------------------------------
def test_mlp_zero_weights_uniform_softmax():
    w = np.zeros(orc.NPARAM)
    X = wl.rng(1).standard_normal((10, 8))
    K = orc.NCLASS
    y = np.array([0, 1, 2, 3, 4, 5, 6, 0, 1, 6], np.int32)
    loss, g = orc.mlp_loss_grad(w, X, y)
    assert loss == pytest.approx(math.log(K), rel=1e-15)
    # dL/db3 = mean(p - onehot) with p = 1/K
    onehot = np.eye(K)[y]
    assert np.allclose(g[-K:], (1 / K - onehot).mean(axis=0), atol=1e-15)
    assert not g[:-K].any()  # hidden layers are all zero, so no other gradient


def test_mlp_forward_special_network():
    # h1 = relu(x) in units 0..7, h2 = h1, logits = (h2_0, ..., h2_6) + b3.
    K = orc.NCLASS
    w = np.zeros(orc.NPARAM)
    for i in range(8):
        w[i * 64 + i] = 1.0                       # W1
        w[512 + 64 + i * 64 + i] = 1.0            # W2
    for c in range(K):
        w[512 + 64 + 4096 + 64 + c * K + c] = 1.0  # W3
    w[-K:] = [0.5, -0.5, 2.0, 1.0, -1.0, 0.25, -2.0]
    X = np.array([[1.0, -2.0, 3.0, 0, 2.0, 0, 0, 0], [-1.0, 4.0, -3.0, 1, 1, 1, 1, 1]])
    z = orc.mlp_forward(w, X)
    assert z.tolist() == [[1.5, -0.5, 5.0, 1.0, 1.0, 0.25, -2.0], [0.5, 3.5, 2.0, 2.0, 0.0, 1.25, -1.0]]


def test_mlp_gradient_matches_finite_differences():
    g0 = wl.rng(3)
    w = g0.standard_normal(orc.NPARAM) * 0.3
    X = g0.standard_normal((16, 8))
    y = g0.integers(0, orc.NCLASS, 16).astype(np.int32)
    loss, g = orc.mlp_loss_grad(w, X, y)
    h = 1e-6
    idx = np.concatenate([np.arange(0, 512, 37), np.arange(512, 576, 5), np.arange(576, 4672, 97),
                          np.arange(4672, 4736, 7), np.arange(4736, orc.NPARAM, 11)])
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (orc.mlp_loss_grad(wp, X, y)[0] - orc.mlp_loss_grad(wm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, i


def test_adam_first_step_is_signed_lr():
    # At t = 1 the bias-corrected moments are g and g^2: step = lr*g/(|g|+eps).
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.ones(4)
    m = np.zeros(4)
    v = np.zeros(4)
    orc.adam_step(w, m, v, g, lr=0.1, t=1)
    assert np.allclose(w, 1.0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_stencil_kappa_closed_form_matches_dense_spectrum():
    """The condition number used by the solution bars of the GPU tests: the
    closed form equals the dense eigen-decomposition on small grids, and
    gives the figures 39.0, 2,248 and 5,032 at 16^3, 128^3 and 192^3."""
    from _cases import stencil_kappa
    for n in (2, 3, 5):
        a = wl.stencil(n)
        D = np.zeros((a.nrows, a.ncols))
        D[a.ai, a.aj] = a.av
        lam = np.linalg.eigvalsh(D)
        assert stencil_kappa(n) == pytest.approx(lam.max() / lam.min(), rel=1e-12)
    assert round(stencil_kappa(16), 1) == 39.0
    assert round(stencil_kappa(128)) == 2248 and round(stencil_kappa(192)) == 5032
