"""Pins of the oracle's HPCG preconditioner (symmetric Gauss-Seidel, the
multigrid V-cycle and PCG; Section VII-D) against what the mathematics fixes:
triangular solves by a library routine, the colour-parallel form of the
multicolour sweep, symmetry and definiteness of the V-cycle, its one- and
two-level forms written with library solves, and PCG reducing to CG.

Every pin takes the oracle module as `m`, so the planted-mistake tests can
run it against a mutated copy."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle as orc
import workloads as wl


def csr_of(a):
    return orc.coo_to_csr(a.nrows, a.ai), a.aj, a.av


def sparse_of(a):
    return sp.csr_matrix((a.av, (a.ai, a.aj)), shape=(a.nrows, a.ncols))


def random_dd(n, seed, density=0.1):
    """Random sparse matrix with a dominant diagonal (nonsymmetric pattern)."""
    g = wl.rng(seed)
    M = sp.random(n, n, density=density, random_state=np.random.RandomState(seed), format="coo")
    M = sp.coo_matrix(M + sp.eye(n) * (2.0 + g.random(n)).max() * n * density)
    M = M.tocsr()
    M.sort_indices()
    c = M.tocoo()
    return wl.Coo(n, n, c.row.astype(np.int32), c.col.astype(np.int32), c.data.copy())


def gs_reference(S, order, r, x, direction):
    """One Gauss-Seidel sweep in `order` by a library triangular solve: with
    P the permutation to `order`, B = P S P^T splits into its lower part with
    the diagonal, L + D, and its strict upper part U; the forward sweep
    solves (L + D) y = P r - U P x, the backward one (U + D) y = P r - L P x."""
    order = np.asarray(order)
    B = S[order][:, order].tocsr()
    Lw = sp.tril(B, 0, format="csr")
    Us = sp.triu(B, 1, format="csr")
    Uw = sp.triu(B, 0, format="csr")
    Ls = sp.tril(B, -1, format="csr")
    pr, px = r[order], x[order]
    if direction > 0:
        y = spl.spsolve_triangular(Lw, pr - Us @ px, lower=True)
    else:
        y = spl.spsolve_triangular(Uw, pr - Ls @ px, lower=False)
    out = np.empty_like(x)
    out[order] = y
    return out


@pytest.mark.parametrize("case", ["stencil5", "random60"])
@pytest.mark.parametrize("order_kind", ["natural", "permuted"])
def test_gs_sweeps_are_triangular_solves(case, order_kind, m=orc):
    a = wl.stencil(5) if case == "stencil5" else random_dd(60, seed=3)
    irp, aj, av = csr_of(a)
    S = sparse_of(a)
    g = wl.rng(7)
    r, x = g.standard_normal(a.nrows), g.standard_normal(a.nrows)
    order = (np.arange(a.nrows) if order_kind == "natural" else g.permutation(a.nrows)).astype(np.int32)
    for d in (1, -1):
        st, got = m.gs_sweep(irp, aj, av, order, r, x, d)
        assert st == 0
        want = gs_reference(S, order, r, x, d)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), d
    st, got = m.symgs(irp, aj, av, order, r, x)
    want = gs_reference(S, order, r, gs_reference(S, order, r, x, 1), -1)
    assert st == 0 and np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_gs_zero_diagonal_is_breakdown(m=orc):
    a = wl.Coo(3, 3, np.array([0, 1, 1, 2], np.int32), np.array([0, 0, 2, 2], np.int32),
               np.array([2.0, 1.0, 1.0, 3.0]))
    irp, aj, av = csr_of(a)
    st, _ = m.symgs(irp, aj, av, np.arange(3, dtype=np.int32), np.ones(3), np.zeros(3))
    assert st == orc.BREAKDOWN


@pytest.mark.parametrize("n", [1, 2, 5, 6])
def test_grid_colours_never_couple_and_count(n, m=orc):
    a = wl.stencil(n)
    c = m.grid_colours(n)
    off = a.ai != a.aj
    assert not np.any(c[a.ai[off]] == c[a.aj[off]])
    h = [(n + 1) // 2, n // 2]
    for k in range(8):
        assert np.sum(c == k) == h[k & 1] * h[(k >> 1) & 1] * h[(k >> 2) & 1]
    order = m.colour_order(n)
    assert np.array_equal(np.sort(order), np.arange(n ** 3))
    assert np.array_equal(c[order], np.concatenate([np.full(np.sum(c == k), k)
                                                    for k in m.COLOUR_SWEEP]))
    for k in range(8):
        assert np.all(np.diff(order[c[order] == k]) > 0)
    assert m.COLOUR_SWEEP[-1] == 0 and sorted(m.COLOUR_SWEEP) == list(range(8))


@pytest.mark.parametrize("n", [4, 7])
def test_multicolour_sweep_is_colour_parallel_update(n, m=orc):
    """Within one colour no point reads another, so the sweep equals updating
    all points of a colour at once (a Jacobi step restricted to the colour),
    colours in sweep order, then in reverse."""
    a = wl.stencil(n)
    irp, aj, av = csr_of(a)
    S = sparse_of(a)
    D = S.diagonal()
    Off = S - sp.diags(D)
    c = orc.grid_colours(n)
    g = wl.rng(n)
    r, x = g.standard_normal(n ** 3), g.standard_normal(n ** 3)
    want = x.copy()
    for k in list(orc.COLOUR_SWEEP) + list(reversed(orc.COLOUR_SWEEP)):
        idx = np.flatnonzero(c == k)
        want[idx] = (r[idx] - Off[idx] @ want) / D[idx]
    st, got = m.symgs(irp, aj, av, m.colour_order(n), r, x)
    assert st == 0 and np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("n", [2, 4, 6])
def test_coarse_points_are_even_coordinates(n, m=orc):
    f = m.coarse_points(n)
    mm = n // 2
    for ic, fi in enumerate(f):
        i, j, k = ic % mm, (ic // mm) % mm, ic // (mm * mm)
        assert fi == 2 * i + 2 * j * n + 2 * k * n * n
    assert np.array_equal(np.sort(np.flatnonzero(orc.grid_colours(n) == 0)), f)


def levels_of(n, L):
    out = []
    for l in range(L):
        a = wl.stencil(n >> l)
        out.append((n >> l, *csr_of(a)))
    return out


@pytest.mark.parametrize("n,L", [(8, 2), (16, 3), (16, 4)])
def test_vcycle_symmetric_positive(n, L, m=orc):
    """With identical symmetric sweeps before and after the coarse correction
    and prolongation the transpose of restriction, M^{-1} is symmetric; it is
    positive definite for an SPD operator."""
    lv = levels_of(n, L)
    g = wl.rng(n + L)
    R = g.standard_normal((3, n ** 3))
    Z = [m.mg_vcycle(lv, r) for r in R]
    for i in range(3):
        assert R[i] @ Z[i] > 0
        for j in range(i):
            assert abs(R[i] @ Z[j] - R[j] @ Z[i]) <= 1e-12 * abs(R[i] @ Z[j])


def test_vcycle_one_level_is_one_sweep(m=orc):
    lv = levels_of(6, 1)
    r = wl.rng(2).standard_normal(216)
    _, irp, aj, av = lv[0]
    st, want = orc.symgs(irp, aj, av, orc.colour_order(6), r, np.zeros(216))
    assert np.array_equal(m.mg_vcycle(lv, r), want)


@pytest.mark.parametrize("n", [4, 8])
def test_vcycle_two_levels_by_library_solves(n, m=orc):
    """Two-level cycle written with the triangular solves of gs_reference:
    pre-sweep, injected residual r_c = (r - A z)[coarse], one sweep on the
    coarse grid, z[coarse] += z_c, post-sweep."""
    S = sparse_of(wl.stencil(n))
    Sc = sparse_of(wl.stencil(n // 2))
    order = orc.colour_order(n)
    order_c = orc.colour_order(n // 2)
    r = wl.rng(n).standard_normal(n ** 3)

    def sym(Smat, o, rr, x):
        return gs_reference(Smat, o, rr, gs_reference(Smat, o, rr, x, 1), -1)

    z = sym(S, order, r, np.zeros(n ** 3))
    mm = n // 2
    ic = np.arange(mm ** 3)
    f = 2 * (ic % mm) + 2 * ((ic // mm) % mm) * n + 2 * (ic // (mm * mm)) * n * n
    rc = (r - S @ z)[f]
    zc = sym(Sc, order_c, rc, np.zeros(mm ** 3))
    z[f] += zc
    want = sym(S, order, r, z)
    got = m.mg_vcycle(levels_of(n, 2), r)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("n", [6, 10])
def test_pcg_identity_preconditioner_is_cg(n, m=orc):
    a = wl.stencil(n)
    irp, aj, av = csr_of(a)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, wl.uniform_vector(a.nrows, seed=n))
    st, x, it, rel, tr = m.pcg(irp, aj, av, b, lambda r: r, tol=1e-10, maxit=500)
    st_c, x_c, it_c, rel_c, tr_c = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=500)
    assert st == st_c == 0 and it == it_c
    assert np.max(np.abs(x - x_c)) <= 1e-10 * np.max(np.abs(x_c))
    assert abs(rel - rel_c) <= 1e-6 * rel_c


def test_pcg_with_vcycle_converges_faster_and_to_ones(m=orc):
    """b = A 1, x0 = 0 (HPCG's problem).  The V-cycle cuts the iteration
    count well below CG's, reaches the tolerance in the true residual and
    stays within two iterations of the same cycle with the natural row order
    in each sweep (HPCG's reference order)."""
    n = 16
    lv = levels_of(n, 3)
    _, irp, aj, av = lv[0]
    b = orc.csr_spmv(irp, aj, av, np.ones(n ** 3))
    st, x, it, rel, tr = m.pcg(irp, aj, av, b, lambda r: m.mg_vcycle(lv, r), tol=1e-9)
    st_n, _, it_n, _, _ = m.pcg(irp, aj, av, b,
                                lambda r: m.mg_vcycle(lv, r, [np.arange(k ** 3, dtype=np.int32)
                                                              for k, *_ in lv]), tol=1e-9)
    st_c, _, it_c, _, _ = m.pcg(irp, aj, av, b, lambda r: r, tol=1e-9)
    assert st == st_n == st_c == 0
    assert it <= 0.6 * it_c and abs(it - it_n) <= 2, (it, it_n, it_c)
    assert rel <= 1e-9 and tr <= 2e-9
    assert np.max(np.abs(x - 1.0)) <= 1e-6
