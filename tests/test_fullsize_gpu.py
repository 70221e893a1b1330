"""Parity at the benchmark's full sizes, in the configuration it times.

* 128^3 stencil (2,097,152 rows, 55,742,968 entries): the device-built
  matrix equals the host generator's bit for bit; SpMV in every format
  (COO, CSR, DIA, ELL, SELL-64-4096, HYB)
  within 1e-12 of the oracle over the whole vector; CG to 1e-9 in every
  format against the oracle's stored run (iterations within 2, sampled x).
* Zipf and banded, 4,000,000 rows: SpMV in every accepted format against the
  oracle on 2,000 seeded rows.
* 192^3 stencil (7,077,888 rows): FP64 CG, mixed refinement and FP32 CG
  with FP64 reliable updates (update factors 0.01 and 0.1, DIA and CSR) to
  1e-10 against the oracle's stored runs of the same methods at 4,098
  sampled rows.

Solution bars.  With b = A*1 the exact solution is x* = 1, and for any x
the error obeys ||x - x*||_2 / ||x*||_2 <= kappa ||b - A x||_2 / ||b||_2
(kappa = lambda_max / lambda_min from the stencil's closed-form spectrum):
that inequality is checked over the whole vector.  Two solutions that both
reach tolerance tol are then within 2 kappa tol of each other in that norm;
the sampled entries are held to the same 2 kappa tol in the max norm, and
so is max |x - 1| (the error of these solves is smooth, so its largest entry
is close to its root mean square; measured errors are about 1e-11).
* 128^3 PCG with HPCG's 4-level multigrid V-cycle against the oracle's run.

Stored oracle results come from tests/golden/make_golden.py.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import rel_maxnorm, stencil_kappa

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    return json.load(open(os.path.join(GOLDEN, name + ".json")))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_solution(x, n, tol, true_rel_resid, g, what):
    """The solution bars above: the kappa inequality over the whole vector,
    then max |x - 1| and the sampled distance to the oracle's solution within
    2 kappa tol."""
    import torch
    kappa = stencil_kappa(n)
    e = x - 1.0
    rel2 = float(torch.linalg.vector_norm(e) / math.sqrt(x.numel()))
    assert rel2 <= kappa * true_rel_resid * 1.01 + 1e-14, (what, rel2, kappa, true_rel_resid)
    bar = 2 * kappa * tol
    assert float(e.abs().max()) <= bar, (what, float(e.abs().max()), bar)
    idx = torch.tensor(g["sample_idx"], device=x.device)
    xo = np.array(g["x_sample"])
    err = np.max(np.abs(x[idx].cpu().numpy() - xo)) / np.max(np.abs(xo))
    assert err <= bar, (what, err, bar)
    return err


def formats_of(mxs, A):
    out = {"coo": A}
    for f in ("csr", "dia", "ell", "sell", "hyb"):
        try:
            out[f] = (A.to_sell(4096) if f == "sell" else A.to_hyb() if f == "hyb" else
                      A.convert(f))
        except mxs.MxsError as e:
            if e.status != -5:
                raise
    for B in out.values():
        B.optimize()
    return out


@pytest.fixture(scope="module")
def stencil128(gpu):
    a = wl.stencil(128)
    A = gpu.stencil(128, fmt="coo")
    mats = formats_of(gpu, A)
    yield a, mats
    for B in mats.values():
        B.close()


def test_stencil128_device_matrix_is_the_generator(gpu, stencil128):
    a, mats = stencil128
    ai, aj, av = mats["coo"].export()
    assert np.array_equal(ai, a.ai) and np.array_equal(aj, a.aj) and np.array_equal(av, a.av)
    assert mats["dia"].ndiag == 27


def test_stencil128_spmv_full_vector(gpu, stencil128):
    a, mats = stencil128
    x = wl.uniform_vector(a.ncols, seed=1)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    xd = to_dev(x)
    for fmt, B in mats.items():
        y = gpu.spmv(B, xd).cpu().numpy()
        assert rel_maxnorm(y, ref) <= 1e-12, fmt


def test_stencil128_every_implementation_full_vector(gpu, stencil128):
    """Every SpMV implementation of COO, CSR and DIA (DIA planned with its
    row-blocked copy, so that all three are reachable) at the benchmark's
    size, the whole vector against the oracle."""
    a, mats = stencil128
    x = wl.uniform_vector(a.ncols, seed=2)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    xd = to_dev(x)
    D = mats["coo"].convert("dia").optimize(gpu.PLAN_DIA_BLOCKED)
    for fmt, B in (("coo", mats["coo"]), ("csr", mats["csr"]), ("dia", D)):
        default = B.impl
        ran = []
        for i in range(B.impl_count()):
            try:
                B.impl = i
            except gpu.MxsError as e:
                assert e.status == -10
                continue
            y = gpu.spmv(B, xd).cpu().numpy()
            assert rel_maxnorm(y, ref) <= 1e-12, (fmt, i)
            ran.append(i)
        B.impl = default
        assert {"coo": {0, 1}, "csr": {0, 1, 2, 3, 5}, "dia": {0, 1, 2}}[fmt] <= set(ran), (fmt, ran)
    D.close()


def test_stencil128_spmv_integer_data_bit_exact(gpu, stencil128):
    a, mats = stencil128
    x = wl.integer_vector(a.ncols, seed=4)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    xd = to_dev(x)
    for fmt, B in mats.items():
        assert np.array_equal(gpu.spmv(B, xd).cpu().numpy(), ref), fmt


def test_stencil128_cg_matches_oracle_run(gpu, stencil128):
    import torch
    g = golden("cg_stencil128_tol1e-9")
    a, mats = stencil128
    b = gpu.spmv(mats["csr"], torch.ones(a.nrows, dtype=torch.float64, device="cuda"))
    for fmt, B in mats.items():
        st, x, r = gpu.cg_solve(B, b, rtol=1e-9, maxit=20000)
        assert st == 0 and r["rel_resid"] <= 1e-9, fmt
        assert abs(r["iters"] - g["iters"]) <= 2, (fmt, r["iters"], g["iters"])
        assert r["true_rel_resid"] <= 2e-9, fmt
        check_solution(x, 128, 1e-9, r["true_rel_resid"], g, fmt)


@pytest.mark.parametrize("family", ["zipf", "banded"])
def test_irregular_4M_spmv_sampled_rows(gpu, family):
    if family == "zipf":
        a = wl.zipf_rows(4_000_000, seed=2)
    else:
        a = wl.banded(4_000_000, ndiag=11, max_offset=2000, seed=3)
    x = wl.uniform_vector(a.ncols, seed=1)
    rows = np.sort(wl.rng(9).choice(a.nrows, 2000, replace=False))
    irp = np.concatenate([[0], np.cumsum(np.bincount(a.ai, minlength=a.nrows))])
    sel = np.concatenate([np.arange(irp[r], irp[r + 1]) for r in rows])
    sub_irp = np.concatenate([[0], np.cumsum(irp[rows + 1] - irp[rows])]).astype(np.int32)
    ref = orc.csr_spmv(sub_irp, a.aj[sel], a.av[sel], x)
    A = gpu.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    mats = formats_of(gpu, A)
    assert ("dia" in mats) == (family == "banded") and ("ell" in mats) == (family == "banded")
    assert "sell" in mats and "hyb" in mats
    xd = to_dev(x)
    for fmt, B in mats.items():
        y = gpu.spmv(B, xd).cpu().numpy()
        assert rel_maxnorm(y[rows], ref) <= 1e-12, fmt
        assert np.all(np.isfinite(y)), fmt
    for B in mats.values():
        B.close()


def test_stencil128_pcg_multigrid_matches_oracle_run(gpu):
    """PCG with HPCG's 4-level V-cycle on 128^3 against the oracle's stored
    run: iterations within 2, true residual 2 tol, solution bars as above."""
    import torch
    g = golden("pcg_mg4_stencil128_tol1e-9")
    M = gpu.Multigrid(128, 4)
    _, A = M.level(0)
    b = gpu.spmv(A, torch.ones(A.nrows, dtype=torch.float64, device="cuda"))
    D = gpu.stencil(128, fmt="coo").convert("dia")
    for B in (None, D):
        st, x, r = M.pcg_solve(b, A=B, rtol=1e-9, maxit=1000)
        assert st == 0 and abs(r["iters"] - g["iters"]) <= 2, (r["iters"], g["iters"])
        assert r["true_rel_resid"] <= 2e-9
        check_solution(x, 128, 1e-9, r["true_rel_resid"], g, "pcg")
    D.close()
    M.close()


@pytest.fixture(scope="module")
def stencil192(gpu):
    """The 192^3 stencil in DIA and CSR (FP64, plans built), with FP32 copies."""
    A = gpu.stencil(192, fmt="coo")
    mats = {f: A.convert(f).optimize() for f in ("dia", "csr")}
    A.close()
    m32 = {f: B.cast(gpu.F32).optimize() for f, B in mats.items()}
    yield mats, m32
    for B in list(m32.values()) + list(mats.values()):
        B.close()


def rhs192(gpu, D):
    import torch
    return gpu.spmv(D, torch.ones(D.nrows, dtype=torch.float64, device="cuda"))


def test_stencil192_fp64_cg_matches_oracle(gpu, stencil192):
    g = golden("cg_stencil192_tol1e-10")
    D = stencil192[0]["dia"]
    b = rhs192(gpu, D)
    st, x, r = gpu.cg_solve(D, b, rtol=1e-10, maxit=20000)
    assert st == 0 and abs(r["iters"] - g["iters"]) <= 2, (r["iters"], g["iters"])
    check_solution(x, 192, 1e-10, r["true_rel_resid"], g, "fp64 cg")


def test_stencil192_mixed_refinement_matches_oracle(gpu, stencil192):
    """FP32 inner CG with FP64 outer residual: true residual at most 1e-10 and
    the solution within the conditioning bound of the oracle's.  Iteration
    counts are reported against the oracle's but not pinned."""
    g = golden("mixed_stencil192_tol1e-10")
    D, D32 = stencil192[0]["dia"], stencil192[1]["dia"]
    b = rhs192(gpu, D)
    st, x, r = gpu.cg_solve(D, b, rtol=1e-10, maxit=20000, mixed=True, A32=D32,
                            inner_rtol=g["inner_rtol"], max_outer=g["max_outer"])
    assert st == 0 and r["true_rel_resid"] <= 1e-10, r
    assert r["outer_iters"] <= g["max_outer"]
    check_solution(x, 192, 1e-10, r["true_rel_resid"], g, "mixed ir")


@pytest.mark.parametrize("delta", [0.01, 0.1])
@pytest.mark.parametrize("fmt", ["dia", "csr"])
def test_stencil192_reliable_updates_match_oracle(gpu, stencil192, fmt, delta):
    """FP32 CG with FP64 reliable updates, the mixed solver the benchmark
    credits, against the oracle's run of the same method at full size:
    converged, true residual (the solver's own FP64 b - A x, and again from
    the other format's FP64 SpMV) at most 1e-10, FP32 iterations within 10%
    of the oracle's (FP32 rounding differs with the summation order, so the
    counts need not agree exactly), the solution bars above."""
    g = golden(f"mixed_ru_stencil192_tol1e-10_delta{delta}")
    assert g["status"] == 0 and g["true_rel_resid"] <= 1e-10
    mats, m32 = stencil192
    A, A32 = mats[fmt], m32[fmt]
    b = rhs192(gpu, A)
    st, x, r = gpu.cg_solve(A, b, rtol=1e-10, maxit=20000, mixed="ru", A32=A32, delta=delta)
    print(f"[ru192] {fmt} delta={delta}: iters {r['iters']} updates {r['outer_iters']} "
          f"(oracle {g['iters']}, {g['updates']})", flush=True)
    assert st == 0 and r["true_rel_resid"] <= 1e-10, r
    other = mats["csr" if fmt == "dia" else "dia"]
    res = b - gpu.spmv(other, x)
    import torch
    rel = float(torch.linalg.vector_norm(res) / torch.linalg.vector_norm(b))
    assert rel <= 1e-10 and rel == pytest.approx(r["true_rel_resid"], rel=1e-3, abs=1e-14)
    assert abs(r["iters"] - g["iters"]) <= 0.1 * g["iters"], (r["iters"], g["iters"])
    assert r["outer_iters"] >= 1
    check_solution(x, 192, 1e-10, r["true_rel_resid"], g, f"ru {fmt} {delta}")


def test_reliable_updates_large_grid_untimed_equals_timed(gpu):
    """Above 8.4M rows the FP32 vector grid has more than 2,048 workgroups and
    a reliable-update step ends with a finish kernel and a separate direction
    update instead of the folded one: that step, in the loop that enqueues
    the residual replacement only when asked, against the loop that launches
    the update kernels in every step (the timed solve) - the same kernels
    in the same order on the device, so the same iterations, updates and x,
    bit for bit; converged, with x within the conditioning bound of 1 (b =
    A*1: the kappa inequality and max |x - 1| <= 2 kappa tol, as above).
    Stencil 208^3 (8,998,912 rows), DIA."""
    import torch
    n = 208
    A = gpu.stencil(n, fmt="dia").optimize()
    A32 = A.cast(gpu.F32).optimize()
    b = gpu.spmv(A, torch.ones(A.nrows, dtype=torch.float64, device="cuda"))
    ws = gpu.cg_workspace(A, mixed=True)
    kw = dict(rtol=1e-10, maxit=20000, mixed="ru", A32=A32, delta=0.1, workspace=ws)
    st_u, x_u, r_u = gpu.cg_solve(A, b, **kw)
    st_t, x_t, r_t = gpu.cg_solve(A, b, timing=True, **kw)
    print(f"[ru208] iters {r_u['iters']} updates {r_u['outer_iters']}", flush=True)
    assert st_u == st_t == 0 and r_u["true_rel_resid"] <= 1e-10
    assert (r_u["iters"], r_u["outer_iters"]) == (r_t["iters"], r_t["outer_iters"])
    assert r_u["outer_iters"] >= 2
    assert torch.equal(x_u, x_t)
    kappa = stencil_kappa(n)
    e = x_u - 1.0
    rel2 = float(torch.linalg.vector_norm(e) / math.sqrt(x_u.numel()))
    assert rel2 <= kappa * r_u["true_rel_resid"] * 1.01 + 1e-14, (rel2, kappa)
    assert float(e.abs().max()) <= 2 * kappa * 1e-10, float(e.abs().max())
    A.close()
    A32.close()
    torch.cuda.empty_cache()


def test_near_int32_entry_limit_all_formats(gpu):
    """A ragged tridiagonal matrix (2, -1, -1) with 2^29 + 7 rows: 1.61e9
    entries, close to the int32 entry limit, built on the device.  Integer x,
    so every format must match the oracle exactly on 4,096 sampled rows (and
    the two end rows)."""
    import torch
    mxs = gpu
    N = (1 << 29) + 7
    i = torch.arange(N, device="cuda", dtype=torch.int32)
    # canonical order: row by row, columns i-1, i, i+1 where they exist
    ai = torch.stack([i, i, i], 1).reshape(-1)
    aj = torch.stack([i - 1, i, i + 1], 1).reshape(-1)
    av = torch.tensor([-1.0, 2.0, -1.0], device="cuda", dtype=torch.float64).repeat(N)
    keep = (aj >= 0) & (aj < N)
    ai, aj, av = ai[keep], aj[keep], av[keep]
    nnz = ai.numel()
    assert nnz == 3 * N - 2 and nnz < 2 ** 31 - 1
    A = mxs.Matrix.coo(N, N, ai, aj, av, borrow=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    x = torch.randint(-8, 9, (N,), generator=g, device="cuda").double()
    rows = np.unique(np.concatenate([wl.rng(4).choice(N, 4096, replace=False), [0, N - 1]]))
    xr = x.cpu().numpy()
    sub = [(r, c) for r in rows for c in (r - 1, r, r + 1) if 0 <= c < N]
    si = np.array([np.searchsorted(rows, r) for r, _ in sub], np.int32)
    sj = np.array([c for _, c in sub], np.int32)
    sv = np.array([2.0 if r == c else -1.0 for r, c in sub])
    ref = orc.coo_spmv(rows.size, si, sj, sv, xr)
    for fmt in ("coo", "csr", "dia"):
        B = A if fmt == "coo" else A.convert(fmt)
        y = mxs.spmv(B, x)
        assert np.array_equal(y[torch.from_numpy(rows).cuda()].cpu().numpy(), ref), fmt
        if B is not A:
            B.close()
        del y
        torch.cuda.empty_cache()
