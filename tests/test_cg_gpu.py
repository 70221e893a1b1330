"""GPU CG (HPCG's solver without preconditioner, Section VII-D) and the
FP32-inner / FP64-outer refinement, against the CPU oracle and the HPCG
verification property b = A*1 => x -> 1."""
import math

import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import stencil_kappa

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def to_dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def build(mxs, a, fmt):
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    return A if fmt == "coo" else A.convert(fmt)


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("n", [8, 16])
def test_cg_stencil_matches_oracle(gpu, n, fmt):
    a = wl.stencil(n)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    tol = 1e-9
    st_o, x_o, it_o, rel_o, _ = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=tol)
    A = build(gpu, a, fmt)
    st, x, res = gpu.cg_solve(A, to_dev(b), rtol=tol, maxit=1000)
    x = x.cpu().numpy()
    print(f"[cg] n={n} {fmt} iters={res['iters']} oracle={it_o}", flush=True)
    assert st == 0 and st_o == 0
    assert abs(res["iters"] - it_o) <= 2
    assert res["rel_resid"] <= tol and res["true_rel_resid"] <= 10 * tol
    kappa = stencil_kappa(n)
    assert np.max(np.abs(x - 1.0)) <= 10 * kappa * tol
    assert np.max(np.abs(x - x_o)) <= 10 * kappa * tol


@pytest.mark.parametrize("fmt", ["coo", "csr"])
def test_cg_random_spd_matches_solve(gpu, fmt):
    g = wl.rng(5)
    n = 40
    M = g.standard_normal((n, n))
    Ad = M @ M.T + n * np.eye(n)
    ai, aj = np.nonzero(Ad)
    a = wl.Coo(n, n, ai.astype(np.int32), aj.astype(np.int32), Ad[ai, aj])
    b = wl.uniform_vector(n, seed=6)
    A = build(gpu, a, fmt)
    st, x, res = gpu.cg_solve(A, to_dev(b), rtol=1e-14, maxit=500, check_every=1)
    xs = np.linalg.solve(Ad, b)
    assert st == 0
    assert np.max(np.abs(x.cpu().numpy() - xs)) <= 1e-12 * np.max(np.abs(xs))


def test_cg_first_iterate_and_maxit(gpu):
    a = wl.stencil(6)
    A = build(gpu, a, "csr")
    b = wl.uniform_vector(a.nrows, seed=8)
    st, x1, res = gpu.cg_solve(A, to_dev(b), rtol=0.0, maxit=1, check_every=1)
    Ab = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, b)
    want = (b @ b) / (b @ Ab) * b
    assert st == 1 and res["iters"] == 1
    assert np.max(np.abs(x1.cpu().numpy() - want)) <= 1e-14 * np.max(np.abs(want))
    st, _, res = gpu.cg_solve(A, to_dev(b), rtol=1e-30, maxit=7, check_every=3)
    assert st == 1 and res["iters"] == 7


def test_cg_statuses(gpu):
    torch = _torch()
    a = wl.stencil(4)
    A = build(gpu, a, "csr")
    z = torch.zeros(a.nrows, dtype=torch.float64, device="cuda")
    st, x, res = gpu.cg_solve(A, z)
    assert st == 0 and res["iters"] == 0 and not x.any()
    bad = z.clone()
    bad[3] = float("nan")
    with pytest.raises(gpu.MxsError) as e:
        gpu.cg_solve(A, bad)
    assert e.value.status == -9
    ind = wl.Coo(2, 2, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    st, _, res = gpu.cg_solve(build(gpu, ind, "csr"), to_dev(np.ones(2)))
    assert st == -8 and res["iters"] == 1
    rect = gpu.Matrix.coo(2, 3, np.array([0], np.int32), np.array([2], np.int32), np.ones(1))
    with pytest.raises(gpu.MxsError) as e:
        gpu.cg_solve(rect, to_dev(np.ones(2)))
    assert e.value.status == -1


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
def test_cg_polling_interval_does_not_change_result(gpu, fmt):
    a = wl.stencil(12)
    A = build(gpu, a, fmt)
    b = to_dev(wl.uniform_vector(a.nrows, seed=3))
    runs = [gpu.cg_solve(A, b, rtol=1e-10, check_every=c) for c in (1, 5, 32)]
    for st, x, res in runs:
        assert st == 0 and res["iters"] == runs[0][2]["iters"]
        assert np.array_equal(x.cpu().numpy().view(np.uint64), runs[0][1].cpu().numpy().view(np.uint64))


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
def test_cg_timing_mode_splits_kernel_classes(gpu, fmt):
    a = wl.stencil(16)
    A = build(gpu, a, fmt)
    b = to_dev(orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols)))
    st0, x0, r0 = gpu.cg_solve(A, b, rtol=1e-9)
    st, x, r = gpu.cg_solve(A, b, rtol=1e-9, timing=True)
    assert st == 0 and abs(r["iters"] - r0["iters"]) <= 2
    assert r["t_spmv_ms"] > 0 and r["t_dot_ms"] > 0 and r["t_axpy_ms"] > 0
    assert np.max(np.abs(x.cpu().numpy() - 1.0)) <= 1e-6


# ---------------------------------------------------------------------------
# Mixed precision
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("n", [16, 24])
def test_mixed_refinement_reaches_fp64_tolerance(gpu, n, fmt):
    a = wl.stencil(n)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    A = build(gpu, a, fmt)
    A32 = A.cast(gpu.F32)
    st, x, res = gpu.cg_solve(A, to_dev(b), rtol=1e-10, mixed=True, A32=A32, inner_rtol=1e-4)
    x = x.cpu().numpy()
    st_o, x_o, outer_o, inner_o, true_o = orc.mixed_ir(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10,
                                                       inner_rtol=1e-4)
    print(f"[mixed] n={n} {fmt} outer={res['outer_iters']} inner={res['iters']} "
          f"oracle outer={outer_o} inner={inner_o}", flush=True)
    assert st == 0 and st_o == 0
    # the final residual, recomputed by the oracle's FP64 SpMV
    r = b - orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    assert res["true_rel_resid"] <= 1e-10
    kappa = stencil_kappa(n)
    assert np.max(np.abs(x - 1.0)) <= 10 * kappa * 1e-10
    assert np.max(np.abs(x - x_o)) <= 20 * kappa * 1e-10
    assert 1 <= res["outer_iters"] <= 6 and res["outer_iters"] <= outer_o + 2


def test_mixed_statuses(gpu):
    a = wl.stencil(6)
    A = build(gpu, a, "csr")
    A32 = A.cast(gpu.F32)
    b = to_dev(wl.uniform_vector(a.nrows, seed=2))
    st, x, res = gpu.cg_solve(A, b, rtol=1e-16, mixed=True, A32=A32, max_outer=2)
    assert st == 1 and res["outer_iters"] == 2
    with pytest.raises(gpu.MxsError) as e:
        gpu.cg_solve(A, b, mixed=True, A32=None)
    assert e.value.status == -1


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("n,delta", [(8, 0.1), (24, 0.1), (24, 0.01), (24, 1e-3)])
def test_reliable_update_reaches_fp64_tolerance(gpu, n, delta, fmt):
    """FP32 CG with FP64 reliable updates against the oracle's run of the same
    method: both reach the FP64 tolerance (residual recomputed by the oracle's
    FP64 SpMV), solutions within the conditioning bound of each other;
    iteration and update counts are reported and bounded, not pinned."""
    a = wl.stencil(n)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    A = build(gpu, a, fmt)
    A32 = A.cast(gpu.F32)
    st, x, res = gpu.cg_solve(A, to_dev(b), rtol=1e-10, mixed="ru", A32=A32, delta=delta)
    x = x.cpu().numpy()
    st_o, x_o, upd_o, it_o, true_o = orc.mixed_ru(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, delta=delta)
    print(f"[ru] n={n} delta={delta} {fmt} iters={res['iters']} updates={res['outer_iters']} "
          f"oracle iters={it_o} updates={upd_o}", flush=True)
    assert st == 0 and st_o == 0
    r = b - orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    assert res["true_rel_resid"] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(b), rel=1e-6)
    kappa = stencil_kappa(n)
    assert np.max(np.abs(x - x_o)) <= 20 * kappa * 1e-10
    assert abs(res["iters"] - it_o) <= max(3, 0.1 * it_o)
    assert res["outer_iters"] >= 1


def test_reliable_update_statuses_and_polling(gpu):
    a = wl.stencil(6)
    A = build(gpu, a, "csr")
    A32 = A.cast(gpu.F32)
    torch = __import__("torch")
    z = torch.zeros(a.nrows, dtype=torch.float64, device="cuda")
    st, x, res = gpu.cg_solve(A, z, mixed="ru", A32=A32)
    assert st == 0 and res["iters"] == 0 and not bool(x.any())
    bad = z.clone()
    bad[3] = float("nan")
    with pytest.raises(gpu.MxsError) as e:
        gpu.cg_solve(A, bad, mixed="ru", A32=A32)
    assert e.value.status == -9
    bh = wl.uniform_vector(a.nrows, seed=2)
    b = to_dev(bh)
    st, x, res = gpu.cg_solve(A, b, rtol=1e-30, mixed="ru", A32=A32, maxit=5)
    assert st == 1 and res["iters"] == 5
    # the reported residual is that of the returned x
    r = bh - orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x.cpu().numpy())
    assert res["true_rel_resid"] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(bh), rel=1e-6)
    # the flag-polling interval changes nothing
    outs = [gpu.cg_solve(A, b, rtol=1e-11, mixed="ru", A32=A32, check_every=c) for c in (1, 7, 64)]
    for st_c, x_c, r_c in outs[1:]:
        assert st_c == outs[0][0] and r_c["iters"] == outs[0][2]["iters"]
        assert torch.equal(x_c, outs[0][1])
    with pytest.raises(gpu.MxsError) as e:
        gpu.cg_solve(A, b, mixed="ru", A32=A32, delta=1.5)
    assert e.value.status == -1
    # the timed solve launches the update kernels in every step (idle unless
    # an update is due), the untimed one only when a step asks for an update:
    # the same kernels in the same order on the device, so the same result
    for delta in (0.1, 0.5):
        for every in (1, 5):
            st_u, x_u, r_u = gpu.cg_solve(A, b, rtol=1e-11, mixed="ru", A32=A32, delta=delta,
                                          check_every=every)
            st_t, x_t, r_t = gpu.cg_solve(A, b, rtol=1e-11, mixed="ru", A32=A32, delta=delta,
                                          check_every=every, timing=True)
            assert st_u == st_t == 0
            assert r_u["outer_iters"] >= 1
            assert (r_u["iters"], r_u["outer_iters"]) == (r_t["iters"], r_t["outer_iters"])
            assert torch.equal(x_u, x_t)
    # the cap reached on a step that also asks for an update (its update is
    # the last one), and on one that does not
    for maxit in range(1, 12):
        st_u, x_u, r_u = gpu.cg_solve(A, b, rtol=1e-30, mixed="ru", A32=A32, delta=0.5, maxit=maxit)
        st_t, x_t, r_t = gpu.cg_solve(A, b, rtol=1e-30, mixed="ru", A32=A32, delta=0.5, maxit=maxit,
                                      timing=True)
        assert st_u == st_t == 1 and r_u["iters"] == r_t["iters"] == maxit
        assert r_u["outer_iters"] == r_t["outer_iters"]
        assert torch.equal(x_u, x_t)
    # indefinite: p.Ap = 0 at the first step
    ind = wl.Coo(2, 2, np.array([0, 1], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    I = build(gpu, ind, "csr")
    st, x, res = gpu.cg_solve(I, to_dev(np.ones(2)), mixed="ru", A32=I.cast(gpu.F32))
    assert st == -8
