"""GPU parity of HPCG's preconditioner (symmetric Gauss-Seidel, the
multigrid V-cycle and PCG; Section VII-D) against the CPU oracle, through the
C ABI.

Bars: level operators equal the stencil generator's CSR arrays bit for bit;
one sweep, one V-cycle within 1e-12 relative max-norm of the oracle (the
same updates in the same order; only the rounding of each row's sum
differs); PCG within two iterations of the oracle's and its solution within
1e-9 of the oracle's."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import rel_maxnorm

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def levels_of(n, L):
    out = []
    for l in range(L):
        a = wl.stencil(n >> l)
        out.append((n >> l, orc.coo_to_csr(a.nrows, a.ai), a.aj, a.av))
    return out


@pytest.mark.parametrize("n,L", [(1, 1), (2, 2), (5, 1), (8, 4), (12, 3)])
def test_level_operators_are_the_stencil(gpu, n, L):
    M = gpu.Multigrid(n, L)
    for l, (m, irp, aj, av) in enumerate(levels_of(n, L)):
        mm, A = M.level(l)
        assert mm == m and A.format == gpu.CSR and A.nrows == m ** 3
        girp, gaj, gav = A.export()
        assert np.array_equal(girp, irp) and np.array_equal(gaj, aj) and np.array_equal(gav, av)
    lib = gpu.load()
    assert lib.mxs_destroy(M.level(0)[1].handle) == -1
    M.close()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 33])
def test_symgs_matches_oracle(gpu, n):
    print(f"[symgs] n={n}", flush=True)
    M = gpu.Multigrid(n, 1)
    _, irp, aj, av = levels_of(n, 1)[0]
    g = wl.rng(n)
    r, x = g.standard_normal(n ** 3), g.standard_normal(n ** 3)
    st, want = orc.symgs(irp, aj, av, orc.colour_order(n), r, x)
    xd = to_dev(x)
    M.symgs(0, to_dev(r), xd)
    assert st == 0 and rel_maxnorm(xd.cpu().numpy(), want) <= 1e-12
    # zero start, twice in a row (the state left behind is the output only)
    x0 = to_dev(np.zeros(n ** 3))
    M.symgs(0, to_dev(r), x0)
    _, want0 = orc.symgs(irp, aj, av, orc.colour_order(n), r, np.zeros(n ** 3))
    assert rel_maxnorm(x0.cpu().numpy(), want0) <= 1e-12
    M.close()


def test_symgs_on_a_coarse_level(gpu):
    M = gpu.Multigrid(16, 3)
    _, irp, aj, av = levels_of(16, 3)[2]
    r = wl.rng(3).standard_normal(64)
    x = to_dev(np.zeros(64))
    M.symgs(2, to_dev(r), x)
    _, want = orc.symgs(irp, aj, av, orc.colour_order(4), r, np.zeros(64))
    assert rel_maxnorm(x.cpu().numpy(), want) <= 1e-12
    M.close()


@pytest.mark.parametrize("n,L", [(2, 2), (8, 2), (8, 4), (16, 3), (16, 4), (32, 4), (40, 3),
                                 (64, 3), (64, 4)])
def test_vcycle_matches_oracle(gpu, n, L):
    print(f"[vcycle] n={n} L={L}", flush=True)
    M = gpu.Multigrid(n, L)
    lv = levels_of(n, L)
    r = wl.rng(n * 10 + L).standard_normal(n ** 3)
    want = orc.mg_vcycle(lv, r)
    z1 = M.apply(to_dev(r)).cpu().numpy()
    assert rel_maxnorm(z1, want) <= 1e-12
    z2 = M.apply(to_dev(r)).cpu().numpy()
    assert np.array_equal(z1, z2)  # deterministic; no state carried between cycles
    M.close()


@pytest.mark.parametrize("fmt", ["own", "csr", "dia", "coo"])
def test_pcg_matches_oracle(gpu, fmt):
    n, L = 16, 3
    lv = levels_of(n, L)
    _, irp, aj, av = lv[0]
    b = orc.csr_spmv(irp, aj, av, np.ones(n ** 3))
    st_o, x_o, it_o, rel_o, tr_o = orc.pcg(irp, aj, av, b, lambda r: orc.mg_vcycle(lv, r), tol=1e-10)
    M = gpu.Multigrid(n, L)
    A = None
    if fmt != "own":
        A = gpu.stencil(n, fmt="coo")
        if fmt != "coo":
            A = A.convert(fmt)
    st, x, res = M.pcg_solve(to_dev(b), A=A, rtol=1e-10, maxit=200)
    print(f"[pcg] {fmt} iters={res['iters']} oracle={it_o}", flush=True)
    assert st == 0 and st_o == 0 and abs(res["iters"] - it_o) <= 2
    assert res["rel_resid"] <= 1e-10 and res["true_rel_resid"] <= 2e-10
    assert np.max(np.abs(x.cpu().numpy() - x_o)) <= 1e-9
    M.close()


def test_pcg_timing_and_cap(gpu):
    n, L = 8, 2
    M = gpu.Multigrid(n, L)
    _, irp, aj, av = levels_of(n, L)[0]
    b = orc.csr_spmv(irp, aj, av, wl.uniform_vector(n ** 3, seed=2))
    st, x, res = M.pcg_solve(to_dev(b), rtol=1e-30, maxit=3, timing=True, check_every=1)
    assert st == 1 and res["iters"] == 3
    assert res["t_precond_ms"] > 0 and res["t_spmv_ms"] > 0 and res["t_dot_ms"] > 0
    # the cap's iterate is the oracle's third iterate
    lv = levels_of(n, L)
    _, x_o, it_o, _, _ = orc.pcg(irp, aj, av, b, lambda r: orc.mg_vcycle(lv, r), tol=1e-30, maxit=3)
    assert it_o == 3 and rel_maxnorm(x.cpu().numpy(), x_o) <= 1e-11
    M.close()


def test_mg_argument_checks(gpu):
    import ctypes as C
    mxs = gpu
    lib = mxs.load()
    import torch
    h = C.c_void_p()
    b = C.c_size_t()
    assert lib.mxs_mg_size(8, 2, C.byref(b)) == 0
    ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
    assert lib.mxs_mg_create(6, 3, mxs._ptr(ws), b.value, C.byref(h), None) == -1  # 6 not divisible by 4
    assert lib.mxs_mg_create(8, 0, mxs._ptr(ws), b.value, C.byref(h), None) == -1
    assert lib.mxs_mg_create(0, 1, mxs._ptr(ws), b.value, C.byref(h), None) == -1
    assert lib.mxs_mg_create(2048, 1, mxs._ptr(ws), b.value, C.byref(h), None) == -10  # beyond int32 rows
    assert lib.mxs_mg_create(8, 2, mxs._ptr(ws), b.value - 1, C.byref(h), None) == -1  # too small
    assert h.value is None
    M = mxs.Multigrid(8, 2)
    x = to_dev(np.zeros(512))
    assert lib.mxs_symgs(M.handle, 2, mxs._ptr(x), mxs._ptr(to_dev(np.zeros(512))), None) == -1
    assert lib.mxs_symgs(M.handle, 0, mxs._ptr(x), mxs._ptr(x), None) == -1      # aliasing
    assert lib.mxs_mg_apply(M.handle, mxs._ptr(x), mxs._ptr(x), None) == -1
    small = mxs.stencil(4, fmt="csr")
    with pytest.raises(mxs.MxsError) as e:
        M.pcg_solve(to_dev(np.ones(512)), A=small)
    assert e.value.status == -1
    M.close()
