"""GPU parity of ELL and SELL-C-sigma (Section IX's further formats; C = 64)
against the CPU oracle, through the C ABI.

Bars: conversion arrays (ELL columns/values; SELL perm, slice offsets,
columns, values) equal the oracle's bit for bit, and so do the round trips
back to COO/CSR; refusals follow the 8-slots-per-entry rule; SpMV within
1e-12 relative max-norm and the per-row rounding bound, bit-exact on
integer data; CG matches the oracle's CG."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import U32, U64, rel_maxnorm, row_bound, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()
IDS = [c[0] for c in CASES]
SIGMAS = (1, 64, 4096)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def csr_of(a):
    return orc.coo_to_csr(a.nrows, a.ai), a.aj, a.av


def ell_or_none(mxs, A):
    try:
        return A.convert("ell")
    except mxs.MxsError as e:
        assert e.status == -5
        return None


def sell_or_none(mxs, A, sigma):
    try:
        return A.to_sell(sigma)
    except mxs.MxsError as e:
        assert e.status == -5
        return None


@pytest.mark.parametrize("src", ["coo", "csr"])
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_ell_conversion_and_spmv(gpu, name, a, src):
    mxs = gpu
    print(f"[ell] {name} {src}", flush=True)
    irp, aj, av = csr_of(a)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    if src == "csr":
        A = A.convert("csr")
    K_o = int(np.max(np.diff(irp))) if a.nrows else 0
    E = ell_or_none(mxs, A)
    if K_o * a.nrows > 8 * a.nnz:
        assert E is None
        return
    assert E is not None and E.format == mxs.ELL and E.ndiag == K_o and E.nnz == a.nnz
    K, col, val = orc.csr_to_ell(irp, aj, av)
    gcol, gval = [t.cpu().numpy() for t in E._keep]
    assert np.array_equal(gcol, col) and np.array_equal(gval, val)
    x = wl.uniform_vector(a.ncols, seed=1)
    y = to_dev(np.full(a.nrows, np.nan))
    mxs.spmv(E, to_dev(x), y)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    y = y.cpu().numpy()
    assert rel_maxnorm(y, ref) <= 1e-12
    assert np.all(np.abs(y - ref) <= row_bound(a, x, U64) + 1e-300)
    # back to COO and CSR, bit for bit
    bi, bj, bv = E.convert("coo").export()
    assert np.array_equal(bi, a.ai) and np.array_equal(bj, a.aj) and np.array_equal(bv, a.av)
    ci, cj, cv = E.convert("csr").export()
    assert np.array_equal(ci, irp) and np.array_equal(cj, aj) and np.array_equal(cv, av)


@pytest.mark.parametrize("sigma", SIGMAS)
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_sell_conversion_and_spmv(gpu, name, a, sigma):
    mxs = gpu
    print(f"[sell] {name} sigma={sigma}", flush=True)
    irp, aj, av = csr_of(a)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).convert("csr")
    perm, cs, col, val = orc.csr_to_sell(irp, aj, av, 64, sigma)
    S = sell_or_none(mxs, A, sigma)
    if int(cs[-1]) > 8 * a.nnz:
        assert S is None
        return
    assert S is not None and S.format == mxs.SELL and S.nnz == a.nnz
    gp, gcs, gcol, gval = [t.cpu().numpy() for t in S._keep]
    assert np.array_equal(gp, perm) and np.array_equal(gcs, cs)
    assert np.array_equal(gcol, col) and np.array_equal(gval, val)
    x = wl.uniform_vector(a.ncols, seed=2)
    y = to_dev(np.full(a.nrows, np.nan))
    mxs.spmv(S, to_dev(x), y)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    y = y.cpu().numpy()
    assert rel_maxnorm(y, ref) <= 1e-12
    assert np.all(np.abs(y - ref) <= row_bound(a, x, U64) + 1e-300)
    ci, cj, cv = S.export()   # SELL exports its CSR form
    assert np.array_equal(ci, irp) and np.array_equal(cj, aj) and np.array_equal(cv, av)
    bi, bj, bv = S.convert("coo").export()
    assert np.array_equal(bi, a.ai) and np.array_equal(bj, a.aj) and np.array_equal(bv, a.av)


@pytest.mark.parametrize("n", [3, 16, 33])
def test_integer_data_bit_exact(gpu, n):
    mxs = gpu
    a = wl.stencil(n)
    x = wl.integer_vector(a.ncols, seed=n)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    for B in (A.convert("ell"), A.to_sell(1), A.to_sell(64), A.to_sell(100000)):
        assert np.array_equal(mxs.spmv(B, to_dev(x)).cpu().numpy(), ref), B.format


def test_fp32_within_rounding_bound(gpu):
    mxs = gpu
    a = wl.zipf_rows(20000, seed=11)
    a32 = a.astype(np.float32)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a32.ai, a32.aj, a32.av)
    x = wl.uniform_vector(a.ncols, seed=3).astype(np.float32)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a32.av.astype(np.float64), x.astype(np.float64))
    S = A.to_sell(4096)
    for B in (S, S.cast(mxs.F64).cast(mxs.F32)):
        y = mxs.spmv(B, to_dev(x)).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(y - ref) <= row_bound(a, x.astype(np.float64), U32) + 1e-30)


@pytest.mark.parametrize("fmt", ["ell", "sell1", "sell64"])
def test_cg_matches_oracle(gpu, fmt):
    mxs = gpu
    a = wl.stencil(12)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    st_o, x_o, it_o, _, _ = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=2000)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    B = A.convert("ell") if fmt == "ell" else A.to_sell(int(fmt[4:]))
    st, x, res = mxs.cg_solve(B, to_dev(b), rtol=1e-10, maxit=2000)
    assert st == 0 and abs(res["iters"] - it_o) <= 2
    assert np.max(np.abs(x.cpu().numpy() - x_o)) <= 1e-8
    # reliable-update mixed solve with an FP32 copy of the same format
    st, x, res = mxs.cg_solve(B, to_dev(b), rtol=1e-10, maxit=5000, mixed="ru", A32=B.cast(mxs.F32))
    assert st == 0 and res["true_rel_resid"] <= 1e-10


def test_unsupported_calls(gpu):
    mxs = gpu
    a = wl.stencil(5)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    E, S = A.convert("ell"), A.to_sell(64)
    assert E.impl_count() == 1 and S.impl_count() == 1 and E.impl == 0
    for call in (lambda: E.convert("dia"), lambda: S.convert("ell"), lambda: mxs.features(E),
                 lambda: mxs.features(S), lambda: E.split(), lambda: S.to_sell(1),
                 lambda: E.to_sell(1)):
        with pytest.raises(mxs.MxsError) as e:
            call()
        assert e.value.status == -10
    lib = mxs.load()
    import ctypes as C
    h = C.c_void_p()
    assert lib.mxs_convert(A.handle, mxs.SELL, None, None, None, C.byref(h), None) == -10
    assert lib.mxs_to_sell(A.handle, 0, None, None, None, None, C.byref(h), None) == -1
