"""Execution plans in caller memory (the optimize stage of Section VI-A's
Table I): mxs_plan_size / mxs_optimize build every plan array in a torch
tensor, calls that run SpMV kernels refuse a handle without one, plans can be
rebuilt with other options into another tensor (the first then freed), and
mxs_spmv_ws lets two streams run SpMV on one handle at once, each with its
own scratch for the carries, all against the CPU oracle."""
import ctypes as C

import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import rel_maxnorm

pytestmark = pytest.mark.gpu

NO_PLAN = -11


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _long_rows(n=30000, seed=3):
    """Rows of 1-9 entries, and every 997th row 3,000 long: rows that span
    entry tiles, so the tile kernels write carries and the fix-up reads them."""
    g = wl.rng(seed)
    lens = g.integers(1, 10, n)
    lens[::997] = 3000
    ai = np.repeat(np.arange(n, dtype=np.int32), lens)
    aj = np.concatenate([np.sort(g.choice(n, k, replace=False)) for k in lens]).astype(np.int32)
    return wl.Coo(n, n, ai, aj, g.standard_normal(ai.shape[0]))


def _mats(mxs, a):
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    return {"coo": A, "csr": A.convert("csr")}


def test_calls_refuse_a_handle_without_plan(gpu):
    import torch
    mxs = gpu
    lib = mxs.load()
    a = wl.stencil(8)
    for fmt in ("coo", "csr", "dia", "ell"):
        A = mxs.Matrix.from_workload(a, fmt)
        assert not A.optimized
        x = torch.ones(a.ncols, dtype=torch.float64, device="cuda")
        y = torch.empty(a.nrows, dtype=torch.float64, device="cuda")
        assert lib.mxs_spmv(A.handle, mxs._ptr(x), mxs._ptr(y), None) == NO_PLAN
        assert lib.mxs_spmv_ws(A.handle, mxs._ptr(x), mxs._ptr(y), None, 0, None) == NO_PLAN
        v = C.c_int32()
        assert lib.mxs_get_impl(A.handle, C.byref(v), None) == NO_PLAN
        assert lib.mxs_set_impl(A.handle, 0, None) == NO_PLAN
        n = C.c_size_t()
        assert lib.mxs_spmv_scratch_size(A.handle, C.byref(n)) == NO_PLAN
        with pytest.raises(mxs.MxsError) as e:
            mxs._check(lib.mxs_tune(A.handle, mxs._ptr(x), mxs._ptr(y), 3, None, None, None), "tune")
        assert e.value.status == NO_PLAN
        A.optimize()
        assert A.optimized
        assert lib.mxs_spmv(A.handle, mxs._ptr(x), mxs._ptr(y), None) == 0
        A.close()


@pytest.mark.parametrize("name", ["stencil24", "long_rows", "banded"])
def test_plan_lives_in_the_callers_tensor(gpu, name):
    """The plan is built in a torch tensor; rebuilt with other options into a
    second tensor, the first tensor can be freed and its memory reused while
    the handle keeps giving the oracle's product."""
    import torch
    mxs = gpu
    a = {"stencil24": lambda: wl.stencil(24), "long_rows": _long_rows,
         "banded": lambda: wl.banded(40000, ndiag=9, max_offset=300, seed=4)}[name]()
    x = wl.uniform_vector(a.ncols, seed=1)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    xd = to_dev(x)
    mats = _mats(mxs, a)
    if name != "long_rows":
        mats["dia"] = mats["coo"].convert("dia")
    for fmt, A in mats.items():
        opts0 = mxs.PLAN_DIA_BLOCKED if fmt == "dia" else 0
        opts1 = mxs.PLAN_NO_ELL if fmt == "csr" else 0
        n0, n1 = A.plan_size(opts0), A.plan_size(opts1)
        if fmt == "dia":   # the blocked copy holds every value again
            assert n0 >= n1 + 8 * a.nrows * A.ndiag
        ws0 = torch.empty(n0, dtype=torch.uint8, device="cuda")
        A.optimize(opts0, workspace=ws0)
        y0 = mxs.spmv(A, xd).cpu().numpy()
        assert rel_maxnorm(y0, ref) <= 1e-12, fmt
        # a workspace one byte short is refused, and the handle has no plan
        small = torch.empty(max(n1 - 1, 0), dtype=torch.uint8, device="cuda")
        lib = mxs.load()
        if n1 > 0:
            assert lib.mxs_optimize(A.handle, opts1, mxs._ptr(small) if small.numel() else None,
                                    n1 - 1, None) == -1
            assert not A.optimized
        ws1 = torch.empty(n1, dtype=torch.uint8, device="cuda")
        A.optimize(opts1, workspace=ws1)
        del ws0, small
        torch.cuda.empty_cache()
        junk = torch.full((n0 // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")
        y1 = mxs.spmv(A, xd).cpu().numpy()
        assert rel_maxnorm(y1, ref) <= 1e-12, fmt
        del junk
    for A in mats.values():
        A.close()


@pytest.mark.parametrize("name", ["long_rows", "stencil24"])
@pytest.mark.parametrize("fmt,impl", [("coo", 0), ("coo", 1), ("csr", 0), ("csr", 2)])
def test_two_streams_on_one_handle(gpu, name, fmt, impl):
    """One optimised handle, two streams, each with its own scratch: 20
    products per stream issued alternately without synchronising, every
    result against the oracle and equal bit for bit to mxs_spmv's."""
    import torch
    mxs = gpu
    a = _long_rows() if name == "long_rows" else wl.stencil(24)
    A = _mats(mxs, a)[fmt]
    A.optimize()
    try:
        A.impl = impl
    except mxs.MxsError:
        pytest.skip("implementation not applicable to this matrix")
    nb = A.spmv_scratch_size()
    if fmt == "coo" and impl == 1:
        assert nb > 0   # segmented tiles always carry
    xs = [wl.uniform_vector(a.ncols, seed=s) for s in (11, 12)]
    refs = [orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x) for x in xs]
    once = [mxs.spmv(A, to_dev(x)).cpu().numpy() for x in xs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    scratch = [torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda") for _ in streams]
    xd = [to_dev(x) for x in xs]
    ys = [[torch.empty(a.nrows, dtype=torch.float64, device="cuda") for _ in range(20)] for _ in streams]
    torch.cuda.synchronize()
    for k in range(20):
        for j, st in enumerate(streams):
            with torch.cuda.stream(st):
                mxs.spmv(A, xd[j], ys[j][k], scratch=scratch[j])
    torch.cuda.synchronize()
    for j in range(2):
        for k in range(20):
            y = ys[j][k].cpu().numpy()
            assert rel_maxnorm(y, refs[j]) <= 1e-12, (j, k)
            assert np.array_equal(y, once[j]), (j, k)
    A.close()


def test_spmv_ws_argument_checks(gpu):
    import torch
    mxs = gpu
    lib = mxs.load()
    a = _long_rows(n=5000)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).optimize()
    A.impl = 1
    nb = A.spmv_scratch_size()
    assert nb > 0
    x = to_dev(wl.uniform_vector(a.ncols, seed=1))
    y = torch.empty(a.nrows, dtype=torch.float64, device="cuda")
    sc = torch.empty(nb, dtype=torch.uint8, device="cuda")
    assert lib.mxs_spmv_ws(A.handle, mxs._ptr(x), mxs._ptr(y), mxs._ptr(sc), nb - 1, None) == -1
    assert lib.mxs_spmv_ws(A.handle, mxs._ptr(x), mxs._ptr(y), None, nb, None) == -1
    assert lib.mxs_spmv_ws(A.handle, mxs._ptr(x), mxs._ptr(y), mxs._ptr(y), nb, None) == -1  # overlaps y
    assert lib.mxs_spmv_ws(A.handle, mxs._ptr(x), mxs._ptr(y), mxs._ptr(sc), nb, None) == 0
    torch.cuda.synchronize()
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x.cpu().numpy())
    assert rel_maxnorm(y.cpu().numpy(), ref) <= 1e-12
    # parts of a split are planned with their parent
    band = wl.banded(5000, ndiag=5, max_offset=40, seed=2)
    H = mxs.Matrix.coo(band.nrows, band.ncols, band.ai, band.aj, band.av).split(0.5, "coo")
    b, r = H.parts()
    n = C.c_size_t()
    assert lib.mxs_plan_size(b.handle, 0, C.byref(n), None) == -1
    assert lib.mxs_optimize(r.handle, 0, None, 0, None) == -1
    assert lib.mxs_plan_size(H.handle, 8, C.byref(n), None) == -1   # unknown option bit
    H.close()
    A.close()


def test_multigrid_lives_in_the_callers_tensor(gpu):
    """mxs_mg_create builds the whole hierarchy in the tensor the binding
    allocated from mxs_mg_size; one V-cycle against the oracle's."""
    import torch
    mxs = gpu
    M = mxs.Multigrid(16, 3)
    lib = mxs.load()
    nb = C.c_size_t()
    assert lib.mxs_mg_size(16, 3, C.byref(nb)) == 0
    assert M._ws.numel() == nb.value
    lv = []
    for m in (16, 8, 4):
        c = wl.stencil(m)
        lv.append((m, orc.coo_to_csr(c.nrows, c.ai), c.aj, c.av))
    r = wl.uniform_vector(16 ** 3, seed=5)
    z = M.apply(to_dev(r)).cpu().numpy()
    zo = orc.mg_vcycle(lv, r)
    assert rel_maxnorm(z, zo) <= 1e-12
    M.close()
