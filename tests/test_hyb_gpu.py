"""GPU parity of HYB (ELL part plus COO remainder; Section IX's hybrid
formats) against the CPU oracle, through the C ABI.

Bars: the width K and both parts' arrays equal the oracle's bit for bit;
SpMV within 1e-12 relative max-norm of the oracle's product of the whole
matrix, bit-exact on integer data; CG matches the oracle's CG."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import U64, rel_maxnorm, row_bound, small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()
IDS = [c[0] for c in CASES]


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("K", [-1, 0, 2, 27])
@pytest.mark.parametrize("src", ["coo", "csr"])
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_hyb_matches_oracle(gpu, name, a, src, K):
    mxs = gpu
    print(f"[hyb] {name} {src} K={K}", flush=True)
    irp = orc.coo_to_csr(a.nrows, a.ai)
    Ko, ecol, evals, ri, rj, rv = orc.csr_to_hyb(irp, a.aj, a.av, None if K < 0 else K)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    if src == "csr":
        A = A.convert("csr")
    if Ko * a.nrows > 8 * a.nnz:
        with pytest.raises(mxs.MxsError) as e:
            A.to_hyb(K)
        assert e.value.status == -5
        return
    assert A.hyb_size(K) == (Ko, ri.size)
    H = A.to_hyb(K)
    assert H.format == mxs.HYB and H.ndiag == Ko and H.nnz == a.nnz
    gc, gv, gi, gj, gr = [t.cpu().numpy() for t in H._keep]
    assert np.array_equal(gc, ecol) and np.array_equal(gv, evals)
    assert np.array_equal(gi, ri) and np.array_equal(gj, rj) and np.array_equal(gr, rv)
    x = wl.uniform_vector(a.ncols, seed=4)
    y = to_dev(np.full(a.nrows, np.nan))
    mxs.spmv(H, to_dev(x), y)
    ref = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x)
    y = y.cpu().numpy()
    assert rel_maxnorm(y, ref) <= 1e-12
    assert np.all(np.abs(y - ref) <= 2 * row_bound(a, x, U64) + 1e-300)
    band, rest = H.parts()
    assert band.format == mxs.ELL and rest.format == mxs.COO and rest.nnz == ri.size


def test_hyb_integer_data_and_zipf(gpu):
    mxs = gpu
    a = wl.zipf_rows(20000, seed=11)
    a.av = np.round(a.av * 4) + 1.0
    x = wl.integer_vector(a.ncols, seed=5)
    H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).to_hyb()
    assert H._keep[2].numel() > 0          # a remainder exists on Zipf rows
    assert np.array_equal(mxs.spmv(H, to_dev(x)).cpu().numpy(),
                          orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, x))


def test_cg_on_hyb_matches_oracle(gpu):
    mxs = gpu
    a = wl.stencil(12)
    b = orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))
    st_o, x_o, it_o, _, _ = orc.cg(a.nrows, a.ai, a.aj, a.av, b, tol=1e-10, maxit=2000)
    for K in (-1, 9):
        H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).to_hyb(K)
        st, x, res = mxs.cg_solve(H, to_dev(b), rtol=1e-10, maxit=2000)
        assert st == 0 and abs(res["iters"] - it_o) <= 2
        assert np.max(np.abs(x.cpu().numpy() - x_o)) <= 1e-8


def test_hyb_unsupported_calls(gpu):
    mxs = gpu
    a = wl.stencil(5)
    H = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av).to_hyb()
    for call in (lambda: H.convert("csr"), lambda: H.cast(mxs.F32), lambda: mxs.features(H),
                 lambda: H.to_hyb(), lambda: H.split()):
        with pytest.raises(mxs.MxsError) as e:
            call()
        assert e.value.status == -10
