"""The allocation-free dot product (mxs_dot_noalloc) against mxs_dot, the
entry point it mirrors: two calls in a row (the second on a smaller input,
so the fixed partials array holds the first call's leftovers), each
bit-identical to mxs_dot on the same inputs and within the FP64 rounding
bound gamma_n sum |a_i b_i| (doubled: both sides round) of the oracle's
sequential dot product; then FP32 inputs, an
empty input, and many calls in one stream without synchronising between
them."""
import ctypes as C

import numpy as np
import pytest

import oracle as orc
import workloads as wl

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(mxs, a, b):
    """(mxs_dot result, mxs_dot_noalloc result) as Python floats, both through
    the C ABI on torch's current stream."""
    import torch
    lib = mxs.load()
    code = 0 if a.dtype == torch.float64 else 1
    ref = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert lib.mxs_dot(a.numel(), code, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                       C.c_void_p(ref.data_ptr()), C.c_void_p(s)) == 0
    assert lib.mxs_dot_noalloc(a.numel(), code, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                               C.c_void_p(out.data_ptr()), C.c_void_p(s)) == 0
    torch.cuda.synchronize()
    return float(ref.item()), float(out.item())


@pytest.mark.parametrize("sizes", [(3_000_001, 1_000_003), (50_000_000, 777)])
def test_two_calls_in_a_row_match_mxs_dot(gpu, sizes):
    for k, n in enumerate(sizes):
        a = wl.uniform_vector(n, seed=20 + k)
        b = wl.uniform_vector(n, seed=30 + k)
        ref, got = _both(gpu, _dev(a), _dev(b))
        assert got == ref, (n, got, ref)
        ref_o = orc.dot(a, b)
        bound = 2 * n * U64 * float(np.dot(np.abs(a), np.abs(b)))
        assert abs(got - ref_o) <= bound, (n, got, ref_o, bound)


def test_fp32_empty_and_back_to_back(gpu):
    import torch
    mxs = gpu
    a32 = torch.linspace(-1, 1, 123_457, dtype=torch.float32, device="cuda")
    b32 = torch.cos(a32)
    ref, got = _both(mxs, a32, b32)
    assert got == ref
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ref, got = _both(mxs, e, e)
    assert got == ref == 0.0
    # twenty calls on one stream, no synchronisation between them: each
    # writes its own result, all equal to mxs_dot's
    xs = [_dev(wl.uniform_vector(n, seed=n)) for n in range(200_000, 220_000, 1000)]
    outs = torch.full((len(xs),), np.nan, dtype=torch.float64, device="cuda")
    for i, x in enumerate(xs):
        mxs.dot_noalloc(x, x, outs[i:i + 1])
    refs = torch.cat([mxs.dot(x, x) for x in xs])
    assert torch.equal(outs, refs)
