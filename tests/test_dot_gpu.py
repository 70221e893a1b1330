"""mxs_dot (the reduction behind CG's timed dot products and the public dot
entry point) against the oracle's sequential FP64 dot product, within the
rounding bound gamma_n sum |a_i b_i| doubled (both sides round): FP64 and
FP32 inputs, lengths with and without a tail past the last 16-byte vector,
and inputs that start off a 16-byte boundary (the kernel's scalar path).
Integer-valued inputs, whose every partial sum is exact, must agree bit for
bit."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _dot(mxs, a, b, offset):
    """mxs.dot over a[offset:], b[offset:] (device views that start `offset`
    elements into their allocations)."""
    import torch
    ta = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    r = mxs.dot(ta[offset:], tb[offset:])
    torch.cuda.synchronize()
    return float(r.item())


@pytest.mark.parametrize("n", [0, 1, 2, 7, 1024, 4097, 1_048_579, 9_000_001])
@pytest.mark.parametrize("offset", [0, 1])
def test_fp64_dot_within_rounding_bound(gpu, n, offset):
    a = wl.uniform_vector(n + offset, seed=41)
    b = wl.uniform_vector(n + offset, seed=42)
    got = _dot(gpu, a, b, offset)
    ref = orc.dot(a[offset:], b[offset:])
    bound = 2 * max(n, 1) * U64 * float(np.dot(np.abs(a[offset:]), np.abs(b[offset:])))
    assert abs(got - ref) <= bound, (n, offset, got, ref, bound)


@pytest.mark.parametrize("n", [3, 4099, 2_000_003])
@pytest.mark.parametrize("offset", [0, 1, 2, 3])
def test_fp32_dot_accumulates_in_fp64(gpu, n, offset):
    a = wl.uniform_vector(n + offset, seed=43, dtype=np.float32)
    b = wl.uniform_vector(n + offset, seed=44, dtype=np.float32)
    got = _dot(gpu, a, b, offset)
    # products of two FP32 values are exact in FP64: the oracle sees the same terms
    ref = orc.dot(a[offset:].astype(np.float64), b[offset:].astype(np.float64))
    bound = 2 * max(n, 1) * U64 * float(np.dot(np.abs(a[offset:].astype(np.float64)),
                                                np.abs(b[offset:].astype(np.float64))))
    assert abs(got - ref) <= bound, (n, offset, got, ref, bound)


@pytest.mark.parametrize("offset", [0, 1])
def test_integer_dot_is_exact(gpu, offset):
    n = 3_000_017
    a = wl.integer_vector(n + offset, seed=45)
    b = wl.integer_vector(n + offset, seed=46)
    got = _dot(gpu, a, b, offset)
    assert got == float(np.dot(a[offset:].astype(np.int64), b[offset:].astype(np.int64)))
