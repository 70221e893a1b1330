"""The C-ABI library: it loads, exports every function mxs.h declares, and
rejects invalid arguments on the host before touching the GPU (so these run
without one)."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2304_09511_amd as mxs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mxs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mxs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mxs.lib_path()):
        pytest.fail("libmxs.so is not built (run __graft_entry__.build())")
    return mxs.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mxs_coo_create", "mxs_csr_create", "mxs_dia_create", "mxs_convert",
                     "mxs_spmv", "mxs_cg_solve", "mxs_features", "mxs_mlp_train_step"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", mxs.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mxs_[a-z0-9_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_binding_signatures_cover_the_header():
    assert set(mxs._SIGS) == set(declared_functions())


def test_status_strings(lib):
    for code, name in mxs.STATUS.items():
        assert lib.mxs_status_string(code).decode() == name
    assert lib.mxs_status_string(12345).decode() == "MXS_UNKNOWN_STATUS"
    assert lib.mxs_version() == 10000


def test_stencil_nnz_closed_form(lib):
    for n in (1, 2, 3, 16, 128, 192):
        assert lib.mxs_stencil_nnz(n, 27) == (3 * n - 2) ** 3
        assert lib.mxs_stencil_nnz(n, 7) == n ** 3 + 6 * (n - 1) * n * n
    assert lib.mxs_stencil_nnz(4, 5) == -1
    assert lib.mxs_stencil_nnz(-1, 27) == -1


P = C.c_void_p
FAKE = C.c_void_p(0x1000)  # never dereferenced: validation fails first


def test_create_rejects_bad_arguments_on_host(lib):
    h = C.c_void_p()
    # null output handle
    assert lib.mxs_coo_create(None, 2, 2, 1, FAKE, FAKE, FAKE, 0, 0, None) == -1
    # negative sizes
    assert lib.mxs_coo_create(C.byref(h), -1, 2, 0, None, None, None, 0, 0, None) == -1
    assert lib.mxs_csr_create(C.byref(h), 2, -2, 0, FAKE, None, None, 0, 0, None) == -1
    assert lib.mxs_dia_create(C.byref(h), 2, 2, -1, None, None, 0, 0, None) == -1
    # unknown dtype and flags
    assert lib.mxs_coo_create(C.byref(h), 2, 2, 0, None, None, None, 7, 0, None) == -1
    assert lib.mxs_coo_create(C.byref(h), 2, 2, 0, None, None, None, 0, 0x10, None) == -1
    # missing arrays for a non-empty matrix
    assert lib.mxs_coo_create(C.byref(h), 2, 2, 3, FAKE, None, FAKE, 0, 0, None) == -1
    assert lib.mxs_csr_create(C.byref(h), 2, 2, 0, None, None, None, 0, 0, None) == -1
    # more diagonals than a 2x2 matrix has
    assert lib.mxs_dia_create(C.byref(h), 2, 2, 4, FAKE, FAKE, 0, 0, None) == -2
    # indices are int32: more than 2^31-1 entries is unsupported
    assert lib.mxs_coo_create(C.byref(h), 2, 2, 2 ** 31, FAKE, FAKE, FAKE, 0, 0, None) == -10
    assert h.value is None  # outputs untouched on failure


def test_calls_reject_null_handles_and_bad_enums(lib):
    assert lib.mxs_spmv(None, FAKE, FAKE, None) == -1
    assert lib.mxs_optimize(None, 0, None, 0, None) == -1
    assert lib.mxs_plan_size(None, 0, FAKE, None) == -1
    assert lib.mxs_plan_info(None, None, None) == -1
    assert lib.mxs_spmv_scratch_size(None, FAKE) == -1
    assert lib.mxs_spmv_ws(None, FAKE, FAKE, FAKE, 64, None) == -1
    assert lib.mxs_impl_count(None) == 0
    assert lib.mxs_split_parts(None, None, None) == -1
    assert lib.mxs_sell_size(None, 1, None, None, None) == -1
    assert lib.mxs_to_sell(None, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1
    assert lib.mxs_hyb_size(None, -1, None, None, None) == -1
    assert lib.mxs_to_hyb(None, -1, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1
    assert lib.mxs_mg_create(8, 2, FAKE, 1 << 20, None, None) == -1   # no output pointer
    assert lib.mxs_mg_create(8, 2, None, 1 << 20, FAKE, None) == -1   # no workspace
    assert lib.mxs_mg_create(8, 2, C.c_void_p(0x1010), 1 << 20, FAKE, None) == -1  # misaligned
    assert lib.mxs_mg_create(6, 3, FAKE, 1 << 20, FAKE, None) == -1   # 6 not divisible by 4
    assert lib.mxs_mg_create(8, 13, FAKE, 1 << 20, FAKE, None) == -1
    assert lib.mxs_mg_create(2048, 1, FAKE, 1 << 20, FAKE, None) == -10  # rows beyond int32
    assert lib.mxs_mg_size(8, 2, None) == -1
    assert lib.mxs_mg_size(6, 3, FAKE) == -1
    assert lib.mxs_mg_size(2048, 1, FAKE) == -10
    assert lib.mxs_mg_destroy(None) == 0
    assert lib.mxs_mg_level(None, 0, None, None) == -1
    assert lib.mxs_symgs(None, 0, FAKE, FAKE, None) == -1
    assert lib.mxs_mg_apply(None, FAKE, FAKE, None) == -1
    assert lib.mxs_pcg_workspace_size(None, FAKE) == -1
    assert lib.mxs_pcg_solve(None, None, FAKE, FAKE, FAKE, FAKE, FAKE, 8, None) == -1
    assert lib.mxs_set_impl(None, 0, None) == -1
    assert lib.mxs_get_impl(None, FAKE, None) == -1
    assert lib.mxs_tune(None, FAKE, FAKE, 5, None, None, None) == -1
    assert lib.mxs_info(None, None, None, None, None, None, None) == -1
    assert lib.mxs_arrays(None, None, None, None) == -1
    assert lib.mxs_convert_size(None, 0, None, None, None) == -1
    assert lib.mxs_convert(None, 1, None, None, None, None, None) == -1
    assert lib.mxs_cast(None, 1, None, None, None) == -1
    assert lib.mxs_features(None, None, None) == -1
    assert lib.mxs_cg_solve(None, None, None, None, None, None, None, 0, None) == -1
    assert lib.mxs_cg_workspace_size(None, 0, None) == -1
    assert lib.mxs_destroy(None) == 0
    assert lib.mxs_dot(-1, 0, None, None, None, None) == -1
    assert lib.mxs_dot(4, 3, FAKE, FAKE, FAKE, None) == -1
    assert lib.mxs_dot_noalloc(-1, 0, None, None, None, None) == -1
    assert lib.mxs_dot_noalloc(4, 3, FAKE, FAKE, FAKE, None) == -1
    assert lib.mxs_dot_noalloc(4, 0, FAKE, FAKE, None, None) == -1
    assert lib.mxs_axpby(4, 0, 1.0, None, 0.0, FAKE, None) == -1
    assert lib.mxs_stencil_coo(4, 9, 26.0, -1.0, FAKE, FAKE, FAKE, 0, None) == -1
    assert lib.mxs_stencil_coo(2000, 27, 26.0, -1.0, FAKE, FAKE, FAKE, 0, None) == -10


def test_mlp_calls_reject_bad_arguments(lib):
    assert lib.mxs_mlp_forward(None, FAKE, 4, FAKE, None) == -1
    assert lib.mxs_mlp_predict(FAKE, None, 4, None, FAKE, None) == -1
    assert lib.mxs_mlp_grad(FAKE, FAKE, FAKE, 4, FAKE, FAKE, FAKE, 0, None) == -1  # workspace too small
    assert lib.mxs_mlp_adam(FAKE, FAKE, FAKE, FAKE, 1e-3, 0, 0.9, 0.999, 1e-8, None) == -1
    assert lib.mxs_mlp_train_step(FAKE, FAKE, FAKE, FAKE, FAKE, 4, 1e-3, 1, FAKE, FAKE, 8, None) == -1
    assert lib.mxs_mlp_workspace_size(128) >= 128 * (4 * 64 + 7 + 1) * 4 + 5191 * 4
    assert lib.mxs_mlp_inputs(None, 3, FAKE, FAKE, FAKE, None) == -1
    assert lib.mxs_mlp_norm_stats(FAKE, 3, None, FAKE, None) == -1


def test_load_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="no fallback"):
        mxs.load(str(tmp_path / "missing.so"))


def test_one_hip_runtime_whatever_the_import_order():
    """Loading libmxs before torch must not put a second HIP/HSA runtime in
    the process (the second one would see no device)."""
    import subprocess
    import sys
    code = ("import re, sys; sys.path.insert(0, %r); import paper_2304_09511_amd as mxs; mxs.load(); "
            "import torch; m = open('/proc/self/maps').read(); "
            "print(len(set(re.findall(r'\\S*libamdhip64\\S*', m))), "
            "len(set(re.findall(r'\\S*libhsa-runtime64\\S*', m))))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout


def test_multigrid_workspace_size_closed_form(lib):
    """mxs_mg_size is host arithmetic: per level the CSR operator, colour
    order, slice offsets, sliced off-diagonal entries (slice widths from the
    stencil's row lengths), diagonal and, below the finest level, two
    vectors; plus the build's temporaries.  It grows with n and levels and is
    bounded below by the operators' and slices' bytes."""
    sizes = {}
    for n, L in ((8, 1), (8, 2), (16, 4), (128, 4)):
        b = C.c_size_t()
        assert lib.mxs_mg_size(n, L, C.byref(b)) == 0
        sizes[(n, L)] = b.value
        low = 0
        for l in range(L):
            m = n >> l
            nnz, rows = (3 * m - 2) ** 3, m ** 3
            # CSR operator (12 bytes an entry) and the slices (off-diagonal
            # entries, 12 bytes each, at least) and the diagonal
            low += 12 * nnz + 4 * (rows + 1) + 12 * (nnz - rows) + 8 * rows + (16 * rows if l else 0)
        assert b.value >= low, (n, L, b.value, low)
        assert b.value <= 1.2 * low + (1 << 20), (n, L, b.value, low)
    assert sizes[(8, 1)] < sizes[(8, 2)] < sizes[(16, 4)] < sizes[(128, 4)]
