"""Python binding of libmxs: SpMV in COO / CSR / DIA and CG on MI355X (gfx950),
after arXiv 2304.09511 ("Morpheus unleashed").

Argument marshalling only: every step runs in the HIP library.  Device memory
belongs to torch tensors; the stream is torch's current stream.  Import works
without a GPU (so host-side validation can be tested); ``load()`` raises if
the built library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "MxsError", "load", "lib_path", "Matrix", "spmv", "dot", "axpby", "cg_solve", "stencil",
    "features", "mlp_inputs", "mlp_norm_stats", "mlp_forward", "mlp_predict", "mlp_grad",
    "mlp_adam", "mlp_train_step", "COO", "CSR", "DIA", "F64", "F32", "NPARAM",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libmxs.so")

COO, CSR, DIA, HDC, ELL, SELL, HYB = 0, 1, 2, 3, 4, 5, 6
F64, F32 = 0, 1
BORROW = 1
NPARAM = 5191  # MXS_MLP_NPARAM: MLP 8-64-64-7
NCLASS = 7     # MXS_NCLASS: outputs (COO, CSR, DIA, ELL, SELL, HYB, HDC)
FORMATS = {"coo": COO, "csr": CSR, "dia": DIA, "ell": ELL}
FORMAT_NAMES = {COO: "coo", CSR: "csr", DIA: "dia", HDC: "hdc", ELL: "ell", SELL: "sell", HYB: "hyb"}

STATUS = {
    0: "MXS_OK", 1: "MXS_NOT_CONVERGED", -1: "MXS_ERR_INVALID_ARG", -2: "MXS_ERR_INDEX_RANGE",
    -3: "MXS_ERR_UNSORTED", -4: "MXS_ERR_DUPLICATE", -5: "MXS_ERR_DIA_TOO_SPARSE",
    -6: "MXS_ERR_OUT_OF_MEMORY", -7: "MXS_ERR_HIP", -8: "MXS_ERR_BREAKDOWN",
    -9: "MXS_ERR_NONFINITE", -10: "MXS_ERR_UNSUPPORTED", -11: "MXS_ERR_NO_PLAN",
}
# plan options (mxs_plan_size, mxs_optimize)
PLAN_NO_ELL, PLAN_NO_COLBLK, PLAN_DIA_BLOCKED = 1, 2, 4


class MxsError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


def lib_path() -> str:
    return _LIB


class CgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int64), ("mixed", C.c_int32),
                ("max_outer", C.c_int32), ("inner_rtol", C.c_double),
                ("check_every", C.c_int32), ("timing", C.c_int32), ("ru_delta", C.c_double)]


class CgResult(C.Structure):
    _fields_ = [("iters", C.c_int64), ("outer_iters", C.c_int64), ("rel_resid", C.c_double),
                ("true_rel_resid", C.c_double), ("t_spmv_ms", C.c_double),
                ("t_dot_ms", C.c_double), ("t_axpy_ms", C.c_double),
                ("t_precond_ms", C.c_double)]


_lib = None
P, I32, I64, U32, D, F, SZ = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double,
                              C.c_float, C.c_size_t)

_SIGS = {
    "mxs_status_string": (C.c_char_p, [I32]),
    "mxs_version": (I32, []),
    "mxs_last_error": (C.c_char_p, []),
    "mxs_coo_create": (I32, [P, I32, I32, I64, P, P, P, I32, U32, P]),
    "mxs_csr_create": (I32, [P, I32, I32, I64, P, P, P, I32, U32, P]),
    "mxs_dia_create": (I32, [P, I32, I32, I32, P, P, I32, U32, P]),
    "mxs_destroy": (I32, [P]),
    "mxs_info": (I32, [P, P, P, P, P, P, P]),
    "mxs_arrays": (I32, [P, P, P, P]),
    "mxs_convert_size": (I32, [P, I32, P, P, P]),
    "mxs_convert": (I32, [P, I32, P, P, P, P, P]),
    "mxs_split_size": (I32, [P, D, P, P, P]),
    "mxs_split": (I32, [P, D, I32, P, P, P, P, P, P, P]),
    "mxs_split_parts": (I32, [P, P, P]),
    "mxs_sell_size": (I32, [P, I32, P, P, P]),
    "mxs_hyb_size": (I32, [P, I32, P, P, P]),
    "mxs_to_hyb": (I32, [P, I32, P, P, P, P, P, P, P]),
    "mxs_to_sell": (I32, [P, I32, P, P, P, P, P, P]),
    "mxs_cast": (I32, [P, I32, P, P, P]),
    "mxs_plan_size": (I32, [P, U32, P, P]),
    "mxs_optimize": (I32, [P, U32, P, SZ, P]),
    "mxs_plan_info": (I32, [P, P, P]),
    "mxs_spmv_scratch_size": (I32, [P, P]),
    "mxs_spmv_ws": (I32, [P, P, P, P, SZ, P]),
    "mxs_impl_count": (I32, [P]),
    "mxs_set_impl": (I32, [P, I32, P]),
    "mxs_get_impl": (I32, [P, P, P]),
    "mxs_tune": (I32, [P, P, P, I32, P, P, P]),
    "mxs_spmv": (I32, [P, P, P, P]),
    "mxs_dot": (I32, [I64, I32, P, P, P, P]),
    "mxs_dot_noalloc": (I32, [I64, I32, P, P, P, P]),
    "mxs_axpby": (I32, [I64, I32, D, P, D, P, P]),
    "mxs_cg_workspace_size": (I32, [P, I32, P]),
    "mxs_cg_solve": (I32, [P, P, P, P, P, P, P, SZ, P]),
    "mxs_mg_size": (I32, [I32, I32, P]),
    "mxs_mg_create": (I32, [I32, I32, P, SZ, P, P]),
    "mxs_mg_destroy": (I32, [P]),
    "mxs_mg_level": (I32, [P, I32, P, P]),
    "mxs_symgs": (I32, [P, I32, P, P, P]),
    "mxs_mg_apply": (I32, [P, P, P, P]),
    "mxs_pcg_workspace_size": (I32, [P, P]),
    "mxs_pcg_solve": (I32, [P, P, P, P, P, P, P, SZ, P]),
    "mxs_stencil_nnz": (I64, [I32, I32]),
    "mxs_stencil_coo": (I32, [I32, I32, D, D, P, P, P, I32, P]),
    "mxs_features": (I32, [P, P, P]),
    "mxs_mlp_inputs": (I32, [P, I32, P, P, P, P]),
    "mxs_mlp_norm_stats": (I32, [P, I32, P, P, P]),
    "mxs_mlp_forward": (I32, [P, P, I32, P, P]),
    "mxs_mlp_predict": (I32, [P, P, I32, P, P, P]),
    "mxs_mlp_workspace_size": (SZ, [I32]),
    "mxs_mlp_grad": (I32, [P, P, P, I32, P, P, P, SZ, P]),
    "mxs_mlp_adam": (I32, [P, P, P, P, F, I32, F, F, F, P]),
    "mxs_mlp_train_step": (I32, [P, P, P, P, P, I32, F, I32, P, P, SZ, P]),
}


def load(path: str | None = None):
    """Loads libmxs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2304_09511_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback path")
    # torch first: its HIP runtime is required by the name libamdhip64.so and
    # carries the soname libamdhip64.so.7, which libmxs requires.  Loaded in
    # this order the process has one HIP runtime; the other order would load
    # a second runtime (and HSA) beside torch's, which then sees no device.
    _torch()
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(st: int, where: str, ok=(0,)):
    if st not in ok:
        if st in (-6, -7) and _lib is not None:
            detail = _lib.mxs_last_error()
            if detail:
                where = f"{where} [{detail.decode(errors='replace')}]"
        raise MxsError(st, where)
    return st


# --------------------------------------------------------------- tensors
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise TypeError("device tensor required")
    if not t.is_contiguous():
        raise TypeError("contiguous tensor required")
    return C.c_void_p(t.data_ptr())


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"values must be float64 or float32, got {t.dtype}")


def _torch_dtype(code):
    torch = _torch()
    return torch.float64 if code == F64 else torch.float32


def _dev(a, dtype=None, device="cuda"):
    """numpy or tensor -> contiguous device tensor."""
    torch = _torch()
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        a = a.to(dtype)
    return a.to(device).contiguous()


# --------------------------------------------------------------- matrices
class Matrix:
    """A libmxs handle plus the tensors whose memory it borrows."""

    def __init__(self, handle, keep=(), owned=True):
        self._h = handle
        self._keep = list(keep)
        self._owned = owned  # False for the parts of a split matrix
        self._plan = None    # the plan's workspace (device memory the handle reads)
        lib = load()
        fmt, dt, nr, nc, nnz, nd = (C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(),
                                    C.c_int64(), C.c_int32())
        _check(lib.mxs_info(handle, C.byref(fmt), C.byref(dt), C.byref(nr), C.byref(nc),
                            C.byref(nnz), C.byref(nd)), "mxs_info")
        self.format, self.dtype = fmt.value, dt.value
        self.nrows, self.ncols, self.nnz, self.ndiag = nr.value, nc.value, nnz.value, nd.value

    # -- construction
    @classmethod
    def coo(cls, nrows, ncols, ai, aj, av, borrow=False):
        torch = _torch()
        ai, aj, av = _dev(ai, torch.int32), _dev(aj, torch.int32), _dev(av)
        h = C.c_void_p()
        _check(load().mxs_coo_create(C.byref(h), nrows, ncols, ai.numel(), _ptr(ai), _ptr(aj),
                                     _ptr(av), _dtype_code(av), BORROW if borrow else 0,
                                     _stream()), "mxs_coo_create")
        return cls(h, (ai, aj, av) if borrow else ())

    @classmethod
    def csr(cls, nrows, ncols, irp, aj, av, borrow=False):
        torch = _torch()
        irp, aj, av = _dev(irp, torch.int32), _dev(aj, torch.int32), _dev(av)
        h = C.c_void_p()
        _check(load().mxs_csr_create(C.byref(h), nrows, ncols, aj.numel(), _ptr(irp), _ptr(aj),
                                     _ptr(av), _dtype_code(av), BORROW if borrow else 0,
                                     _stream()), "mxs_csr_create")
        return cls(h, (irp, aj, av) if borrow else ())

    @classmethod
    def dia(cls, nrows, ncols, doff, av, borrow=False):
        """av is diagonal-major: av[d*nrows + i] multiplies x[i + doff[d]]."""
        torch = _torch()
        doff, av = _dev(doff, torch.int32), _dev(av)
        h = C.c_void_p()
        _check(load().mxs_dia_create(C.byref(h), nrows, ncols, doff.numel(), _ptr(doff),
                                     _ptr(av), _dtype_code(av), BORROW if borrow else 0,
                                     _stream()), "mxs_dia_create")
        return cls(h, (doff, av) if borrow else ())

    @classmethod
    def from_workload(cls, coo, fmt="coo", dtype=None):
        """A workloads.Coo uploaded as COO and converted to `fmt` on the device."""
        av = coo.av if dtype is None else coo.av.astype(dtype)
        A = cls.coo(coo.nrows, coo.ncols, coo.ai, coo.aj, av)
        if FORMATS.get(fmt, fmt) == COO:
            return A
        B = A.convert(fmt)
        A.close()
        return B

    # -- queries
    @property
    def handle(self):
        return self._h

    def arrays_ptr(self):
        i0, i1, v = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(load().mxs_arrays(self._h, C.byref(i0), C.byref(i1), C.byref(v)), "mxs_arrays")
        return i0.value, i1.value, v.value

    def convert_size(self, fmt):
        cnt, nd = C.c_int64(), C.c_int32()
        _check(load().mxs_convert_size(self._h, FORMATS.get(fmt, fmt), C.byref(cnt), C.byref(nd),
                                       _stream()), "mxs_convert_size")
        return cnt.value, nd.value

    def convert(self, fmt):
        """Converts into freshly allocated tensors; returns the new Matrix."""
        torch = _torch()
        f = FORMATS.get(fmt, fmt)
        cnt, nd = self.convert_size(f)
        dev = "cuda"
        vals = torch.empty(max(cnt, 0), dtype=_torch_dtype(self.dtype), device=dev)
        if f == COO:
            i0 = torch.empty(cnt, dtype=torch.int32, device=dev)
            i1 = torch.empty(cnt, dtype=torch.int32, device=dev)
        elif f == CSR:
            i0 = torch.empty(self.nrows + 1, dtype=torch.int32, device=dev)
            i1 = torch.empty(cnt, dtype=torch.int32, device=dev)
        elif f == ELL:
            i0 = torch.empty(cnt, dtype=torch.int32, device=dev)
            i1 = None
        else:
            i0 = torch.empty(nd, dtype=torch.int32, device=dev)
            i1 = None
        h = C.c_void_p()
        _check(load().mxs_convert(self._h, f, _ptr(i0) if i0.numel() else None,
                                  _ptr(i1) if i1 is not None and i1.numel() else None,
                                  _ptr(vals) if vals.numel() else None, C.byref(h), _stream()),
               "mxs_convert")
        return Matrix(h, [t for t in (i0, i1, vals) if t is not None])

    def split_size(self, min_fill=0.5):
        nd, rn = C.c_int32(), C.c_int64()
        _check(load().mxs_split_size(self._h, min_fill, C.byref(nd), C.byref(rn), _stream()),
               "mxs_split_size")
        return nd.value, rn.value

    def split(self, min_fill=0.5, rest="csr", x=None, reps=10, model=None):
        """A DIA band (diagonals at least min_fill full) plus the remaining
        entries in `rest` ("coo" or "csr"), as an HDC Matrix on fresh tensors.
        rest="auto" splits both ways, tunes each (tune(), on x or a seeded
        uniform vector) and keeps the faster split; its choice is in
        .tuning.  rest="select" asks the format selector's network (`model`,
        default the committed one) for COO or CSR on the remainder's
        features; its choice is in .selection."""
        torch = _torch()
        if rest == "select":
            from . import selector as S
            m = model if model is not None else S.Selector.load(str(S.MODEL_PATH))
            H = self.split(min_fill, "coo")
            r = S.select_rest(m, H.parts()[1])
            if r != "coo":
                H.close()
                H = self.split(min_fill, r)
            H.selection = {"rest_format": r}
            return H
        if rest == "auto":
            if x is None:
                g = torch.Generator(device="cuda")
                g.manual_seed(1)
                x = (torch.rand(self.ncols, generator=g, device="cuda",
                                dtype=torch.float64) * 2 - 1).to(_torch_dtype(self.dtype))
            best = None
            for r in ("coo", "csr"):
                H = self.split(min_fill, r)
                H.tuning = H.tune(x, reps=reps)
                H.tuning["rest_format"] = r
                if best is None or H.tuning["ms"] < best.tuning["ms"]:
                    if best is not None:
                        best.close()
                    best = H
                else:
                    H.close()
            return best
        f = FORMATS.get(rest, rest)
        nd, rn = self.split_size(min_fill)
        dt = _torch_dtype(self.dtype)
        doff = torch.empty(nd, dtype=torch.int32, device="cuda")
        band = torch.empty(nd * self.nrows, dtype=dt, device="cuda")
        i0 = torch.empty(self.nrows + 1 if f == CSR else rn, dtype=torch.int32, device="cuda")
        i1 = torch.empty(rn, dtype=torch.int32, device="cuda")
        vals = torch.empty(rn, dtype=dt, device="cuda")
        h = C.c_void_p()
        nz = lambda t: _ptr(t) if t.numel() else None
        _check(load().mxs_split(self._h, min_fill, f, nz(doff), nz(band), nz(i0), nz(i1), nz(vals),
                                C.byref(h), _stream()), "mxs_split")
        return Matrix(h, [doff, band, i0, i1, vals])

    def hyb_size(self, K=-1):
        k, r = C.c_int32(), C.c_int64()
        _check(load().mxs_hyb_size(self._h, int(K), C.byref(k), C.byref(r), _stream()),
               "mxs_hyb_size")
        return k.value, r.value

    def to_hyb(self, K=-1):
        """HYB on fresh tensors (K < 0: the width rule), kept as
        [ell_col, ell_val, rest_ai, rest_aj, rest_av]."""
        torch = _torch()
        k, r = self.hyb_size(K)
        dt = _torch_dtype(self.dtype)
        ecol = torch.empty(max(k * self.nrows, 1), dtype=torch.int32, device="cuda")
        ev = torch.empty(max(k * self.nrows, 1), dtype=dt, device="cuda")
        ri = torch.empty(max(r, 1), dtype=torch.int32, device="cuda")
        rj = torch.empty(max(r, 1), dtype=torch.int32, device="cuda")
        rv = torch.empty(max(r, 1), dtype=dt, device="cuda")
        h = C.c_void_p()
        _check(load().mxs_to_hyb(self._h, int(K), _ptr(ecol), _ptr(ev), _ptr(ri), _ptr(rj), _ptr(rv),
                                 C.byref(h), _stream()), "mxs_to_hyb")
        n = k * self.nrows
        return Matrix(h, [ecol[:n], ev[:n], ri[:r], rj[:r], rv[:r]])

    def sell_size(self, sigma=1):
        sl, ns = C.c_int64(), C.c_int32()
        _check(load().mxs_sell_size(self._h, int(sigma), C.byref(sl), C.byref(ns), _stream()),
               "mxs_sell_size")
        return sl.value, ns.value

    def to_sell(self, sigma=1):
        """SELL-64-sigma on fresh tensors, kept as [perm, cs, col, vals]."""
        torch = _torch()
        slots, ns = self.sell_size(sigma)
        perm = torch.empty(max(self.nrows, 1), dtype=torch.int32, device="cuda")
        cs = torch.empty(ns + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(slots, 1), dtype=torch.int32, device="cuda")
        vals = torch.empty(max(slots, 1), dtype=_torch_dtype(self.dtype), device="cuda")
        h = C.c_void_p()
        _check(load().mxs_to_sell(self._h, int(sigma), _ptr(perm), _ptr(cs), _ptr(col), _ptr(vals),
                                  C.byref(h), _stream()), "mxs_to_sell")
        M = Matrix(h, [perm[:self.nrows], cs, col[:slots], vals[:slots]])
        M._slots = slots
        return M

    def cast(self, dtype):
        torch = _torch()
        code = F32 if dtype in (F32, torch.float32, np.float32, "f32") else F64
        n = (self.ndiag * self.nrows if self.format in (DIA, ELL) else
             self._slots if self.format == SELL else self.nnz)
        vals = torch.empty(n, dtype=_torch_dtype(code), device="cuda")
        h = C.c_void_p()
        _check(load().mxs_cast(self._h, code, _ptr(vals) if n else None, C.byref(h), _stream()),
               "mxs_cast")
        M = Matrix(h, [vals, self])
        if self.format == SELL:
            M._slots = self._slots
        return M

    def export(self):
        """Copies of the canonical arrays as CPU numpy arrays: COO (ai, aj, av),
        CSR (irp, aj, av), DIA (doff, av), ELL (col, val); SELL exports its
        CSR form (irp, aj, av)."""
        B = self.convert(CSR if self.format == SELL else self.format)
        out = [t.cpu().numpy() for t in B._keep]
        B.close()
        return tuple(out)

    def plan_size(self, opts=0):
        """Bytes of device workspace the plan needs with these options."""
        n = C.c_size_t()
        _check(load().mxs_plan_size(self._h, int(opts), C.byref(n), _stream()), "mxs_plan_size")
        return n.value

    def optimize(self, opts=0, workspace=None):
        """Builds the plan in a torch tensor (allocated here unless given),
        kept with this Matrix until close() or the next optimize()."""
        torch = _torch()
        n = self.plan_size(opts)
        if workspace is None:
            workspace = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
        if workspace.numel() * workspace.element_size() < n:
            raise ValueError("plan workspace too small")
        _check(load().mxs_optimize(self._h, int(opts), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream()),
               "mxs_optimize")
        self._plan = workspace
        return self

    @property
    def optimized(self):
        v = C.c_int32()
        _check(load().mxs_plan_info(self._h, C.byref(v), None), "mxs_plan_info")
        return bool(v.value)

    def ensure_plan(self):
        """Builds the default plan if the handle has none (the C library never
        builds one implicitly)."""
        if not self.optimized:
            self.optimize()
        return self

    def spmv_scratch_size(self):
        n = C.c_size_t()
        _check(load().mxs_spmv_scratch_size(self._h, C.byref(n)), "mxs_spmv_scratch_size")
        return n.value

    # SpMV implementations of the format (ids as in mxs_set_impl)
    IMPL_NAMES = {COO: ("row_tiles", "segmented", "column_blocks"),
                  CSR: ("entry_tiles", "row_per_thread", "staged_gather", "ell_copy", "column_blocks",
                        "wave_per_row"),
                  DIA: ("blocked_shared_x", "blocked", "diagonal_major")}

    @property
    def impl(self):
        self.ensure_plan()
        v = C.c_int32()
        _check(load().mxs_get_impl(self._h, C.byref(v), _stream()), "mxs_get_impl")
        return v.value

    @impl.setter
    def impl(self, i):
        self.ensure_plan()
        _check(load().mxs_set_impl(self._h, int(i), _stream()), "mxs_set_impl")

    def impl_count(self):
        return load().mxs_impl_count(self._h)

    def parts(self):
        """(band, rest) of a split or HYB matrix: handles owned by this one."""
        self.ensure_plan()  # the parts are planned with this matrix
        b, r = C.c_void_p(), C.c_void_p()
        _check(load().mxs_split_parts(self._h, C.byref(b), C.byref(r)), "mxs_split_parts")
        return Matrix(b, [self], owned=False), Matrix(r, [self], owned=False)

    def tune(self, x, y=None, reps=10):
        """Times every applicable implementation on y = A x, keeps the
        fastest; returns (id, [median ms per id, None where not applicable]).
        A split matrix tunes its two parts and returns a dict: each part's
        choice and times, and the median time of the whole product ("ms")."""
        torch = _torch()
        if y is None:
            y = torch.empty(self.nrows, dtype=x.dtype, device=x.device)
        if self.format == HDC:
            band, rest = self.parts()
            out = {"band": band.tune(x, y, reps), "rest": rest.tune(x, y, reps)}
            out["ms"] = _median_ms(torch, lambda: spmv(self, x, y), reps)
            return out
        if _dtype_code(x) != self.dtype or _dtype_code(y) != self.dtype:
            raise TypeError("x and y must have the matrix's dtype")
        if x.numel() != self.ncols or y.numel() != self.nrows:
            raise ValueError("vector lengths do not match the matrix")
        self.ensure_plan()
        n = max(self.impl_count(), 1)
        ms = (C.c_double * n)()
        best = C.c_int32()
        _check(load().mxs_tune(self._h, _ptr(x), _ptr(y), int(reps), C.byref(best), ms,
                               _stream()), "mxs_tune")
        return best.value, [None if m < 0 else m for m in ms[:self.impl_count()]]

    def close(self):
        if self._h is not None and _lib is not None and self._owned:
            _check(_lib.mxs_destroy(self._h), "mxs_destroy")
        self._h = None
        self._keep = []
        self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _median_ms(torch, fn, reps):
    for _ in range(3):
        fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


# --------------------------------------------------------------- operations
def spmv(A: Matrix, x, y=None, scratch=None):
    """y = A x on the device (y allocated when not given; A's default plan
    built first if it has none).  With `scratch` (a device tensor of at least
    A.spmv_scratch_size() bytes) the carries go there (mxs_spmv_ws), so calls
    on A from several streams may overlap."""
    torch = _torch()
    if y is None:
        y = torch.empty(A.nrows, dtype=x.dtype, device=x.device)
    if _dtype_code(x) != A.dtype or _dtype_code(y) != A.dtype:
        raise TypeError("x and y must have the matrix's dtype")
    if x.numel() != A.ncols or y.numel() != A.nrows:
        raise ValueError("vector lengths do not match the matrix")
    A.ensure_plan()
    if scratch is None:
        _check(load().mxs_spmv(A.handle, _ptr(x), _ptr(y), _stream()), "mxs_spmv")
    else:
        nb = scratch.numel() * scratch.element_size()
        _check(load().mxs_spmv_ws(A.handle, _ptr(x), _ptr(y), _ptr(scratch) if nb else None, nb,
                                  _stream()), "mxs_spmv_ws")
    return y


def dot(a, b):
    """a.b accumulated in FP64, as a device scalar tensor."""
    torch = _torch()
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    _check(load().mxs_dot(a.numel(), _dtype_code(a), _ptr(a), _ptr(b), _ptr(out), _stream()),
           "mxs_dot")
    return out


def dot_noalloc(a, b, out):
    """a.b into the caller's FP64 device tensor `out` (one element) through
    the allocation-free entry point (no device memory is allocated)."""
    if a.numel() != b.numel() or _dtype_code(a) != _dtype_code(b):
        raise ValueError("a and b must have the same length and dtype")
    if out.numel() < 1 or _dtype_code(out) != 0:
        raise TypeError("out must be an FP64 device tensor with at least one element")
    _check(load().mxs_dot_noalloc(a.numel(), _dtype_code(a), _ptr(a), _ptr(b), _ptr(out),
                                  _stream()), "mxs_dot_noalloc", ok=(0,))
    return out


def axpby(alpha, x, beta, y):
    _check(load().mxs_axpby(x.numel(), _dtype_code(x), alpha, _ptr(x), beta, _ptr(y), _stream()),
           "mxs_axpby")
    return y


def cg_workspace(A: Matrix, mixed=False):
    torch = _torch()
    n = C.c_size_t()
    _check(load().mxs_cg_workspace_size(A.handle, 1 if mixed else 0, C.byref(n)),
           "mxs_cg_workspace_size")
    return torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")


MIXED_MODES = {False: 0, True: 1, 0: 0, 1: 1, 2: 2, "fp64": 0, "ir": 1, "ru": 2}


def cg_solve(A: Matrix, b, x0=None, rtol=1e-9, maxit=10000, mixed=False, A32=None,
             inner_rtol=1e-4, max_outer=20, check_every=16, timing=False, workspace=None,
             delta=0.1):
    """Solves A x = b.  mixed: False (FP64 CG), True or "ir" (iterative
    refinement with FP32 inner CG), "ru" (FP32 CG with FP64 reliable
    updates).  Returns (status, x, CgResult as a dict)."""
    torch = _torch()
    mode = MIXED_MODES[mixed]
    A.ensure_plan()
    if A32 is not None:
        A32.ensure_plan()
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    ws = workspace if workspace is not None else cg_workspace(A, mode)
    o = CgOpts(rtol, maxit, mode, max_outer, inner_rtol, check_every, 1 if timing else 0, delta)
    r = CgResult()
    st = load().mxs_cg_solve(A.handle, A32.handle if A32 is not None else None, _ptr(b), _ptr(x),
                             C.byref(o), C.byref(r), _ptr(ws), ws.numel(), _stream())
    _check(st, "mxs_cg_solve", ok=(0, 1, -8))
    res = {k: getattr(r, k) for k, _ in CgResult._fields_}
    return st, x, res


class Multigrid:
    """HPCG's multigrid preconditioner on the n^3 27-point stencil (levels
    grids, finest first)."""

    def __init__(self, n, levels=4):
        torch = _torch()
        nb = C.c_size_t()
        _check(load().mxs_mg_size(int(n), int(levels), C.byref(nb)), "mxs_mg_size")
        self._ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _check(load().mxs_mg_create(int(n), int(levels), _ptr(self._ws), nb.value, C.byref(h),
                                    _stream()), "mxs_mg_create")
        self._h, self.n, self.levels = h, n, levels
        self._lv = {}  # level -> (n, operator Matrix), kept: a plan built on one lives here

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("closed multigrid hierarchy")
        return self._h

    def level(self, l):
        """(grid edge, operator Matrix owned by the hierarchy) of level l."""
        if l not in self._lv or self._lv[l][1]._h is None:
            n, a = C.c_int32(), C.c_void_p()
            _check(load().mxs_mg_level(self.handle, int(l), C.byref(n), C.byref(a)), "mxs_mg_level")
            self._lv[l] = (n.value, Matrix(a, [], owned=False))
        return self._lv[l]

    def symgs(self, level, r, x):
        """One symmetric Gauss-Seidel sweep of `level` on x in place."""
        _check(load().mxs_symgs(self.handle, int(level), _ptr(r), _ptr(x), _stream()), "mxs_symgs")
        return x

    def apply(self, r, z=None):
        """z = M^{-1} r (one V-cycle)."""
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        _check(load().mxs_mg_apply(self.handle, _ptr(r), _ptr(z), _stream()), "mxs_mg_apply")
        return z

    def pcg_solve(self, b, x0=None, A=None, rtol=1e-9, maxit=10000, check_every=4,
                  timing=False, workspace=None):
        """PCG on A x = b preconditioned by this hierarchy (A: the finest
        operator in any format, default the hierarchy's CSR).  Returns
        (status, x, CgResult as a dict)."""
        torch = _torch()
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        if workspace is None:
            nb = C.c_size_t()
            _check(load().mxs_pcg_workspace_size(self.handle, C.byref(nb)), "mxs_pcg_workspace_size")
            workspace = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
        (A if A is not None else self.level(0)[1]).ensure_plan()
        o = CgOpts(rtol, maxit, 0, 0, 0.0, check_every, 1 if timing else 0, 0.0)
        r = CgResult()
        st = load().mxs_pcg_solve(self.handle, A.handle if A is not None else None, _ptr(b),
                                  _ptr(x), C.byref(o), C.byref(r), _ptr(workspace),
                                  workspace.numel(), _stream())
        _check(st, "mxs_pcg_solve", ok=(0, 1, -8))
        return st, x, {k: getattr(r, k) for k, _ in CgResult._fields_}

    def close(self):
        if self._h is not None and _lib is not None:
            _check(_lib.mxs_mg_destroy(self._h), "mxs_mg_destroy")
        self._h = None
        for _, m in self._lv.values():
            m._h, m._plan = None, None
        self._lv = {}
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stencil(n, points=27, diag=None, offdiag=-1.0, dtype=F64, fmt="coo"):
    """The HPCG stencil generated on the device, as a Matrix in `fmt`."""
    torch = _torch()
    diag = (26.0 if points == 27 else 6.0) if diag is None else diag
    lib = load()
    nnz = lib.mxs_stencil_nnz(n, points)
    ai = torch.empty(nnz, dtype=torch.int32, device="cuda")
    aj = torch.empty(nnz, dtype=torch.int32, device="cuda")
    av = torch.empty(nnz, dtype=_torch_dtype(dtype), device="cuda")
    _check(lib.mxs_stencil_coo(n, points, diag, offdiag, _ptr(ai), _ptr(aj), _ptr(av), dtype,
                               _stream()), "mxs_stencil_coo")
    A = Matrix.coo(n ** 3, n ** 3, ai, aj, av, borrow=True)
    if FORMATS.get(fmt, fmt) == COO:
        return A
    B = A.convert(fmt)
    A.close()
    return B


def features(A: Matrix):
    out = (C.c_double * 8)()
    _check(load().mxs_features(A.handle, out, _stream()), "mxs_features")
    return np.array(out[:], dtype=np.float64)


# --------------------------------------------------------------- selector MLP
def mlp_norm_stats(raw):
    torch = _torch()
    mu = torch.empty(8, dtype=torch.float32, device="cuda")
    sd = torch.empty(8, dtype=torch.float32, device="cuda")
    _check(load().mxs_mlp_norm_stats(_ptr(raw), raw.shape[0], _ptr(mu), _ptr(sd), _stream()),
           "mxs_mlp_norm_stats")
    return mu, sd


def mlp_inputs(raw, mu, sd):
    torch = _torch()
    X = torch.empty(raw.shape[0], 8, dtype=torch.float32, device="cuda")
    _check(load().mxs_mlp_inputs(_ptr(raw), raw.shape[0], _ptr(mu), _ptr(sd), _ptr(X),
                                 _stream()), "mxs_mlp_inputs")
    return X


def _mlp_shapes(w, X, feasible=None):
    """The ABI takes raw pointers: check sizes here so no kernel reads or
    writes past an array."""
    if w.numel() != NPARAM or X.dim() != 2 or X.shape[1] != 8:
        raise ValueError("w must hold NPARAM values and X be [n][8]")
    if feasible is not None and feasible.numel() != X.shape[0] * NCLASS:
        raise ValueError("feasible must be [n][NCLASS]")


def mlp_forward(w, X):
    torch = _torch()
    _mlp_shapes(w, X)
    z = torch.empty(X.shape[0], NCLASS, dtype=torch.float32, device="cuda")
    _check(load().mxs_mlp_forward(_ptr(w), _ptr(X), X.shape[0], _ptr(z), _stream()),
           "mxs_mlp_forward")
    return z


def mlp_predict(w, X, feasible=None):
    torch = _torch()
    _mlp_shapes(w, X, feasible)
    out = torch.empty(X.shape[0], dtype=torch.int32, device="cuda")
    _check(load().mxs_mlp_predict(_ptr(w), _ptr(X), X.shape[0], _ptr(feasible), _ptr(out),
                                  _stream()), "mxs_mlp_predict")
    return out


def mlp_workspace(n):
    torch = _torch()
    return torch.empty(load().mxs_mlp_workspace_size(n), dtype=torch.uint8, device="cuda")


def mlp_grad(w, X, labels, workspace=None):
    torch = _torch()
    n = X.shape[0]
    _mlp_shapes(w, X)
    ws = workspace if workspace is not None else mlp_workspace(n)
    g = torch.empty(NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(load().mxs_mlp_grad(_ptr(w), _ptr(X), _ptr(labels), n, _ptr(g), _ptr(loss), _ptr(ws),
                               ws.numel(), _stream()), "mxs_mlp_grad")
    return loss, g


def mlp_adam(w, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    _check(load().mxs_mlp_adam(_ptr(w), _ptr(m), _ptr(v), _ptr(g), lr, t, b1, b2, eps,
                               _stream()), "mxs_mlp_adam")


def mlp_train_step(w, m, v, X, labels, lr, t, workspace=None):
    torch = _torch()
    n = X.shape[0]
    _mlp_shapes(w, X)
    ws = workspace if workspace is not None else mlp_workspace(n)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(load().mxs_mlp_train_step(_ptr(w), _ptr(m), _ptr(v), _ptr(X), _ptr(labels), n, lr, t,
                                     _ptr(loss), _ptr(ws), ws.numel(), _stream()),
           "mxs_mlp_train_step")
    return loss
