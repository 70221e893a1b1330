"""Python view of the CPU oracle (``oracle.c``): a plain FP64 reference for the
SpMV / CG path of arXiv 2304.09511.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it.  It shares no code with the GPU library and never imports it.
Inputs come from ``workloads`` (structure and values only).

Functions take and return numpy arrays; the index base is 0 and all ranges are
half-open, as in the loops of Algorithms 1-3.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, INDEX_RANGE, UNSORTED, DUPLICATE, BREAKDOWN, NONFINITE = 0, 1, -2, -3, -4, -8, -9
NPARAM = 5191
NFEAT = 8
NCLASS = 7


def build(out: str | None = None, src: str | None = None) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    out = out or _LIB_PATH
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", out, src or _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


class use_library:
    """Context manager: route every call through another build of the oracle
    (used by the tests that plant mistakes in a copy of the source)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _load(path: str | None = None):
    """The oracle library; ORACLE_LIB names another build of it (the
    sanitizer run of the pins uses that)."""
    global _lib
    if path is not None:
        return _bind(C.CDLL(path))
    if _lib is None:
        other = os.environ.get("ORACLE_LIB")
        if other:
            _lib = _bind(C.CDLL(other))
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(C.CDLL(_LIB_PATH))
    return _lib


P = C.c_void_p
I64 = C.c_int64
D = C.c_double


def _bind(lib):
    sig = {
        "orc_coo_spmv": (None, [I64, I64, P, P, P, P, P]),
        "orc_coo_spmv_f32": (None, [I64, I64, P, P, P, P, P]),
        "orc_csr_spmv": (None, [I64, P, P, P, P, P]),
        "orc_dia_spmv": (None, [I64, I64, I64, P, P, P, P]),
        "orc_coo_check": (C.c_int, [I64, I64, I64, P, P]),
        "orc_csr_check": (C.c_int, [I64, I64, I64, P, P]),
        "orc_coo_sort": (None, [I64, I64, I64, P, P, P]),
        "orc_coo_to_csr": (None, [I64, I64, P, P]),
        "orc_csr_to_coo": (None, [I64, P, P]),
        "orc_dia_offsets": (I64, [I64, I64, I64, P, P, P]),
        "orc_coo_to_dia": (None, [I64, I64, P, P, P, I64, P, P]),
        "orc_dia_nnz": (I64, [I64, I64, I64, P, P]),
        "orc_dia_slots": (I64, [I64, I64, I64, P]),
        "orc_dia_to_coo": (None, [I64, I64, I64, P, P, P, P, P]),
        "orc_dot": (D, [I64, P, P]),
        "orc_cg": (C.c_int, [I64, I64, P, P, P, P, P, D, I64, P, P]),
        "orc_mixed_ir": (C.c_int, [I64, I64, P, P, P, P, P, D, D, I64, I64, P, P]),
        "orc_split_offsets": (I64, [I64, I64, I64, P, P, D, P]),
        "orc_mixed_ru": (C.c_int, [I64, I64, P, P, P, P, P, D, D, I64, P, P]),
        "orc_features": (None, [I64, I64, I64, P, P, P]),
        "orc_mlp_nparam": (I64, []),
        "orc_mlp_forward": (None, [P, P, I64, P]),
        "orc_mlp_loss_grad": (D, [P, P, P, I64, P]),
        "orc_adam_step": (None, [I64, P, P, P, P, D, I64, D, D, D]),
        "orc_symgs": (C.c_int, [I64, P, P, P, P, P, P]),
        "orc_ell_width": (I64, [I64, P]),
        "orc_hyb_width": (I64, [I64, P]),
        "orc_hyb_rest": (I64, [I64, P, I64]),
        "orc_csr_to_hyb": (None, [I64, P, P, P, I64, P, P, P, P, P]),
        "orc_csr_to_ell": (None, [I64, P, P, P, I64, P, P]),
        "orc_ell_spmv": (None, [I64, I64, P, P, P, P]),
        "orc_sell_perm": (None, [I64, P, I64, P]),
        "orc_sell_offsets": (I64, [I64, P, P, I64, P]),
        "orc_csr_to_sell": (None, [I64, P, P, P, I64, P, P, P, P]),
        "orc_sell_spmv": (None, [I64, I64, P, P, P, P, P, P]),
        "orc_gs_sweep": (C.c_int, [I64, P, P, P, P, C.c_int, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ----------------------------------------------------------------- SpMV
def coo_spmv(nrows, ai, aj, av, x):
    """Algorithm 1 over all stored entries, y cleared first: y = A x (FP64)."""
    ai, aj, av, x = _i32(ai), _i32(aj), _f64(av), _f64(x)
    y = np.empty(nrows, np.float64)
    _load().orc_coo_spmv(nrows, ai.shape[0], _p(ai), _p(aj), _p(av), _p(x), _p(y))
    return y


def coo_spmv_f32(nrows, ai, aj, av, x):
    """Algorithm 1 in float arithmetic (float products, float accumulation)."""
    ai, aj, av, x = _i32(ai), _i32(aj), _f32(av), _f32(x)
    y = np.empty(nrows, np.float32)
    _load().orc_coo_spmv_f32(nrows, ai.shape[0], _p(ai), _p(aj), _p(av), _p(x), _p(y))
    return y


def csr_spmv(irp, aj, av, x):
    """Algorithm 2: per-row sums assigned to y."""
    irp, aj, av, x = _i32(irp), _i32(aj), _f64(av), _f64(x)
    nrows = irp.shape[0] - 1
    y = np.empty(nrows, np.float64)
    _load().orc_csr_spmv(nrows, _p(irp), _p(aj), _p(av), _p(x), _p(y))
    return y


def dia_spmv(nrows, ncols, doff, av_dia, x):
    """Algorithm 3 with N = ncols; av_dia is diagonal-major [ndiag][nrows]."""
    doff, av_dia, x = _i32(doff), _f64(av_dia), _f64(x)
    y = np.empty(nrows, np.float64)
    _load().orc_dia_spmv(nrows, ncols, doff.shape[0], _p(doff), _p(av_dia), _p(x), _p(y))
    return y


# ----------------------------------------------------------- conversions
def coo_check(nrows, ncols, ai, aj) -> int:
    ai, aj = _i32(ai), _i32(aj)
    return int(_load().orc_coo_check(nrows, ncols, ai.shape[0], _p(ai), _p(aj)))


def csr_check(nrows, ncols, irp, aj) -> int:
    irp, aj = _i32(irp), _i32(aj)
    return int(_load().orc_csr_check(nrows, ncols, aj.shape[0], _p(irp), _p(aj)))


def coo_sort(nrows, ncols, ai, aj, av):
    """Triples sorted by (row, col), stably.  Returns new arrays."""
    ai, aj, av = _i32(ai).copy(), _i32(aj).copy(), _f64(av).copy()
    _load().orc_coo_sort(nrows, ncols, ai.shape[0], _p(ai), _p(aj), _p(av))
    return ai, aj, av


def coo_to_csr(nrows, ai):
    ai = _i32(ai)
    irp = np.empty(nrows + 1, np.int32)
    _load().orc_coo_to_csr(nrows, ai.shape[0], _p(ai), _p(irp))
    return irp


def csr_to_coo(irp):
    irp = _i32(irp)
    nrows = irp.shape[0] - 1
    ai = np.empty(int(irp[-1]) if nrows >= 0 else 0, np.int32)
    _load().orc_csr_to_coo(nrows, _p(irp), _p(ai))
    return ai


def dia_offsets(nrows, ncols, ai, aj):
    ai, aj = _i32(ai), _i32(aj)
    buf = np.empty(max(nrows + ncols - 1, 1), np.int32)
    nd = _load().orc_dia_offsets(nrows, ncols, ai.shape[0], _p(ai), _p(aj), _p(buf))
    return buf[:nd].copy()


def coo_to_dia(nrows, ncols, ai, aj, av):
    """(doff, av_dia[ndiag*nrows]) of a sorted COO matrix."""
    ai, aj, av = _i32(ai), _i32(aj), _f64(av)
    doff = dia_offsets(nrows, ncols, ai, aj)
    av_dia = np.empty(doff.shape[0] * nrows, np.float64)
    _load().orc_coo_to_dia(nrows, ai.shape[0], _p(ai), _p(aj), _p(av), doff.shape[0],
                           _p(doff), _p(av_dia))
    return doff, av_dia


def dia_slots(nrows, ncols, doff) -> int:
    doff = _i32(doff)
    return int(_load().orc_dia_slots(nrows, ncols, doff.shape[0], _p(doff)))


def dia_to_coo(nrows, ncols, doff, av_dia):
    doff, av_dia = _i32(doff), _f64(av_dia)
    nd = doff.shape[0]
    lib = _load()
    nnz = int(lib.orc_dia_nnz(nrows, ncols, nd, _p(doff), _p(av_dia)))
    ai = np.empty(nnz, np.int32)
    aj = np.empty(nnz, np.int32)
    av = np.empty(nnz, np.float64)
    lib.orc_dia_to_coo(nrows, ncols, nd, _p(doff), _p(av_dia), _p(ai), _p(aj), _p(av))
    return ai, aj, av


# ------------------------------------------------------------------ CG
def dot(a, b) -> float:
    a, b = _f64(a), _f64(b)
    return float(_load().orc_dot(a.shape[0], _p(a), _p(b)))


def cg(n, ai, aj, av, b, x0=None, tol=1e-9, maxit=10000):
    """Unpreconditioned CG.  Returns (status, x, iters, rel_resid, true_rel_resid)."""
    ai, aj, av, b = _i32(ai), _i32(aj), _f64(av), _f64(b)
    x = np.zeros(n, np.float64) if x0 is None else _f64(x0).copy()
    iters = np.zeros(1, np.int64)
    out = np.zeros(2, np.float64)
    st = _load().orc_cg(n, ai.shape[0], _p(ai), _p(aj), _p(av), _p(b), _p(x), tol, maxit,
                        _p(iters), _p(out))
    return int(st), x, int(iters[0]), float(out[0]), float(out[1])


def mixed_ir(n, ai, aj, av, b, x0=None, tol=1e-10, inner_rtol=1e-4, inner_maxit=10000,
             max_outer=20):
    """FP64-outer / FP32-inner refinement.
    Returns (status, x, corrections, inner_iters_total, true_rel_resid)."""
    ai, aj, av, b = _i32(ai), _i32(aj), _f64(av), _f64(b)
    x = np.zeros(n, np.float64) if x0 is None else _f64(x0).copy()
    counts = np.zeros(2, np.int64)
    out = np.zeros(1, np.float64)
    st = _load().orc_mixed_ir(n, ai.shape[0], _p(ai), _p(aj), _p(av), _p(b), _p(x), tol,
                              inner_rtol, inner_maxit, max_outer, _p(counts), _p(out))
    return int(st), x, int(counts[0]), int(counts[1]), float(out[0])


def mixed_ru(n, ai, aj, av, b, x0=None, tol=1e-10, delta=0.1, maxit=10000):
    """FP32 CG with FP64 reliable updates (residual replacement).
    Returns (status, x, updates, iters, true_rel_resid)."""
    ai, aj, av, b = _i32(ai), _i32(aj), _f64(av), _f64(b)
    x = np.zeros(n, np.float64) if x0 is None else _f64(x0).copy()
    counts = np.zeros(2, np.int64)
    out = np.zeros(1, np.float64)
    st = _load().orc_mixed_ru(n, ai.shape[0], _p(ai), _p(aj), _p(av), _p(b), _p(x), tol, delta,
                              maxit, _p(counts), _p(out))
    return int(st), x, int(counts[0]), int(counts[1]), float(out[0])


def split_offsets(nrows, ncols, ai, aj, min_fill=0.5):
    """Offsets of the band of a split (ascending)."""
    ai, aj = _i32(ai), _i32(aj)
    out = np.empty(max(nrows + ncols - 1, 1), np.int32)
    nd = _load().orc_split_offsets(nrows, ncols, ai.shape[0], _p(ai), _p(aj), min_fill, _p(out))
    return out[:nd].copy()


# ------------------------------------------------------------ selector
def features(nrows, ncols, ai, aj):
    ai, aj = _i32(ai), _i32(aj)
    f = np.empty(NFEAT, np.float64)
    _load().orc_features(nrows, ncols, ai.shape[0], _p(ai), _p(aj), _p(f))
    return f


def mlp_forward(w, X):
    w, X = _f64(w), _f64(X).reshape(-1, NFEAT)
    z = np.empty((X.shape[0], NCLASS), np.float64)
    _load().orc_mlp_forward(_p(w), _p(X), X.shape[0], _p(z))
    return z


def mlp_loss_grad(w, X, labels):
    w, X, labels = _f64(w), _f64(X).reshape(-1, NFEAT), _i32(labels)
    g = np.empty(NPARAM, np.float64)
    loss = _load().orc_mlp_loss_grad(_p(w), _p(X), _p(labels), X.shape[0], _p(g))
    return float(loss), g


def adam_step(w, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays w, m, v."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    _load().orc_adam_step(w.shape[0], _p(w), _p(m), _p(v), _p(g), lr, t, b1, b2, eps)


# ------------------------------------------- ELL and SELL-C-sigma (Sec. IX)
def csr_to_ell(irp, aj, av):
    """(K, col[K*nrows], val[K*nrows]): ELL, column-major, padding col -1."""
    irp, aj, av = _i32(irp), _i32(aj), _f64(av)
    n = irp.shape[0] - 1
    lib = _load()
    K = int(lib.orc_ell_width(n, _p(irp)))
    col = np.empty(K * n, np.int32)
    val = np.empty(K * n, np.float64)
    lib.orc_csr_to_ell(n, _p(irp), _p(aj), _p(av), K, _p(col), _p(val))
    return K, col, val


def ell_spmv(nrows, K, col, val, x):
    col, val, x = _i32(col), _f64(val), _f64(x)
    y = np.empty(nrows, np.float64)
    _load().orc_ell_spmv(nrows, K, _p(col), _p(val), _p(x), _p(y))
    return y


def ell_to_csr(nrows, K, col, val):
    """Back to canonical CSR: a row's non-padding slots in slot order."""
    col = np.asarray(col).reshape(K, nrows)
    val = np.asarray(val).reshape(K, nrows)
    keep = col >= 0
    lens = keep.sum(axis=0)
    irp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    return irp, col.T[keep.T].astype(np.int32), val.T[keep.T].astype(np.float64)


def hyb_width(irp):
    """HYB's ELL width by the rule of Bell and Garland."""
    irp = _i32(irp)
    return int(_load().orc_hyb_width(irp.shape[0] - 1, _p(irp)))


def csr_to_hyb(irp, aj, av, K=None):
    """(K, ELL col, ELL val, COO ai, aj, av of the remainder)."""
    irp, aj, av = _i32(irp), _i32(aj), _f64(av)
    n = irp.shape[0] - 1
    lib = _load()
    K = hyb_width(irp) if K is None else int(K)
    nr = int(lib.orc_hyb_rest(n, _p(irp), K))
    ecol, evals = np.empty(K * n, np.int32), np.empty(K * n, np.float64)
    ri, rj, rv = np.empty(nr, np.int32), np.empty(nr, np.int32), np.empty(nr, np.float64)
    lib.orc_csr_to_hyb(n, _p(irp), _p(aj), _p(av), K, _p(ecol), _p(evals), _p(ri), _p(rj), _p(rv))
    return K, ecol, evals, ri, rj, rv


def sell_layout(irp, C, sigma):
    """(perm, cs) of SELL-C-sigma for the row lengths of irp."""
    irp = _i32(irp)
    n = irp.shape[0] - 1
    lib = _load()
    perm = np.empty(n, np.int32)
    lib.orc_sell_perm(n, _p(irp), sigma, _p(perm))
    cs = np.empty((n + C - 1) // C + 1, np.int64)
    lib.orc_sell_offsets(n, _p(irp), _p(perm), C, _p(cs))
    return perm, cs


def csr_to_sell(irp, aj, av, C, sigma):
    """(perm, cs, col[cs[-1]], val[cs[-1]]) of SELL-C-sigma."""
    irp, aj, av = _i32(irp), _i32(aj), _f64(av)
    n = irp.shape[0] - 1
    perm, cs = sell_layout(irp, C, sigma)
    col = np.empty(int(cs[-1]), np.int32)
    val = np.empty(int(cs[-1]), np.float64)
    _load().orc_csr_to_sell(n, _p(irp), _p(aj), _p(av), C, _p(perm), _p(cs), _p(col), _p(val))
    return perm, cs, col, val


def sell_spmv(nrows, C, perm, cs, col, val, x):
    perm, cs, col, val, x = _i32(perm), np.ascontiguousarray(cs, np.int64), _i32(col), _f64(val), _f64(x)
    y = np.empty(nrows, np.float64)
    _load().orc_sell_spmv(nrows, C, _p(perm), _p(cs), _p(col), _p(val), _p(x), _p(y))
    return y


def sell_to_csr(nrows, C, perm, cs, col, val):
    """Back to canonical CSR (rows in their original order)."""
    rows_c, rows_v = [None] * nrows, [None] * nrows
    for p in range(nrows):
        s, r = divmod(p, C)
        w = (int(cs[s + 1]) - int(cs[s])) // C
        q = int(cs[s]) + np.arange(w) * C + r
        keep = col[q] >= 0
        rows_c[perm[p]] = col[q][keep]
        rows_v[perm[p]] = val[q][keep]
    lens = np.array([len(c) for c in rows_c], np.int64)
    irp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cat = lambda parts, t: np.concatenate(parts).astype(t) if nrows else np.zeros(0, t)
    return irp, cat(rows_c, np.int32), cat(rows_v, np.float64)


# ------------------------------------------------- HPCG's preconditioner
# Section VII-D: HPCG runs CG preconditioned by a multigrid V-cycle whose
# smoother is symmetric Gauss-Seidel.  The paper gives no further detail; the
# cycle below is HPCG's (one pre- and one post-smoothing sweep, injection
# between a grid and the grid of every second point, the 27-point operator
# on every level, one sweep on the coarsest level).
def symgs(irp, aj, av, order, r, x):
    """One symmetric Gauss-Seidel sweep (forward over `order`, backward over
    its reverse) on a copy of x; returns (status, x)."""
    irp, aj, av, order, r = _i32(irp), _i32(aj), _f64(av), _i32(order), _f64(r)
    x = _f64(x).copy()
    st = _load().orc_symgs(order.shape[0], _p(irp), _p(aj), _p(av), _p(order), _p(r), _p(x))
    return int(st), x


def gs_sweep(irp, aj, av, order, r, x, direction):
    """One forward (direction 1) or backward (-1) sweep on a copy of x."""
    irp, aj, av, order, r = _i32(irp), _i32(aj), _f64(av), _i32(order), _f64(r)
    x = _f64(x).copy()
    st = _load().orc_gs_sweep(order.shape[0], _p(irp), _p(aj), _p(av), _p(order), int(direction),
                              _p(r), _p(x))
    return int(st), x


def grid_colours(n):
    """Colour of each point of an n^3 grid (x fastest): the parities of its
    three coordinates, c = (ix & 1) + 2 (iy & 1) + 4 (iz & 1).  Two points of
    one colour differ by an even amount in every coordinate, so no 27-point
    coupling joins them."""
    i = np.arange(n ** 3, dtype=np.int64)
    ix, iy, iz = i % n, (i // n) % n, i // (n * n)
    return ((ix & 1) + 2 * (iy & 1) + 4 * (iz & 1)).astype(np.int32)


# Sweep order of the colours: colour 0 (the points a coarser grid keeps)
# last, so the forward sweep of the post-smoother reads the coarse
# correction before it recomputes those points.
COLOUR_SWEEP = (1, 2, 3, 4, 5, 6, 7, 0)


def colour_order(n):
    """Row order of the multicolour sweep: colours in COLOUR_SWEEP order,
    ascending row ids within a colour."""
    c = grid_colours(n)
    return np.concatenate([np.flatnonzero(c == k) for k in COLOUR_SWEEP]).astype(np.int32)


def coarse_points(n):
    """Fine row of each coarse point: coarse (i, j, k) of the (n/2)^3 grid is
    fine (2i, 2j, 2k); listed in coarse row order."""
    m = n // 2
    i = np.arange(m ** 3, dtype=np.int64)
    ci, cj, ck = i % m, (i // m) % m, i // (m * m)
    return (2 * ci + 2 * cj * n + 2 * ck * n * n).astype(np.int64)


def mg_vcycle(levels, r, orders=None):
    """z = M^{-1} r for HPCG's V-cycle.  levels[l] = (n_l, irp, aj, av), the
    27-point operator on the n_l^3 grid, finest first, n_{l+1} = n_l / 2.
    orders[l] is the sweep order of level l (default colour_order)."""
    orders = orders or [colour_order(lv[0]) for lv in levels]

    def cycle(l, rl):
        n, irp, aj, av = levels[l]
        z = np.zeros(n ** 3)
        st, z = symgs(irp, aj, av, orders[l], rl, z)
        if st != OK:
            raise ArithmeticError("zero diagonal")
        if l == len(levels) - 1:
            return z
        f = coarse_points(n)
        az = csr_spmv(irp, aj, av, z)
        zc = cycle(l + 1, rl[f] - az[f])
        z[f] += zc
        st, z = symgs(irp, aj, av, orders[l], rl, z)
        return z

    return cycle(0, _f64(r))


def pcg(irp, aj, av, b, precond, x0=None, tol=1e-9, maxit=1000):
    """Preconditioned CG as HPCG runs it: z = M^{-1} r, p = z on the first
    iteration and z + (r.z / r_old.z_old) p after, alpha = r.z / p.Ap; stop
    when ||r|| <= tol ||r_0||.  Returns (status, x, iters, rel_resid,
    true_rel_resid)."""
    b = _f64(b)
    x = np.zeros(b.shape[0]) if x0 is None else _f64(x0).copy()
    r = b - csr_spmv(irp, aj, av, x)
    rr0 = dot(r, r)
    rr, k, st = rr0, 0, NOT_CONVERGED
    if rr0 == 0.0:
        st = OK
    p, rz_old = None, 0.0
    while st == NOT_CONVERGED and k < maxit:
        z = _f64(precond(r))
        rz = dot(r, z)
        p = z.copy() if k == 0 else z + (rz / rz_old) * p
        rz_old = rz
        q = csr_spmv(irp, aj, av, p)
        sigma = dot(p, q)
        k += 1
        if not (sigma > 0.0) or not np.isfinite(sigma):
            st = BREAKDOWN
            break
        alpha = rz / sigma
        x = x + alpha * p
        r = r - alpha * q
        rr = dot(r, r)
        if np.sqrt(rr) <= tol * np.sqrt(rr0):
            st = OK
    t = b - csr_spmv(irp, aj, av, x)
    bn = np.sqrt(dot(b, b))
    rel = np.sqrt(rr) / np.sqrt(rr0) if rr0 > 0 else 0.0
    return st, x, k, float(rel), float(np.sqrt(dot(t, t)) / bn if bn > 0 else np.sqrt(dot(t, t)))
