"""Writes the oracle's results for the full-size stencil solves (too slow to
recompute inside a GPU test or a benchmark run).  Calls only `oracle` and the
seeded generators in `workloads`.

    python tests/golden/make_golden.py [--only NAME]

Each JSON file holds the oracle's status, iteration counts, residuals and the
solution x at 4,096 seeded sample indices (plus the first and last rows).
Cited method: unpreconditioned conjugate gradients on the HPCG 27-point
operator with b = A*1 and x0 = 0 (Section VII-D), stopping on the recursive
relative residual; mixed-precision refinement with an FP32 inner CG and an
FP64 outer residual and update (the mixed precision named in Section I);
an FP32 CG whose residual is replaced by the FP64 b - A*x at reliable
updates (the same mixed-precision aim); PCG with HPCG's multigrid V-cycle (symmetric Gauss-Seidel smoother; Section
VII-D describes HPCG's preconditioner).
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402
import workloads as wl  # noqa: E402


def sample_indices(n, k=4096, seed=8):
    idx = np.random.Generator(np.random.PCG64(seed)).choice(n, size=min(k, n), replace=False)
    return np.unique(np.concatenate([idx, [0, n - 1]])).astype(np.int64)


def host_info():
    """The machine the oracle ran on (one thread): CPU model and core count."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "cores_on_host": os.cpu_count(), "threads_used": 1}


def stencil_rhs(a):
    return orc.coo_spmv(a.nrows, a.ai, a.aj, a.av, np.ones(a.ncols))


def cg_case(n, tol):
    a = wl.stencil(n)
    b = stencil_rhs(a)
    t = time.time()
    st, x, iters, rel, true_rel = orc.cg(a.nrows, a.ai, a.aj, a.av, b, np.zeros(a.nrows), tol, 20000)
    idx = sample_indices(a.nrows)
    return {"what": f"oracle FP64 CG, 27-point stencil {n}^3, b = A*1, x0 = 0, tol {tol}",
            "n": n, "rows": a.nrows, "nnz": a.nnz, "tol": tol, "status": st, "iters": iters,
            "rel_resid": rel, "true_rel_resid": true_rel, "sample_idx": idx.tolist(),
            "x_sample": x[idx].tolist(), "oracle_seconds": round(time.time() - t, 1)}


def mixed_case(n, tol, inner_rtol, max_outer):
    a = wl.stencil(n)
    b = stencil_rhs(a)
    t = time.time()
    st, x, outer, inner, true_rel = orc.mixed_ir(a.nrows, a.ai, a.aj, a.av, b, np.zeros(a.nrows), tol=tol,
                                                 inner_rtol=inner_rtol, inner_maxit=20000,
                                                 max_outer=max_outer)
    idx = sample_indices(a.nrows)
    return {"what": f"oracle mixed refinement (FP32 inner CG to {inner_rtol}, FP64 outer), "
                    f"27-point stencil {n}^3, b = A*1, x0 = 0, tol {tol}",
            "n": n, "rows": a.nrows, "nnz": a.nnz, "tol": tol, "inner_rtol": inner_rtol,
            "max_outer": max_outer, "status": st, "outer_iters": outer, "inner_iters": inner,
            "true_rel_resid": true_rel, "sample_idx": idx.tolist(), "x_sample": x[idx].tolist(),
            "oracle_seconds": round(time.time() - t, 1)}


def pcg_case(n, levels, tol):
    lv = []
    for l in range(levels):
        a = wl.stencil(n >> l)
        lv.append((n >> l, orc.coo_to_csr(a.nrows, a.ai), a.aj, a.av))
    _, irp, aj, av = lv[0]
    b = orc.csr_spmv(irp, aj, av, np.ones(n ** 3))
    t = time.time()
    st, x, iters, rel, true_rel = orc.pcg(irp, aj, av, b, lambda r: orc.mg_vcycle(lv, r), tol=tol,
                                          maxit=1000)
    idx = sample_indices(n ** 3)
    return {"what": f"oracle PCG with HPCG's {levels}-level V-cycle (multicolour symmetric "
                    f"Gauss-Seidel), 27-point stencil {n}^3, b = A*1, x0 = 0, tol {tol}",
            "n": n, "levels": levels, "rows": n ** 3, "tol": tol, "status": st, "iters": iters,
            "rel_resid": rel, "true_rel_resid": true_rel, "sample_idx": idx.tolist(),
            "x_sample": x[idx].tolist(), "oracle_seconds": round(time.time() - t, 1)}


def mixed_ru_case(n, tol, delta):
    a = wl.stencil(n)
    b = stencil_rhs(a)
    t = time.time()
    st, x, upd, iters, true_rel = orc.mixed_ru(a.nrows, a.ai, a.aj, a.av, b, np.zeros(a.nrows),
                                               tol=tol, delta=delta, maxit=20000)
    idx = sample_indices(a.nrows)
    return {"what": f"oracle FP32 CG with FP64 reliable updates (update when the recursive "
                    f"residual falls to {delta} times its largest value since the last one), "
                    f"27-point stencil {n}^3, b = A*1, x0 = 0, tol {tol}",
            "n": n, "rows": a.nrows, "nnz": a.nnz, "tol": tol, "delta": delta, "status": st,
            "iters": iters, "updates": upd, "true_rel_resid": true_rel,
            "max_abs_x_minus_1": float(np.max(np.abs(x - 1.0))),
            "sample_idx": idx.tolist(), "x_sample": x[idx].tolist(),
            "oracle_seconds": round(time.time() - t, 1), "host": host_info()}


CASES = {
    "pcg_mg4_stencil128_tol1e-9": lambda: pcg_case(128, 4, 1e-9),
    "cg_stencil128_tol1e-9": lambda: cg_case(128, 1e-9),
    "cg_stencil192_tol1e-10": lambda: cg_case(192, 1e-10),
    "mixed_stencil192_tol1e-10": lambda: mixed_case(192, 1e-10, 1e-4, 20),
    "mixed_ru_stencil192_tol1e-10_delta0.01": lambda: mixed_ru_case(192, 1e-10, 0.01),
    "mixed_ru_stencil192_tol1e-10_delta0.1": lambda: mixed_ru_case(192, 1e-10, 0.1),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    for name, fn in CASES.items():
        if args.only and name != args.only:
            continue
        t = time.time()
        rec = fn()
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(rec, fh)
        print(f"{name}: status {rec['status']} ({time.time() - t:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
