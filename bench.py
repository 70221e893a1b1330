"""Benchmark: SpMV effective HBM bandwidth per format and CG time-to-tolerance on
one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the HPCG 27-point stencil on a 128^3 grid (2,097,152 rows,
55,742,968 stored entries, FP64 values, int32 indices), resident in HBM in
COO, CSR and DIA.  One step = one SpMV in each of the three formats.  The JSON
line reports the aggregate algorithmic bytes of a step over its time (GB/s),
each format's share, the HBM roofline of the dominant kernel, CG to 1e-9 in
each format with the SpMV / dot / vector-update split, FP64 vs mixed CG to
1e-10 on the 192^3 stencil, and the CPU oracle timed on this host.

Algorithmic bytes per SpMV (x read once, y written once, nothing else):
    COO: nnz*(8+s) + s*(ncols+nrows)
    CSR: nnz*(4+s) + 4*(nrows+1) + s*(ncols+nrows)
    DIA: s*(in-range slots) + 4*ndiag + s*(ncols+nrows)
with s the value size.  Only kernel time on resident data is timed.

    python bench.py --pmc FMT   runs a few SpMVs of one format plus a 1 GiB
copy (the counter calibration) for rocprofv3 --pmc.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "SpMV effective HBM GB/s (% of peak) per format; mixed vs FP64 CG time-to-tol"
FORMATS = ("coo", "csr", "dia")
# kernel of each format's implementation (ids as in mxs_set_impl)
KERNEL_NAMES = {"coo": ("coo_rows_kernel", "coo_spmv_kernel", "coo_spmv_kernel"),
                "csr": ("csr_spmv_kernel", "csr_rowwise_kernel", "csr_spmv_kernel", "ell_spmv_kernel",
                        "csr_spmv_kernel", "csr_vector_kernel"),
                "dia": ("dia_spmv_kernel",) * 3}
SPMV_SRC = os.path.join(ROOT, "paper_2304_09511_amd", "csrc", "spmv.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(A, fmt, s=8):
    if fmt == "coo":
        return A.nnz * (8 + s) + s * (A.ncols + A.nrows)
    if fmt == "csr":
        return A.nnz * (4 + s) + 4 * (A.nrows + 1) + s * (A.ncols + A.nrows)
    return s * A.nnz + 4 * A.ndiag + s * (A.ncols + A.nrows)  # DIA: nnz = in-range slots


def split_bytes(H, rest):
    """Algorithmic bytes of a split SpMV: the band as DIA, the remainder as
    COO or CSR, x read once and y written once (the accumulate pass's read
    of y is the method's own traffic and is not counted)."""
    band_slots = H.nnz - H._keep[3].numel()
    rn = H._keep[3].numel()
    rest_bytes = rn * 16 if rest == "coo" else rn * 12 + 4 * (H.nrows + 1)
    return 8 * band_slots + 4 * H.ndiag + rest_bytes + 8 * (H.ncols + H.nrows)


def source_sha(path=None):
    return hashlib.sha256(open(path or SPMV_SRC, "rb").read()).hexdigest()[:16]


MG_SRC = os.path.join(ROOT, "paper_2304_09511_amd", "csrc", "mg.hip")
ELL_SRC = os.path.join(ROOT, "paper_2304_09511_amd", "csrc", "ell.hip")


def symgs_traffic_from_profile(n):
    """HBM bytes of one finest-level symmetric sweep from the committed
    counter summary, if it was taken on the current mg.hip."""
    path = os.path.join(ROOT, "profiles", f"symgs_sweep_stencil{n}_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"^source_sha256_16:\s*(\w+)", text, re.M)
    m_b = re.search(r"^hbm_bytes_per_sweep:\s*([0-9.eE+]+)", text, re.M)
    if not m_sha or not m_b or m_sha.group(1) != source_sha(MG_SRC):
        return None
    return float(m_b.group(1))


def traffic_from_profile(fmt, workload_tag, src=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (`src`: the kernel's file,
    spmv.hip by default)."""
    path = os.path.join(ROOT, "profiles", f"{fmt}_spmv_{workload_tag}_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"^source_sha256_16:\s*(\w+)", text, re.M)
    m_b = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m_sha or not m_b or m_sha.group(1) != source_sha(src):
        return None
    return float(m_b.group(1))


def build_matrices(mxs, n):
    t = time.time()
    coo = mxs.stencil(n, 27, fmt="coo")
    mats = {"coo": coo, "csr": coo.convert("csr"), "dia": coo.convert("dia")}
    for A in mats.values():
        A.optimize()
    log(f"[bench] {n}^3 stencil on device: {coo.nrows} rows, {coo.nnz} nnz, "
        f"DIA {mats['dia'].ndiag} diagonals, {mats['dia'].nnz} slots ({time.time() - t:.1f}s)")
    return mats


def time_calls(torch, fn, batches=10, per_batch=100, warm=5):
    """Median, mean and min per call over `batches` batches of back-to-back calls."""
    for _ in range(warm):
        fn()
    out = []
    for _ in range(batches):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(per_batch):
            fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b) / per_batch)
    return {"median_ms": statistics.median(out), "mean_ms": statistics.fmean(out), "min_ms": min(out)}


def cg_runs(torch, mxs, mats, rtol, label):
    res = {}
    n = mats["csr"].nrows
    ones = torch.ones(n, dtype=torch.float64, device="cuda")
    b = mxs.spmv(mats["csr"], ones)
    bn = float(torch.linalg.vector_norm(b))
    for fmt, A in mats.items():
        ws = mxs.cg_workspace(A)
        mxs.cg_solve(A, b, rtol=rtol, maxit=20000, workspace=ws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, x, r = mxs.cg_solve(A, b, rtol=rtol, maxit=20000, workspace=ws)
        torch.cuda.synchronize()
        t_tol = (time.perf_counter() - t0) * 1e3
        _, _, rt = mxs.cg_solve(A, b, rtol=rtol, maxit=20000, workspace=ws, timing=True)
        err1 = float((x - 1.0).abs().max())
        res[fmt] = {"status": st, "iters": r["iters"], "time_to_tol_ms": round(t_tol, 3),
                    "ms_per_iter": round(t_tol / max(r["iters"], 1), 4),
                    "rel_resid": r["rel_resid"], "true_rel_resid": r["true_rel_resid"],
                    "max_abs_err_vs_ones": err1,
                    "timed_split_ms": {"spmv": round(rt["t_spmv_ms"], 3), "dot": round(rt["t_dot_ms"], 3),
                                       "axpy": round(rt["t_axpy_ms"], 3)}}
        log(f"[bench] {label} CG {fmt}: {r['iters']} it, {t_tol:.1f} ms, true rel resid "
            f"{r['true_rel_resid']:.2e}, |x-1|max {err1:.1e}")
        del ws
    return res, bn


def cg16_run(torch, mxs):
    """GPU FP64 CG to 1e-9 on the 16^3 stencil (DIA), time to tolerance after
    a warm-up solve: the GPU side of the oracle's 16^3 CG timing."""
    A = mxs.stencil(16, fmt="dia").optimize()
    b = mxs.spmv(A, torch.ones(A.nrows, dtype=torch.float64, device="cuda"))
    ws = mxs.cg_workspace(A)
    mxs.cg_solve(A, b, rtol=1e-9, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, x, r = mxs.cg_solve(A, b, rtol=1e-9, workspace=ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) * 1e3
    A.close()
    return {"status": st, "iters": r["iters"], "time_to_tol_ms": round(t, 3), "format": "dia"}


def padded_bytes(A, nnz, s=8):
    """Algorithmic bytes of an ELL or SELL SpMV: the entries (column and
    value; padding slots are the format's overhead, not the operation's),
    SELL's permutation and slice offsets, x read once and y written once."""
    b = nnz * (4 + s) + s * (A.ncols + A.nrows)
    if A.format == 5:
        b += 4 * A.nrows + 8 * (A.ndiag + 1)
    return b


def other_formats(torch, mxs, coo, x, y, label):
    """ELL and SELL-64-sigma SpMV (Section IX's further formats): protocol
    median of 10 x 100 calls, GB/s of algorithmic bytes, stored slots."""
    out = {}
    for name, make in (("ell", lambda: coo.convert("ell")), ("sell_sigma1", lambda: coo.to_sell(1)),
                       ("sell_sigma4096", lambda: coo.to_sell(4096)), ("hyb", lambda: coo.to_hyb())):
        try:
            B = make()
        except mxs.MxsError as e:
            if e.status != -5:
                raise
            out[name] = {"refused": "MXS_ERR_DIA_TOO_SPARSE (more than 8 slots per entry)"}
            continue
        tc = time_calls(torch, lambda: mxs.spmv(B, x, y))
        nb = padded_bytes(B, coo.nnz)
        if name == "hyb":
            nb += 4 * B._keep[2].numel()   # the remainder's row ids
        slots = (B.ndiag * B.nrows + (B._keep[2].numel() if name == "hyb" else 0)
                 if name in ("ell", "hyb") else int(B._slots))
        med = tc["median_ms"] * 1e-3
        out[name] = {"us_per_call": round(med * 1e6, 2), "algorithmic_bytes": nb,
                     "GBps": round(nb / med / 1e9, 1), "frac_of_peak": round(nb / med / 1e9 / PEAK_HBM_GBS, 4),
                     "slots_per_entry": round(slots / max(coo.nnz, 1), 4)}
        log(f"[bench] {label} {name}: {out[name]['us_per_call']} us, {out[name]['GBps']} GB/s, "
            f"{out[name]['slots_per_entry']} slots/entry")
        B.close()
    return out


# colour order of a symmetric sweep (mxs.h): forward over colours 1, ..., 7, 0,
# backward over the reverse without repeating colour 0
SWEEP_PASSES = (1, 2, 3, 4, 5, 6, 7, 0, 7, 6, 5, 4, 3, 2, 1)


def symgs_bytes(nn):
    """Algorithmic bytes of one symmetric sweep on the nn^3 stencil: every
    colour pass reads its rows' off-diagonal entries (4-byte column, 8-byte
    value), diagonal, right-hand side and row id, writes their x, and reads
    x once; 15 passes (the backward sweep repeats no colour).  A point's
    colour is the parity of its coordinates, (ix&1) + 2(iy&1) + 4(iz&1)."""
    rows = nn ** 3
    i = np.arange(rows)
    ax = [i % nn, (i // nn) % nn, i // (nn * nn)]
    col = (ax[0] & 1) + 2 * (ax[1] & 1) + 4 * (ax[2] & 1)
    # off-diagonal entries per row of the 27-point stencil: (product of
    # neighbours in range along each axis) - 1
    span = np.ones(rows, np.int64)
    for a in ax:
        span *= 1 + (a > 0) + (a < nn - 1)
    offd = span - 1
    total = 0
    for c in SWEEP_PASSES:
        sel = col == c
        total += int(offd[sel].sum()) * 12 + int(sel.sum()) * (8 + 8 + 4 + 8) + rows * 8
    return total


def pcg_runs(torch, mxs, n, levels, rtol, mats_for_spmv):
    """PCG with HPCG's V-cycle to rtol: time to tolerance after a warm-up
    solve, the timed split per kernel class, one V-cycle and one finest-level
    sweep timed on their own, and the solution against the oracle's run."""
    M = mxs.Multigrid(n, levels)
    _, A0 = M.level(0)
    b = mxs.spmv(A0, torch.ones(A0.nrows, dtype=torch.float64, device="cuda"))
    out = {"config": f"27-point stencil {n}^3, {levels} levels, b = A*1, x0 = 0, PCG to {rtol} "
                     f"(||r_k|| / ||r_0||), one V-cycle per iteration: one symmetric "
                     f"multicolour Gauss-Seidel sweep before and after the coarse correction"}
    for name, A in (("csr", None), ("dia", mats_for_spmv.get("dia"))):
        if name != "csr" and A is None:
            continue
        M.pcg_solve(b, A=A, rtol=rtol, maxit=1000)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, x, r = M.pcg_solve(b, A=A, rtol=rtol, maxit=1000)
        torch.cuda.synchronize()
        t_tol = (time.perf_counter() - t0) * 1e3
        _, _, rt = M.pcg_solve(b, A=A, rtol=rtol, maxit=1000, timing=True)
        rec = {"status": st, "iters": r["iters"], "time_to_tol_ms": round(t_tol, 3),
               "ms_per_iter": round(t_tol / max(r["iters"], 1), 4),
               "true_rel_resid": r["true_rel_resid"],
               "max_abs_err_vs_ones": float((x - 1.0).abs().max()),
               "timed_split_ms": {k: round(rt["t_" + k + "_ms"], 3)
                                  for k in ("precond", "spmv", "dot", "axpy")}}
        g = load_golden(f"pcg_mg{levels}_stencil{n}_tol{rtol:.0e}".replace("e-0", "e-"))
        if g is not None:
            idx = torch.tensor(g["sample_idx"], device="cuda")
            xo = np.array(g["x_sample"])
            rec["oracle_iters"] = g["iters"]
            rec["max_rel_err_vs_oracle_sample"] = float(np.max(np.abs(x[idx].cpu().numpy() - xo))
                                                        / np.max(np.abs(xo)))
        out["spmv_" + name] = rec
        log(f"[bench] PCG-MG {n}^3 ({name} SpMV): {r['iters']} it, {t_tol:.1f} ms, "
            f"split {rec['timed_split_ms']}")
    r0 = torch.rand(A0.nrows, dtype=torch.float64, device="cuda")
    z0 = torch.empty_like(r0)
    tc = time_calls(torch, lambda: M.apply(r0, z0), batches=5, per_batch=20)
    out["vcycle_ms"] = round(tc["median_ms"], 4)
    xs = torch.zeros_like(r0)
    tc = time_calls(torch, lambda: M.symgs(0, r0, xs), batches=5, per_batch=20)
    sb = symgs_bytes(n)
    out["symgs_finest"] = {"ms": round(tc["median_ms"], 4), "algorithmic_bytes": sb,
                           "GBps": round(sb / (tc["median_ms"] * 1e-3) / 1e9, 1),
                           "frac_of_peak": round(sb / (tc["median_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                           "launches": 15, "traffic": symgs_traffic_from_profile(n)}
    log(f"[bench] V-cycle {out['vcycle_ms']} ms; finest symmetric sweep {tc['median_ms']:.4f} ms, "
        f"{out['symgs_finest']['GBps']} GB/s")
    M.close()
    return out


MIXED_VARIANTS = (("fp64", {}),
                  ("ir_inner1e-4", dict(mixed="ir", inner_rtol=1e-4, max_outer=20)),
                  ("ir_inner1e-5", dict(mixed="ir", inner_rtol=1e-5, max_outer=20)),
                  ("ir_inner1e-6", dict(mixed="ir", inner_rtol=1e-6, max_outer=20)),
                  ("ru_delta0.1", dict(mixed="ru", delta=0.1)),
                  ("ru_delta0.01", dict(mixed="ru", delta=0.01)))


def mixed_vs_fp64(torch, mxs, n, fmts=("dia", "csr")):
    """FP64 CG against the two mixed-precision solvers (iterative refinement
    with an FP32 inner CG; FP32 CG with FP64 reliable updates) to 1e-10, each
    timed to tolerance after one warm-up solve, with the solution's error
    against the oracle's stored FP64 solution at sampled rows."""
    mats = build_matrices(mxs, n)
    out = {"workload": f"27-point stencil {n}^3 ({mats['csr'].nrows} rows, {mats['csr'].nnz} nnz), "
                       f"b = A*1, x0 = 0, tol 1e-10 on ||b - A x|| / ||b|| (FP64 CG: recursive)"}
    ones = torch.ones(mats["csr"].nrows, dtype=torch.float64, device="cuda")
    b = mxs.spmv(mats["csr"], ones)
    gold = {"fp64": load_golden(f"cg_stencil{n}_tol1e-10"), "ir": load_golden(f"mixed_stencil{n}_tol1e-10"),
            "ru_delta0.1": load_golden(f"mixed_ru_stencil{n}_tol1e-10_delta0.1"),
            "ru_delta0.01": load_golden(f"mixed_ru_stencil{n}_tol1e-10_delta0.01")}
    # the oracle's run of the same method (iterative refinement: inner 1e-4 only)
    same = {"fp64": "fp64", "ir_inner1e-4": "ir", "ru_delta0.1": "ru_delta0.1", "ru_delta0.01": "ru_delta0.01"}
    for fmt in fmts:
        A = mats[fmt]
        A32 = A.cast(mxs.F32)
        A32.optimize()
        ws64 = mxs.cg_workspace(A)
        wsm = mxs.cg_workspace(A, mixed=True)
        rows = {}
        for name, kw in MIXED_VARIANTS:
            kw = dict(kw, rtol=1e-10, maxit=20000)
            if kw.get("mixed"):
                kw.update(A32=A32, workspace=wsm)
            else:
                kw.update(workspace=ws64)
            mxs.cg_solve(A, b, **kw)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, x, r = mxs.cg_solve(A, b, **kw)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) * 1e3
            rec = {"status": st, "time_to_tol_ms": round(t, 3), "iters": r["iters"],
                   "outer_iters": r["outer_iters"], "true_rel_resid": r["true_rel_resid"],
                   "max_abs_err_vs_ones": float((x - 1.0).abs().max())}
            g = gold["fp64"]
            if g is not None:
                idx = torch.tensor(g["sample_idx"], dtype=torch.int64, device="cuda")
                xo = torch.tensor(g["x_sample"], dtype=torch.float64, device="cuda")
                rec["max_rel_err_vs_oracle_fp64_x_sampled"] = float((x[idx] - xo).abs().max() / xo.abs().max())
            gs = gold.get(same.get(name, ""))
            if gs is not None:
                idx = torch.tensor(gs["sample_idx"], dtype=torch.int64, device="cuda")
                xo = torch.tensor(gs["x_sample"], dtype=torch.float64, device="cuda")
                rec["oracle_same_method"] = {
                    "iters": gs.get("iters", gs.get("inner_iters")),
                    "updates_or_corrections": gs.get("updates", gs.get("outer_iters")),
                    "true_rel_resid": gs["true_rel_resid"],
                    "max_rel_err_x_sampled": float((x[idx] - xo).abs().max() / xo.abs().max()),
                    "source": "tests/golden/" + gs["_file"]}
            rows[name] = rec
        fp = rows["fp64"]["time_to_tol_ms"]
        for name in rows:
            rows[name]["speedup_over_fp64"] = round(fp / rows[name]["time_to_tol_ms"], 3)
        best = max((k for k in rows if k != "fp64" and rows[k]["status"] == 0),
                   key=lambda k: rows[k]["speedup_over_fp64"], default=None)
        rows["best_mixed"] = best
        out[fmt] = rows
        log(f"[bench] {n}^3 {fmt}: " + ", ".join(
            f"{k} {v['time_to_tol_ms']:.1f} ms ({v['iters']} it)" for k, v in rows.items() if isinstance(v, dict)))
        A32.close()
    out["oracle"] = {k: (None if g is None else {kk: g.get(kk) for kk in ("iters", "outer_iters", "inner_iters",
                                                                          "updates", "true_rel_resid",
                                                                          "inner_rtol", "delta")})
                     for k, g in gold.items()}
    out["oracle"]["source"] = "tests/golden/*.json (tests/golden/make_golden.py, oracle only)"
    for A in mats.values():
        A.close()
    return out


def host_cpu():
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline(orc, coo_host, nbytes, budget_s=8.0, gpu_cg=None):
    """The oracle on this host, one thread: its COO SpMV (Algorithm 1)
    repeated for about `budget_s` seconds on the benchmark's matrix, and its
    FP64 CG to 1e-9 on the 16^3 and 128^3 stencils (b = A*1, x0 = 0) beside
    the GPU's CG on the same problem; the 192^3 FP64 CG comes from the stored
    oracle run with the CPU it ran on."""
    import workloads as wl
    ai, aj, av, nrows = coo_host
    x = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, nrows)
    times = []
    t_end = time.perf_counter() + budget_s
    while time.perf_counter() < t_end or len(times) < 3:
        t0 = time.perf_counter()
        orc.coo_spmv(nrows, ai, aj, av, x)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    cores, model = host_cpu()
    cg = {}
    for n, coo in ((16, None), (128, (ai, aj, av))):
        if coo is None:
            a = wl.stencil(n)
            cai, caj, cav = a.ai, a.aj, a.av
        else:
            cai, caj, cav = coo
        b = orc.coo_spmv(n ** 3, cai, caj, cav, np.ones(n ** 3))
        t0 = time.perf_counter()
        st, xo, it, rel, true_rel = orc.cg(n ** 3, cai, caj, cav, b, None, 1e-9, 20000)
        t = time.perf_counter() - t0
        rec = {"status": st, "iters": it, "time_to_tol_ms": round(t * 1e3, 2),
               "true_rel_resid": true_rel}
        g = (gpu_cg or {}).get(n)
        if g:
            rec["gpu_time_to_tol_ms"] = g["time_to_tol_ms"]
            rec["gpu_iters"] = g["iters"]
            rec["gpu_format"] = g["format"]
            rec["speedup_gpu_over_oracle"] = round(rec["time_to_tol_ms"] / g["time_to_tol_ms"], 1)
        cg[f"stencil{n}_tol1e-9"] = rec
    g192 = load_golden("cg_stencil192_tol1e-10")
    if g192 is not None:
        cg["stencil192_tol1e-10"] = {
            "status": g192["status"], "iters": g192["iters"],
            "time_to_tol_ms": round(1e3 * g192["oracle_seconds"], 1),
            "source": "tests/golden/cg_stencil192_tol1e-10.json (stored oracle run, one thread of "
                      "the CPU of the machine that wrote the stored runs, not this host)"}
    return {"value": round(nbytes / med / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle COO SpMV (Algorithm 1, FP64, single thread) on the same 128^3 "
                      f"stencil, {len(times)} calls in {sum(times):.1f} s, median {med * 1e3:.1f} ms/call; "
                      f"oracle FP64 CG to 1e-9 on the 16^3 and 128^3 stencils",
            "host_cores_available": cores, "host_cpu": model, "cg": cg}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    g["_file"] = name + ".json"
    return g


def compare_golden(section, name, x_by_fmt=None):
    """Adds the oracle's stored iteration count (written by
    tests/golden/make_golden.py) beside the GPU's."""
    g = load_golden(name)
    if g is None:
        section["oracle"] = None
        return None
    section["oracle"] = {"iters": g.get("iters"), "outer_iters": g.get("outer_iters"),
                         "inner_iters": g.get("inner_iters"), "true_rel_resid": g["true_rel_resid"],
                         "source": f"tests/golden/{name}.json"}
    return g


def csr_arrays_line(torch, mxs, A, x, y, nbytes):
    """CSR's entry-tile kernel, which reads the CSR arrays themselves (the
    default implementation may read a plan copy instead): protocol timing
    against CSR's algorithmic bytes; the default is restored afterwards."""
    default = A.impl
    A.impl = 0
    tc = time_calls(torch, lambda: mxs.spmv(A, x, y))
    A.impl = default
    med = tc["median_ms"] * 1e-3
    return {"implementation": "entry_tiles", "kernel": "csr_spmv_kernel",
            "protocol_10x100_median_us": round(med * 1e6, 2), "algorithmic_bytes": nbytes,
            "GBps": round(nbytes / med / 1e9, 1), "frac_of_peak": round(nbytes / med / 1e9 / PEAK_HBM_GBS, 4)}


def fp32_lines(torch, mxs, mats, fp64_bytes):
    """The FP32 SpMVs of the mixed solvers (values rounded to FP32, FP32 x and
    y) on the same stencil: protocol timing against the FP32 algorithmic
    bytes (s = 4)."""
    out = {}
    n = mats["csr"].nrows
    x32 = (torch.rand(n, dtype=torch.float64, device="cuda") * 2 - 1).float()
    y32 = torch.empty(n, dtype=torch.float32, device="cuda")
    for f in FORMATS:
        B = mats[f].cast(mxs.F32)
        B.optimize()
        nb = algorithmic_bytes(B, f, s=4)
        tc = time_calls(torch, lambda: mxs.spmv(B, x32, y32))
        med = tc["median_ms"] * 1e-3
        names = mxs.Matrix.IMPL_NAMES[B.format]
        kern = KERNEL_NAMES[f][B.impl]
        traffic = traffic_from_profile(f"{f}_fp32", f"stencil{round(n ** (1 / 3))}",
                                       ELL_SRC if kern.startswith("ell") else None)
        out[f] = {"us_per_call": round(med * 1e6, 2), "algorithmic_bytes": nb,
                  "GBps": round(nb / med / 1e9, 1), "frac_of_peak": round(nb / med / 1e9 / PEAK_HBM_GBS, 4),
                  "bytes_vs_fp64": round(nb / fp64_bytes[f], 3), "implementation": names[B.impl],
                  "kernel": kern, "traffic": traffic,
                  "traffic_over_algorithmic": None if traffic is None else round(traffic / nb, 4)}
        log(f"[bench]   fp32 {f}: {out[f]['us_per_call']} us, {out[f]['GBps']} GB/s "
            f"({100 * out[f]['frac_of_peak']:.1f}%)")
        B.close()
    return out


def impl_report(mxs, A, x, y, reps=20):
    """Every applicable implementation of A's format timed by mxs_tune (median
    of `reps` calls after 3 warm-ups); the default implementation is restored
    afterwards, so the other figures stay those of the default plan."""
    names = mxs.Matrix.IMPL_NAMES[A.format]
    default = A.impl
    best, ms = A.tune(x, y, reps=reps)
    A.impl = default
    return {"default": names[default], "default_id": default, "fastest": names[best],
            "median_us": {names[i]: (None if m is None else round(m * 1e3, 2))
                          for i, m in enumerate(ms)}}


def irregular_runs(torch, mxs, checks):
    """SpMV on the two irregular 4,000,000-row workloads in every format the
    container accepts: protocol median of 10 x 100 calls, GB/s, GFLOP/s.  The
    outputs of 2,000 seeded rows go to the oracle check of the CPU leg."""
    import workloads as wl
    gens = {
        "zipf_4M": ("row lengths L = min(5000, floor(3.04109 k + u)), k ~ Zipf(2) on [1, 5000], "
                    "distinct uniform columns, N(0,1) values, 4,000,000 rows, seed 2",
                    lambda: wl.device_zipf_rows(4_000_000, seed=2)),
        "banded_4M": ("11 distinct diagonal offsets uniform in [-2000, 2000], every in-range slot "
                      "N(0,1), 4,000,000 rows, seed 3",
                      lambda: wl.device_banded(4_000_000, 11, 2000, seed=3)),
        "banded_noise40k_4M": ("the banded 4M matrix plus 40,000 entries at uniform random "
                               "positions (long-range couplings), N(0,1), seed 3",
                               lambda: wl.device_banded_noise(4_000_000, 11, 2000, 40_000, seed=3)),
        "banded_noise1600k_4M": ("the banded 4M matrix plus 1,600,000 entries at uniform random "
                                 "positions, N(0,1), seed 3",
                                 lambda: wl.device_banded_noise(4_000_000, 11, 2000, 1_600_000, seed=3)),
    }
    out = {}
    for name, (desc, gen) in gens.items():
        t0 = time.time()
        nr, nc, ai, aj, av = gen()
        coo = mxs.Matrix.coo(nr, nc, ai, aj, av, borrow=True)
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        x = torch.rand(nc, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        y = torch.empty(nr, dtype=torch.float64, device="cuda")
        rows = np.sort(np.random.Generator(np.random.PCG64(9)).choice(nr, 2000, replace=False))
        irp = torch.zeros(nr + 1, dtype=torch.int64, device="cuda")
        irp[1:] = torch.cumsum(torch.bincount(ai.long(), minlength=nr), 0)
        irp_h = irp.cpu().numpy()
        starts, ends = irp_h[rows], irp_h[rows + 1]
        sel = torch.from_numpy(np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)])).cuda()
        sub = (len(rows), nc, np.concatenate([[0], np.cumsum(ends - starts)]).astype(np.int32),
               aj[sel].cpu().numpy(), av[sel].cpu().numpy())
        x_h = x.cpu().numpy()
        rec = {"workload": desc, "rows": nr, "nnz": coo.nnz, "x": "U[-1,1) (torch generator, seed 1)"}
        fmts = FORMATS + (("hdc_csr", "hdc_coo") if "noise" in name else ())
        for fmt in fmts:
            if fmt == "coo":
                A = coo
            elif fmt.startswith("hdc"):
                A = coo.split(0.5, fmt[4:])
            else:
                try:
                    A = coo.convert(fmt)
                except mxs.MxsError as e:
                    if e.status == -5:
                        rec[fmt] = {"refused": "MXS_ERR_DIA_TOO_SPARSE"}
                        continue
                    raise
            A.optimize()
            tc = time_calls(torch, lambda: mxs.spmv(A, x, y))
            nb = algorithmic_bytes(A, fmt) if not fmt.startswith("hdc") else split_bytes(A, fmt[4:])
            med = tc["median_ms"] * 1e-3
            rec[fmt] = {"us_per_call": round(med * 1e6, 2), "mean_us": round(tc["mean_ms"] * 1e3, 2),
                        "min_us": round(tc["min_ms"] * 1e3, 2), "algorithmic_bytes": nb,
                        "GBps": round(nb / med / 1e9, 1), "frac_of_peak": round(nb / med / 1e9 / PEAK_HBM_GBS, 4),
                        "GFLOPs": round(2 * coo.nnz / med / 1e9, 1)}
            if fmt == "dia" or fmt.startswith("hdc"):
                rec[fmt]["ndiag"] = A.ndiag
            if fmt.startswith("hdc"):
                rec[fmt]["band_diagonals_min_fill"] = 0.5
                rec[fmt]["remainder_entries"] = int(A._keep[3].numel())
            checks.append({"name": f"{name}/{fmt}", "csr_rows": sub, "x": x_h, "y": y.cpu().numpy()[rows]})
            log(f"[bench] {name} {fmt}: {rec[fmt]['us_per_call']} us, {rec[fmt]['GBps']} GB/s, "
                f"{rec[fmt]['GFLOPs']} GFLOP/s")
            if not fmt.startswith("hdc"):
                rec[fmt]["implementations"] = impl_report(mxs, A, x, y)
                log(f"[bench]   implementations: {rec[fmt]['implementations']['median_us']}")
            else:
                # each part's implementation chosen by mxs_tune
                t = A.tune(x, y, reps=20)
                names = mxs.Matrix.IMPL_NAMES
                rest_fmt = mxs.FORMATS[fmt[4:]]
                tc = time_calls(torch, lambda: mxs.spmv(A, x, y))
                rec[fmt]["tuned"] = {"band": names[mxs.DIA][t["band"][0]],
                                     "rest": names[rest_fmt][t["rest"][0]],
                                     "us_per_call": round(tc["median_ms"] * 1e3, 2),
                                     "timing": "protocol median of 10 x 100 calls after tuning"}
                log(f"[bench]   tuned parts: {rec[fmt]['tuned']}")
            if A is not coo:
                A.close()
        rec["other_formats"] = other_formats(torch, mxs, coo, x, y, name)
        coo.close()
        del coo, ai, aj, av, x, y, irp, sel
        torch.cuda.empty_cache()
        rec["setup_s"] = round(time.time() - t0, 2)
        out[name] = rec
    return out


def device_facts(torch):
    """What the device reports about itself (names, counts, sizes)."""
    pr = torch.cuda.get_device_properties(0)
    out = {"name": pr.name, "arch": getattr(pr, "gcnArchName", None),
           "compute_units": pr.multi_processor_count, "hbm_bytes": pr.total_memory,
           "wavefront": getattr(pr, "warp_size", None)}
    l2 = getattr(pr, "L2_cache_size", None)
    if l2:
        out["l2_bytes_reported"] = l2
    return out


def stream_reference(torch, mxs, mib=512, reps=10):
    """Bandwidth of plain streams on this device, for scale beside the SpMV
    figures: a device copy (torch, reads and writes `mib` MiB each way) and a
    read-only stream (the library's dot product of two `mib` MiB FP64
    vectors).  Median of `reps` timed calls after two warm-ups."""
    n = mib * 2 ** 20 // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)

    def med(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return statistics.median(ts)
    t_copy = med(lambda: c.copy_(a))
    t_read = med(lambda: mxs.dot(a, b))
    out = {"copy_GBps": round(2 * n * 8 / t_copy / 1e9, 1), "copy_bytes_each_way": n * 8,
           "read_stream_GBps": round(2 * n * 8 / t_read / 1e9, 1), "read_stream_bytes": 2 * n * 8,
           "read_stream_kernel": "dot_kernel (mxs_dot: two arrays read together, plus its finish kernel)",
           "timing": f"median of {reps} calls, HIP events around each"}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def conversion_costs(torch, mxs, coo, spmv_ms, reps=3):
    """Runtime format switching has a price (Section IV): wall time of each
    conversion from the 128^3 COO handle (and back), and of building each
    format's plan (mxs_optimize), in ms and in SpMVs of the target format.
    Matrix.convert includes its host-synchronous sizing call and the
    allocation of the new arrays from torch's caching allocator."""
    def wall(fn):
        r = fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            del r
        return statistics.median(ts) * 1e3
    out = {}
    csr = coo.convert("csr")
    dia = coo.convert("dia")
    for name, fn, tgt in (("coo_to_csr", lambda: coo.convert("csr"), "csr"),
                          ("coo_to_dia", lambda: coo.convert("dia"), "dia"),
                          ("csr_to_coo", lambda: csr.convert("coo"), "coo"),
                          ("csr_to_dia", lambda: csr.convert("dia"), "dia"),
                          ("dia_to_csr", lambda: dia.convert("csr"), "csr"),
                          ("dia_to_coo", lambda: dia.convert("coo"), "coo")):
        ms = wall(fn)
        out[name] = {"ms": round(ms, 3), "spmv_equivalents": round(ms / spmv_ms[tgt], 1)}
    for name, A, tgt in (("optimize_csr", csr, "csr"), ("optimize_dia", dia, "dia"),
                         ("optimize_coo", coo, "coo")):
        ms = wall(lambda A=A: A.optimize())
        out[name] = {"ms": round(ms, 3), "spmv_equivalents": round(ms / spmv_ms[tgt], 1)}
    csr.close()
    dia.close()
    torch.cuda.empty_cache()
    return out


def selector_eval(torch, mxs, n_live=100):
    """The committed selector on its 700 held-out matrices (stored timings;
    also per group of families, with each format's label count and recall),
    and live on a seeded sample of them re-timed on this GPU: accuracy, mean
    regret against the run-first tuner, the always-CSR baseline, and the
    selection cost of each."""
    from paper_2304_09511_amd import selector as S
    model = S.Selector.load(str(S.MODEL_PATH))
    recs, F, T, y = S.load_dataset(str(S.DATA_PATH))
    tr, te = S.dataset_split(len(recs))
    base, ext = te[te < S.N_BASE], te[te >= S.N_BASE]
    out = {"stored_held_out": S.evaluate(model, F[te], T[te]),
           "stored_held_out_base_families": S.evaluate(model, F[base], T[base]),
           "stored_held_out_further_families": S.evaluate(model, F[ext], T[ext]) if ext.size else None,
           "labels_per_format_all": {f: int((y == k).sum()) for k, f in enumerate(S.FORMATS)}}
    pick = np.sort(np.random.Generator(np.random.PCG64(12)).choice(te, n_live, replace=False))
    Tl, choice, t_model, t_tuner = [], [], [], []
    for i in pick:
        A = S.generate(recs[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = model.select(A)
        t_model.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        best, times = S.exhaustive_select(A)
        t_tuner.append(time.perf_counter() - t0)
        Tl.append([times[k] for k in S.FORMATS])
        choice.append(S.FORMATS.index(f))
        A.close()
        torch.cuda.empty_cache()
    Tl = np.array(Tl)
    choice = np.array(choice)
    best = Tl.argmin(axis=1)
    out["live"] = {"matrices": int(n_live), "accuracy": float(np.mean(choice == best)),
                   "mean_regret": S.regret(Tl, choice),
                   "always_csr_regret": S.regret(Tl, np.ones(len(Tl), int)),
                   "model_select_ms_median": round(1e3 * statistics.median(t_model), 3),
                   "tuner_select_ms_median": round(1e3 * statistics.median(t_tuner), 3)}
    log(f"[bench] selector held out: {out['stored_held_out']}; live: {out['live']}")
    return out


def parity_checks(orc, checks):
    """Relative max-norm of each GPU output against the oracle: the full
    vector for the stencil, the sampled rows for the irregular matrices."""
    res = {}
    ref_cache = {}
    for c in checks:
        if "coo" in c:
            key = id(c["coo"][1])
            if key not in ref_cache:
                nrows, ai, aj, av = c["coo"]
                ref_cache[key] = orc.coo_spmv(nrows, ai, aj, av, c["x"])
            ref = ref_cache[key]
        else:
            m, ncols, irp, aj, av = c["csr_rows"]
            ref = orc.csr_spmv(irp, aj, av, c["x"])
        den = float(np.max(np.abs(ref))) if ref.size else 1.0
        res[c["name"]] = float(np.max(np.abs(c["y"] - ref)) / (den if den > 0 else 1.0)) if ref.size else 0.0
    return res


def pmc_mode(args):
    import torch

    import paper_2304_09511_amd as mxs
    mxs.load()
    value_bytes = 8
    if args.pmc == "symgs":
        M = mxs.Multigrid(args.n, 4)
        r = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, args.n ** 3)).cuda()
        x = torch.zeros_like(r)
        for _ in range(args.steps):
            M.symgs(0, r, x)
    elif args.pmc.startswith("zipf-"):
        # the 4M-row Zipf matrix of the irregular runs, COO or CSR, one implementation
        import workloads as wl
        fmt, impl = args.pmc[len("zipf-"):len("zipf-") + 3], int(args.pmc[len("zipf-") + 3:])
        nr, nc, ai, aj, av = wl.device_zipf_rows(4_000_000, seed=2)
        A = mxs.Matrix.coo(nr, nc, ai, aj, av, borrow=True)
        A = (A.convert("csr") if fmt == "csr" else A).optimize()
        A.impl = impl
        x = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, A.ncols)).cuda()
        y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
        for _ in range(args.steps):
            mxs.spmv(A, x, y)
        args.pmc = fmt
    else:
        # a stencil format with its default implementation, csr0: CSR's
        # entry tiles (the kernel that reads the CSR arrays), or <fmt>32: the
        # FP32 copy of a format (values rounded, FP32 x and y) as the mixed
        # solvers run it
        mats = build_matrices(mxs, args.n)
        A = mats[args.pmc[:3]]
        fp32 = args.pmc.endswith("32")
        if fp32:
            A = A.cast(mxs.F32).optimize()
            value_bytes = 4
        if args.pmc == "csr0":
            A.impl = 0
        args.pmc = args.pmc[:3]
        x = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, A.ncols)).cuda()
        if fp32:
            x = x.float()
        y = torch.empty(A.nrows, dtype=x.dtype, device="cuda")
        for _ in range(args.steps):
            mxs.spmv(A, x, y)
    # calibration: a plain copy of 1 GiB (reads 1 GiB, writes 1 GiB)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    if args.pmc == "symgs":
        print(json.dumps({"pmc": "symgs", "bytes_per_sweep": symgs_bytes(args.n),
                          "copy_bytes_each_way": src.numel() * 8,
                          "source_sha256_16": source_sha(MG_SRC)}))
        return
    print(json.dumps({"pmc": args.pmc, "bytes_per_launch": algorithmic_bytes(A, args.pmc, s=value_bytes),
                      "copy_bytes_each_way": src.numel() * 8, "source_sha256_16": source_sha()}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--mixed-n", type=int, default=192)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-irregular", action="store_true")
    ap.add_argument("--no-selector", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--pmc", choices=FORMATS + ("csr0", "symgs", "zipf-csr0", "zipf-csr4", "zipf-coo0", "zipf-coo2",
                                                "coo32", "csr32", "dia32"),
                    default=None)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.pmc:
        return pmc_mode(args)

    import torch

    import paper_2304_09511_amd as mxs
    mxs.load()
    torch.cuda.set_device(0)
    mats = build_matrices(mxs, args.n)
    n = mats["csr"].nrows
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, n)).cuda()
    ys = {f: torch.empty(n, dtype=torch.float64, device="cuda") for f in FORMATS}
    bytes_f = {f: algorithmic_bytes(mats[f], f) for f in FORMATS}
    step_bytes = sum(bytes_f.values())

    # outputs of this exact configuration, checked against the oracle in the
    # CPU leg below; and the 16^3 stencil (x ~ U[-1,1), seed 1) in each format
    checks = []
    ai, aj, av = mats["coo"].export()
    x_host = x.cpu().numpy()
    for f in FORMATS:
        y = mxs.spmv(mats[f], x, ys[f]).cpu().numpy()
        checks.append({"name": f"stencil{args.n}/{f}", "coo": (n, ai, aj, av), "x": x_host, "y": y})
    small = build_matrices(mxs, 16)
    n16 = small["coo"].nrows
    x16 = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, n16)
    c16 = small["coo"].export()
    for f in FORMATS:
        y16 = mxs.spmv(small[f], torch.from_numpy(x16).cuda()).cpu().numpy()
        checks.append({"name": f"stencil16/{f}", "coo": (n16, *c16), "x": x16, "y": y16})
    for A in small.values():
        A.close()

    # ---- timed region: K steps, one SpMV per format per step ----
    ev = {f: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for f in FORMATS}
    for _ in range(args.warmup):
        for f in FORMATS:
            mxs.spmv(mats[f], x, ys[f])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for f in FORMATS:
            ev[f][k][0].record()
            mxs.spmv(mats[f], x, ys[f])
            ev[f][k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = step_bytes / (wall / args.steps) / 1e9
    per = {}
    for f in FORMATS:
        ms = statistics.fmean(a.elapsed_time(b) for a, b in ev[f])
        per[f] = {"timing": "HIP events around each launch inside the timed steps",
                  "us_per_call": round(ms * 1e3, 2), "algorithmic_bytes": bytes_f[f],
                  "GBps": round(bytes_f[f] / (ms * 1e-3) / 1e9, 1),
                  "frac_of_peak": round(bytes_f[f] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                  "GFLOPs": round(2 * mats["coo"].nnz / (ms * 1e-3) / 1e9, 1)}
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} GB/s aggregate")
    for f in FORMATS:
        log(f"[bench]   {f}: {per[f]['us_per_call']} us, {per[f]['GBps']} GB/s "
            f"({100 * per[f]['frac_of_peak']:.1f}% of 8 TB/s)")

    # paper's protocol: 10 runs of 100 back-to-back SpMVs, median per call
    for f in FORMATS:
        tc = time_calls(torch, lambda f=f: mxs.spmv(mats[f], x, ys[f]))
        per[f]["protocol_10x100"] = {k: round(v * 1e3, 2) for k, v in tc.items()}
        per[f]["protocol_10x100"]["unit"] = "us"
        gbps = bytes_f[f] / (tc["median_ms"] * 1e-3) / 1e9
        per[f]["protocol_10x100"]["GBps"] = round(gbps, 1)
        per[f]["protocol_10x100"]["frac_of_peak"] = round(gbps / PEAK_HBM_GBS, 4)
        log(f"[bench]   {f} protocol (median of 10 x 100 back-to-back): "
            f"{tc['median_ms'] * 1e3:.2f} us, {gbps:.1f} GB/s ({100 * gbps / PEAK_HBM_GBS:.1f}%)")

    for f in FORMATS:
        per[f]["implementations"] = impl_report(mxs, mats[f], x, ys[f])
        d = per[f]["implementations"]["default_id"]
        per[f]["implementation"] = per[f]["implementations"]["default"]
        per[f]["kernel"] = KERNEL_NAMES[f][d]
        log(f"[bench]   {f} implementations (median us): {per[f]['implementations']['median_us']}")
    if per["csr"]["kernel"] == "ell_spmv_kernel":
        # the default reads the plan's ELL copy
        per["csr"]["note"] = ("the default implementation runs ell_spmv_kernel over the plan's ELL copy "
                              "(rows of near-equal length); algorithmic_bytes are the CSR operation's; "
                              "csr_arrays_kernel is the kernel that reads the CSR arrays")
    per["csr"]["csr_arrays_kernel"] = csr_arrays_line(torch, mxs, mats["csr"], x, ys["csr"], bytes_f["csr"])
    log(f"[bench]   csr entry tiles (CSR arrays): {per['csr']['csr_arrays_kernel']}")
    out_fp32 = fp32_lines(torch, mxs, mats, bytes_f)

    out_other = other_formats(torch, mxs, mats["coo"], x, ys["coo"], f"stencil{args.n}")

    # scale: plain streams on the same device, and what switching formats costs
    stream = stream_reference(torch, mxs)
    for f in FORMATS:
        per[f]["frac_of_read_stream"] = round(per[f]["protocol_10x100"]["GBps"] / stream["read_stream_GBps"], 4)
    log(f"[bench] streams: copy {stream['copy_GBps']} GB/s, read {stream['read_stream_GBps']} GB/s")
    conv = conversion_costs(torch, mxs, mats["coo"],
                            {f: per[f]["protocol_10x100"]["median_ms"] * 1e-3 for f in FORMATS})
    conv_s = ", ".join(f"{k} {v['ms']}" for k, v in conv.items())
    log(f"[bench] conversions and plans (ms): {conv_s}")

    # dominant kernel of the step and its roofline
    dom = max(FORMATS, key=lambda f: per[f]["us_per_call"])
    achieved = bytes_f[dom] / (per[dom]["us_per_call"] * 1e-6) / 1e9
    tag = f"stencil{args.n}"
    traffic = traffic_from_profile(dom, tag)
    roofline = {"kernel": KERNEL_NAMES[dom][per[dom]["implementations"]["default_id"]],
                "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic,
                "algorithmic_bytes_per_launch": bytes_f[dom]}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"HPCG 27-point stencil {args.n}^3 ({n} rows, {mats['coo'].nnz} nnz, "
                                  f"FP64 values 26/-1, int32 indices), resident in HBM; one step = one "
                                  f"SpMV in each of COO, CSR, DIA",
                      "x": "U[-1,1) seed 1", "formats": list(FORMATS)},
           "per_format": per, "fp32_spmv": out_fp32, "other_formats": out_other, "roofline": roofline,
           "device": device_facts(torch), "stream_reference": stream, "conversion": conv}

    if not args.no_cg:
        out["cg"], _ = cg_runs(torch, mxs, mats, 1e-9, f"{args.n}^3")
        out["cg"]["config"] = f"b = A*1, x0 = 0, unpreconditioned CG to 1e-9 (||r_k|| / ||r_0||)"
        compare_golden(out["cg"], f"cg_stencil{args.n}_tol1e-9")
        out["cg16"] = cg16_run(torch, mxs)
    if not args.no_pcg:
        out["pcg_mg"] = pcg_runs(torch, mxs, args.n, 4, 1e-9, mats)
    for A in mats.values():
        A.close()
    del ys
    torch.cuda.empty_cache()
    if not args.no_irregular:
        out["irregular"] = irregular_runs(torch, mxs, checks)
    if not args.no_mixed:
        out["mixed_cg"] = mixed_vs_fp64(torch, mxs, args.mixed_n)
    if not args.no_selector:
        out["selector"] = selector_eval(torch, mxs)
    if not args.no_cpu:
        import oracle as orc
        gpu_cg = {}
        if "cg" in out:
            best = min(FORMATS, key=lambda f: out["cg"][f]["time_to_tol_ms"])
            gpu_cg[args.n] = dict(out["cg"][best], format=best)
        if "cg16" in out:
            gpu_cg[16] = out["cg16"]
        out["cpu_baseline"] = cpu_baseline(orc, (ai, aj, av, n), bytes_f["coo"], args.cpu_seconds,
                                           gpu_cg=gpu_cg)
        log(f"[bench] CPU oracle: {out['cpu_baseline']['value']} GB/s ({out['cpu_baseline']['sample']})")
        out["parity_vs_oracle"] = parity_checks(orc, checks)
        bad = {k: v for k, v in out["parity_vs_oracle"].items() if not v <= 1e-12}
        assert not bad, bad
    else:
        out["parity_vs_oracle"] = "not run (--no-cpu): the oracle runs only in the CPU leg"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
