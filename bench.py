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
KERNEL_NAMES = {"coo": "coo_spmv_kernel", "csr": "csr_spmv_kernel", "dia": "dia_spmv_kernel"}
SPMV_SRC = os.path.join(ROOT, "paper_2304_09511_amd", "csrc", "spmv.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(A, fmt, s=8):
    if fmt == "coo":
        return A.nnz * (8 + s) + s * (A.ncols + A.nrows)
    if fmt == "csr":
        return A.nnz * (4 + s) + 4 * (A.nrows + 1) + s * (A.ncols + A.nrows)
    return s * A.nnz + 4 * A.ndiag + s * (A.ncols + A.nrows)  # DIA: nnz = in-range slots


def source_sha():
    return hashlib.sha256(open(SPMV_SRC, "rb").read()).hexdigest()[:16]


def traffic_from_profile(fmt, workload_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{fmt}_spmv_{workload_tag}_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"^source_sha256_16:\s*(\w+)", text, re.M)
    m_b = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m_sha or not m_b or m_sha.group(1) != source_sha():
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


def mixed_vs_fp64(torch, mxs, n, fmts=("dia", "csr")):
    mats = build_matrices(mxs, n)
    out = {"workload": f"27-point stencil {n}^3 ({mats['csr'].nrows} rows, {mats['csr'].nnz} nnz), "
                       f"b = A*1, x0 = 0, tol 1e-10 on ||b - A x|| / ||b||"}
    ones = torch.ones(mats["csr"].nrows, dtype=torch.float64, device="cuda")
    b = mxs.spmv(mats["csr"], ones)
    for fmt in fmts:
        A = mats[fmt]
        A32 = A.cast(mxs.F32)
        A32.optimize()
        ws64 = mxs.cg_workspace(A)
        wsm = mxs.cg_workspace(A, mixed=True)
        rows = {}
        for mode in ("fp64", "mixed"):
            kw = dict(rtol=1e-10, maxit=20000)
            if mode == "mixed":
                kw.update(mixed=True, A32=A32, inner_rtol=1e-4, max_outer=20, workspace=wsm)
            else:
                kw.update(workspace=ws64)
            mxs.cg_solve(A, b, **kw)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, x, r = mxs.cg_solve(A, b, **kw)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) * 1e3
            rows[mode] = {"status": st, "time_to_tol_ms": round(t, 3), "iters": r["iters"],
                          "outer_iters": r["outer_iters"], "true_rel_resid": r["true_rel_resid"],
                          "max_abs_err_vs_ones": float((x - 1.0).abs().max())}
            rows[mode + "_x"] = x
        rows["max_abs_diff_mixed_vs_fp64"] = float((rows.pop("mixed_x") - rows.pop("fp64_x")).abs().max())
        rows["speedup_mixed_over_fp64"] = round(rows["fp64"]["time_to_tol_ms"] / rows["mixed"]["time_to_tol_ms"], 3)
        out[fmt] = rows
        log(f"[bench] {n}^3 {fmt}: fp64 {rows['fp64']['time_to_tol_ms']:.1f} ms ({rows['fp64']['iters']} it), "
            f"mixed {rows['mixed']['time_to_tol_ms']:.1f} ms ({rows['mixed']['outer_iters']} outer, "
            f"{rows['mixed']['iters']} inner), speedup {rows['speedup_mixed_over_fp64']}")
        A32.close()
    for A in mats.values():
        A.close()
    return out


def cpu_baseline(orc, coo_host, nbytes, budget_s=12.0):
    """The oracle's COO SpMV (single thread) on this host, repeated for about
    `budget_s` seconds."""
    ai, aj, av, nrows = coo_host
    x = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, nrows)
    times = []
    t_end = time.perf_counter() + budget_s
    while time.perf_counter() < t_end or len(times) < 3:
        t0 = time.perf_counter()
        orc.coo_spmv(nrows, ai, aj, av, x)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
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
    return {"value": round(nbytes / med / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle COO SpMV (Algorithm 1, FP64, single thread) on the same 128^3 "
                      f"stencil, {len(times)} calls in {sum(times):.1f} s, median {med * 1e3:.1f} ms/call",
            "host_cores_available": cores, "host_cpu": model}


def pmc_mode(args):
    import torch

    import paper_2304_09511_amd as mxs
    mxs.load()
    mats = build_matrices(mxs, args.n)
    A = mats[args.pmc]
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, A.ncols)).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    for _ in range(args.steps):
        mxs.spmv(A, x, y)
    # calibration: a plain copy of 1 GiB (reads 1 GiB, writes 1 GiB)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc": args.pmc, "bytes_per_launch": algorithmic_bytes(A, args.pmc),
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
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--pmc", choices=FORMATS, default=None)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see DESIGN.md for how the SpMV/CG path would shard)", file=sys.stderr)
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

    # parity of this exact configuration against the oracle (full vector)
    import oracle as orc
    t = time.time()
    ai, aj, av = mats["coo"].export()
    ref = orc.coo_spmv(n, ai, aj, av, x.cpu().numpy())
    parity = {}
    for f in FORMATS:
        y = mxs.spmv(mats[f], x, ys[f]).cpu().numpy()
        parity[f] = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
    log(f"[bench] parity vs oracle (rel max-norm): {parity} ({time.time() - t:.1f}s)")
    assert all(v <= 1e-12 for v in parity.values()), parity

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
        per[f] = {"us_per_call": round(ms * 1e3, 2), "algorithmic_bytes": bytes_f[f],
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

    # dominant kernel of the step and its roofline
    dom = max(FORMATS, key=lambda f: per[f]["us_per_call"])
    achieved = bytes_f[dom] / (per[dom]["us_per_call"] * 1e-6) / 1e9
    tag = f"stencil{args.n}"
    traffic = traffic_from_profile(dom, tag)
    roofline = {"kernel": KERNEL_NAMES[dom] + ("+coo_fixup_kernel" if dom == "coo" else ""),
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
           "per_format": per, "parity_rel_maxnorm": parity, "roofline": roofline}

    if not args.no_cg:
        out["cg"], _ = cg_runs(torch, mxs, mats, 1e-9, f"{args.n}^3")
        out["cg"]["config"] = f"b = A*1, x0 = 0, unpreconditioned CG to 1e-9 (||r_k|| / ||r_0||)"
    coo_host = (ai, aj, av, n)
    for A in mats.values():
        A.close()
    del ys
    torch.cuda.empty_cache()
    if not args.no_mixed:
        out["mixed_cg"] = mixed_vs_fp64(torch, mxs, args.mixed_n)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(orc, coo_host, bytes_f["coo"], args.cpu_seconds)
        log(f"[bench] CPU oracle: {out['cpu_baseline']['value']} GB/s ({out['cpu_baseline']['sample']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
