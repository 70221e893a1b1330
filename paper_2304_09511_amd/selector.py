"""Storage-format selection for SpMV.

The paper's HPCG runs pick each process's format with a run-first auto-tuner
(time every format, keep the fastest; Section VII-D, Table III) and name a
dynamic selection mechanism as further work (Section IX).  This module
provides both:

* ``exhaustive_select`` -- the run-first tuner: time one SpMV in every
  feasible format (median of repeats) and keep the fastest;
* ``Selector`` -- an MLP 8-64-64-7 over eight matrix features
  (``mxs.features``), trained and evaluated on the GPU by the library's own
  kernels (``mlp_train_step``, ``mlp_predict``), with the formats the
  containers refuse masked out.  Without a model, selection falls back to
  the tuner.

The label set is COO, CSR, DIA and the further formats Section IX names:
ELL, SELL-64-1 (slices of 64 rows, no sorting), HYB (ELL part plus COO
remainder) and HDC (the diagonals at least half full as a DIA band plus a
COO remainder, the local/remote split of Table III on one GPU).

The dataset builder labels synthetic matrices (8 families, rows log-uniform
in [1e4, 1e7]) by the tuner's timings; labels are written as JSON lines and
the builder resumes an interrupted file.

    python -m paper_2304_09511_amd.selector label --n 3200 --out labels.jsonl
    python -m paper_2304_09511_amd.selector train --data labels.jsonl --out model.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import pathlib
import statistics
import sys
import time

import numpy as np

import paper_2304_09511_amd as mxs

DATA_DIR = pathlib.Path(__file__).resolve().parent / "selector_data"
DATA_PATH = DATA_DIR / "labels.jsonl"
MODEL_PATH = DATA_DIR / "model.json"
FAMILIES = ("stencil7", "stencil27", "banded", "zipf", "block")
# matrices 2000 onward: a band with scattered entries (uniform, or gathered
# in a few long rows), hypersparse matrices (most rows empty), and rows of
# near-equal length at random columns near the diagonal with a few long rows
EXT_FAMILIES = ("bandscatter", "hypersparse", "windowed")
N_BASE, N_TOTAL = 2000, 3200
FORMATS = ("coo", "csr", "dia", "ell", "sell", "hyb", "hdc")
# equal medians: the general-purpose format first, the two-part ones last
TIE_ORDER = ("csr", "dia", "ell", "sell", "coo", "hyb", "hdc")
SELL_SIGMA = 1
HDC_MIN_FILL = 0.5  # band diagonals hold at least this share of their slots


# ---------------------------------------------------------------------------
# Run-first tuner
# ---------------------------------------------------------------------------
def time_spmv(A, x, y, reps=10, warm=3):
    """Median time (ms) of one SpMV over `reps` individually timed calls."""
    import torch
    for _ in range(warm):
        mxs.spmv(A, x, y)
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        mxs.spmv(A, x, y)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def two_part_feasible(A, f):
    """HYB and HDC count only with both parts non-empty: an empty remainder
    leaves ELL (HYB) or DIA (HDC), an empty first part COO."""
    k, rest = A.hyb_size() if f == "hyb" else A.split_size(HDC_MIN_FILL)
    return k > 0 and rest > 0


def convert_to(A_coo, f):
    """A_coo in format f (a new Matrix), or None where the container refuses
    or a two-part format would have an empty part."""
    try:
        if f == "sell":
            return A_coo.to_sell(SELL_SIGMA)
        if f in ("hyb", "hdc"):
            if not two_part_feasible(A_coo, f):
                return None
            return A_coo.to_hyb() if f == "hyb" else A_coo.split(HDC_MIN_FILL, "coo")
        return A_coo.convert(f)
    except mxs.MxsError as e:
        if e.status == -5:
            return None
        raise


def time_formats(A_coo, reps=10, warm=3, seed=1):
    """Median SpMV time per format (inf where the format is refused)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dt = torch.float64 if A_coo.dtype == mxs.F64 else torch.float32
    x = torch.rand(A_coo.ncols, generator=g, device="cuda", dtype=dt) * 2 - 1
    y = torch.empty(A_coo.nrows, device="cuda", dtype=dt)
    out = {}
    for f in FORMATS:
        B = A_coo if f == "coo" else convert_to(A_coo, f)
        if B is None:
            out[f] = math.inf
            continue
        B.optimize()
        out[f] = time_spmv(B, x, y, reps, warm)
        if B is not A_coo:
            B.close()
    return out


def best_format(times):
    m = min(times.values())
    for f in TIE_ORDER:
        if times.get(f, math.inf) == m:
            return f
    return "csr"


def exhaustive_select(A_coo, reps=10, warm=3):
    """The run-first tuner: (fastest format, per-format times)."""
    t = time_formats(A_coo, reps, warm)
    return best_format(t), t


# ---------------------------------------------------------------------------
# Dataset
# ---------------------------------------------------------------------------
def matrix_spec(i, seed=4):
    """Family, row count and seed of dataset matrix i (400 per family):
    the five base families cycle over matrices 0-1999, the two further ones
    over 2000-2799."""
    g = np.random.Generator(np.random.PCG64([seed, i]))
    fam = FAMILIES[i % len(FAMILIES)] if i < N_BASE else EXT_FAMILIES[(i - N_BASE) % len(EXT_FAMILIES)]
    rows = int(round(10 ** g.uniform(4.0, 7.0)))
    spec = {"i": i, "family": fam, "seed": int(g.integers(1, 2 ** 31 - 1))}
    if fam.startswith("stencil"):
        spec["n"] = max(2, int(round(rows ** (1.0 / 3.0))))
    elif fam == "block":
        spec["nblockrows"] = max(1, rows // 8)
    else:
        spec["rows"] = rows
        if fam in ("banded", "bandscatter"):
            spec["ndiag"] = int(g.integers(3, 65))
        if fam == "bandscatter":
            spec["frac"] = float(10 ** g.uniform(-3.0, math.log10(0.4)))
            spec["concentrated"] = bool(g.integers(0, 2))
        if fam == "hypersparse":
            spec["per_row"] = float(10 ** g.uniform(math.log10(0.02), math.log10(0.5)))
        if fam == "windowed":
            spec["length"] = int(g.integers(4, 33))
            spec["width"] = int(10 ** g.uniform(2.0, 4.7))
            spec["tail_frac"] = float(10 ** g.uniform(-2.0, math.log10(0.5)))
    return spec


def generate_arrays(spec, device="cuda"):
    """(nrows, ncols, ai, aj, av) of a spec's matrix as tensors on `device`."""
    import workloads as wl
    fam = spec["family"]
    if fam == "stencil7":
        return wl.device_stencil(spec["n"], 7, device=device)
    if fam == "stencil27":
        return wl.device_stencil(spec["n"], 27, device=device)
    if fam == "banded":
        return wl.device_banded(spec["rows"], spec["ndiag"], 2000, spec["seed"], device=device)
    if fam == "zipf":
        return wl.device_zipf_rows(spec["rows"], spec["seed"], device=device)
    if fam == "bandscatter":
        return wl.device_banded_scatter(spec["rows"], spec["ndiag"], 2000, spec["frac"],
                                        spec["concentrated"], spec["seed"], device=device)
    if fam == "hypersparse":
        return wl.device_hypersparse(spec["rows"], spec["per_row"], spec["seed"], device=device)
    if fam == "windowed":
        return wl.device_windowed_rows(spec["rows"], spec["length"], spec["width"], spec["tail_frac"],
                                       spec["seed"], device=device)
    return wl.device_block_random(spec["nblockrows"], spec["seed"], device=device)


def generate(spec, dtype=None):
    """The matrix of a spec as a borrowing COO Matrix on the device."""
    nr, nc, ai, aj, av = generate_arrays(spec)
    if dtype is not None:
        av = av.to(dtype)
    return mxs.Matrix.coo(nr, nc, ai, aj, av, borrow=True)


def label_dataset(n, out, seed=4, reps=10, warm=3, log=sys.stderr):
    """Appends one JSON line per matrix to `out`, skipping indices already
    there (so an interrupted run resumes)."""
    import torch
    done = set()
    if os.path.exists(out):
        for line in open(out):
            try:
                done.add(json.loads(line)["i"])
            except (ValueError, KeyError):
                pass
    t_start = time.time()
    with open(out, "a") as fh:
        for i in range(n):
            if i in done:
                continue
            spec = matrix_spec(i, seed)
            t0 = time.time()
            A = generate(spec)
            feats = mxs.features(A)
            times = time_formats(A, reps, warm)
            rec = dict(spec, nrows=A.nrows, nnz=A.nnz, features=feats.tolist(),
                       times_ms={f: (None if math.isinf(v) else v) for f, v in times.items()},
                       label=best_format(times))
            A.close()
            del A
            torch.cuda.empty_cache()
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
            print(f"[label] {i} {spec['family']} rows={rec['nrows']} nnz={rec['nnz']} "
                  f"-> {rec['label']} {rec['times_ms']} ({time.time() - t0:.2f}s, "
                  f"total {time.time() - t_start:.0f}s)", file=log, flush=True)


def load_dataset(path):
    recs = [json.loads(line) for line in open(path) if line.strip()]
    recs.sort(key=lambda r: r["i"])
    F = np.array([r["features"] for r in recs], dtype=np.float64)
    T = np.array([[math.inf if r["times_ms"][f] is None else r["times_ms"][f] for f in FORMATS]
                  for r in recs], dtype=np.float64)
    y = np.array([FORMATS.index(r["label"]) for r in recs], dtype=np.int32)
    return recs, F, T, y


def split(n, n_train, seed=4):
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(n)
    return np.sort(perm[:n_train]), np.sort(perm[n_train:])


def dataset_split(n):
    """Training and held-out indices of the first n matrices: the base
    matrices' fixed 1,500 / 500 split, and three quarters / one quarter of
    the further families' (seed 5)."""
    tr, te = split(min(n, N_BASE), min(n, N_BASE) * 3 // 4)
    if n > N_BASE:
        m = n - N_BASE
        etr, ete = split(m, m * 3 // 4, seed=5)
        tr = np.concatenate([tr, N_BASE + etr])
        te = np.concatenate([te, N_BASE + ete])
    return tr, te


def regret(T, choice):
    """Mean of t(chosen)/min_f t(f) - 1 over the rows of T."""
    best = T.min(axis=1)
    return float(np.mean(T[np.arange(T.shape[0]), choice] / best - 1.0))


# ---------------------------------------------------------------------------
# The network
# ---------------------------------------------------------------------------
NI, NH, NO = 8, 64, len(FORMATS)


def he_init(seed=6):
    """He-normal weights (std sqrt(2/fan_in)), zero biases, in the layout of
    mxs_mlp_forward: W1[8][64], b1, W2[64][64], b2, W3[64][7], b3."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = [g.standard_normal(NI * NH) * math.sqrt(2.0 / NI), np.zeros(NH),
             g.standard_normal(NH * NH) * math.sqrt(2.0 / NH), np.zeros(NH),
             g.standard_normal(NH * NO) * math.sqrt(2.0 / NH), np.zeros(NO)]
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == mxs.NPARAM
    return w


class Selector:
    """MLP 8-64-64-7 format selector; parameters and normalisation live on
    the device while training and predicting."""

    def __init__(self, w=None, mu=None, sd=None):
        self.w = None if w is None else np.asarray(w, np.float32)
        self.mu = None if mu is None else np.asarray(mu, np.float32)
        self.sd = None if sd is None else np.asarray(sd, np.float32)
        self.loss_curve = []

    def _dev(self, a, dt=None):
        import torch
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt) if dt else \
            torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def fit(self, F, y, epochs=300, lr=1e-3, batch=128, seed=6):
        import torch
        raw = self._dev(F.astype(np.float64))
        mu, sd = mxs.mlp_norm_stats(raw)
        X = mxs.mlp_inputs(raw, mu, sd)
        Y = self._dev(y.astype(np.int32))
        w = self._dev(he_init(seed))
        m = torch.zeros_like(w)
        v = torch.zeros_like(w)
        n = X.shape[0]
        ws = mxs.mlp_workspace(min(batch, n))
        order = np.random.Generator(np.random.PCG64(seed))
        step = 0
        for ep in range(epochs):
            perm = torch.from_numpy(order.permutation(n)).cuda()
            tot = torch.zeros(1, dtype=torch.float64, device="cuda")
            for s0 in range(0, n, batch):
                idx = perm[s0:s0 + batch]
                Xb = X.index_select(0, idx).contiguous()
                Yb = Y.index_select(0, idx).contiguous()
                step += 1
                loss = mxs.mlp_train_step(w, m, v, Xb, Yb, lr, step, workspace=ws)
                tot += loss.double() * Xb.shape[0]
            self.loss_curve.append(float(tot) / n)
        self.w = w.cpu().numpy()
        self.mu = mu.cpu().numpy()
        self.sd = sd.cpu().numpy()
        return self

    def predict(self, F, feasible=None):
        """Format index per row of F (raw features); feasible: bool [n][7]."""
        import torch
        raw = self._dev(np.atleast_2d(F).astype(np.float64))
        X = mxs.mlp_inputs(raw, self._dev(self.mu), self._dev(self.sd))
        fz = None if feasible is None else self._dev(np.asarray(feasible, np.uint8))
        out = mxs.mlp_predict(self._dev(self.w), X, fz)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def select(self, A):
        """Format name for a COO/CSR Matrix.  DIA and ELL are masked by the
        containers' refusal rules, which the features decide.  SELL's rule
        depends on slice maxima, HYB's and HDC's on the sizes of their parts,
        so a refused choice of these is masked and the network asked again."""
        f = mxs.features(A)
        feas = [True, True, dia_feasible(f), ell_feasible(f), True, True, True]
        while True:
            name = FORMATS[int(self.predict(f[None, :], [feas])[0])]
            if name == "sell":
                try:
                    A.sell_size(SELL_SIGMA)
                except mxs.MxsError as e:
                    if e.status != -5:
                        raise
                    feas[FORMATS.index("sell")] = False
                    continue
            if name in ("hyb", "hdc") and not two_part_feasible(A, name):
                feas[FORMATS.index(name)] = False
                continue
            return name

    def save(self, path):
        json.dump({"layout": "W1[8][64] b1 W2[64][64] b2 W3[64][7] b3",
                   "formats": list(FORMATS), "sell_sigma": SELL_SIGMA, "w": self.w.tolist(),
                   "mu": self.mu.tolist(), "sd": self.sd.tolist(),
                   "loss_curve": self.loss_curve}, open(path, "w"))

    @classmethod
    def load(cls, path):
        d = json.load(open(path))
        s = cls(d["w"], d["mu"], d["sd"])
        s.loss_curve = d.get("loss_curve", [])
        return s


def dia_feasible(features):
    """The container's refusal rule: ndiag * rows <= 8 * nnz."""
    return features[5] * features[0] <= 8 * features[1]


def ell_feasible(features):
    """ELL's refusal rule: (longest row) * rows <= 8 * nnz."""
    return features[4] * features[0] <= 8 * features[1]


def select_rest(model, R):
    """COO or CSR for the remainder R of a split (a COO part handle): the
    network's choice on R's features with every other format masked."""
    f = mxs.features(R)
    feas = [f_ in ("coo", "csr") for f_ in FORMATS]
    return FORMATS[int(model.predict(f[None, :], [feas])[0])]


def select_format(A, model=None):
    """The learned choice when a model is given, else the run-first tuner."""
    if model is not None:
        return model.select(A)
    return exhaustive_select(A)[0]


def evaluate(model, F, T):
    """Accuracy, mean regret of the model and of always-CSR, and per format
    the labels (fastest) and the recall of the model on them, on rows of F/T."""
    feas = np.isfinite(T)
    choice = model.predict(F, feas)
    best = np.array([FORMATS.index(best_format(dict(zip(FORMATS, t)))) for t in T])
    per = {}
    for k, f in enumerate(FORMATS):
        sel = best == k
        per[f] = {"labels": int(sel.sum()),
                  "recall": None if not sel.any() else float(np.mean(choice[sel] == k))}
    return {"n": int(F.shape[0]), "accuracy": float(np.mean(choice == best)),
            "mean_regret": regret(T, choice), "always_csr_regret": regret(T, np.ones(len(T), int)),
            "exhaustive_cost_x_one_spmv": float(len(FORMATS)), "per_format": per}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--n", type=int, default=N_TOTAL)
    a.add_argument("--out", required=True)
    a.add_argument("--seed", type=int, default=4)
    b = sub.add_parser("train")
    b.add_argument("--data", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--epochs", type=int, default=300)
    args = ap.parse_args(argv)
    mxs.load()
    if args.cmd == "label":
        label_dataset(args.n, args.out, args.seed)
    else:
        recs, F, T, y = load_dataset(args.data)
        tr, te = dataset_split(len(recs))
        model = Selector().fit(F[tr], y[tr], epochs=args.epochs)
        model.save(args.out)
        base = te[te < N_BASE]
        ext = te[te >= N_BASE]
        print(json.dumps({"train": evaluate(model, F[tr], T[tr]),
                          "held_out": evaluate(model, F[te], T[te]),
                          "held_out_base_families": evaluate(model, F[base], T[base]),
                          "held_out_further_families": evaluate(model, F[ext], T[ext]) if ext.size else None}))


if __name__ == "__main__":
    main()
