"""GPU parity of the format selector's kernels against the CPU oracle, through
the C ABI: the eight features, network inputs, forward pass, gradient, Adam,
masked prediction, and the trained selector's regret on the labelled set.

Bars: integer features bit-exact, real features within 1e-12 relative; FP32
logits within 1e-5 and gradients within 1e-4 of the FP64 oracle (relative to
the largest magnitude); Adam within FP32 rounding of the oracle step.
"""
import math

import numpy as np
import pytest

import oracle as orc
import workloads as wl
from _cases import small_cases

pytestmark = pytest.mark.gpu

CASES = small_cases()
IDS = [c[0] for c in CASES]


def _torch():
    import torch
    return torch


def dev(a, dtype=None):
    t = _torch().from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def matrix(mxs, a, fmt):
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    if fmt == "coo":
        return A
    try:
        return A.convert(fmt)
    except mxs.MxsError as e:
        if e.status == -5:
            return None
        raise


U = 2.0 ** -53


def features_close(f, ref):
    """Integer features bit-exact; mean, fill and bandwidth within a few
    roundings.  The variance is exact on the device (integer moments) while
    the oracle sums nrows squared deviations in FP64, so the bar there is that
    sum's rounding bound, about 4 (nrows + 2) u (var + mean^2)."""
    for k in (0, 1, 4, 5):   # integers
        assert f[k] == ref[k], (k, f[k], ref[k])
    for k in (2, 6, 7):
        assert abs(f[k] - ref[k]) <= 4 * U * abs(ref[k]), (k, f[k], ref[k])
    tol = 4 * (ref[0] + 2) * U * (ref[3] + ref[2] ** 2)
    assert abs(f[3] - ref[3]) <= tol, (3, f[3], ref[3], tol)


@pytest.mark.parametrize("fmt", ["coo", "csr", "dia"])
@pytest.mark.parametrize("name,a", CASES, ids=IDS)
def test_features_match_oracle(gpu, name, a, fmt):
    mxs = gpu
    if not np.all(a.av != 0):
        pytest.skip("explicit zeros: DIA features count non-zero slots")
    A = matrix(mxs, a, fmt)
    if A is None:
        pytest.skip("DIA refused")
    features_close(mxs.features(A), orc.features(a.nrows, a.ncols, a.ai, a.aj))


def test_features_stencil_closed_forms(gpu):
    """Mean ((3n-2)/n)^3 and population variance ((9n-10)/n)^3 - mean^2 of
    the 27-point stencil's row lengths (products of per-axis counts 2 or 3)."""
    mxs = gpu
    for n in (16, 40):
        A = mxs.stencil(n, fmt="csr")
        f = mxs.features(A)
        mean = ((3 * n - 2) / n) ** 3
        var = ((9 * n - 10) / n) ** 3 - mean ** 2
        assert f[0] == n ** 3 and f[1] == (3 * n - 2) ** 3 and f[4] == 27 and f[5] == 27
        assert f[2] == pytest.approx(mean, rel=1e-14)
        assert f[3] == pytest.approx(var, rel=1e-12)
        assert f[6] == pytest.approx((3 * n - 2) ** 3 / (27 * n ** 3), rel=1e-14)


def _inputs_reference(raw, mu, sd):
    t = raw.astype(np.float64).copy()
    t[:, :6] = np.log1p(t[:, :6])
    return (t - mu.astype(np.float64)) / sd.astype(np.float64)


def test_norm_stats_and_inputs(gpu):
    mxs = gpu
    g = np.random.Generator(np.random.PCG64(21))
    raw = np.abs(g.standard_normal((333, 8))) * 10.0 ** g.integers(0, 7, (333, 8))
    raw[:, 7] = g.uniform(0, 1, 333)
    raw[:, 5] = 4.0                                 # constant feature: sd replaced by 1
    mu, sd = mxs.mlp_norm_stats(dev(raw))
    t = raw.copy()
    t[:, :6] = np.log1p(t[:, :6])
    mu_ref = t.mean(axis=0)
    sd_ref = t.std(axis=0)
    sd_ref[sd_ref <= 1e-6 * np.abs(mu_ref)] = 1.0
    np.testing.assert_allclose(mu.cpu().numpy(), mu_ref, rtol=2e-7, atol=1e-7)
    np.testing.assert_allclose(sd.cpu().numpy(), sd_ref, rtol=2e-6)
    assert sd.cpu().numpy()[5] == 1.0
    X = mxs.mlp_inputs(dev(raw), mu, sd).cpu().numpy()
    ref = _inputs_reference(raw, mu.cpu().numpy(), sd.cpu().numpy())
    np.testing.assert_allclose(X, ref, rtol=1e-5, atol=1e-5)


def _net(seed, scale=1.0):
    from paper_2304_09511_amd import selector as S
    w = S.he_init(seed) * np.float32(scale)
    g = np.random.Generator(np.random.PCG64(seed + 1))
    w[512:576] = g.uniform(-0.1, 0.1, 64)      # non-zero biases exercise every term
    w[4672:4736] = g.uniform(-0.1, 0.1, 64)
    w[orc.NPARAM - orc.NCLASS:] = g.uniform(-0.1, 0.1, orc.NCLASS)
    return w.astype(np.float32)


def _data(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    X = g.standard_normal((n, 8)).astype(np.float32)
    y = g.integers(0, orc.NCLASS, n).astype(np.int32)
    return X, y


@pytest.mark.parametrize("n", [1, 7, 128, 1000])
def test_forward_matches_oracle(gpu, n):
    mxs = gpu
    w = _net(6)
    X, _ = _data(n, 30 + n)
    z = mxs.mlp_forward(dev(w), dev(X)).cpu().numpy()
    ref = orc.mlp_forward(w.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(z - ref)) <= 1e-5 * max(np.max(np.abs(ref)), 1.0)


@pytest.mark.parametrize("n", [1, 5, 128, 777])
def test_gradient_matches_oracle(gpu, n):
    mxs = gpu
    w = _net(8)
    X, y = _data(n, 40 + n)
    loss, g = mxs.mlp_grad(dev(w), dev(X), dev(y))
    lref, gref = orc.mlp_loss_grad(w.astype(np.float64), X.astype(np.float64), y)
    assert float(loss.cpu()) == pytest.approx(lref, rel=1e-5)
    g = g.cpu().numpy()
    assert np.max(np.abs(g - gref)) <= 1e-4 * np.max(np.abs(gref))


@pytest.mark.parametrize("lead", [3, 4, 5, 6])
def test_gradient_with_a_dominant_late_logit(gpu, lead):
    """One of the formats after the first three (ELL, SELL, HYB, HDC) leads
    every other logit by more than 100: a softmax shifted by anything but the
    largest logit overflows FP32's exponential there (e^100 > FLT_MAX)."""
    mxs = gpu
    w = _net(12)
    w[orc.NPARAM - orc.NCLASS + lead] = np.float32(150.0)
    X, y = _data(64, 70 + lead)
    z = orc.mlp_forward(w.astype(np.float64), X.astype(np.float64)).reshape(-1, orc.NCLASS)
    others = np.delete(z, lead, axis=1)
    assert np.min(z[:, lead] - others.max(axis=1)) > 100.0
    loss, g = mxs.mlp_grad(dev(w), dev(X), dev(y))
    lref, gref = orc.mlp_loss_grad(w.astype(np.float64), X.astype(np.float64), y)
    g = g.cpu().numpy()
    assert np.all(np.isfinite(g)) and math.isfinite(float(loss.cpu()))
    assert float(loss.cpu()) == pytest.approx(lref, rel=1e-5)
    assert np.max(np.abs(g - gref)) <= 1e-4 * np.max(np.abs(gref))


def test_gradient_deterministic(gpu):
    mxs = gpu
    w = _net(9)
    X, y = _data(500, 50)
    a = mxs.mlp_grad(dev(w), dev(X), dev(y))[1].cpu().numpy()
    b = mxs.mlp_grad(dev(w), dev(X), dev(y))[1].cpu().numpy()
    assert np.array_equal(a, b)


def test_adam_matches_oracle(gpu):
    mxs = gpu
    g0 = np.random.Generator(np.random.PCG64(60))
    w = g0.standard_normal(orc.NPARAM).astype(np.float32)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    wd, md, vd = dev(w), dev(m), dev(v)
    w64, m64, v64 = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    mag = np.zeros(orc.NPARAM)          # the same moving average of |g|
    for t in range(1, 6):
        grad = (g0.standard_normal(orc.NPARAM) * 10.0 ** g0.integers(-4, 1, orc.NPARAM)).astype(np.float32)
        mxs.mlp_adam(wd, md, vd, dev(grad), 1e-3, t)
        orc.adam_step(w64, m64, v64, grad.astype(np.float64), 1e-3, t)
        mag = 0.9 * mag + 0.1 * np.abs(grad.astype(np.float64))
    np.testing.assert_allclose(wd.cpu().numpy(), w64, rtol=0, atol=1e-6)
    # FP32 rounding of the first moment: at most a few units of 2^-24 per
    # step relative to the magnitudes summed (m may cancel to near zero)
    err = np.abs(md.cpu().numpy() - m64)
    assert np.all(err <= 5 * 4 * 2.0 ** -24 * mag + 1e-30)


def test_train_step_is_grad_then_adam(gpu):
    mxs = gpu
    torch = _torch()
    w = _net(10)
    X, y = _data(128, 70)
    wa, ma, va = dev(w), torch.zeros(orc.NPARAM, device="cuda"), torch.zeros(orc.NPARAM, device="cuda")
    wb, mb, vb = dev(w), torch.zeros_like(ma), torch.zeros_like(va)
    la = mxs.mlp_train_step(wa, ma, va, dev(X), dev(y), 1e-3, 1)
    lb, g = mxs.mlp_grad(wb, dev(X), dev(y))
    mxs.mlp_adam(wb, mb, vb, g, 1e-3, 1)
    assert torch.equal(wa, wb) and torch.equal(la, lb)


def test_predict_is_masked_argmax(gpu):
    mxs = gpu
    w = _net(11, scale=3.0)
    X, _ = _data(2000, 80)
    g = np.random.Generator(np.random.PCG64(81))
    feas = g.integers(0, 2, (2000, orc.NCLASS)).astype(np.uint8)
    feas[:20] = 0                                   # nothing feasible -> -1
    out = mxs.mlp_predict(dev(w), dev(X), dev(feas)).cpu().numpy()
    free = mxs.mlp_predict(dev(w), dev(X)).cpu().numpy()
    z = orc.mlp_forward(w.astype(np.float64), X.astype(np.float64))
    zs = np.sort(z, axis=1)
    clear = (zs[:, -1] - zs[:, -2]) > 1e-4 * np.maximum(1.0, np.abs(zs[:, -1]))
    assert np.array_equal(free[clear], np.argmax(z, axis=1)[clear])
    zm = np.where(feas > 0, z, -np.inf)
    exp = np.where(feas.any(axis=1), np.argmax(zm, axis=1), -1)
    zms = np.sort(zm, axis=1)
    with np.errstate(invalid="ignore"):
        gap = zms[:, -1] - zms[:, -2]
    ok = ~feas.any(axis=1) | (feas.sum(axis=1) == 1) | (gap > 1e-4 * np.maximum(1.0, np.abs(zms[:, -1])))
    assert ok.mean() > 0.9
    assert np.array_equal(out[ok], exp[ok])
    assert np.all(out[:20] == -1)
    assert np.all((out == -1) | (feas[np.arange(2000), np.maximum(out, 0)] > 0))


def test_training_reduces_loss_and_learns_a_rule(gpu):
    """A rule-labelled synthetic set: training drives the loss well below
    ln 5 and fits the rule."""
    from paper_2304_09511_amd import selector as S
    g = np.random.Generator(np.random.PCG64(90))
    F = np.abs(g.standard_normal((1200, 8))) * 10.0 ** g.integers(2, 7, (1200, 8))
    F[:, 6] = g.uniform(0, 1, 1200)
    F[:, 7] = g.uniform(0, 1, 1200)
    y = np.where(F[:, 6] > 0.6, 2, np.where(F[:, 7] > 0.5, 0, 1)).astype(np.int32)
    sel = S.Selector().fit(F, y, epochs=150)
    assert sel.loss_curve[-1] < 0.3 and sel.loss_curve[-1] < 0.3 * sel.loss_curve[0]
    acc = np.mean(sel.predict(F) == y)
    assert acc > 0.93


def test_exhaustive_tuner_times_every_feasible_format(gpu):
    mxs = gpu
    from paper_2304_09511_amd import selector as S
    a = wl.banded(200000, 11, 2000, seed=3)
    A = mxs.Matrix.coo(a.nrows, a.ncols, a.ai, a.aj, a.av)
    fmt, t = S.exhaustive_select(A, reps=5, warm=2)
    assert set(t) == set(S.FORMATS)
    # every row of the banded matrix fits HYB's ELL part and every entry the
    # DIA band: the two-part formats would have an empty remainder
    assert math.isinf(t["hdc"]) and math.isinf(t["hyb"])
    assert all(math.isfinite(v) and v > 0 for f, v in t.items() if f not in ("hdc", "hyb"))
    # scattered entries added: both parts non-empty (DIA itself is refused:
    # each scattered entry opens a diagonal)
    from test_split_gpu import merge
    g = wl.rng(5)
    rows = np.sort(g.choice(a.nrows, 4000, replace=False)).astype(np.int32)
    extra = wl.Coo(a.nrows, a.ncols, rows, g.integers(0, a.ncols, rows.size).astype(np.int32),
                   g.standard_normal(rows.size))
    bn = merge(a, extra)
    B = mxs.Matrix.coo(bn.nrows, bn.ncols, bn.ai, bn.aj, bn.av)
    fb, tb = S.exhaustive_select(B, reps=3, warm=1)
    assert math.isinf(tb["dia"]) and tb[fb] == min(tb.values())
    assert all(math.isfinite(v) and v > 0 for f, v in tb.items() if f != "dia")
    assert t[fmt] == min(t.values())
    z = wl.zipf_rows(100000, seed=2)
    Z = mxs.Matrix.coo(z.nrows, z.ncols, z.ai, z.aj, z.av)
    fz, tz = S.exhaustive_select(Z, reps=3, warm=1)
    assert math.isinf(tz["dia"]) and math.isinf(tz["ell"]) and math.isinf(tz["hdc"])
    assert fz in ("coo", "csr", "sell", "hyb")


def test_device_dataset_generators_match_oracle_features(gpu):
    """Matrices built on the device by the dataset generators: canonical
    (accepted by the container check) with the oracle's features."""
    mxs = gpu
    from paper_2304_09511_amd import selector as S
    for spec in ({"family": "stencil7", "n": 13}, {"family": "stencil27", "n": 11},
                 {"family": "banded", "rows": 30000, "ndiag": 23, "seed": 5},
                 {"family": "zipf", "rows": 30000, "seed": 6},
                 {"family": "block", "nblockrows": 3000, "seed": 7}):
        nr, nc, ai, aj, av = S.generate_arrays(spec)
        A = mxs.Matrix.coo(nr, nc, ai, aj, av, borrow=True)
        f = mxs.features(A)
        features_close(f, orc.features(nr, nc, ai.cpu().numpy(), aj.cpu().numpy()))


def test_trained_selector_beats_always_csr(gpu):
    """On the committed labelled set (timings of this GPU): the selector
    trained on the 2,400 training matrices has held-out mean regret at most
    5 % and below the always-CSR baseline's, on all 800 held-out matrices and
    on each group of families; every one of the seven formats is the fastest
    for some matrix of the set."""
    from paper_2304_09511_amd import selector as S
    if not S.DATA_PATH.exists():
        pytest.skip("no labelled dataset committed")
    recs, F, T, y = S.load_dataset(str(S.DATA_PATH))
    assert set(np.unique(y).tolist()) == set(range(len(S.FORMATS)))
    tr, te = S.dataset_split(len(recs))
    sel = S.Selector().fit(F[tr], y[tr], epochs=300)
    for part in (te, te[te < S.N_BASE], te[te >= S.N_BASE]):
        ev = S.evaluate(sel, F[part], T[part])
        assert ev["mean_regret"] <= 0.05, ev
        assert ev["mean_regret"] < ev["always_csr_regret"], ev
