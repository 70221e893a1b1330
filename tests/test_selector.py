"""Host logic of the format selector: dataset specification, labels, regret,
initialisation, and the oracle's features on the selector families."""
import math

import numpy as np
import pytest

import oracle as orc
import workloads as wl
from paper_2304_09511_amd import selector as S


def test_dataset_spec_is_deterministic_and_balanced():
    specs = [S.matrix_spec(i) for i in range(S.N_TOTAL)]
    assert S.N_TOTAL == S.N_BASE + 400 * len(S.EXT_FAMILIES)
    assert specs == [S.matrix_spec(i) for i in range(S.N_TOTAL)]
    fams = [s["family"] for s in specs]
    for f in S.FAMILIES + S.EXT_FAMILIES:
        assert fams.count(f) == 400
    assert set(fams[:S.N_BASE]) == set(S.FAMILIES)
    rows = []
    for s in specs:
        if s["family"].startswith("stencil"):
            rows.append(s["n"] ** 3)
        elif s["family"] == "block":
            rows.append(8 * s["nblockrows"])
        else:
            rows.append(s["rows"])
            if s["family"] in ("banded", "bandscatter"):
                assert 3 <= s["ndiag"] <= 64
            if s["family"] == "bandscatter":
                assert 0.001 <= s["frac"] <= 0.4 and isinstance(s["concentrated"], bool)
            if s["family"] == "hypersparse":
                assert 0.02 <= s["per_row"] <= 0.5
            if s["family"] == "windowed":
                assert 4 <= s["length"] <= 32 and 100 <= s["width"] <= 50200
                assert 0.01 <= s["tail_frac"] <= 0.5
    rows = np.array(rows)
    assert rows.min() >= 9000 and rows.max() <= 10_100_000
    # log-uniform: about a third of the matrices in each decade
    dec = np.floor(np.log10(rows)).clip(4, 6)
    for d in (4, 5, 6):
        assert 0.28 < np.mean(dec == d) < 0.39


def test_best_format_tie_order_and_regret():
    inf = math.inf
    assert S.best_format({"coo": 1.0, "csr": 1.0, "dia": 1.0, "ell": 1.0, "sell": 1.0}) == "csr"
    assert S.best_format({"coo": 1.0, "csr": 2.0, "dia": 1.0, "ell": 1.0, "sell": 1.0}) == "dia"
    assert S.best_format({"coo": 1.0, "csr": 2.0, "dia": inf, "ell": 1.0, "sell": 1.0}) == "ell"
    assert S.best_format({"coo": 1.0, "csr": 2.0, "dia": inf, "ell": inf, "sell": 1.0}) == "sell"
    assert S.best_format({"coo": 0.5, "csr": 2.0, "dia": inf, "ell": inf, "sell": 0.7}) == "coo"
    T = np.array([[3.0, 2.0, 1.0], [1.0, 2.0, np.inf], [2.0, 2.0, 4.0]])
    best = np.array([2, 0, 0])
    assert S.regret(T, best) == 0.0
    assert S.regret(T, np.array([1, 1, 1])) == pytest.approx((1.0 + 1.0 + 0.0) / 3)


def test_split_is_a_partition():
    tr, te = S.split(2000, 1500)
    assert len(tr) == 1500 and len(te) == 500
    assert np.array_equal(np.sort(np.concatenate([tr, te])), np.arange(2000))
    # the whole set: the base matrices keep that split, the further families
    # split three to one
    tr2, te2 = S.dataset_split(S.N_TOTAL)
    assert len(tr2) == 2400 and len(te2) == 800
    assert np.array_equal(np.sort(np.concatenate([tr2, te2])), np.arange(S.N_TOTAL))
    assert np.array_equal(tr2[tr2 < S.N_BASE], tr) and np.array_equal(te2[te2 < S.N_BASE], te)


@pytest.mark.parametrize("concentrated", [False, True])
def test_band_scatter_and_hypersparse_generators(concentrated):
    """Canonical COO (sorted, distinct, in range); the band keeps every
    in-range slot of its offsets; scattered entries add about frac of the
    band's count, gathered in at most 1% of the rows when concentrated."""
    import torch
    N = 30000
    nr, nc, ai, aj, av = wl.device_banded_scatter(N, 9, 300, 0.2, concentrated, seed=11, device="cpu")
    b_nr, _, b_ai, b_aj, _ = wl.device_banded(N, 9, 300, 11, device="cpu")
    key = ai.long() * nc + aj.long()
    assert bool((key[1:] > key[:-1]).all()) and nr == nc == N
    bkey = b_ai.long() * N + b_aj.long()
    assert bool(torch.isin(bkey, key).all())
    extra = key.numel() - bkey.numel()
    assert 0.15 * bkey.numel() <= extra <= 0.2 * bkey.numel()
    off = ~torch.isin(key, bkey)
    if concentrated:
        assert torch.unique(ai[off]).numel() <= N // 100
    nr, nc, ai, aj, av = wl.device_hypersparse(N, 0.3, seed=12, device="cpu")
    key = ai.long() * nc + aj.long()
    assert bool((key[1:] > key[:-1]).all())
    assert 0.29 * N <= key.numel() <= 0.3 * N and av.numel() == key.numel()
    nr, nc, ai, aj, av = wl.device_windowed_rows(N, 12, 500, 0.1, seed=13, device="cpu")
    key = ai.long() * nc + aj.long()
    assert bool((key[1:] > key[:-1]).all())
    lens = torch.bincount(ai.long(), minlength=N)
    # the body: at most length + 1 entries a row outside the long rows
    assert int(torch.quantile(lens.double(), 0.9)) <= 13 and int(lens.max()) > 13
    body = (aj.long() - ai.long()).abs() <= 500
    assert float(body.double().mean()) > 0.85


def test_he_init_layout_and_scale():
    w = S.he_init(6)
    assert w.dtype == np.float32 and w.size == orc.NPARAM
    W1, b1 = w[:512], w[512:576]
    W2, b2 = w[576:576 + 4096], w[4672:4736]
    W3, b3 = w[4736:4736 + 64 * S.NO], w[4736 + 64 * S.NO:]
    assert not b1.any() and not b2.any() and not b3.any()
    assert np.std(W1) == pytest.approx(math.sqrt(2 / 8), rel=0.15)
    assert np.std(W2) == pytest.approx(math.sqrt(2 / 64), rel=0.05)
    assert np.std(W3) == pytest.approx(math.sqrt(2 / 64), rel=0.15)


def test_dia_feasibility_rule_matches_oracle_slot_count():
    """The mask the selector uses is the container's refusal rule."""
    for coo in (wl.stencil(6), wl.banded(3000, 11, 200, seed=3),
                wl.zipf_rows(3000, seed=2), wl.block_random(200, seed=5)):
        f = orc.features(coo.nrows, coo.ncols, coo.ai, coo.aj)
        nd = int(f[5])
        assert S.dia_feasible(f) == (nd * coo.nrows <= 8 * coo.nnz)
    assert S.dia_feasible(orc.features(*(lambda c: (c.nrows, c.ncols, c.ai, c.aj))(wl.stencil(6))))
    z = wl.zipf_rows(3000, seed=2)
    assert not S.dia_feasible(orc.features(z.nrows, z.ncols, z.ai, z.aj))


def test_ell_feasibility_rule_matches_oracle_width():
    """ELL's mask is its refusal rule with the oracle's width (longest row)."""
    for coo in (wl.stencil(6), wl.banded(3000, 11, 200, seed=3),
                wl.zipf_rows(3000, seed=2), wl.block_random(200, seed=5)):
        f = orc.features(coo.nrows, coo.ncols, coo.ai, coo.aj)
        K, _, _ = orc.csr_to_ell(orc.coo_to_csr(coo.nrows, coo.ai), coo.aj, coo.av)
        assert f[4] == K and S.ell_feasible(f) == (K * coo.nrows <= 8 * coo.nnz)


@pytest.mark.parametrize("fam", ["banded", "zipf", "block"])
def test_device_generators_canonical_on_cpu(fam):
    """The torch generators emit sorted, distinct, in-range triples with the
    family's structure (run on the CPU device)."""
    import torch
    if fam == "banded":
        nr, nc, ai, aj, av = wl.device_banded(5000, 17, 300, 11, device="cpu")
        d = (aj.long() - ai.long()).unique()
        assert d.numel() == 17 and int(d.abs().max()) <= 300
    elif fam == "zipf":
        nr, nc, ai, aj, av = wl.device_zipf_rows(20000, 9, device="cpu")
        lens = torch.bincount(ai.long(), minlength=nr).double()
        assert 14.0 < float(lens.mean()) < 18.5 and int(lens.max()) <= 5000
    else:
        nr, nc, ai, aj, av = wl.device_block_random(300, 3, device="cpu")
        lens = torch.bincount(ai.long(), minlength=nr)
        assert bool(((lens % 8) == 0).all()) and int(lens.min()) >= 8 and int(lens.max()) <= 64
    key = ai.long() * nc + aj.long()
    assert bool((key[1:] > key[:-1]).all())
    assert int(ai.min()) >= 0 and int(ai.max()) < nr and int(aj.min()) >= 0 and int(aj.max()) < nc
    assert av.dtype == torch.float64 and av.numel() == ai.numel()


def test_committed_labels_are_consistent():
    """Every committed label is the argmin of its recorded times (tie rule),
    and the recorded features equal the oracle's for the matrix the spec
    names (checked on the small ones)."""
    path = S.DATA_PATH
    if not path.exists():
        pytest.skip("no labelled dataset committed")
    recs, F, T, y = S.load_dataset(str(path))
    assert len(recs) == S.N_TOTAL and [r["i"] for r in recs] == list(range(S.N_TOTAL))
    for r in recs:
        t = {f: (math.inf if r["times_ms"][f] is None else r["times_ms"][f]) for f in S.FORMATS}
        assert r["label"] == S.best_format(t)
        assert (r["times_ms"]["dia"] is None) == (not S.dia_feasible(r["features"]))
        assert (r["times_ms"]["ell"] is None) == (not S.ell_feasible(r["features"]))
        assert dict((k, v) for k, v in r.items() if k in S.matrix_spec(r["i"])) == S.matrix_spec(r["i"])
    # stencils are deterministic and banded features depend only on the
    # offsets (numpy-seeded), so these regenerate identically on the CPU;
    # the other families draw from torch's device generator
    checked = 0
    det = [r for r in recs if r["family"] in ("stencil7", "stencil27", "banded")]
    for r in sorted(det, key=lambda r: r["nnz"])[:10]:
        spec = S.matrix_spec(r["i"])
        nr, nc, ai, aj, _ = S.generate_arrays(spec, device="cpu")
        f = orc.features(nr, nc, ai.numpy(), aj.numpy())
        np.testing.assert_allclose(r["features"], f, rtol=1e-12)
        checked += 1
    assert checked == 10
