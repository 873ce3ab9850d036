"""GPU parity of the HIP path against the FP64 oracle, through the C-ABI.

Tolerances (written here, derived in the design notes):
  * lookups, Philox words, hit counts and hit checksums: bit-exact;
  * per-trial loss:  |Y_gpu - Y_oracle| <= 1e-5 * G_oracle (+1e-3 absolute),
    G = the trial's gross loss sum_k X_k (FP32 error enters at that scale
    because every clamp of the method is 1-Lipschitz);
  * PML / TVaR end to end: 1e-6 relative;
  * PML on the same YLT: bit-identical to numpy's k-th largest; TVaR 1e-12.
"""
import json
import math

import numpy as np
import pytest

import oracle
from tests.tiny import (GOLDEN, A, B, golden_worked_cases, random_tiny_case, worked_example,
                        yet_from_lists)
from workloads import config_small, make_yet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

T2 = 1e-5


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ara():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06326_amd import Ara
    a = Ara(0)
    yield a
    a.close()


def check_t2(got, ref, what):
    g = got.double().cpu().numpy() if hasattr(got, "cpu") else got
    err = np.abs(g - ref["ylt"])
    tol = T2 * ref["gross"] + 1e-3
    bad = np.argwhere(err > tol)
    assert bad.size == 0, (what, bad[:5], g[tuple(bad[0])], ref["ylt"][tuple(bad[0])])
    return float((err / np.maximum(ref["gross"], 1.0)).max())


# --------------------------------------------------------------------------
def test_philox_bit_exact(ara):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(1 << 20, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4096] = 0
    ctr[:4096, 0] = np.arange(4096)
    for key in (0, 150106326, 0xFFFFFFFFFFFFFFFF, 0x9ABCDEF012345678):
        say("philox key", key)
        got = ara.debug_philox(ctr, key)
        ref = oracle.philox4x32_10(ctr, np.array([key & 0xFFFFFFFF, key >> 32], np.uint32))
        assert np.array_equal(got, ref)


QUANTILE_SHAPES = [(2.75, 8.25), (1.0, 1.0), (1.0, 3.0), (3.0, 1.0), (1.2, 3.0), (30.0, 70.0),
                   (200.0, 300.0), (1.01, 50.0), (50.0, 1.01), (0.5, 0.5), (0.7, 5.0),
                   (5.0, 0.7), (0.01, 0.02), (2000.0, 3000.0)]


@pytest.mark.parametrize("a,b", QUANTILE_SHAPES)
def test_beta_quantile_accuracy(ara, a, b):
    """Per-draw accuracy against the FP64 oracle on the 2^-24 draw grid.
    Bound: the paper's convergence criterion (relative error < 1e-6,
    section 5.1) on |x - x_ref| / max(x_ref, mean), i.e. relative to the
    root where it is not tiny and to the distribution's mean below that."""
    rng = np.random.default_rng(7)
    j = np.concatenate([np.array([1, 3, 2 ** 23 - 1, 2 ** 23 + 1, 2 ** 24 - 3, 2 ** 24 - 1]),
                        (rng.integers(0, 2 ** 23, size=20000) * 2 + 1)]).astype(np.float64)
    z = j / 2 ** 24
    zc = (2 ** 24 - j) / 2 ** 24
    af = np.float32(a)
    bf = np.float32(b)
    say("quantile shape", a, b)
    x, path = ara.debug_beta_quantile(np.full(z.size, af), np.full(z.size, bf), z, zc)
    ref = oracle.betaincinv(float(af), float(bf), z, zc)
    assert np.all(np.isfinite(x))
    scale = np.maximum(ref, float(af) / (float(af) + float(bf)))
    err = np.abs(x.astype(np.float64) - ref) / scale
    say(f"  path64 share {path.mean():.4f}  max {err.max():.3g}  p99 {np.percentile(err, 99):.3g}")
    assert err.max() < 1e-6
    in_f32 = 1.0 <= af <= 32.0 and 1.0 <= bf <= 32.0
    if in_f32:
        # inside the FP32 domain (almost) every grid point stays on the FP32 path
        assert path.mean() < 1e-3


SHAPE_TABLE_SHAPES = [(2.75, 8.25), (1.0, 1.0), (1.0, 3.0), (3.0, 1.0), (1.2, 3.0), (1.0, 32.0),
                      (32.0, 1.0), (32.0, 32.0), (1.01, 30.0), (7.5, 2.5)]


@pytest.mark.parametrize("a,b", SHAPE_TABLE_SHAPES)
def test_beta_quantile_shape_table_accuracy(ara, a, b):
    """The path of rows whose Beta shape has a table (started from the
    shape's interpolated logit table, one Halley step when the start is
    close), over the same kind of grid points, tails included; every point
    stays on the FP32 path.  Bound: the paper's 1e-6 (section 5.1) for shapes
    within a factor 4 of symmetric; 2e-6 for the more skewed ones, where the
    FP32 prefactor's rounding (a few 1e-7) is amplified by the cancellation
    in 1 - I on the direct branch (a host emulation of both starting paths
    over 160 random shapes of the FP32 domain gives at most 1.6e-6)."""
    rng = np.random.default_rng(8)
    j = np.concatenate([np.array([1, 3, 5, 2 ** 23 - 1, 2 ** 23 + 1, 2 ** 24 - 5, 2 ** 24 - 3,
                                  2 ** 24 - 1]),
                        (rng.integers(0, 2 ** 23, size=20000) * 2 + 1)]).astype(np.float64)
    z = j / 2 ** 24
    zc = (2 ** 24 - j) / 2 ** 24
    say("quantile shape table", a, b)
    x, path = ara.debug_beta_quantile_shape(a, b, z, zc)
    af, bf = float(np.float32(a)), float(np.float32(b))
    ref = oracle.betaincinv(af, bf, z, zc)
    assert np.all(np.isfinite(x))
    err = np.abs(x.astype(np.float64) - ref) / np.maximum(ref, af / (af + bf))
    say(f"  path64 share {path.mean():.4f}  max {err.max():.3g}  p99 {np.percentile(err, 99):.3g}")
    assert err.max() < (1e-6 if max(af, bf) <= 4.0 * min(af, bf) else 2e-6)
    assert path.mean() < 1e-3


def test_worked_example_exact(ara):
    yet, pf = worked_example(trials=[[A, B, A], [B], [], [A, A, A]])
    say("worked example PU")
    y = ara.load_yet(yet)
    p = ara.load_portfolio(pf, yet.n_catalogue)
    r = ara.run(y, p)
    assert r["ylt"].cpu().numpy()[0].tolist() == [6.0e5, 0.0, 0.0, 3.4e6]
    pf.su_enabled = True     # sigma = 0 rows: the secondary-uncertainty kernel must agree
    p2 = ara.load_portfolio(pf, yet.n_catalogue)
    r2 = ara.run(y, p2, diagnostics=True)
    assert r2["ylt"].cpu().numpy()[0].tolist() == [6.0e5, 0.0, 0.0, 3.4e6]
    assert r2["hits"].cpu().numpy()[0].tolist() == [5, 1, 0, 6]


@pytest.mark.parametrize("su", [False, True])
def test_ragged_long_trials(ara, su):
    """Trial lengths around every boundary of the kernels (one wavefront of
    64 occurrences, a 512-occurrence segment, a 1,280-id pass) and one trial
    of 50,000 occurrences (about a hundred segments): YLT, hit counts and the
    occurrence view against the oracle."""
    from workloads import INF
    rng = np.random.default_rng(21)
    lengths = [50_000, 0, 1, 63, 64, 65, 511, 512, 513, 1025, 1279, 1280, 1281, 3000, 0, 7]
    w = config_small(su=su, n_trials=1)
    trials = [list(rng.integers(0, w.yet.n_catalogue, size=n)) for n in lengths]
    yet = yet_from_lists(trials, w.yet.n_catalogue)
    pf = w.portfolio
    pf.layers[0].agg_limit = INF                     # keep the long trial's loss informative
    say("ragged long trials, su", su)
    ref = oracle.run_ara(yet, pf, occ_view=True)
    y = ara.load_yet(yet)
    p = ara.load_portfolio(pf, yet.n_catalogue)
    r = ara.run(y, p, diagnostics=su, occ_view=True)
    check_t2(r["ylt"], ref, "ragged")
    if su:
        assert np.array_equal(r["hits"].cpu().numpy(), ref["hits"])
        assert np.array_equal(r["hit_chk"].cpu().numpy().view(np.uint64), ref["hit_chk"])
    d = r["occ_view"].double().cpu().numpy()
    G = np.repeat(ref["gross"], np.diff(yet.offsets), axis=1)
    assert np.all(np.abs(d - ref["occ_view"]) <= 2 * (1e-5 * G + 1e-3))
    lean = ara.run(y, p, occ_view=True)              # the lean pass: the same view
    assert torch.equal(lean["occ_view"], r["occ_view"])
    ara.free_portfolio(p)
    ara.free_yet(y)


def test_empty_inputs(ara):
    """A YET whose trials are all empty (no occurrence, so no event-id array
    is needed on the device) through both kernels, with the occurrence view
    and the hit counts, and a run over no trial: every YLT entry is 0."""
    yet = yet_from_lists([[], [], [], []], 4)
    _, pf = worked_example()
    say("empty inputs")
    y = ara.load_yet(yet)
    for su in (False, True):
        pf.su_enabled = su
        p = ara.load_portfolio(pf, yet.n_catalogue)
        r = ara.run(y, p, diagnostics=su, occ_view=True)
        assert r["ylt"].cpu().numpy().tolist() == [[0.0] * 4], su
        assert r["ylt_pf"].cpu().numpy().tolist() == [0.0] * 4, su
        if su:
            assert r["hits"].cpu().numpy().tolist() == [[0] * 4]
        r0 = ara.run(y, p, trial_begin=2, trial_count=0)
        assert tuple(r0["ylt"].shape) == (1, 0) and r0["ylt_pf"].numel() == 0
        ara.free_portfolio(p)
    ara.free_yet(y)


@pytest.mark.parametrize("corr", [False, True])
def test_small_config_vs_stored_oracle(ara, corr):
    """Against the oracle's stored results (tests/golden/oracle_small.json),
    without running the oracle: hit count exact, PML / TVaR 1e-6 relative."""
    with open(GOLDEN / "oracle_small.json") as f:
        case = json.load(f)["cases"][int(corr)]
    w = config_small(corr=corr)
    assert w.name == case["workload"]
    say("stored oracle results:", w.name)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p, diagnostics=True)
    assert int(r["hits"].sum().item()) == case["hits"]
    pml, tvar = ara.pml_tvar(r["ylt_pf"], case["return_periods"])
    np.testing.assert_allclose(pml, case["pml"], rtol=1e-6)
    np.testing.assert_allclose(tvar, case["tvar"], rtol=1e-6)
    ara.free_portfolio(p)
    ara.free_yet(y)


def test_worked_example_golden_fixture(ara):
    """The hand-worked fixture through both kernels: exact values."""
    for name, yet, pf, ex in golden_worked_cases():
        say("golden worked example:", name)
        y = ara.load_yet(yet)
        for su in (False, True):
            pf.su_enabled = su
            p = ara.load_portfolio(pf, yet.n_catalogue)
            r = ara.run(y, p, diagnostics=su, occ_view=True)
            assert r["ylt"].cpu().numpy()[0].tolist() == ex["ylt"], (name, su)
            if ex["occ_view"]:
                assert r["occ_view"].cpu().numpy()[0].tolist() == ex["occ_view"], (name, su)
            if su:
                assert r["hits"].cpu().numpy()[0].tolist() == ex["hits"], (name, su)
            ara.free_portfolio(p)
        ara.free_yet(y)


@pytest.mark.parametrize("su", [False, True])
def test_small_config_parity(ara, su):
    w = config_small(su=su)
    say("small config su", su, w.yet.n_trials, w.yet.n_occ)
    ref = oracle.run_ara(w.yet, w.portfolio)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p, diagnostics=su)
    m = check_t2(r["ylt"], ref, "small")
    say(f"  max |dY|/G = {m:.3g}")
    pf_ref = ref["ylt_pf"]
    pf_got = r["ylt_pf"].double().cpu().numpy()
    assert np.all(np.abs(pf_got - pf_ref) <= T2 * ref["gross"].sum(0) + 1e-3)
    if su:
        assert np.array_equal(r["hits"].cpu().numpy(), ref["hits"])
        assert np.array_equal(r["hit_chk"].cpu().numpy().view(np.uint64), ref["hit_chk"])
    pml, tvar = ara.pml_tvar(r["ylt_pf"], w.return_periods)
    opml, otvar = oracle.pml_tvar(pf_ref, w.return_periods)
    say(f"  PML {pml} vs {opml}; TVaR {tvar} vs {otvar}")
    np.testing.assert_allclose(pml, opml, rtol=1e-6)
    np.testing.assert_allclose(tvar, otvar, rtol=1e-6)


def test_small_config_correlated(ara):
    w = config_small(corr=True, n_trials=3000)
    say("small correlated", w.yet.n_trials)
    ref = oracle.run_ara(w.yet, w.portfolio)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p, diagnostics=True)
    check_t2(r["ylt"], ref, "corr")
    assert np.array_equal(r["hits"].cpu().numpy(), ref["hits"])


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("su,corr", [(False, False), (True, False), (True, True)])
def test_tiny_random_portfolios(ara, seed, su, corr):
    rng = np.random.default_rng(1000 + seed)
    yet, pf = random_tiny_case(rng, n_cat=40, n_layers=3, max_elts=4, max_occ=30, n_trials=64,
                               dyadic=False, su=su, corr=corr)
    say("tiny", seed, su, corr)
    ref = oracle.run_ara(yet, pf)
    y = ara.load_yet(yet)
    p = ara.load_portfolio(pf, yet.n_catalogue)
    r = ara.run(y, p, diagnostics=su)
    check_t2(r["ylt"], ref, f"tiny {seed}")
    if su:
        assert np.array_equal(r["hits"].cpu().numpy(), ref["hits"])


def test_determinism_and_slicing(ara):
    w = config_small(n_trials=3000)
    say("determinism")
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    a = ara.run(y, p)["ylt"].cpu().numpy()
    b = ara.run(y, p)["ylt"].cpu().numpy()
    assert np.array_equal(a, b)
    c1 = ara.run(y, p, trial_begin=0, trial_count=1234)["ylt"].cpu().numpy()
    c2 = ara.run(y, p, trial_begin=1234, trial_count=3000 - 1234)["ylt"].cpu().numpy()
    assert np.array_equal(np.concatenate([c1, c2], axis=1), a)


@pytest.mark.parametrize("su", [False, True])
def test_small_trial_ranges(ara, su):
    """Ranges far below one block of wavefronts (1, 7, 17 trials, odd starts)
    give the same YLT entries as the whole run: a trial's result does not
    depend on the grid that computed it."""
    w = config_small(su=su, n_trials=3000)
    say("small trial ranges", su)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    full = ara.run(y, p)["ylt"].cpu().numpy()
    for tb, tc in [(0, 1), (5, 7), (100, 17), (2983, 17), (1, 2999)]:
        part = ara.run(y, p, trial_begin=tb, trial_count=tc)["ylt"].cpu().numpy()
        assert np.array_equal(part, full[:, tb:tb + tc]), (tb, tc)
    ara.free_portfolio(p)
    ara.free_yet(y)


@pytest.mark.parametrize("mode", ["naive32", "kahan32", "f64"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sum_modes(ara, mode, dtype):
    w = config_small(n_trials=2000)
    say("sum mode", mode, dtype)
    ref = oracle.run_ara(w.yet, w.portfolio)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p, sum_mode=mode, ylt_dtype=dtype)
    assert r["ylt"].dtype == (torch.float64 if dtype == "f64" else torch.float32)
    check_t2(r["ylt"], ref, mode)


def test_pml_tvar_on_same_ylt(ara):
    rng = np.random.default_rng(5)
    for n, dt in [(1_000_000, np.float32), (12345, np.float32), (777, np.float64), (50, np.float32)]:
        v = rng.lognormal(14, 2, size=n).astype(dt)
        v[rng.random(n) < 0.3] = 0
        v[:10] = v[10]           # ties
        t = torch.from_numpy(v).cuda()
        rps = [100.0, 250.0, 1.0, 2.0, 1e9]
        say("pml", n, dt)
        pml, tvar = ara.pml_tvar(t, rps)
        s = np.sort(v.astype(np.float64))[::-1]
        for r_, rp in enumerate(rps):
            k = max(1, int(math.floor(n / rp)))
            assert pml[r_] == s[k - 1]
            assert abs(tvar[r_] - math.fsum(s[:k]) / k) <= 1e-12 * abs(tvar[r_]) + 1e-300


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_pml_tvar_many_return_periods(ara, dt):
    """Return periods are selected in groups of up to eight: 19 periods (three
    groups) with duplicates, periods whose k-th largest values share their
    leading digits, k = 1, k = N (and a period below 1, whose k is clamped to
    N), negative zeros, two calls in a row; FP32 and FP64 losses."""
    rng = np.random.default_rng(11)
    n = 200_003
    v = rng.lognormal(14, 1.5, size=n).astype(dt)
    v[rng.random(n) < 0.4] = 0
    v[rng.random(n) < 0.05] = -0.0
    v[100:200] = v[99]                              # a run of ties
    t = torch.from_numpy(v).cuda()
    rps = [100.0, 101.0, 99.5, 250.0, 250.0, 1.0, 1.5, 2.0, 1e9, 3.0, 10.0, 20.0, 50.0, 200.0,
           500.0, 1000.0, 5000.0, 0.5, 1.0001]
    s = np.sort(v.astype(np.float64))[::-1]
    for call in range(2):
        say("pml many return periods", dt.__name__, "call", call)
        pml, tvar = ara.pml_tvar(t, rps)
        for r_, rp in enumerate(rps):
            k = min(n, max(1, int(math.floor(n / rp))))
            assert pml[r_] == s[k - 1], (rp, pml[r_], s[k - 1])
            assert abs(tvar[r_] - math.fsum(s[:k]) / k) <= 1e-12 * abs(tvar[r_]) + 1e-300, rp
        # a shorter YLT through the same scratch
        pml2, tvar2 = ara.pml_tvar(t[:1000], [7.0, 1.0, 1000.0])
        s2 = np.sort(v[:1000].astype(np.float64))[::-1]
        for r_, rp in enumerate([7.0, 1.0, 1000.0]):
            k = max(1, int(math.floor(1000 / rp)))
            assert pml2[r_] == s2[k - 1]
            assert abs(tvar2[r_] - math.fsum(s2[:k]) / k) <= 1e-12 * abs(tvar2[r_]) + 1e-300


def test_input_errors(ara):
    from paper_1501_06326_amd.ara import (ARA_E_BAD_ELT_ROW, ARA_E_EVENT_ID_RANGE,
                                          ARA_E_OFFSETS_NOT_MONOTONE, ARA_E_TIMES_UNSORTED,
                                          AraError)
    yet, pf = worked_example()
    say("errors")
    bad = make_yet(5, 4.0, 4, 1)
    bad.event_ids[3] = 7
    with pytest.raises(AraError) as e:
        ara.load_yet(bad)
    assert e.value.code == ARA_E_EVENT_ID_RANGE
    bad = make_yet(5, 4.0, 4, 1)
    bad.times[bad.offsets[1]:bad.offsets[2]] = bad.times[bad.offsets[1]:bad.offsets[2]][::-1]
    if bad.offsets[2] - bad.offsets[1] > 1 and bad.times[bad.offsets[1]] != bad.times[bad.offsets[1] + 1]:
        with pytest.raises(AraError) as e:
            ara.load_yet(bad)
        assert e.value.code == ARA_E_TIMES_UNSORTED
    from tests.tiny import yet_from_lists
    bad = yet_from_lists([[0, 1, 2], [3, 0], [1, 1, 2], [0, 3]], 4)
    bad.offsets[2] = 2                                  # offsets 0, 3, 2, 8, 10
    with pytest.raises(AraError) as e:
        ara.load_yet(bad)
    assert e.value.code == ARA_E_OFFSETS_NOT_MONOTONE
    e1 = pf.layers[0].elts[0]
    e1.event_ids = np.array([A, A], np.int32)        # duplicate event in one ELT
    with pytest.raises(AraError) as e:
        ara.load_portfolio(pf, 4)
    assert e.value.code == ARA_E_BAD_ELT_ROW
    yet, pf = worked_example()
    pf.su_enabled = True
    e1 = pf.layers[0].elts[0]
    e1.sigma_i = np.array([1.0, 1.0], np.float32)
    e1.max_loss = e1.mean.copy()                        # mean >= max_loss with sigma > 0
    with pytest.raises(AraError) as e:
        ara.load_portfolio(pf, 4)
    assert e.value.code == ARA_E_BAD_ELT_ROW
    yet, pf = worked_example()
    y = ara.load_yet(yet)
    p = ara.load_portfolio(pf, 8)                       # catalogue mismatch
    with pytest.raises(AraError):
        ara.run(y, p)


def test_numeric_failure_reported(ara):
    """The convergence check behind ARA_E_NUMERIC (section 5.1's criterion
    on the quantile): with ARA_DEBUG_QUANTILE_ONE_STEP every draw takes the
    FP64 quantile and may take one step only, so draws are reported as
    non-converging through ara_sync_status, with a (trial, occurrence,
    elt_id) that is a real hit of the run; every kernel still ends."""
    from paper_1501_06326_amd.ara import (ARA_DEBUG_QUANTILE_ONE_STEP, ARA_E_NUMERIC, AraError)
    w = config_small(n_trials=300)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    say("numeric failure")
    with pytest.raises(AraError) as e:
        ara.run(y, p, trial_begin=100, trial_count=150, debug_flags=ARA_DEBUG_QUANTILE_ONE_STEP)
    assert e.value.code == ARA_E_NUMERIC
    import re
    m = re.search(r"trial (\d+), occurrence (\d+), elt_id (\d+)", str(e.value))
    assert m, str(e.value)
    t, k, elt = (int(v) for v in m.groups())
    assert 100 <= t < 250
    off = w.yet.offsets
    assert 0 <= k < off[t + 1] - off[t]
    ev = int(w.yet.event_ids[off[t] + k])
    rows = [x for x in w.portfolio.layers[0].elts if x.elt_id == elt]
    assert rows and ev in set(rows[0].event_ids.tolist())
    # the flag is cleared by the report: a normal run afterwards is clean and
    # matches the oracle
    r = ara.run(y, p, trial_begin=100, trial_count=150)
    ref = oracle.run_ara(w.yet, w.portfolio, 100, 150)
    check_t2(r["ylt"], ref, "after numeric failure")
    # an unknown flag is rejected before anything is enqueued
    with pytest.raises(AraError) as e:
        ara.run(y, p, debug_flags=4)
    assert e.value.code == -1


def test_run_requires_scratch(ara):
    """ara_run allocates nothing: a secondary-uncertainty run without scratch,
    or with too little, fails with ARA_E_WORKSPACE_TOO_SMALL; a primary-
    uncertainty run needs none."""
    from paper_1501_06326_amd.ara import ARA_E_WORKSPACE_TOO_SMALL, AraError
    w = config_small(n_trials=200)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    small = torch.empty(16, dtype=torch.uint8, device=ara.device)
    with pytest.raises(AraError) as e:
        ara.run(y, p, scratch=small)
    assert e.value.code == ARA_E_WORKSPACE_TOO_SMALL
    from paper_1501_06326_amd import ara as AB
    o = AB.ara_run_opts(trial_begin=0, trial_count=200, sum_mode=0, ylt_dtype=0, tail_band=0.0,
                        debug_flags=0, d_hits=None, d_hit_chk=None, d_scratch=None,
                        scratch_bytes=0, d_occ_view=None, occ_view_stride=0)
    out = torch.empty(200, dtype=torch.float32, device=ara.device)
    rc = AB.lib().ara_run(ara.ctx, y.handle, p.handle, o, None, out.data_ptr(), None)
    assert rc == ARA_E_WORKSPACE_TOO_SMALL
    pu = config_small(n_trials=200, su=False)
    q = ara.load_portfolio(pu.portfolio, pu.yet.n_catalogue)
    rc = AB.lib().ara_run(ara.ctx, y.handle, q.handle, o, None, out.data_ptr(), None)
    assert rc == 0
    torch.cuda.synchronize()
    ref = oracle.run_ara(pu.yet, pu.portfolio)
    check_t2(out.view(1, -1), {"ylt": ref["ylt_pf"][None, :], "gross": ref["gross"]}, "pu")


def test_concurrent_runs_on_two_streams(ara):
    """Two runs whose trials go through the FP64-capable second pass (rows
    with sigma_C > 0 and rows of varied shapes), enqueued on two streams at
    once, each with its own scratch: each equals the same run alone."""
    from workloads import varied_shapes
    w = config_small(corr=True, n_trials=3000)
    y = ara.load_yet(w.yet)
    p1 = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    p2 = ara.load_portfolio(varied_shapes(config_small(n_trials=10).portfolio),
                            w.yet.n_catalogue)
    alone1 = ara.run(y, p1)["ylt"].clone()
    alone2 = ara.run(y, p2)["ylt"].clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    say("two streams")
    for _ in range(3):
        r1 = ara.run(y, p1, stream=s1, sync=False)
        r2 = ara.run(y, p2, stream=s2, sync=False)
        torch.cuda.synchronize()
        ara.sync_status()
        assert torch.equal(r1["ylt"], alone1)
        assert torch.equal(r2["ylt"], alone2)
