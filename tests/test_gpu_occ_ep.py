"""GPU parity of the occurrence view and the exceedance-probability curve.

Occurrence view (d_k = A_k - A_{k-1}, aggregate terms over the running sum of
the occurrence losses in stored order): per occurrence against the FP64
oracle with the per-trial tolerance of the YLT (the same FP32 error in the
occurrence losses enters every A_k: |d_gpu - d_orc| <= 2 (1e-5 G + 1e-3),
G the trial's gross loss); the increments of a trial add up to its YLT
entry.  EP curve: the sorted losses equal the oracle's sort of the same YLT
bit for bit, the FP64 running means agree to 1e-12, and the points at a
return period equal ara_pml_tvar (PML bit-identical, TVaR 1e-12)."""
import math

import numpy as np
import pytest

import oracle
from workloads import config_small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def per_occurrence_gross(yet, tb, tc, gross):
    """The trial's gross loss repeated over its occurrences: [n_layers, n_occ]."""
    off = yet.offsets[tb:tb + tc + 1]
    reps = np.diff(off)
    return np.repeat(gross, reps, axis=1)


@pytest.mark.parametrize("su,sum_mode,dtype", [(True, "naive32", "f32"), (False, "naive32", "f32"),
                                               (True, "f64", "f64"), (False, "kahan32", "f32")])
def test_occurrence_view_vs_oracle(ara, su, sum_mode, dtype):
    w = config_small(su=su, n_trials=2000)
    tb, tc = 300, 1500
    say("occ view", su, sum_mode, dtype)
    ref = oracle.run_ara(w.yet, w.portfolio, tb, tc, occ_view=True)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p, trial_begin=tb, trial_count=tc, sum_mode=sum_mode, ylt_dtype=dtype,
                occ_view=True)
    d = r["occ_view"].double().cpu().numpy()
    G = per_occurrence_gross(w.yet, tb, tc, ref["gross"])
    err = np.abs(d - ref["occ_view"])
    assert np.all(err <= 2 * (1e-5 * G + 1e-3)), err.max()
    # a trial's increments add up to its layer loss
    off = w.yet.offsets[tb:tb + tc + 1] - w.yet.offsets[tb]
    sums = np.add.reduceat(d, off[:-1], axis=1) * (np.diff(off) > 0)
    ylt = r["ylt"].double().cpu().numpy()
    assert np.all(np.abs(sums - ylt) <= 1e-6 * ref["gross"] + 1e-3)
    ara.free_portfolio(p)
    ara.free_yet(y)


@pytest.mark.parametrize("corr", [False, True])
def test_occurrence_view_lean_equals_diagnostic(ara, corr):
    """Without hit counts the view comes from the lean pass (only the rows that
    can pay are visited); with them, from the diagnostic pass (every row).
    The rows the lean pass skips add +0, so the two views are bit-identical;
    the correlated case sends trials through the FP64-capable second pass."""
    w = config_small(corr=corr, n_trials=3000)
    tb, tc = 100, 2700
    say("occ view lean vs diagnostic, corr", corr)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    lean = ara.run(y, p, trial_begin=tb, trial_count=tc, occ_view=True)
    diag = ara.run(y, p, trial_begin=tb, trial_count=tc, occ_view=True, diagnostics=True)
    assert torch.equal(lean["occ_view"], diag["occ_view"])
    assert torch.equal(lean["ylt"], diag["ylt"])
    plain = ara.run(y, p, trial_begin=tb, trial_count=tc)
    assert torch.equal(lean["ylt"], plain["ylt"])
    ara.free_portfolio(p)
    ara.free_yet(y)


@pytest.mark.parametrize("n_catalogue", [1_000_000])
def test_occurrence_view_table_layouts(ara, n_catalogue):
    """Without secondary uncertainty the view reads the per-event table from
    LDS, dense (the golden worked example) or sparse (the small workload,
    above), or from global memory when it is too large for LDS (here)."""
    from workloads import config_full
    w = config_full(n_trials=300, with_times=False, su=False, n_catalogue=n_catalogue)
    say("occ view table layout, catalogue", n_catalogue, w.yet.n_occ)
    ref = oracle.run_ara(w.yet, w.portfolio, occ_view=True)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p, occ_view=True)
    d = r["occ_view"].double().cpu().numpy()
    G = per_occurrence_gross(w.yet, 0, w.yet.n_trials, ref["gross"])
    err = np.abs(d - ref["occ_view"])
    assert np.all(err <= 2 * (1e-5 * G + 1e-3)), err.max()
    ara.free_portfolio(p)
    ara.free_yet(y)


def test_occurrence_view_stride_too_small(ara):
    from paper_1501_06326_amd.ara import ARA_E_WORKSPACE_TOO_SMALL, AraError
    w = config_small(n_trials=200)
    say("occ view small stride")
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    n_occ = int(w.yet.offsets[200] - w.yet.offsets[0])
    with pytest.raises(AraError) as e:
        ara.run(y, p, occ_view=True, occ_view_stride=n_occ // 2)
    assert e.value.code == ARA_E_WORKSPACE_TOO_SMALL
    r = ara.run(y, p, occ_view=True)              # the context is usable again
    assert r["occ_view"].shape[1] == n_occ
    ara.free_portfolio(p)
    ara.free_yet(y)


def ep_cases():
    rng = np.random.default_rng(11)
    yield "lognormal_1M", rng.lognormal(14, 2, size=1_000_003).astype(np.float32)
    yield "ties", np.repeat(rng.lognormal(14, 2, size=300).astype(np.float32), 37)
    yield "zeros_negzero", np.array([0.0, -0.0, 3.0, 0.0, -0.0, 1.0], np.float32)
    yield "one", np.array([42.0], np.float32)
    yield "tile_edge", rng.lognormal(10, 1, size=2049).astype(np.float32)
    yield "f64", rng.lognormal(14, 2, size=100_001)


@pytest.mark.parametrize("case", [c for c, _ in ep_cases()])
def test_ep_curve(ara, case):
    y = dict(ep_cases())[case]
    say("ep curve", case, y.shape[0])
    yt = torch.from_numpy(y).to(ara.device)
    srt, tm = ara.ep_curve(yt)
    s = srt.cpu().numpy()
    ref_s, ref_tm = oracle.ep_curve(y.astype(np.float64))
    assert np.array_equal(s.astype(np.float64), ref_s)
    assert not np.any(np.signbit(s))
    t = tm.cpu().numpy()
    assert np.all(np.abs(t - ref_tm) <= 1e-12 * np.abs(ref_tm))
    rps = [1.0, 2.0, 10.0, 100.0, 250.0, 1e9]
    pml, tvar = ara.pml_tvar(yt, rps)
    for j, rp in enumerate(rps):
        k = max(1, int(math.floor(y.shape[0] / rp)))
        assert pml[j] == float(s[k - 1])
        assert abs(tvar[j] - t[k - 1]) <= 1e-12 * abs(tvar[j]) + 1e-300


def test_ep_curve_of_a_ylt(ara):
    """The EP curve of a GPU YLT equals the oracle's curve of that YLT."""
    w = config_small(n_trials=10_000)
    say("ep curve of ylt")
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    r = ara.run(y, p)
    srt, tm = ara.ep_curve(r["ylt_pf"])
    ref_s, ref_tm = oracle.ep_curve(r["ylt_pf"].double().cpu().numpy())
    assert np.array_equal(srt.double().cpu().numpy(), ref_s)
    assert np.all(np.abs(tm.cpu().numpy() - ref_tm) <= 1e-12 * np.abs(ref_tm) + 1e-300)
    ara.free_portfolio(p)
    ara.free_yet(y)
