"""Full-shape parity: the 1,000,000-trial x Poisson(1000) workload with 16 ELTs,
run in the launch configuration the benchmark times, checked against the FP64
oracle: end to end against the oracle's stored results for the whole YET
(PML / TVaR at 1e-6 relative, the 10,000 largest trial losses and 2,000
uniform trials per trial at 1e-5 of the trial's gross loss, the lookup counts
and checksums summed over every trial bit-exact), on freshly computed sampled
trials, and through properties that hold at any size."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads import config_full, full_portfolio

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06326_amd import Ara
    w = config_full(n_trials=1_000_000, with_times=False)
    print("full shape generated", w.yet.n_occ, flush=True)
    a = Ara(0)
    y = a.load_yet(w.yet)
    yield a, w, y
    a.close()


def sample_trials(n, k=160, seed=11):
    rng = np.random.default_rng(seed)
    s = set(rng.choice(n, size=k, replace=False).tolist()) | {0, 1, n - 2, n - 1}
    return sorted(s)


@pytest.mark.parametrize("su", [True, False])
def test_full_shape_sampled_parity(full, su):
    ara, w, y = full
    pf = w.portfolio if su else full_portfolio(su=False)
    print("full shape su", su, flush=True)
    p = ara.load_portfolio(pf, w.yet.n_catalogue)
    r = ara.run(y, p, diagnostics=su)
    ylt = r["ylt"][0].cpu().numpy().astype(np.float64)
    idx = sample_trials(w.yet.n_trials)
    ref = oracle.run_ara(w.yet, pf, trials=idx)
    err = np.abs(ylt[idx] - ref["ylt"][0])
    tol = 1e-5 * ref["gross"][0] + 1e-3
    assert np.all(err <= tol), (np.max(err / np.maximum(ref["gross"][0], 1)))
    if su:
        assert np.array_equal(r["hits"][0].cpu().numpy()[idx], ref["hits"][0])
        assert np.array_equal(r["hit_chk"][0].cpu().numpy().view(np.uint64)[idx],
                              ref["hit_chk"][0])
    # properties at full size: bounds, determinism, slicing, PML on the same YLT
    layer = pf.layers[0]
    assert np.all(ylt >= 0) and np.all(ylt <= layer.agg_limit)
    r2 = ara.run(y, p)
    assert torch.equal(r2["ylt"], r["ylt"])
    part = ara.run(y, p, trial_begin=400_000, trial_count=123_457)["ylt"][0]
    assert torch.equal(part, r["ylt"][0][400_000:400_000 + 123_457])
    pml, tvar = ara.pml_tvar(r["ylt_pf"], [100.0, 250.0])
    s = np.sort(r["ylt_pf"].cpu().numpy().astype(np.float64))[::-1]
    for j, rp in enumerate([100.0, 250.0]):
        k = int(math.floor(s.size / rp))
        assert pml[j] == s[k - 1]
        assert abs(tvar[j] - math.fsum(s[:k]) / k) <= 1e-12 * tvar[j]


GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_full.json")


@pytest.mark.parametrize("case", ["su", "pu"])
def test_full_shape_end_to_end_vs_stored_oracle(full, case):
    """The headline configuration (lean pass, compensated FP32 sums, FP32
    YLT) against the FP64 oracle run once over all 1,000,000 trials
    (tests/golden/make_oracle_full.py): the YLT and its metrics of section
    2.3 at the full size."""
    ara, w, y = full
    with open(GOLD_PATH) as f:
        gold = json.load(f)
    assert gold["n_occurrences"] == w.yet.n_occ
    assert gold["event_id_sum"] == int(w.yet.event_ids.sum(dtype=np.int64))
    g = gold["cases"][case]
    pf = w.portfolio if case == "su" else full_portfolio(su=False)
    print("end to end", case, flush=True)
    p = ara.load_portfolio(pf, w.yet.n_catalogue)
    r = ara.run(y, p, sum_mode="kahan32")
    rps = g["return_periods"]
    pml, tvar = ara.pml_tvar(r["ylt_pf"], rps)
    rel_pml = np.abs(pml - np.array(g["pml"])) / np.array(g["pml"])
    rel_tvar = np.abs(tvar - np.array(g["tvar"])) / np.array(g["tvar"])
    print(f"{case}: PML rel err {rel_pml}, TVaR rel err {rel_tvar}", flush=True)
    assert np.all(rel_pml <= 1e-6) and np.all(rel_tvar <= 1e-6)
    yg = r["ylt_pf"].cpu().numpy().astype(np.float64)
    for key in ("top", "sample"):
        idx = np.asarray(g[key + "_index"], np.int64)
        ref = np.asarray(g[key + "_y"])
        gross = np.asarray(g[key + "_gross"])
        err = np.abs(yg[idx] - ref)
        bad = np.flatnonzero(err > 1e-5 * gross + 1e-3)
        strict = err / np.maximum(ref, 1.0)
        print(f"{case} {key}: max err/G {np.max(err / np.maximum(gross, 1.0)):.3g}, "
              f"strict rel max {strict.max():.3g} median {np.median(strict):.3g}", flush=True)
        assert bad.size == 0, (key, idx[bad[:5]], yg[idx[bad[:5]]], ref[bad[:5]])
    ysum = math.fsum(yg.tolist())
    assert abs(ysum - g["ylt_sum"]) <= 1e-6 * g["ylt_sum"], (ysum, g["ylt_sum"])
    # a trial's loss sits at 0 below the aggregate retention: FP32 rounding may
    # move a trial within 1e-5 of its gross across that edge, never many
    assert abs(int((yg > 0).sum()) - g["positive_trials"]) <= 50
    if case == "su":
        d = ara.run(y, p, diagnostics=True)
        assert int(d["hits"].sum().item()) == g["hits_total"]
        chk = d["hit_chk"].cpu().numpy().view(np.uint64)
        assert int(np.sum(chk, dtype=np.uint64)) == g["hit_chk_total"]
