"""Full-shape parity: the 1,000,000-trial x Poisson(1000) workload with 16 ELTs,
run in the launch configuration the benchmark times, checked against the FP64
oracle on sampled trials (per-trial tolerance 1e-5 of the trial's gross loss,
hit counts bit-exact) and through properties that hold at any size."""
import math

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
