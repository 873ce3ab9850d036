"""GPU parity of the method's other readings and regimes against the oracle:

  * the keying of section 3.1's inputs (z_(Prog,E) per occurrence and
    program, z_(E) per event), with and without the correlated part, alone
    and in a batch;
  * rows whose fit hits the sigma cap of section 3.3 (near-Bernoulli shapes,
    the FP64 quantile path);
  * the large-catalogue case of the paper's direct-access example (16 ELTs of
    20,000 rows over 1,000,000 events), secondary and primary uncertainty.

Tolerances as for the headline path: hit counts and checksums bit-exact,
per-trial |Y_gpu - Y_orc| <= 1e-5 G + 1e-3."""
import copy

import numpy as np
import pytest

import oracle
from workloads import config_full, config_small, sigma_capped, varied_shapes

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


def parity(ara, yet, pf, diagnostics=True):
    ref = oracle.run_ara(yet, pf)
    y = ara.load_yet(yet)
    p = ara.load_portfolio(pf, yet.n_catalogue)
    r = ara.run(y, p, diagnostics=diagnostics and pf.su_enabled)
    g = r["ylt"].double().cpu().numpy()
    err = np.abs(g - ref["ylt"])
    assert np.all(err <= 1e-5 * ref["gross"] + 1e-3), float((err / np.maximum(ref["gross"], 1)).max())
    if diagnostics and pf.su_enabled:
        assert np.array_equal(r["hits"].cpu().numpy(), ref["hits"])
        assert np.array_equal(r["hit_chk"].cpu().numpy().astype(np.uint64), ref["hit_chk"])
    ara.free_portfolio(p)
    ara.free_yet(y)
    return r, ref


def two_programs(pf):
    """The small portfolio's ELTs split over two layers of two programs."""
    out = copy.deepcopy(pf)
    layer = out.layers[0]
    second = copy.deepcopy(layer)
    layer.elts, second.elts = layer.elts[:2], layer.elts[2:]
    layer.program_id, second.program_id = 3, 4
    out.layers.append(second)
    out.keying = 1
    return out


@pytest.mark.parametrize("corr", [False, True])
def test_paper_keying_parity(ara, corr):
    w = config_small(corr=corr, n_trials=3000)
    say("paper keying", corr)
    r, ref = parity(ara, w.yet, two_programs(w.portfolio))
    # the keying changes the draws: the YLT differs from the default keying's
    r0 = oracle.run_ara(w.yet, w.portfolio)
    assert not np.allclose(ref["ylt_pf"], r0["ylt_pf"])


def test_paper_keying_in_a_batch(ara):
    w = config_small(n_trials=2000)
    say("paper keying batch")
    pfs = [w.portfolio, two_programs(w.portfolio)]
    y = ara.load_yet(w.yet)
    dps = [ara.load_portfolio(pf, w.yet.n_catalogue) for pf in pfs]
    alone = [ara.run(y, d) for d in dps]
    for cfg in [None, (2, 16, 1)]:
        outs = ara.run_batch(y, dps, cfg=cfg)
        for o, a in zip(outs, alone):
            assert torch.equal(o["ylt"], a["ylt"])
    for d in dps:
        ara.free_portfolio(d)
    ara.free_yet(y)


@pytest.mark.parametrize("corr", [False, True])
def test_sigma_capped_rows(ara, corr):
    """Rows above the sigma cap take the FP64 quantile in the second pass
    (without mixed rows its 4-wavefront form, the diagnostic pass its
    1-wavefront form): parity with the oracle, and the fast pass gives the
    diagnostic pass's YLT bit for bit."""
    w = config_small(corr=corr, n_trials=2000)
    say("sigma capped rows", corr)
    pf = sigma_capped(w.portfolio)
    r, ref = parity(ara, w.yet, pf)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(pf, w.yet.n_catalogue)
    assert torch.equal(ara.run(y, p)["ylt"], r["ylt"])
    ara.free_portfolio(p)
    ara.free_yet(y)


@pytest.mark.parametrize("corr", [False, True])
def test_varied_shapes(ara, corr):
    """Every row its own shape: parity with the oracle, and the diagnostic
    pass (which also draws the rows that cannot pay, so its batches mix other
    draws) gives the fast pass's YLT bit for bit, as does a batch."""
    w = config_small(corr=corr, n_trials=3000)
    pf = varied_shapes(w.portfolio)
    say("varied shapes", corr)
    r, ref = parity(ara, w.yet, pf)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(pf, w.yet.n_catalogue)
    fast = ara.run(y, p)
    assert torch.equal(fast["ylt"], r["ylt"])
    p0 = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    outs = ara.run_batch(y, [p0, p])
    assert torch.equal(outs[1]["ylt"], fast["ylt"])
    for d in (p, p0):
        ara.free_portfolio(d)
    ara.free_yet(y)


@pytest.mark.parametrize("su", [True, False])
def test_large_catalogue(ara, su):
    w = config_full(n_trials=400, with_times=False, su=su, n_catalogue=1_000_000)
    say("large catalogue", su, w.yet.n_occ)
    parity(ara, w.yet, w.portfolio)
