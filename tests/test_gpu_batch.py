"""Batched portfolios on the GPU: one persistent launch must reproduce, bit for
bit, each secondary-uncertainty portfolio run alone (the draws are keyed by
absolute trial, occurrence and elt_id, and a trial's arithmetic does not
depend on its neighbours); a primary-uncertainty portfolio in a batch runs
ara_run's per-event table pass after the launch, so it too equals ara_run bit
for bit.  Graph replays must reproduce the eager batch on every replay."""
import numpy as np
import pytest

import oracle
from workloads import batched_portfolios, make_yet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06326_amd import Ara
    yet = make_yet(6000, 120.0, 20_000, 77)
    pfs = batched_portfolios(n=7, n_catalogue=20_000, seed=9, layer_hi=4, elt_hi=6,
                             rows_lo=200, rows_hi=4000)
    pfs[PU_INDEX].su_enabled = False        # a primary-uncertainty portfolio in the mix
    a = Ara(0)
    y = a.load_yet(yet)
    dps = [a.load_portfolio(pf, yet.n_catalogue) for pf in pfs]
    alone = [a.run(y, d) for d in dps]
    yield a, yet, y, pfs, dps, alone
    a.close()


PU_INDEX = 2


def same(outs, alone):
    for k, (o, r) in enumerate(zip(outs, alone)):
        assert torch.equal(o["ylt"], r["ylt"])
        assert torch.equal(o["ylt_pf"], r["ylt_pf"])


def test_batch_equals_alone(setup):
    a, yet, y, pfs, dps, alone = setup
    say("batch vs alone, portfolios", len(dps))
    for cfg in [None, (1, 0, 0), (3, 0, 1), (1, 8, 0), (8, 20, 0), (3, 4, 0), (1, 8, 1),
                (4, 16, 1), (3, 4, 1)]:
        outs = a.run_batch(y, dps, cfg=cfg)
        same(outs, alone)


def test_batch_one_portfolio_vs_oracle(setup):
    a, yet, y, pfs, dps, alone = setup
    say("batch vs oracle")
    outs = a.run_batch(y, dps)
    for k in (0, PU_INDEX):
        ref = oracle.run_ara(yet, pfs[k])
        err = np.abs(outs[k]["ylt"].double().cpu().numpy() - ref["ylt"])
        assert np.all(err <= 1e-5 * ref["gross"] + 1e-3)


def test_batch_trial_subrange(setup):
    a, yet, y, pfs, dps, alone = setup
    say("batch subrange")
    for cfg in (None, (2, 16, 0), (2, 16, 1), (2, 0, 0), (1, 0, 1)):
        outs = a.run_batch(y, dps, trial_begin=1000, trial_count=2500, cfg=cfg)
        for k, (o, r) in enumerate(zip(outs, alone)):
            assert torch.equal(o["ylt"], r["ylt"][:, 1000:3500])


def test_batch_graph_replays(setup):
    a, yet, y, pfs, dps, alone = setup
    say("batch graph")
    g, outs, sc = a.batch_graph(y, dps, cfg=(2, 12))
    for rep in range(3):
        for o in outs:
            o["ylt"].fill_(-1.0)
            o["ylt_pf"].fill_(-1.0)
        a.graph_launch(g)
        torch.cuda.synchronize()
        same(outs, alone)
        a.run(y, dps[0])                        # eager work between replays
        torch.cuda.synchronize()
    a.graph_destroy(g)


def test_batch_autotune(setup):
    a, yet, y, pfs, dps, alone = setup
    say("autotune")
    cfg, ms = a.batch_autotune(y, dps, trial_count=2000)
    assert cfg[0] in (1, 2, 4) and cfg[1] in (0, 16, 20) and cfg[2] in (0, 1) and ms > 0
    same(a.run_batch(y, dps, cfg=cfg), alone)
