"""Serving loop on the GPU (ara_server_*): requests submitted together, run in
batched launches on several streams, must give each request exactly the result
it gets when submitted alone (bit for bit: YLT, PML and TVaR), and for a
secondary-uncertainty portfolio the same YLT as ara_run; a pool too small for
the largest request and any other at once still serves every request; a request that can never fit
is refused at submission; a request with an invalid ELT fails alone."""
import copy

import numpy as np
import pytest

from workloads import batched_portfolios, make_yet

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RPS = (2.0, 10.0, 50.0, 100.0)
N_CAT = 20_000
PU_INDEX = 1


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06326_amd import Ara
    yet = make_yet(5000, 120.0, N_CAT, 78)
    pfs = batched_portfolios(n=5, n_catalogue=N_CAT, seed=11, layer_hi=3, elt_hi=5,
                             rows_lo=200, rows_hi=3000)
    pfs[PU_INDEX].su_enabled = False
    a = Ara(0)
    y = a.load_yet(yet)
    yield a, yet, y, pfs
    a.close()


def collect(srv, ids, timeout_s=60.0):
    import time
    want = set(ids)
    got = {}
    t0 = time.time()
    while want - set(got):
        assert time.time() - t0 < timeout_s, "server did not finish"
        for r in srv.poll(64, wait_s=0.5):
            got[r["id"]] = r
    return got


# (portfolio index, trial_begin, trial_count)
REQS = [(0, 0, 5000), (1, 0, 5000), (2, 1000, 3000), (3, 0, 4999), (4, 17, 2500),
        (0, 2500, 2500), (2, 0, 5000), (3, 4000, 1000)]


def serve(yet, pfs, reqs, together, borrow=False, **kw):
    from paper_1501_06326_amd import Server
    with Server(yet, **kw) as srv:
        if together:
            ids = [srv.submit(pfs[k], b, c, RPS, want_ylt=True, borrow=borrow)
                   for k, b, c in reqs]
            got = collect(srv, ids)
        else:
            got = {}
            ids = []
            for k, b, c in reqs:
                i = srv.submit(pfs[k], b, c, RPS, want_ylt=True)
                got.update(collect(srv, [i]))
                ids.append(i)
    return [got[i] for i in ids]


def test_serve_mix_equals_alone(setup):
    a, yet, y, pfs = setup
    say("serve alone")
    alone = serve(yet, pfs, REQS, False, pool_bytes=256 << 20, max_inflight=3, max_batch=4)
    say("serve together")
    mix = serve(yet, pfs, REQS, True, pool_bytes=256 << 20, max_inflight=3, max_batch=4)
    say("serve together, borrowed descriptions")
    lent = serve(yet, pfs, REQS, True, borrow=True, pool_bytes=256 << 20, max_inflight=2,
                 max_batch=3)
    for r0, r1 in zip(alone, lent):
        assert r1["status"] == 0 and np.array_equal(r0["ylt"], r1["ylt"])
    for r0, r1 in zip(alone, mix):
        assert r0["status"] == 0 and r1["status"] == 0
        assert np.array_equal(r0["ylt"], r1["ylt"])
        assert np.array_equal(r0["pml"], r1["pml"]) and np.array_equal(r0["tvar"], r1["tvar"])
        assert r1["latency_s"] >= r1["queue_s"] >= 0.0


def test_serve_matches_ara_run(setup):
    a, yet, y, pfs = setup
    say("serve vs ara_run")
    res = serve(yet, pfs, REQS, True, pool_bytes=256 << 20, max_inflight=2, max_batch=3)
    for (k, b, c), r in zip(REQS, res):
        d = a.load_portfolio(pfs[k], N_CAT)
        ref = a.run(y, d, trial_begin=b, trial_count=c)["ylt_pf"]
        a.free_portfolio(d)
        got = torch.from_numpy(r["ylt"]).to(ref.device)
        assert torch.equal(got, ref)
        pml, tvar = a.pml_tvar(ref, RPS)
        assert np.array_equal(np.asarray(pml), r["pml"])
        assert np.allclose(np.asarray(tvar), r["tvar"], rtol=1e-12, atol=0.0)


def up(n):
    return (n + 255) // 256 * 256


def footprint(a, pf, count):
    """An upper bound of a request's pool region."""
    from paper_1501_06326_amd.ara import ara_pml_tvar_scratch_size
    return (up(a.workspace_size(pf, N_CAT)) + up(4 * len(pf.layers) * count) + up(4 * count)
            + up(ara_pml_tvar_scratch_size(count)))


def slot_scratch(slots, batch, n_trials):
    from paper_1501_06326_amd.ara import ara_batch_scratch_size
    return slots * up(ara_batch_scratch_size(batch, (n_trials + batch - 1) // batch))


def test_serve_small_pool_serialises(setup):
    a, yet, y, pfs = setup
    say("serve small pool")
    big = max(footprint(a, pfs[k], c) for k, b, c in REQS[:5])
    small = min(footprint(a, pfs[k], c) for k, b, c in REQS[:5])
    # room for the slots' scratch and the largest request, which then has the
    # pool to itself: admission must hold the others back meanwhile
    pool = slot_scratch(3, 4, 5000) + big + small // 2
    alone = serve(yet, pfs, REQS[:5], False, pool_bytes=256 << 20, max_inflight=3, max_batch=4)
    tight = serve(yet, pfs, REQS[:5], True, pool_bytes=pool, max_inflight=3, max_batch=4)
    for r0, r1 in zip(alone, tight):
        assert r1["status"] == 0
        assert np.array_equal(r0["ylt"], r1["ylt"])
        assert np.array_equal(r0["pml"], r1["pml"])


def test_serve_refuses_request_that_never_fits(setup):
    a, yet, y, pfs = setup
    say("serve refuse")
    from paper_1501_06326_amd import Server
    from paper_1501_06326_amd.ara import ARA_E_WORKSPACE_TOO_SMALL, AraError
    pool = slot_scratch(1, 1, 5000) + footprint(a, pfs[0], 5000) // 2
    with Server(yet, pool_bytes=pool, max_inflight=1, max_batch=1) as srv:
        with pytest.raises(AraError) as e:
            srv.submit(pfs[0], 0, 5000, RPS)
        assert e.value.code == ARA_E_WORKSPACE_TOO_SMALL
        with pytest.raises(AraError):
            srv.submit(pfs[0], 4000, 2000, RPS)          # past the last trial


def test_serve_bad_request_fails_alone(setup):
    a, yet, y, pfs = setup
    say("serve bad request")
    from paper_1501_06326_amd.ara import ARA_E_EVENT_ID_RANGE
    bad = copy.deepcopy(pfs[2])
    ev = np.array(bad.layers[0].elts[0].event_ids, dtype=np.int32, copy=True)
    ev[len(ev) // 2] = N_CAT + 5                          # outside the catalogue
    bad.layers[0].elts[0].event_ids = ev
    mixed = list(pfs) + [bad]
    reqs = [(0, 0, 5000), (5, 0, 5000), (3, 0, 4999), (5, 100, 200), (4, 17, 2500)]
    res = serve(yet, mixed, reqs, True, pool_bytes=256 << 20, max_inflight=2, max_batch=8)
    alone = serve(yet, mixed, [q for q in reqs if q[0] != 5], False, pool_bytes=256 << 20,
                  max_inflight=1, max_batch=1)
    good = [r for q, r in zip(reqs, res) if q[0] != 5]
    for r in (res[1], res[3]):
        assert r["status"] == ARA_E_EVENT_ID_RANGE
    for r0, r1 in zip(alone, good):
        assert r1["status"] == 0
        assert np.array_equal(r0["ylt"], r1["ylt"])
