"""Small hand-made inputs shared by the oracle pins and the GPU parity tests."""
import json
from pathlib import Path

import numpy as np

from workloads import ELT, INF, YET, Layer, Portfolio


def yet_from_lists(trials, n_catalogue, times=True):
    counts = [len(t) for t in trials]
    off = np.zeros(len(trials) + 1, np.int64)
    off[1:] = np.cumsum(counts)
    ids = np.asarray([e for t in trials for e in t], np.int32)
    tm = None
    if times:
        tm = np.concatenate([np.linspace(1.0, 300.0, max(c, 1))[:c] for c in counts]
                            ).astype(np.float32) if sum(counts) else np.zeros(0, np.float32)
    return YET(offsets=off, event_ids=ids, times=tm, n_catalogue=n_catalogue)


def elt_from_dict(elt_id, rows, retention=0.0, limit=INF, share=1.0, sigma=None, max_loss=None,
                  sigma_c=None):
    """rows: {event: mean}.  sigma / max_loss: {event: value} (default 0 / 4*mean)."""
    ev = np.asarray(sorted(rows), np.int32)
    mean = np.asarray([rows[e] for e in ev], np.float32)
    si = np.asarray([(sigma or {}).get(int(e), 0.0) for e in ev], np.float32)
    sc = np.asarray([(sigma_c or {}).get(int(e), 0.0) for e in ev], np.float32)
    mx = np.asarray([(max_loss or {}).get(int(e), 4.0 * rows[e]) for e in ev], np.float32)
    return ELT(elt_id=elt_id, event_ids=ev, mean=mean, sigma_i=si, sigma_c=sc, max_loss=mx,
               retention=retention, limit=limit, share=share)


# The hand-worked example: events A = 0, B = 1 in a 4-event catalogue.
A, B = 0, 1


def worked_example(agg_limit=1e8, share1=1.0, trials=None):
    """ELT1 = {A: 3.0e6, B: 5.0e5}, ELT2 = {A: 1.0e6}; ELT terms (1e5, 5e6, s);
    occurrence terms (1e6, 2e7); aggregate terms (5e6, AggL); trial [A, B, A]."""
    elt1 = elt_from_dict(0, {A: 3.0e6, B: 5.0e5}, 1e5, 5e6, share1)
    elt2 = elt_from_dict(1, {A: 1.0e6}, 1e5, 5e6, 1.0)
    layer = Layer(elts=[elt1, elt2], occ_retention=1e6, occ_limit=2e7,
                  agg_retention=5e6, agg_limit=agg_limit)
    pf = Portfolio(layers=[layer], seed=1, su_enabled=False)
    yet = yet_from_lists(trials if trials is not None else [[A, B, A]], 4)
    return yet, pf


def random_tiny_case(rng, n_cat=12, n_layers=2, max_elts=3, max_occ=8, n_trials=20,
                     dyadic=True, su=False, corr=False):
    """Tiny random portfolio.  With ``dyadic`` every number is a small dyadic
    rational so FP64 arithmetic on it is exact."""
    trials = [list(rng.integers(0, n_cat, size=int(rng.integers(0, max_occ + 1))))
              for _ in range(n_trials)]
    yet = yet_from_lists(trials, n_cat)
    layers = []
    eid = 0
    for _ in range(n_layers):
        elts = []
        for _ in range(int(rng.integers(1, max_elts + 1))):
            n_rows = int(rng.integers(0, n_cat + 1))
            evs = rng.choice(n_cat, size=n_rows, replace=False)
            if dyadic:
                rows = {int(e): float(rng.integers(1, 64)) * 1024.0 for e in evs}
                ret = float(rng.integers(0, 20)) * 1024.0
                lim = INF if rng.random() < 0.3 else float(rng.integers(1, 64)) * 1024.0
                share = float(rng.choice([0.25, 0.5, 0.75, 1.0]))
            else:
                rows = {int(e): float(np.float32(np.exp(rng.normal(12, 1.5)))) for e in evs}
                ret = float(np.float32(rng.uniform(0, 2e5)))
                lim = INF if rng.random() < 0.3 else float(np.float32(rng.uniform(1e5, 5e6)))
                share = float(np.float32(rng.uniform(0.1, 1.0)))
            # secondary-uncertainty parameters vary per row so that rows fit
            # different Beta shapes (std 5%-90% of the mean, exposure 1.5-10x)
            frac = {e: float(np.float32(rng.uniform(0.05, 0.9))) for e in rows}
            sig = {e: float(np.float32(frac[e] * m)) for e, m in rows.items()}
            mxl = {e: float(np.float32(rng.uniform(1.5, 10.0) * m)) for e, m in rows.items()}
            sigc = None
            if corr:
                sig = {e: float(np.float32(0.5 * v)) for e, v in sig.items()}
                sigc = {e: float(np.float32(rng.uniform(0.0, 1.0) * v)) for e, v in sig.items()}
            elts.append(elt_from_dict(eid, rows, ret, lim, share, sigma=sig, sigma_c=sigc,
                                      max_loss=mxl))
            eid += 1
        if dyadic:
            t = [float(rng.integers(0, 40)) * 1024.0, float(rng.integers(1, 200)) * 1024.0,
                 float(rng.integers(0, 100)) * 1024.0, float(rng.integers(1, 400)) * 1024.0]
        else:
            t = [float(np.float32(v)) for v in (rng.uniform(0, 1e6), rng.uniform(1e6, 2e7),
                                                 rng.uniform(0, 5e6), rng.uniform(1e6, 1e8))]
        if rng.random() < 0.25:
            t[1] = INF
        if rng.random() < 0.25:
            t[3] = INF
        layers.append(Layer(elts=elts, occ_retention=t[0], occ_limit=t[1],
                            agg_retention=t[2], agg_limit=t[3]))
    return yet, Portfolio(layers=layers, seed=int(rng.integers(0, 2**63)), su_enabled=su)


GOLDEN = Path(__file__).resolve().parent / "golden"


def golden_worked_cases():
    """The hand-worked fixture ``golden/worked_example.json``: yields (name,
    yet, portfolio, expected) with expected holding ylt, gross, hits and the
    flattened occurrence view of the single layer."""
    with open(GOLDEN / "worked_example.json") as f:
        g = json.load(f)
    ev = g["events"]
    lay = g["layer"]
    for case in g["cases"]:
        elts = []
        for j, d in enumerate(g["elts"]):
            share = case.get("share0", d["share"]) if j == 0 else d["share"]
            elts.append(elt_from_dict(d["elt_id"], {ev[k]: v for k, v in d["rows"].items()},
                                      d["retention"], d["limit"], share))
        layer = Layer(elts=elts, occ_retention=lay["occ_retention"], occ_limit=lay["occ_limit"],
                      agg_retention=lay["agg_retention"],
                      agg_limit=case.get("agg_limit", lay["agg_limit"]))
        pf = Portfolio(layers=[layer], seed=1, su_enabled=False)
        yet = yet_from_lists([[ev[k] for k in t] for t in case["trials"]], g["catalogue"])
        expect = {"ylt": case["ylt"], "gross": case["gross"], "hits": case["hits"],
                  "occ_view": [d for t in case["occurrence_view"] for d in t]}
        yield case["name"], yet, pf, expect
