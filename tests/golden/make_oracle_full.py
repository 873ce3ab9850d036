"""Writes ``oracle_full.json``: the FP64 oracle's results on the full-shape
workload (1,000,000 trials x Poisson(1000) over a 100,000-event catalogue, one
layer of 16 ELTs x 20,000 rows), with and without secondary uncertainty.

For each case it stores what the Year Loss Table and its metrics (section 2.3)
fix at this size: PML and TVaR at return periods 100 and 250 of the portfolio
YLT, the YLT's exact sum and its count of positive trials, the totals of the
non-zero lookup counts and of the lookup checksums over every trial, and per
trial (index, loss Y, gross loss G = sum of the event losses before the
occurrence and aggregate terms) for the 10,000 trials with the largest losses
(the ones that decide PML and TVaR at these return periods) and for 2,000
trials drawn uniformly.  It calls only the oracle and the seeded input
generators.  With secondary uncertainty on it runs about 25 minutes on 8 host
cores.

    python tests/golden/make_oracle_full.py [--threads N] [--case su|pu|both]
"""
import argparse
import json
import math
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from workloads import config_full, full_portfolio  # noqa: E402

OUT = Path(__file__).resolve().parent / "oracle_full.json"
N_TRIALS = 1_000_000
N_TOP = 10_000
N_SAMPLE = 2_000
SAMPLE_SEED = 17


def top_trials(y: np.ndarray, n: int) -> np.ndarray:
    """Indices of the n largest losses, largest first (ties: lower index first)."""
    order = np.lexsort((np.arange(y.size), -y))
    return order[:n]


def case(w, pf, threads):
    t0 = time.time()
    r = oracle.run_ara(w.yet, pf, threads=threads)
    dt = time.time() - t0
    y = r["ylt_pf"]
    g = r["gross"][0]
    pml, tvar = oracle.pml_tvar(y, w.return_periods)
    top = top_trials(y, N_TOP)
    rng = np.random.default_rng(SAMPLE_SEED)
    samp = np.sort(rng.choice(y.size, size=N_SAMPLE, replace=False))
    chk = int(np.sum(r["hit_chk"][0], dtype=np.uint64))   # wraps modulo 2^64
    print(f"{'su' if pf.su_enabled else 'pu'}: oracle {dt:.0f} s, PML {pml} TVaR {tvar}",
          flush=True)
    return {
        "secondary_uncertainty": bool(pf.su_enabled),
        "return_periods": list(w.return_periods),
        "pml": [float(v) for v in pml],
        "tvar": [float(v) for v in tvar],
        "ylt_sum": math.fsum(y.tolist()),
        "positive_trials": int((y > 0).sum()),
        "hits_total": int(r["hits"].sum()),
        "hit_chk_total": chk,
        "top_index": [int(v) for v in top],
        "top_y": [float(v) for v in y[top]],
        "top_gross": [float("%.10g" % v) for v in g[top]],
        "sample_index": [int(v) for v in samp],
        "sample_y": [float(v) for v in y[samp]],
        "sample_gross": [float("%.10g" % v) for v in g[samp]],
        "oracle_seconds": round(dt, 1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--case", choices=["su", "pu", "both"], default="both")
    a = ap.parse_args()
    w = config_full(n_trials=N_TRIALS, with_times=False)
    print(f"generated {w.name}: {w.yet.n_occ} occurrences", flush=True)
    doc = {}
    if OUT.exists():
        doc = json.loads(OUT.read_text())
    doc["source"] = ("written by tests/golden/make_oracle_full.py from the FP64 oracle on "
                     "seeded synthetic inputs")
    doc["workload"] = w.name
    doc["n_trials"] = w.yet.n_trials
    doc["n_occurrences"] = w.yet.n_occ
    doc["event_id_sum"] = int(w.yet.event_ids.sum(dtype=np.int64))
    cases = doc.setdefault("cases", {})
    if a.case in ("pu", "both"):
        cases["pu"] = case(w, full_portfolio(su=False), a.threads)
    if a.case in ("su", "both"):
        cases["su"] = case(w, w.portfolio, a.threads)
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
