"""Writes ``oracle_small.json``: the FP64 oracle's results on the small
workload (10,000 trials x Poisson(100) over a 10,000-event catalogue, one
layer of 3 ELTs x 2,000 rows), with independent and with correlated secondary
uncertainty.  It calls only the oracle and the seeded input generators.

    python tests/golden/make_oracle_small.py
"""
import json
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from workloads import config_small  # noqa: E402

OUT = Path(__file__).resolve().parent / "oracle_small.json"


def summary(corr):
    w = config_small(corr=corr)
    r = oracle.run_ara(w.yet, w.portfolio)
    pml, tvar = oracle.pml_tvar(r["ylt_pf"], w.return_periods)
    return {
        "workload": w.name,
        "return_periods": list(w.return_periods),
        "pml": [float(v) for v in pml],
        "tvar": [float(v) for v in tvar],
        "hits": int(r["hits"].sum()),
        "ylt_sum": float(r["ylt_pf"].sum()),
        "ylt_head": [float(v) for v in r["ylt_pf"][:16]],
        "positive_trials": int((r["ylt_pf"] > 0).sum()),
    }


def main():
    doc = {"source": "written by tests/golden/make_oracle_small.py from the FP64 oracle "
                      "on seeded synthetic inputs",
           "cases": [summary(False), summary(True)]}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
