"""Benchmark: Aggregate Risk Analysis on one MI355X.

One step = one pass of the whole path over the full-shape workload
(1,000,000 trials x Poisson(1000) occurrences over a 100,000-event catalogue,
one layer of 16 ELTs x 20,000 rows, secondary uncertainty on): ara_run (YET
lookup, Philox draw, Beta quantile, ELT / occurrence / aggregate terms, YLT)
followed by ara_pml_tvar (PML and TVaR at 1-in-100 and 1-in-250).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

Metric: trial x event x ELT evaluations per second (every ELT lookup of every
occurrence counts, zero losses included).  Also reported: the primary-
uncertainty variant of the same workload against the HBM roofline, the
dominant kernel against its roofline, and the FP64 oracle timed on a bounded
sample of trials on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# VALU issue peak in 32-bit lane operations: the FP32 vector peak of
# 157.3 TFLOP/s counts an FMA as two flops, i.e. 256 CUs x 128 lanes x 2.4 GHz
# = 78.6e12 lane operations per second.
PEAK_VALU_TOPS = 157.3 / 2.0
# VALU lane operations per secondary-uncertainty draw of the main kernel at the
# full-shape workload: SQ_INSTS_VALU x 64 / draws from rocprofv3 (profiles/).
VALU_OPS_PER_DRAW = float(os.environ.get("ARA_VALU_OPS_PER_DRAW", "659"))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--trials", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sum-mode", default="naive32")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a known-size kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by trial range, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_06326_amd import Ara, evaluations
    from workloads import config_full, full_portfolio

    t0 = time.time()
    w = config_full(n_trials=args.trials)
    yet, pf = w.yet, w.portfolio
    log(f"generated {w.name}: {yet.n_occ} occurrences in {time.time() - t0:.1f}s")
    evals = evaluations(yet, pf)
    rps = list(w.return_periods)

    ara = Ara(0)
    dev = ara.device
    off = torch.from_numpy(yet.offsets).to(dev)
    ev = torch.from_numpy(yet.event_ids).to(dev)
    tm = torch.from_numpy(yet.times).to(dev) if yet.times is not None else None
    y = ara.load_yet(yet, device_arrays=(off, ev, tm))
    p = ara.load_portfolio(pf, yet.n_catalogue)
    n = yet.n_trials
    out_l = torch.empty((1, n), dtype=torch.float32, device=dev)
    out_p = torch.empty(n, dtype=torch.float32, device=dev)
    scratch = torch.empty(ara.run_scratch_size(n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    log("loaded YET and portfolio")
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(portfolio):
        ara.run(y, portfolio, sum_mode=args.sum_mode, out_layers=out_l, out_pf=out_p,
                scratch=scratch, sync=False)
        return ara.pml_tvar(out_p, rps)

    # warmup, also the numeric-status check
    for _ in range(max(1, args.warmup)):
        step(p)
    ara.run(y, p, out_layers=out_l, out_pf=out_p, scratch=scratch, sync=True)
    torch.cuda.synchronize()

    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev0[k].record(stream)
        ara.run(y, p, sum_mode=args.sum_mode, out_layers=out_l, out_pf=out_p, scratch=scratch,
                sync=False)
        ev1[k].record(stream)
        pml, tvar = ara.pml_tvar(out_p, rps)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = 1e3 * t_total / args.steps
    run_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))
    log(f"SU: {ms_step:.3f} ms/step, ara_run {run_ms:.3f} ms; PML {pml} TVaR {tvar}")

    # draws of the run (non-zero lookups): the unit of the SU kernel's work
    hits = ara.run(y, p, diagnostics=True, out_pf=out_p)["hits"].sum().item()
    result = {
        "metric": "trial*event*ELT evaluations/s (1M-trial YET, secondary uncertainty)",
        "value": evals / (ms_step / 1e3),
        "unit": "evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 in the quantile tail band and the TVaR sum)",
        "data": "synthetic (seeded numpy generator; lognormal ELT means)",
        "config": {"workload": w.name, "trials": n, "occurrences": yet.n_occ,
                   "catalogue": yet.n_catalogue, "layers": 1, "elts": 16,
                   "rows_per_elt": 20000, "secondary_uncertainty": True,
                   "sum_mode": args.sum_mode, "return_periods": rps,
                   "evaluations_per_step": evals, "draws_per_step": int(hits)},
        "pml": [float(v) for v in pml],
        "tvar": [float(v) for v in tvar],
    }
    ops = VALU_OPS_PER_DRAW * hits
    result["roofline"] = {
        "kernel": "k_ara_su (+ k_ara_su_redo), ara_run",
        "bound": "alu",
        "achieved": (ops / (run_ms / 1e3) / 1e12) if ops else None,
        "peak": PEAK_VALU_TOPS,
        "unit": "TOP/s",
        "frac": (ops / (run_ms / 1e3) / 1e12 / PEAK_VALU_TOPS) if ops else None,
        "traffic": None,
        "launch_ms": run_ms,
        "draws_per_s": hits / (run_ms / 1e3),
        "valu_ops_per_draw": VALU_OPS_PER_DRAW or None,
    }

    if not args.no_pu:
        pf_pu = full_portfolio(su=False)
        p_pu = ara.load_portfolio(pf_pu, yet.n_catalogue)
        for _ in range(3):
            ara.run(y, p_pu, out_layers=out_l, out_pf=out_p, sync=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            ara.run(y, p_pu, out_layers=out_l, out_pf=out_p, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        pu_ms = e0.elapsed_time(e1) / reps
        # algorithmic HBM bytes of one run: event ids + trial offsets + the
        # per-event occurrence-loss table + the two YLT outputs
        byts = 4 * yet.n_occ + 8 * (n + 1) + 4 * yet.n_catalogue + 2 * 4 * n
        gbs = byts / (pu_ms / 1e3) / 1e9
        result["pu_path"] = {
            "ms_per_run": pu_ms, "evaluations_per_s": evals / (pu_ms / 1e3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "traffic": None, "bytes": byts},
        }
        log(f"PU: {pu_ms:.3f} ms/run, {gbs:.0f} GB/s")

    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        # calibrate on a few trials, then a sample sized to ~cpu_seconds
        tc = time.perf_counter()
        oracle.run_ara(yet, pf, 0, 64, threads=cores)
        dt = time.perf_counter() - tc
        m = int(max(64, min(n, 64 * args.cpu_seconds / max(dt, 1e-3))))
        tc = time.perf_counter()
        oracle.run_ara(yet, pf, 0, m, threads=cores)
        dt = time.perf_counter() - tc
        ev_s = evaluations(yet, pf, 0, m)
        result["cpu_baseline"] = {"value": ev_s / dt, "unit": "evaluations/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"trials [0, {m}) of the same workload, "
                                            f"{ev_s} evaluations in {dt:.1f} s"}
        log(f"oracle: {ev_s / dt:.3g} evals/s on {cores} threads ({m} trials)")

    print(json.dumps(result), flush=True)
    ara.close()


if __name__ == "__main__":
    main()
