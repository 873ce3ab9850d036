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

Two further modes print their own JSON line:
  --mode batched  64 portfolios (1-16 layers, 2-48 ELTs per layer, 1,000-50,000
                  rows per ELT) on the same YET: one persistent batched launch
                  against 64 sequential ara_run calls.
  --mode precision  8 layers (4-32 ELTs each, per-layer terms log-uniform on
                  [1e5, 1e9]) on the same YET in the three sum modes: time per
                  mode, and per-trial / PML / TVaR errors against the oracle on
                  a sample of trials.
  --mode served   the serving loop under Poisson arrivals of requests (1-8
                  layers, 2-32 ELTs per layer, trial ranges of 1e4-1e6 trials):
                  p50 / p99 latency and throughput at several offered loads,
                  against a one-at-a-time server with the measured service times.
  --mode probes   the measurement probes behind the roofline figures: the VALU
                  issue rate of single instruction kinds, the streaming read
                  bandwidth, and the per-draw arithmetic alone (Philox and the
                  FP32 Beta quantile at the full-shape row shape).
  --mode variants the full-shape YET with the secondary-uncertainty laws that
                  use the FP64-capable second pass: sigma_I = sigma_C = mean/4
                  (section 3.2's two-normal mix), rows of varied Beta shapes
                  (sigma_I / mean 0.15-0.9, max / mean 1.5-10) and 30 % of rows
                  above the sigma cap (section 3.3); time per run and evaluations/s
                  beside the headline law.
  --mode views    the outputs either side of the YLT on the full shape: ara_run
                  with the per-occurrence view (secondary uncertainty on and
                  off; 1e9 FP32 increments written) and ara_ep_curve on the
                  1,000,000-entry YLT.
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
# VALU lane-operation peak of the non-packed instructions the kernels are
# built with: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane
# operations per second (an FMA is one operation).  The FP32 vector figure of
# 157.3 TFLOP/s counts an FMA as two flops and a packed instruction as two
# lanes: 157.3 / 4 = 39.3.  Dependent chains of v_fma_f32, v_mul_f32,
# v_mul_hi_u32, v_mad_u64_u32 or v_xor/v_add reach 0.96 of it at the clock the
# part holds under load (bench.py --mode probes).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Counter figures of the current kernel sources (rocprofv3, one MI355X),
# reported only while the sources hash to the value they were taken with and
# null otherwise.
#  * draw_arith_ops: arithmetic lane operations per draw of the method's own
#    per-draw work -- Philox4x32-10 and the FP32 Beta quantile at the
#    full-shape row shape, run alone by k_probe_draws with the shape table --
#    counted as SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32 + _INT32 + _INT64 per
#    wavefront of 64 draws (moves, selects, compares and lane operations are
#    not the method's arithmetic and are left out).
#  * su_main_bytes / pu_bytes: HBM-side traffic of one launch at 1,000,000
#    trials, FETCH_SIZE and WRITE_SIZE each scaled by what the counter reads
#    for an elementwise kernel that reads and writes 1 GiB (FETCH 2.0,
#    WRITE 1.0).
PROFILED = {
    "sources_sha256": "5b33c6d22be38d8a2aa2655bdb6200c3fe8cce3fdbcded3ac6b52e3e3ef18298",
    "draw_arith_ops": 207.0,        # profiles/ara_su_full_counters.md (k_probe_draws)
    "su_main_bytes": 4.4169e9 + 1.2172e8,    # k_ara_su: fetch + write, 1M trials
    "pu_bytes": 4.0934e9 + 9.714e6,          # k_ara_pu: fetch + write, 1M trials
}


def kernel_sources_sha256():
    """Hash of the kernel sources with comments and blank space removed, so
    documentation edits keep the profiled figures while code edits drop them."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1501_06326_amd", "csrc")
    for f in ("ara_kernels.hip", "ara_math.h", "ara_internal.h", "ara_kernels.h",
              "ara_probe.hip"):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def profiled(key):
    if kernel_sources_sha256() != PROFILED["sources_sha256"]:
        return None
    return PROFILED[key]


def live_draws(yet, pf):
    """Non-zero lookups whose row can pay: the draws the SU kernel performs."""
    n_cat = yet.n_catalogue
    live = np.zeros(n_cat, np.int64)
    for layer in pf.layers:
        for e in layer.elts:
            det = (np.asarray(e.sigma_i, np.float64) + np.asarray(e.sigma_c, np.float64)) == 0.0
            scale = np.where(det, np.asarray(e.mean, np.float32), np.asarray(e.max_loss, np.float32))
            ok = (scale > np.float32(e.retention)) & (np.float32(e.limit) != 0) & \
                 (np.float32(e.share) != 0)
            np.add.at(live, np.asarray(e.event_ids)[ok], 1)
    occ = np.bincount(yet.event_ids, minlength=n_cat)
    return int((occ.astype(np.int64) * live).sum())


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--trials", type=int, default=1_000_000)
    ap.add_argument("--catalogue", type=int, default=100_000,
                    help="events in the catalogue (1,000,000: the large-catalogue variant)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sum-mode", default="kahan32")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise kernel that reads and writes 1 GiB (a "
                         "known-size kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--mode", choices=["step", "batched", "served", "precision", "views",
                                       "probes", "variants", "footprint"], default="step")
    ap.add_argument("--oracle-trials", type=int, default=3000, help="precision mode")
    ap.add_argument("--portfolios", type=int, default=64, help="batched mode")
    ap.add_argument("--graph", action="store_true", help="batched mode: also time a graph replay")
    ap.add_argument("--pu", action="store_true",
                    help="batched mode: the portfolios without secondary uncertainty")
    ap.add_argument("--requests", type=int, default=2000, help="served mode: requests per load")
    ap.add_argument("--loads", default="0.5,0.8,0.95,1.5",
                    help="served mode: offered loads as fractions of one-at-a-time capacity")
    ap.add_argument("--max-inflight", type=int, default=2, help="served mode: streams")
    ap.add_argument("--max-batch", type=int, default=4, help="served mode: requests per launch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by trial range, see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "served":
        return bench_served(args)
    if args.mode == "precision":
        return bench_precision(args)
    if args.mode == "views":
        return bench_views(args)
    if args.mode == "probes":
        return bench_probes(args)
    if args.mode == "variants":
        return bench_variants(args)
    if args.mode == "footprint":
        return bench_footprint(args)

    import torch
    from paper_1501_06326_amd import Ara, evaluations
    from workloads import config_full, full_portfolio

    t0 = time.time()
    w = config_full(n_trials=args.trials, n_catalogue=args.catalogue)
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
        # an elementwise kernel that reads 1 GiB and writes 1 GiB (a device copy
        # would go to a DMA engine, which the counters do not see)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
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

    # non-zero lookups of the run, and the draws performed (the SU kernel's unit of work)
    hits = ara.run(y, p, diagnostics=True, out_pf=out_p)["hits"].sum().item()
    draws = live_draws(yet, pf)
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
        "dtype": "f32 (FP64 for the TVaR sum and the quantile of shapes outside the FP32 domain)",
        "data": "synthetic (seeded numpy generator; lognormal ELT means)",
        "config": {"workload": w.name, "trials": n, "occurrences": yet.n_occ,
                   "catalogue": yet.n_catalogue, "layers": 1, "elts": 16,
                   "rows_per_elt": 20000, "secondary_uncertainty": True,
                   "sum_mode": args.sum_mode, "return_periods": rps,
                   "evaluations_per_step": evals, "nonzero_lookups_per_step": int(hits),
                   "draws_per_step": int(draws)},
        "pml": [float(v) for v in pml],
        "tvar": [float(v) for v in tvar],
    }
    # live ceilings of the same part in the same run: the streaming read of the
    # event-id array (4 GB, 16-byte non-temporal loads) and the per-draw
    # arithmetic alone at the full-shape row shape (k_probe_draws)
    from paper_1501_06326_amd import ara as A
    sh = stream.cuda_stream
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = (4 * yet.n_occ) // 16 * 16
    ev_s = torch.cuda.Event(enable_timing=True)
    ev_e = torch.cuda.Event(enable_timing=True)
    A.ara_probe_stream_read(ara.ctx, ev.data_ptr(), nbytes, sink.data_ptr(), sh)
    ev_s.record(stream)
    for _ in range(5):
        A.ara_probe_stream_read(ara.ctx, ev.data_ptr(), nbytes, sink.data_ptr(), sh)
    ev_e.record(stream)
    torch.cuda.synchronize()
    b9_gbs = nbytes / (ev_s.elapsed_time(ev_e) / 5 / 1e3) / 1e9
    nd = 1 << 27
    xd = torch.empty(nd, dtype=torch.float32, device=dev)
    A.ara_probe_draws(ara.ctx, nd, pf.seed, 3, 2.75, 8.25, True, xd.data_ptr(), sh)
    t0d = time.perf_counter()
    A.ara_probe_draws(ara.ctx, nd, pf.seed, 3, 2.75, 8.25, True, xd.data_ptr(), sh)
    draw_ceiling = nd / (time.perf_counter() - t0d)       # synchronous call: wall time
    del xd
    log(f"ceilings: stream read {b9_gbs:.0f} GB/s, draw arithmetic alone {draw_ceiling:.3e} draws/s")

    # algorithmic HBM bytes of one SU run: event ids + trial offsets + the
    # layer's tables read once (pairs and compact records) + the two YLT outputs
    su_bytes = 4 * yet.n_occ + 8 * (n + 1) + 8 * yet.n_catalogue + 32 * 20000 * 16 + 2 * 4 * n
    arith = profiled("draw_arith_ops")
    ops = arith * draws if arith else None
    result["roofline"] = {
        "kernel": "k_ara_su (+ k_ara_su_redo), ara_run",
        "bound": "alu",
        "achieved": (ops / (run_ms / 1e3) / 1e12) if ops else None,
        "peak": PEAK_VALU_TOPS,
        "unit": "T lane-ops/s",
        "frac": (ops / (run_ms / 1e3) / 1e12 / PEAK_VALU_TOPS) if ops else None,
        "traffic": profiled("su_main_bytes") if (args.trials == 1_000_000 and
                                                  args.catalogue == 100_000) else None,
        "launch_ms": run_ms,
        "draws_per_s": draws / (run_ms / 1e3),
        "draw_arith_ops": arith,
        "draw_arithmetic_ceiling_draws_per_s": draw_ceiling,
        "frac_of_draw_arithmetic_ceiling": draws / (run_ms / 1e3) / draw_ceiling,
        "hbm": {"bytes": su_bytes, "achieved_gbs": su_bytes / (run_ms / 1e3) / 1e9,
                "frac_of_peak": su_bytes / (run_ms / 1e3) / 1e9 / PEAK_HBM_GBS,
                "stream_read_gbs": b9_gbs,
                "frac_of_stream_read": su_bytes / (run_ms / 1e3) / 1e9 / b9_gbs},
    }

    if not args.no_pu:
        pf_pu = full_portfolio(su=False, n_catalogue=args.catalogue)
        # the per-event occurrence-loss table is built at load: row upload,
        # Beta-fit kernel, per-event fill and sparse form (synchronous call)
        ara.load_portfolio(pf_pu, yet.n_catalogue)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        p_pu = ara.load_portfolio(pf_pu, yet.n_catalogue)
        build_ms = 1e3 * (time.perf_counter() - tb)
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
            "table_build_ms": build_ms,
            "evaluations_per_s_with_table_build": evals / ((pu_ms + build_ms) / 1e3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "frac_of_stream_read": gbs / b9_gbs,
                         "traffic": profiled("pu_bytes") if args.catalogue == 100_000 else None,
                         "bytes": byts},
        }
        log(f"PU: {pu_ms:.3f} ms/run, {gbs:.0f} GB/s; table build {build_ms:.2f} ms")

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
        # one thread on a smaller sample (about a quarter of the time) for the per-core rate
        m1 = int(max(8, m * 0.25 / cores))
        tc = time.perf_counter()
        oracle.run_ara(yet, pf, 0, m1, threads=1)
        dt1 = time.perf_counter() - tc
        ev1 = evaluations(yet, pf, 0, m1)
        result["cpu_baseline"] = {"value": ev_s / dt, "unit": "evaluations/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"trials [0, {m}) of the same workload, "
                                            f"{ev_s} evaluations in {dt:.1f} s",
                                  "per_core": {"value": ev1 / dt1, "threads": 1,
                                               "sample": f"trials [0, {m1}), {ev1} evaluations "
                                                         f"in {dt1:.1f} s"}}
        log(f"oracle: {ev_s / dt:.3g} evals/s on {cores} threads ({m} trials); "
            f"{ev1 / dt1:.3g} on one thread ({m1} trials)")

    print(json.dumps(result), flush=True)
    ara.close()


def _full_yet(n_trials):
    from workloads import SEED_YET_FULL, make_yet
    t0 = time.time()
    yet = make_yet(n_trials, 1000.0, 100_000, SEED_YET_FULL, with_times=False)
    log(f"generated YET: {n_trials} trials, {yet.n_occ} occurrences in {time.time() - t0:.1f}s")
    return yet


def bench_probes(args):
    """VALU issue rates per instruction kind, the streaming read bandwidth and
    the per-draw arithmetic alone (one JSON line)."""
    import torch
    from paper_1501_06326_amd import Ara
    from paper_1501_06326_amd import ara as A

    ara = Ara(0)
    dev = ara.device
    props = torch.cuda.get_device_properties(dev)
    n_cu = props.multi_processor_count
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {"metric": "probes", "n_cu": n_cu, "valu": {}}
    wps, iters = 8, 8192
    out = torch.empty(A.ara_probe_valu_lanes(ara.ctx, wps), dtype=torch.float32, device=dev)
    for name, kind in A.PROBE_KINDS.items():
        instr = [0]

        def run():
            instr[0] = A.ara_probe_valu(ara.ctx, kind, wps, iters, out.data_ptr(), sh)
        ms = timed(run, 5)
        rate = instr[0] / (ms / 1e3)
        # wave instructions per SIMD per cycle at the 2.4 GHz peak engine clock
        per_simd_clk = rate / (n_cu * 4 * 2.4e9)
        res["valu"][name] = {"ms": ms, "wave_instr": instr[0], "wave_instr_per_s": rate,
                             "lane_ops_per_s": 64 * rate, "per_simd_per_clk_at_2.4GHz": per_simd_clk}
        log(f"valu {name}: {ms:.3f} ms, {64 * rate / 1e12:.1f} T lane-ops/s, "
            f"{per_simd_clk:.3f} wave-instr per SIMD-clock")
    # streaming read of 4 GiB (the size of the full-shape event-id stream)
    nbytes = 4 << 30
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    ms = timed(lambda: A.ara_probe_stream_read(ara.ctx, buf.data_ptr(), nbytes, sink.data_ptr(),
                                               sh), 10)
    res["stream_read"] = {"bytes": nbytes, "ms": ms, "gbs": nbytes / (ms / 1e3) / 1e9}
    log(f"stream read: {ms:.3f} ms for 4 GiB, {nbytes / (ms / 1e3) / 1e9:.0f} GB/s")
    del buf
    # the per-draw arithmetic alone at the full-shape row shape (mean/max 1/4,
    # sigma/max 1/8: alpha = 2.75, beta = 8.25)
    nd = 1 << 28
    x = torch.empty(nd, dtype=torch.float32, device=dev)
    for tab in (True, False):
        ms = timed(lambda: A.ara_probe_draws(ara.ctx, nd, 150106326, 3, 2.75, 8.25, tab,
                                             x.data_ptr(), sh), 5)
        bad = int((x < 0).sum().item())
        key = "draws" if tab else "draws_closed_form_guess"
        res[key] = {"n": nd, "shape": [2.75, 8.25], "shape_table": tab, "ms": ms,
                    "draws_per_s": nd / (ms / 1e3), "not_converged": bad}
        log(f"draws alone ({'shape table' if tab else 'closed-form guess'}): {ms:.3f} ms for "
            f"{nd}, {nd / (ms / 1e3):.3e} draws/s, {bad} not converged")
    print(json.dumps(res), flush=True)
    ara.close()


def bench_variants(args):
    """Full-shape runs under the laws that use the FP64-capable second pass."""
    import copy
    import torch
    from paper_1501_06326_amd import Ara, evaluations
    from workloads import (SEED_ELT_BASE, Layer, Portfolio, SEED_PHILOX, config_full, make_elt,
                           sigma_capped, varied_shapes)

    w = config_full(n_trials=args.trials, with_times=False)
    yet, base = w.yet, w.portfolio
    lay = base.layers[0]
    corr = Portfolio(layers=[Layer(elts=[make_elt(e, 20_000, yet.n_catalogue, SEED_ELT_BASE + e,
                                                  corr=True, retention=1e6, limit=5e7)
                                         for e in range(16)],
                                   occ_retention=lay.occ_retention, occ_limit=lay.occ_limit,
                                   agg_retention=lay.agg_retention, agg_limit=lay.agg_limit)],
                     seed=SEED_PHILOX, su_enabled=True)
    cases = [("headline", base), ("two_normal_mix", corr), ("varied_shapes", varied_shapes(base)),
             ("sigma_capped_30pct", sigma_capped(base))]
    ara = Ara(0)
    dev = ara.device
    off = torch.from_numpy(yet.offsets).to(dev)
    ev = torch.from_numpy(yet.event_ids).to(dev)
    y = ara.load_yet(yet, device_arrays=(off, ev, None))
    stream = torch.cuda.current_stream()
    n = yet.n_trials
    out_p = torch.empty(n, dtype=torch.float32, device=dev)
    scratch = torch.empty(ara.run_scratch_size(n), dtype=torch.uint8, device=dev)
    res = {}
    for name, pf in cases:
        p = ara.load_portfolio(pf, yet.n_catalogue)
        ara.run(y, p, out_pf=out_p, layers=False, scratch=scratch)      # warmup, status check
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            ara.run(y, p, out_pf=out_p, layers=False, scratch=scratch, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ara.sync_status()
        ms = e0.elapsed_time(e1) / args.steps
        ev_n = evaluations(yet, pf)
        res[name] = {"ms_per_run": ms, "evaluations_per_s": ev_n / (ms / 1e3)}
        log(f"{name}: {ms:.2f} ms per run, {ev_n / (ms / 1e3):.3e} evaluations/s")
        ara.free_portfolio(p)
        del p
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "trial*event*ELT evaluations/s per secondary-uncertainty law",
                      "n_gpus": 1, "steps": args.steps, "dtype": "f32 (FP64 second pass)",
                      "data": "synthetic (seeded numpy generator; lognormal ELT means)",
                      "config": {"workload": w.name, "trials": n, "occurrences": yet.n_occ,
                                 "elts": 16, "sum_mode": "kahan32"}, **res}), flush=True)
    ara.close()


def bench_footprint(args):
    """The lean secondary-uncertainty pass at a fixed number of hits per
    occurrence while the paying-row table grows: catalogues of 12,500 to
    200,000 events, 16 ELTs of catalogue / 5 rows each (the full shape's
    density), Poisson(1000) occurrences, --trials trials (default 300,000 in
    this mode).  The row records and (first row, count) pairs the pass
    gathers grow with the catalogue, so the time per occurrence shows what
    those gathers' cache misses cost."""
    import torch
    from paper_1501_06326_amd import Ara
    from workloads import (SEED_ELT_BASE, SEED_PHILOX, SEED_YET_FULL, Layer, Portfolio, make_elt,
                           make_yet)

    trials = args.trials if args.trials != 1_000_000 else 300_000
    ara = Ara(0)
    dev = ara.device
    stream = torch.cuda.current_stream()
    rows_out = []
    for cat in (12_500, 25_000, 50_000, 100_000, 200_000):
        yet = make_yet(trials, 1000.0, cat, SEED_YET_FULL, with_times=False)
        elts = [make_elt(e, cat // 5, cat, SEED_ELT_BASE + e, retention=1e6, limit=5e7)
                for e in range(16)]
        pf = Portfolio(layers=[Layer(elts=elts, occ_retention=1e7, occ_limit=2e8,
                                     agg_retention=5e7, agg_limit=1e9)],
                       seed=SEED_PHILOX, su_enabled=True)
        off = torch.from_numpy(yet.offsets).to(dev)
        ev = torch.from_numpy(yet.event_ids).to(dev)
        y = ara.load_yet(yet, device_arrays=(off, ev, None))
        p = ara.load_portfolio(pf, cat)
        n = yet.n_trials
        out_p = torch.empty(n, dtype=torch.float32, device=dev)
        scratch = torch.empty(ara.run_scratch_size(n), dtype=torch.uint8, device=dev)
        ara.run(y, p, out_pf=out_p, layers=False, scratch=scratch)      # warmup, status check
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            ara.run(y, p, out_pf=out_p, layers=False, scratch=scratch, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ara.sync_status()
        ms = e0.elapsed_time(e1) / args.steps
        hits = ara.run(y, p, diagnostics=True, out_pf=out_p)["hits"].sum().item()
        row = {"catalogue": cat, "rows_per_elt": cat // 5, "occurrences": yet.n_occ,
               "ms_per_run": ms, "ns_per_occurrence": 1e6 * ms / yet.n_occ,
               "nonzero_lookups_per_occurrence": hits / yet.n_occ}
        rows_out.append(row)
        log(f"catalogue {cat}: {ms:.3f} ms, {row['ns_per_occurrence']:.4f} ns per occurrence")
        ara.free_portfolio(p)
        del p, y, off, ev, out_p, scratch
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "lean secondary-uncertainty pass time vs paying-row footprint",
                      "n_gpus": 1, "steps": args.steps, "trials": trials,
                      "data": "synthetic (seeded numpy generator; lognormal ELT means)",
                      "runs": rows_out}), flush=True)
    ara.close()


def bench_batched(args):
    """64 portfolios on one YET: one batched launch vs sequential ara_run."""
    import torch
    from paper_1501_06326_amd import Ara, evaluations
    from workloads import batched_portfolios

    yet = _full_yet(args.trials)
    n = yet.n_trials
    t0 = time.time()
    pfs = batched_portfolios(args.portfolios, su=not args.pu)
    log(f"generated {len(pfs)} portfolios, {sum(p.n_elts for p in pfs)} ELTs "
        f"in {time.time() - t0:.1f}s")
    evals = sum(evaluations(yet, p) for p in pfs)
    ara = Ara(0)
    min_bytes = 4 * yet.n_occ + 8 * (n + 1)
    dev = ara.device
    off = torch.from_numpy(yet.offsets).to(dev)
    ev = torch.from_numpy(yet.event_ids).to(dev)
    y = ara.load_yet(yet, device_arrays=(off, ev, None))
    dps = []
    for k, pf in enumerate(pfs):
        dps.append(ara.load_portfolio(pf, yet.n_catalogue))
        if k % 16 == 15:
            log(f"loaded {k + 1} portfolios")
    ws = sum(d.workspace.numel() for d in dps)
    outs = [{"ylt": torch.empty((d.n_layers, n), dtype=torch.float32, device=dev),
             "ylt_pf": torch.empty(n, dtype=torch.float32, device=dev)} for d in dps]
    seq = [{"ylt": torch.empty_like(o["ylt"]), "ylt_pf": torch.empty_like(o["ylt_pf"])}
           for o in outs]
    scratch = torch.empty(ara.run_scratch_size(n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    sub = min(n, 4_000)
    cfg, tune_ms = ara.batch_autotune(y, dps, trial_count=sub)
    log(f"autotuned (trial_tile, waves_per_cu) = {cfg} on {sub} trials ({tune_ms:.2f} ms)")
    # warmup on a prefix of the trials
    ara.run_batch(y, dps, trial_count=sub, cfg=cfg)
    for d in dps:
        ara.run(y, d, trial_count=sub, scratch=scratch)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record(stream)
    for d, o in zip(dps, seq):
        ara.run(y, d, out_layers=o["ylt"], out_pf=o["ylt_pf"], scratch=scratch, sync=False)
    e[1].record(stream)
    torch.cuda.synchronize()
    ara.sync_status()
    seq_ms = e[0].elapsed_time(e[1])
    log(f"sequential: {seq_ms:.1f} ms")
    e[2].record(stream)
    ara.run_batch(y, dps, cfg=cfg, outs=outs, sync=False)
    e[3].record(stream)
    torch.cuda.synchronize()
    ara.sync_status()
    bat_ms = e[2].elapsed_time(e[3])
    log(f"batched: {bat_ms:.1f} ms")
    identical = all(torch.equal(a["ylt"], b["ylt"]) and torch.equal(a["ylt_pf"], b["ylt_pf"])
                    for a, b in zip(outs, seq))
    result = {
        "metric": "batched trial*event*ELT evaluations/s (64 portfolios on the 1M-trial YET"
                  + (", primary uncertainty)" if args.pu else ")"),
        "value": evals / (bat_ms / 1e3), "unit": "evaluations/s", "n_gpus": 1,
        "ms_per_step": bat_ms, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic (seeded numpy generator; lognormal ELT means)",
        "config": {"workload": f"ara_batched_{len(pfs)}_portfolios_{n}_trials",
                   "portfolios": len(pfs), "layers": sum(len(p.layers) for p in pfs),
                   "elts": sum(p.n_elts for p in pfs), "trials": n, "occurrences": yet.n_occ,
                   "evaluations_per_step": evals, "workspace_bytes": ws,
                   "batch_config": {"trial_tile": cfg[0], "waves_per_cu": cfg[1],
                                    "order": ["portfolio-major", "trial-major"][cfg[2]]}},
        "sequential": {"ms": seq_ms, "evaluations_per_s": evals / (seq_ms / 1e3)},
        "speedup_vs_sequential": seq_ms / bat_ms,
        "batched_equals_sequential": identical,
        # the least a batch must read: the YET's event ids and offsets once
        "hbm": {"min_bytes": min_bytes, "gbs": min_bytes / (bat_ms / 1e3) / 1e9,
                "frac_of_peak": min_bytes / (bat_ms / 1e3) / 1e9 / PEAK_HBM_GBS},
    }
    if args.graph:
        g, gouts, gsc = ara.batch_graph(y, dps, cfg=cfg)
        ara.graph_launch(g)
        torch.cuda.synchronize()
        e[0].record(stream)
        ara.graph_launch(g)
        e[1].record(stream)
        torch.cuda.synchronize()
        result["graph_ms"] = e[0].elapsed_time(e[1])
        result["graph_evaluations_per_s"] = evals / (result["graph_ms"] / 1e3)
        result["graph_equals_eager"] = all(torch.equal(a["ylt_pf"], b["ylt_pf"])
                                           for a, b in zip(gouts, outs))
        ara.graph_destroy(g)
    print(json.dumps(result), flush=True)
    ara.close()


def bench_precision(args):
    """Sum modes on the 8-layer precision-study portfolio: GPU time per mode and
    error distributions against the oracle on the first --oracle-trials trials."""
    import torch
    import oracle
    from paper_1501_06326_amd import Ara, evaluations
    from workloads import multilayer_portfolio

    yet = _full_yet(args.trials)
    pf = multilayer_portfolio()
    evals = evaluations(yet, pf)
    ara = Ara(0)
    dev = ara.device
    off = torch.from_numpy(yet.offsets).to(dev)
    ev = torch.from_numpy(yet.event_ids).to(dev)
    y = ara.load_yet(yet, device_arrays=(off, ev, None))
    p = ara.load_portfolio(pf, yet.n_catalogue)
    m = min(args.oracle_trials, yet.n_trials)
    t0 = time.time()
    cores = len(os.sched_getaffinity(0))
    ref = oracle.run_ara(yet, pf, 0, m, threads=cores)
    log(f"oracle: {m} trials in {time.time() - t0:.1f}s on {cores} threads")
    rps = [100.0, 250.0]
    rp_ref, rt_ref = oracle.pml_tvar(ref["ylt_pf"], rps)
    stream = torch.cuda.current_stream()
    modes = {}
    for mode in ("naive32", "kahan32", "f64"):
        dt = "f64" if mode == "f64" else "f32"
        r = ara.run(y, p, sum_mode=mode, ylt_dtype=dt)        # warmup and status check
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = ara.run(y, p, sum_mode=mode, ylt_dtype=dt, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        g = r["ylt"][:, :m].double().cpu().numpy()
        gp = r["ylt_pf"][:m].double().cpu().numpy()

        def dist(err, scale, y_ref):
            rel_g = err / np.maximum(scale, 1.0)
            pos = y_ref > 0
            rel_y = err[pos] / y_ref[pos] if pos.any() else np.zeros(1)
            return {"max_over_G": float(rel_g.max()), "p99_over_G": _pct(rel_g, 99),
                    "median_over_G": _pct(rel_g, 50), "max_rel": float(rel_y.max()),
                    "p99_rel": _pct(rel_y, 99), "median_rel": _pct(rel_y, 50)}

        layers = [dist(np.abs(g[l] - ref["ylt"][l]), ref["gross"][l], ref["ylt"][l])
                  for l in range(len(pf.layers))]
        port = dist(np.abs(gp - ref["ylt_pf"]), ref["gross"].sum(axis=0), ref["ylt_pf"])
        pml, tvar = ara.pml_tvar(r["ylt_pf"][:m].contiguous(), rps)
        modes[mode] = {
            "ms_per_run": ms, "evaluations_per_s": evals / (ms / 1e3),
            "layers": layers, "portfolio": port,
            "pml_rel_err": [abs(a - b) / b for a, b in zip(pml, rp_ref)],
            "tvar_rel_err": [abs(a - b) / b for a, b in zip(tvar, rt_ref)],
        }
        log(f"{mode}: {ms:.1f} ms, portfolio max err/G {port['max_over_G']:.3g}, "
            f"PML err {modes[mode]['pml_rel_err']}")
    result = {"metric": "precision study: per-trial and PML/TVaR errors by sum mode",
              "n_gpus": 1, "data": "synthetic (seeded numpy generator; lognormal ELT means)",
              "config": {"workload": f"ara_precision_8_layers_{yet.n_trials}_trials",
                         "layers": len(pf.layers), "elts": pf.n_elts, "trials": yet.n_trials,
                         "oracle_trials": m, "return_periods": rps,
                         "evaluations_per_run": evals},
              "modes": modes}
    print(json.dumps(result), flush=True)
    ara.close()


def bench_views(args):
    """The occurrence view (the per-occurrence increments of the aggregate
    loss, in stored order) and the exceedance-probability curve, on the
    full-shape workload, timed with HIP events on the launch stream."""
    import torch
    from paper_1501_06326_amd import Ara
    from workloads import config_full, full_portfolio

    w = config_full(n_trials=args.trials, n_catalogue=args.catalogue)
    yet, pf_su = w.yet, w.portfolio
    pf_pu = full_portfolio(su=False, n_catalogue=args.catalogue)
    ara = Ara(0)
    dev = ara.device
    off = torch.from_numpy(yet.offsets).to(dev)
    ev = torch.from_numpy(yet.event_ids).to(dev)
    tm = torch.from_numpy(yet.times).to(dev) if yet.times is not None else None
    y = ara.load_yet(yet, device_arrays=(off, ev, tm))
    stream = torch.cuda.current_stream()
    n_occ = int(yet.n_occ)
    out = {}

    def timed(fn, reps):
        fn()                                               # warmup and status check
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r = fn(sync=False)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            del r
        return float(np.mean(ms))

    for name, pf in (("su", pf_su), ("pu", pf_pu)):
        p = ara.load_portfolio(pf, yet.n_catalogue)
        ms = timed(lambda sync=True: ara.run(y, p, occ_view=True, sync=sync), args.steps)
        # written: one FP32 increment per occurrence (the binding's zero fill of
        # that buffer is inside the timed region); read: the event ids
        out[name] = {"ms_per_run": ms, "occurrences_per_s": n_occ / (ms / 1e3),
                     "view_bytes": 4 * n_occ,
                     "view_gb_per_s": 4 * n_occ / (ms / 1e3) / 1e9}
        log(f"occurrence view ({name}): {ms:.2f} ms for {n_occ} occurrences")
        ara.free_portfolio(p)
        torch.cuda.empty_cache()

    p = ara.load_portfolio(pf_su, yet.n_catalogue)
    ylt = ara.run(y, p)["ylt_pf"]
    ms = timed(lambda sync=True: ara.ep_curve(ylt), args.steps)
    out["ep_curve"] = {"ms_per_call": ms, "entries": int(ylt.numel()),
                       "entries_per_s": ylt.numel() / (ms / 1e3)}
    log(f"EP curve: {ms:.3f} ms for {ylt.numel()} entries")
    result = {"metric": "occurrence view and exceedance-probability curve",
              "n_gpus": 1, "steps": args.steps, "dtype": "f32 (FP64 running means)",
              "data": "synthetic (seeded numpy generator; lognormal ELT means)",
              "config": {"workload": w.name, "trials": yet.n_trials, "occurrences": n_occ,
                         "catalogue": yet.n_catalogue, "layers": 1, "elts": 16},
              **out}
    print(json.dumps(result), flush=True)
    ara.close()


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def bench_served(args):
    """Serving loop under Poisson arrivals against a one-at-a-time server."""
    import threading

    import torch
    from paper_1501_06326_amd import Ara, Server, evaluations
    from workloads import poisson_arrivals, served_requests

    yet = _full_yet(args.trials)
    t0 = time.time()
    reqs = served_requests(args.requests, yet.n_trials)
    log(f"generated {len(reqs)} requests in {time.time() - t0:.1f}s")
    req_evals = [evaluations(yet, r.portfolio, r.trial_begin, r.trial_count) for r in reqs]
    rps = [100.0, 250.0]
    ara = Ara(0)
    dev = ara.device
    off = torch.from_numpy(yet.offsets).to(dev)
    ev = torch.from_numpy(yet.event_ids).to(dev)
    y = ara.load_yet(yet, device_arrays=(off, ev, None))

    # one-at-a-time: load, run, PML / TVaR, free -- per request, synchronously
    for r in reqs[:4]:
        d = ara.load_portfolio(r.portfolio, yet.n_catalogue)
        ara.pml_tvar(ara.run(y, d, r.trial_begin, r.trial_count)["ylt_pf"], rps)
        ara.free_portfolio(d)
    svc = []
    for i, r in enumerate(reqs):
        ts = time.perf_counter()
        d = ara.load_portfolio(r.portfolio, yet.n_catalogue)
        ara.pml_tvar(ara.run(y, d, r.trial_begin, r.trial_count)["ylt_pf"], rps)
        ara.free_portfolio(d)
        svc.append(time.perf_counter() - ts)
        if i % 200 == 199:
            log(f"one-at-a-time: {i + 1} requests, mean service {np.mean(svc) * 1e3:.1f} ms")
    svc = np.asarray(svc)
    capacity = len(reqs) / svc.sum()
    total_evals = float(sum(req_evals))
    log(f"one-at-a-time capacity {capacity:.2f} req/s, "
        f"{total_evals / svc.sum():.3g} evaluations/s")
    torch.cuda.empty_cache()

    points = []
    for f in [float(x) for x in args.loads.split(",")]:
        rate = f * capacity
        arr = poisson_arrivals(len(reqs), rate, seed=6 + int(f * 1000))
        # one-at-a-time FIFO server with the measured service times
        fin = 0.0
        lat1 = []
        for a, s_i in zip(arr, svc):
            fin = max(a, fin) + s_i
            lat1.append(fin - a)
        with Server(yet, device_arrays=(off, ev), pool_bytes=32 << 30,
                    max_inflight=args.max_inflight, max_batch=args.max_batch) as srv:
            ids = {}
            start = time.perf_counter() + 0.05
            lock = threading.Lock()

            def submitter():
                for i, r in enumerate(reqs):
                    dt = start + arr[i] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                    rid = srv.submit(r.portfolio, r.trial_begin, r.trial_count, rps, borrow=True)
                    with lock:
                        ids[rid] = i

            th = threading.Thread(target=submitter)
            th.start()
            lat, done_t, n_err = [], [], 0
            while len(lat) < len(reqs):
                for res in srv.poll(64, wait_s=0.02):
                    now = time.perf_counter()
                    with lock:
                        i = ids.get(res["id"])
                    while i is None:           # result before the submitter recorded the id
                        time.sleep(1e-4)
                        with lock:
                            i = ids.get(res["id"])
                    n_err += res["status"] != 0
                    lat.append(now - (start + arr[i]))
                    done_t.append(now - start)
                    if len(lat) % 250 == 0:
                        log(f"load {f}: {len(lat)} done")
            th.join()
        span = max(done_t) - arr[0]
        pt = {"offered_load": f, "rate_req_s": rate, "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99),
              "mean_s": float(np.mean(lat)), "achieved_req_s": len(reqs) / span,
              "evaluations_per_s": total_evals / span, "errors": int(n_err),
              "one_at_a_time": {"p50_s": _pct(lat1, 50), "p99_s": _pct(lat1, 99),
                                "mean_s": float(np.mean(lat1))}}
        log(f"load {f}: p50 {pt['p50_s'] * 1e3:.1f} ms p99 {pt['p99_s'] * 1e3:.1f} ms "
            f"(one-at-a-time {pt['one_at_a_time']['p50_s'] * 1e3:.1f} / "
            f"{pt['one_at_a_time']['p99_s'] * 1e3:.1f} ms), {pt['evaluations_per_s']:.3g} evals/s")
        points.append(pt)
    result = {
        "metric": "served latency p50/p99 (s) and evaluations/s under Poisson arrivals",
        "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
        "data": "synthetic (seeded numpy generator; lognormal ELT means)",
        "config": {"workload": f"ara_served_{n_trials_label(yet)}_yet",
                   "requests_per_load": len(reqs), "distinct_portfolios": 32,
                   "trials": yet.n_trials, "max_inflight": args.max_inflight,
                   "max_batch": args.max_batch, "return_periods": rps},
        "one_at_a_time": {"capacity_req_s": capacity,
                          "evaluations_per_s": total_evals / svc.sum(),
                          "mean_service_s": float(svc.mean()),
                          "p50_service_s": _pct(svc, 50), "p99_service_s": _pct(svc, 99)},
        "points": points,
    }
    print(json.dumps(result), flush=True)
    ara.close()


def n_trials_label(yet):
    return f"{yet.n_trials // 1000}k" if yet.n_trials < 1_000_000 else f"{yet.n_trials // 1_000_000}M"


if __name__ == "__main__":
    main()
