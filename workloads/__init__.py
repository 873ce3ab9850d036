"""Seeded synthetic inputs for Aggregate Risk Analysis (ARA).

This module only *draws inputs*: Year Event Tables (YET), Event Loss Tables
(ELT / extended XELT rows) and portfolios of layers with their terms.  It holds
none of the method's arithmetic (no lookups, no secondary uncertainty, no
financial terms, no risk metrics); both the FP64 oracle and the GPU library
consume what it produces.

Data model (paper section 2.1 "Inputs" and section 3.1):
  * YET: trials T_i, each an ordered list of (event id, time stamp) in
    ascending time.  Stored as CSR: ``offsets[int64, T+1]``,
    ``event_ids[int32, n_occ]``, ``times[float32, n_occ]`` (optional).
  * ELT / XELT: rows {E, mean loss mu, sigma_I, sigma_C, max loss} plus the
    ELT financial terms (retention, limit, share).
  * Portfolio -> layers; a layer holds a list of ELTs and the occurrence /
    aggregate terms (OccR, OccL, AggR, AggL).

Generator rules (shared by every configuration):
  * numpy ``Generator(PCG64(SeedSequence([...])))``; YET chunks of
    ``YET_CHUNK`` trials draw from their own seed sequences so chunks can be
    generated in parallel threads and the result does not depend on the
    thread count.
  * occurrence counts per trial ~ Poisson(lambda); event ids uniform with
    replacement over the catalogue; time stamps uniform on [0, 365) and
    sorted, drawn as normalised cumulative exponential spacings (the order
    statistics of uniforms) so no per-trial sort is needed.
  * an ELT's non-zero event set is drawn uniformly without replacement and
    stored in ascending event order; mean = exp(N(12, 1.5^2)) rounded to
    float32; std = 0.5 * mean; max loss (exposure) = 4 * mean (both exact in
    float32).
  * financial terms are rounded to float32 so that an FP32 consumer sees the
    same values as an FP64 one.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

YET_CHUNK = 8192

# Seeds: arbitrary, printed with every result.
SEED_YET_SMALL = 1501
SEED_YET_FULL = 1502
SEED_ELT_BASE = 6326
SEED_PHILOX = 150106326
SEED_TERMS = 3

INF = float("inf")


# --------------------------------------------------------------------------
# data classes
# --------------------------------------------------------------------------
@dataclass
class YET:
    offsets: np.ndarray            # int64 [n_trials + 1], offsets[0] == 0
    event_ids: np.ndarray          # int32 [n_occ]
    times: Optional[np.ndarray]    # float32 [n_occ] or None
    n_catalogue: int

    @property
    def n_trials(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_occ(self) -> int:
        return int(self.offsets[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)

    def slice(self, begin: int, count: int) -> "YET":
        """Trials [begin, begin+count) as a standalone YET (offsets rebased)."""
        o = self.offsets[begin:begin + count + 1]
        lo, hi = int(o[0]), int(o[-1])
        return YET(offsets=(o - lo).astype(np.int64),
                   event_ids=self.event_ids[lo:hi],
                   times=None if self.times is None else self.times[lo:hi],
                   n_catalogue=self.n_catalogue)


@dataclass
class ELT:
    elt_id: int                    # caller's 32-bit id (keys the random draws)
    event_ids: np.ndarray          # int32 [n_rows], distinct
    mean: np.ndarray               # float32 [n_rows]
    sigma_i: np.ndarray            # float32 [n_rows]
    sigma_c: np.ndarray            # float32 [n_rows]
    max_loss: np.ndarray           # float32 [n_rows]
    retention: float = 0.0
    limit: float = INF
    share: float = 1.0

    @property
    def n_rows(self) -> int:
        return int(self.event_ids.shape[0])


@dataclass
class Layer:
    elts: List[ELT]
    occ_retention: float = 0.0
    occ_limit: float = INF
    agg_retention: float = 0.0
    agg_limit: float = INF
    program_id: int = 0


@dataclass
class Portfolio:
    layers: List[Layer]
    seed: int = SEED_PHILOX
    su_enabled: bool = True
    keying: int = 0                # 0: per-occurrence keys; 1: section 3.1's layout

    @property
    def n_elts(self) -> int:
        return sum(len(l.elts) for l in self.layers)


@dataclass
class Workload:
    name: str
    yet: YET
    portfolio: Portfolio
    return_periods: Sequence[float] = (100.0, 250.0)
    extra: dict = field(default_factory=dict)


def f32(x: float) -> float:
    """Round a Python float to the nearest float32 value (kept as float)."""
    if math.isinf(x):
        return x
    return float(np.float32(x))


# --------------------------------------------------------------------------
# YET
# --------------------------------------------------------------------------
def _n_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def make_yet(n_trials: int, lam: float, n_catalogue: int, seed: int,
             with_times: bool = True, threads: Optional[int] = None) -> YET:
    """Poisson(lam) occurrences per trial, ids uniform over the catalogue."""
    n_chunks = (n_trials + YET_CHUNK - 1) // YET_CHUNK
    counts = np.empty(n_trials, dtype=np.int64)
    for c in range(n_chunks):
        lo, hi = c * YET_CHUNK, min(n_trials, (c + 1) * YET_CHUNK)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c, 0])))
        counts[lo:hi] = rng.poisson(lam, size=hi - lo)
    offsets = np.zeros(n_trials + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n_occ = int(offsets[-1])
    event_ids = np.empty(n_occ, dtype=np.int32)
    times = np.empty(n_occ, dtype=np.float32) if with_times else None
    top = np.float32(np.nextafter(np.float32(365.0), np.float32(0.0)))

    def chunk(c: int) -> None:
        lo, hi = c * YET_CHUNK, min(n_trials, (c + 1) * YET_CHUNK)
        a, b = int(offsets[lo]), int(offsets[hi])
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c, 1])))
        event_ids[a:b] = rng.integers(0, n_catalogue, size=b - a, dtype=np.int32)
        if times is None or b == a:
            return
        rng_t = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c, 2])))
        cnt = counts[lo:hi]
        # n_i + 1 exponential spacings per trial; the first n_i partial sums
        # divided by the total are the sorted uniforms of that trial.
        sp = rng_t.standard_exponential(size=(b - a) + (hi - lo))
        cs = np.cumsum(sp)
        ends = np.cumsum(cnt + 1) - 1                  # index of each trial's total
        starts = ends - cnt                             # first spacing of the trial
        base = np.where(starts > 0, cs[np.maximum(starts - 1, 0)], 0.0)
        total = cs[ends] - base
        keep = np.ones(cs.shape[0], dtype=bool)
        keep[ends] = False
        trial_of = np.repeat(np.arange(hi - lo), cnt)
        t = (cs[keep] - base[trial_of]) / total[trial_of] * 365.0
        times[a:b] = np.minimum(t.astype(np.float32), top)

    nt = threads or _n_threads()
    if nt > 1 and n_chunks > 1:
        with ThreadPoolExecutor(nt) as ex:
            list(ex.map(chunk, range(n_chunks)))
    else:
        for c in range(n_chunks):
            chunk(c)
    return YET(offsets=offsets, event_ids=event_ids, times=times, n_catalogue=n_catalogue)


# --------------------------------------------------------------------------
# ELTs
# --------------------------------------------------------------------------
def make_elt(elt_id: int, n_rows: int, n_catalogue: int, seed: int,
             corr: bool = False, retention: float = 0.0, limit: float = INF,
             share: float = 1.0, mu_log: float = 12.0, sigma_log: float = 1.5) -> ELT:
    """One ELT with ``n_rows`` distinct events and lognormal mean losses.

    std = 0.5 * mean; exposure (max loss) = 4 * mean.  With ``corr`` the std is
    split evenly into an independent and a correlated part
    (sigma_I = sigma_C = 0.25 * mean), otherwise sigma_I = std, sigma_C = 0.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    ev = np.sort(rng.choice(n_catalogue, size=n_rows, replace=False)).astype(np.int32)
    mean = np.exp(rng.normal(mu_log, sigma_log, size=n_rows)).astype(np.float32)
    if corr:
        si = (mean * np.float32(0.25)).astype(np.float32)
        sc = si.copy()
    else:
        si = (mean * np.float32(0.5)).astype(np.float32)
        sc = np.zeros(n_rows, dtype=np.float32)
    mx = (mean * np.float32(4.0)).astype(np.float32)
    return ELT(elt_id=int(elt_id), event_ids=ev, mean=mean, sigma_i=si, sigma_c=sc,
               max_loss=mx, retention=f32(retention), limit=f32(limit), share=f32(share))


def _log_uniform(rng: np.random.Generator, lo: float, hi: float, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


# --------------------------------------------------------------------------
# the configurations
# --------------------------------------------------------------------------
def config_small(corr: bool = False, su: bool = True, with_times: bool = True,
                 n_trials: int = 10_000) -> Workload:
    """Small parity case: 10,000 trials x Poisson(100) over a 10,000-event
    catalogue; one layer of 3 ELTs x 2,000 rows; ELT terms (1e5, 5e6, 1.0),
    occurrence terms (1e6, 2e7), aggregate terms (5e6, 1e8); RP 100 and 250."""
    yet = make_yet(n_trials, 100.0, 10_000, SEED_YET_SMALL, with_times=with_times)
    elts = [make_elt(e, 2_000, 10_000, SEED_ELT_BASE + e, corr=corr,
                     retention=1e5, limit=5e6, share=1.0) for e in range(3)]
    layer = Layer(elts=elts, occ_retention=1e6, occ_limit=2e7,
                  agg_retention=5e6, agg_limit=1e8)
    name = "ara_small_10k_trials_3_elts" + ("_corr" if corr else "")
    return Workload(name=name, yet=yet,
                    portfolio=Portfolio(layers=[layer], seed=SEED_PHILOX, su_enabled=su))


def full_portfolio(su: bool = True, n_catalogue: int = 100_000) -> Portfolio:
    """One layer of 16 ELTs x 20,000 rows, the small case's terms scaled x10."""
    elts = [make_elt(e, 20_000, n_catalogue, SEED_ELT_BASE + e,
                     retention=1e6, limit=5e7, share=1.0) for e in range(16)]
    layer = Layer(elts=elts, occ_retention=1e7, occ_limit=2e8,
                  agg_retention=5e7, agg_limit=1e9)
    return Portfolio(layers=[layer], seed=SEED_PHILOX, su_enabled=su)


def config_full(n_trials: int = 1_000_000, with_times: bool = True, su: bool = True,
                lam: float = 1000.0, n_catalogue: int = 100_000) -> Workload:
    """Full shape: 1,000,000 trials x Poisson(1000) over a 100,000-event
    catalogue; one layer of 16 ELTs x 20,000 rows.  n_catalogue = 1,000,000
    is the large-catalogue variant of the paper's direct-access example (16
    ELTs of 20,000 non-zero rows over a 1,000,000-event catalogue)."""
    yet = make_yet(n_trials, lam, n_catalogue, SEED_YET_FULL, with_times=with_times)
    tag = "" if n_catalogue == 100_000 else f"_catalogue_{n_catalogue}"
    return Workload(name=f"ara_full_{n_trials}_trials_16_elts{tag}", yet=yet,
                    portfolio=full_portfolio(su=su, n_catalogue=n_catalogue))


def sigma_capped(pf: Portfolio, fraction: float = 0.3, seed: int = 8) -> Portfolio:
    """A copy of pf where a fraction of each ELT's rows have sigma_I = 3 mean
    (with max = 4 mean that is sigma_beta = 0.75 > sigma_beta_max ~ 0.433, so
    the fit hits the cap of section 3.3 and the shape is near-Bernoulli)."""
    import copy
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    out = copy.deepcopy(pf)
    for layer in out.layers:
        for e in layer.elts:
            pick = rng.random(len(e.mean)) < fraction
            si = np.array(e.sigma_i, np.float32, copy=True)
            si[pick] = (np.float32(3.0) * np.asarray(e.mean, np.float32)[pick]).astype(np.float32)
            e.sigma_i = si
    return out


def varied_shapes(pf: Portfolio, seed: int = 9) -> Portfolio:
    """A copy of pf whose rows each get their own Beta shape: sigma_I = mean x
    U(0.15, 0.9) and max = mean x U(1.5, 10), so one batch of draws mixes
    shapes (and continued-fraction term counts) across its lanes."""
    import copy
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    out = copy.deepcopy(pf)
    for layer in out.layers:
        for e in layer.elts:
            m = np.asarray(e.mean, np.float32)
            e.sigma_i = (m * rng.uniform(0.15, 0.9, m.size)).astype(np.float32)
            e.max_loss = (m * rng.uniform(1.5, 10.0, m.size)).astype(np.float32)
    return out


def random_layer_terms(rng: np.random.Generator, lo: float = 1e5, hi: float = 1e9):
    """Per-layer OccR, OccL, AggR, AggL, each log-uniform on [lo, hi]."""
    v = _log_uniform(rng, lo, hi, size=4)
    return tuple(f32(float(x)) for x in v)


def multilayer_portfolio(n_layers: int = 8, elt_lo: int = 4, elt_hi: int = 32,
                         n_catalogue: int = 100_000, rows: int = 20_000,
                         seed: int = SEED_TERMS, su: bool = True) -> Portfolio:
    """Precision-study portfolio: 8 layers, ELT counts uniform on [4, 32],
    per-layer terms log-uniform on [1e5, 1e9]; ELTs follow the full-shape law."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    layers = []
    eid = 0
    for _ in range(n_layers):
        n = int(rng.integers(elt_lo, elt_hi + 1))
        occr, occl, aggr, aggl = random_layer_terms(rng)
        elts = []
        for _ in range(n):
            elts.append(make_elt(eid, rows, n_catalogue, SEED_ELT_BASE + eid,
                                 retention=1e6, limit=5e7, share=1.0))
            eid += 1
        layers.append(Layer(elts=elts, occ_retention=occr, occ_limit=occl,
                            agg_retention=aggr, agg_limit=aggl))
    return Portfolio(layers=layers, seed=SEED_PHILOX, su_enabled=su)


def random_portfolio(rng: np.random.Generator, layer_lo: int, layer_hi: int,
                     elt_lo: int, elt_hi: int, rows_lo: int, rows_hi: int,
                     n_catalogue: int, elt_id_base: int, su: bool = True,
                     seed: int = SEED_PHILOX) -> Portfolio:
    """Batched / served portfolios: uniform layer and ELT counts, ELT row counts
    log-uniform on [rows_lo, rows_hi], layer terms log-uniform on [1e5, 1e9]."""
    n_layers = int(rng.integers(layer_lo, layer_hi + 1))
    layers = []
    eid = elt_id_base
    for _ in range(n_layers):
        n = int(rng.integers(elt_lo, elt_hi + 1))
        occr, occl, aggr, aggl = random_layer_terms(rng)
        elts = []
        for _ in range(n):
            nr = int(round(float(_log_uniform(rng, rows_lo, rows_hi))))
            nr = max(1, min(n_catalogue, nr))
            elts.append(make_elt(eid, nr, n_catalogue, SEED_ELT_BASE + eid,
                                 retention=1e6, limit=5e7, share=1.0))
            eid += 1
        layers.append(Layer(elts=elts, occ_retention=occr, occ_limit=occl,
                            agg_retention=aggr, agg_limit=aggl))
    return Portfolio(layers=layers, seed=seed, su_enabled=su)


def batched_portfolios(n: int = 64, n_catalogue: int = 100_000, seed: int = 4,
                       layer_hi: int = 16, elt_hi: int = 48, rows_lo: int = 1_000,
                       rows_hi: int = 50_000, su: bool = True) -> List[Portfolio]:
    """64 portfolios: layers uniform 1-16, ELTs per layer uniform 2-48, rows
    log-uniform 1,000-50,000 over a 100,000-event catalogue."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    out = []
    base = 0
    for _ in range(n):
        pf = random_portfolio(rng, 1, layer_hi, 2, elt_hi, rows_lo, rows_hi,
                              n_catalogue, base, su=su)
        base += pf.n_elts
        out.append(pf)
    return out


@dataclass
class Request:
    portfolio: Portfolio
    trial_begin: int
    trial_count: int


def served_requests(n: int, n_trials: int, n_distinct: int = 32, n_catalogue: int = 100_000,
                    seed: int = 5, sub_lo: int = 10_000, sub_hi: int = 1_000_000,
                    su: bool = True) -> List[Request]:
    """Serving workload: n requests cycling over n_distinct portfolios (layers
    uniform 1-8, ELTs per layer uniform 2-32, rows log-uniform 1,000-50,000);
    each request prices a contiguous trial range whose length is log-uniform on
    [sub_lo, sub_hi] (clipped to the YET) with a uniformly random start."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    pfs = []
    base = 0
    for _ in range(n_distinct):
        pf = random_portfolio(rng, 1, 8, 2, 32, 1_000, 50_000, n_catalogue, base, su=su)
        base += pf.n_elts
        pfs.append(pf)
    out = []
    for i in range(n):
        c = int(round(float(_log_uniform(rng, sub_lo, sub_hi))))
        c = max(1, min(n_trials, c))
        b = int(rng.integers(0, n_trials - c + 1))
        out.append(Request(portfolio=pfs[int(rng.integers(0, n_distinct))], trial_begin=b,
                           trial_count=c))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 6) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed])))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
