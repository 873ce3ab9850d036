"""Pins of the FP64 oracle against things other than itself.

Each test names what fixes the expected value: the paper's formulas worked by
hand (section 2.2 terms), closed forms, exact rational brute force, library
special functions (scipy, mpmath, statistics), rocRAND's Philox engine, and
invariants of the method.  No expected value comes from the GPU library.
"""
import json
import math
import statistics
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sp
import scipy.stats as st

import oracle as O
from tests.tiny import (GOLDEN, A, B, elt_from_dict, golden_worked_cases, random_tiny_case, worked_example,
                        yet_from_lists)
from workloads import INF, Layer, Portfolio, config_small, make_yet

# --------------------------------------------------------------------------
# independent brute-force references written from the paper (section 2.2)
# --------------------------------------------------------------------------


def _F(x):
    return None if math.isinf(x) else Fraction(x)


def _clamp(x, ret, lim):
    """min(max(x - ret, 0), lim) with lim = None meaning no limit."""
    v = x - ret
    if v < 0:
        v = Fraction(0)
    if lim is not None and v > lim:
        v = lim
    return v


def frac_ara(yet, pf, loss_fn=None):
    """Algorithm 1 in exact rational arithmetic.  loss_fn(elt, row, k, i) gives
    the (secondary-uncertainty) loss of a hit, default the mean."""
    out = []
    gross = []
    views = []
    for layer in pf.layers:
        tabs = []
        for elt in layer.elts:
            tabs.append({int(e): r for r, e in enumerate(elt.event_ids)})
        occR, occL = _F(layer.occ_retention), _F(layer.occ_limit)
        aggR, aggL = _F(layer.agg_retention), _F(layer.agg_limit)
        ys, gs, vs = [], [], []
        for i in range(yet.n_trials):
            S = Fraction(0)
            A_prev = Fraction(0)
            G = Fraction(0)
            for k, E in enumerate(yet.event_ids[yet.offsets[i]:yet.offsets[i + 1]]):
                X = Fraction(0)
                for elt, tab in zip(layer.elts, tabs):
                    r = tab.get(int(E))
                    if r is None:
                        continue
                    loss = (Fraction(float(elt.mean[r])) if loss_fn is None
                            else loss_fn(elt, r, k, i))
                    X += Fraction(elt.share) * _clamp(loss, Fraction(elt.retention),
                                                      _F(elt.limit))
                G += X
                S += _clamp(X, occR, occL)
                Acur = _clamp(S, aggR, aggL)
                vs.append(Acur - A_prev)
                A_prev = Acur
            ys.append(A_prev)
            gs.append(G)
        out.append(ys)
        gross.append(gs)
        views.append(vs)
    return out, gross, views


# --------------------------------------------------------------------------
# P1: the hand-worked example
# --------------------------------------------------------------------------
def test_worked_example_exact():
    # X = [2.9e6 + 0.9e6, 0.4e6, 3.8e6]; O = X - 1e6 clipped at 0:
    # [2.8e6, 0, 2.8e6]; S = [2.8e6, 2.8e6, 5.6e6]; A = S - 5e6 clipped:
    # [0, 0, 0.6e6] -> Y = 6.0e5, G = 8.0e6, d = [0, 0, 6e5].
    yet, pf = worked_example()
    r = O.run_ara(yet, pf, occ_view=True)
    assert r["ylt"][0, 0] == 6.0e5
    assert r["gross"][0, 0] == 8.0e6
    assert list(r["occ_view"][0]) == [0.0, 0.0, 6.0e5]
    assert r["hits"][0, 0] == 5                      # A hits both ELTs (x2), B hits ELT1
    assert r["ylt_pf"][0] == 6.0e5


def test_worked_example_variants():
    yet, pf = worked_example(agg_limit=5e5)          # aggregate limit binds
    assert O.run_ara(yet, pf)["ylt"][0, 0] == 5.0e5
    # ELT1 share 0.5: X_A = 0.5*2.9e6 + 0.9e6 = 2.35e6 -> O = 1.35e6 twice;
    # S = 2.7e6 < AggR -> Y = 0
    yet, pf = worked_example(share1=0.5)
    r = O.run_ara(yet, pf, occ_view=True)
    assert r["ylt"][0, 0] == 0.0
    assert r["gross"][0, 0] == 2.35e6 * 2 + 0.2e6
    yet, pf = worked_example(trials=[[B], [], [A, A, A], [A, B, A]])
    r = O.run_ara(yet, pf)
    # [B]: X = 4e5 < OccR -> 0; []: 0; [A,A,A]: S = 8.4e6 -> 3.4e6
    assert list(r["ylt"][0]) == [0.0, 0.0, 3.4e6, 6.0e5]


def test_worked_example_golden_fixture():
    """Every case of the hand-worked fixture, exactly (all values are dyadic
    multiples of 1e5, so FP64 reaches them without rounding), and the exact
    rational brute force agrees."""
    n = 0
    for name, yet, pf, ex in golden_worked_cases():
        r = O.run_ara(yet, pf, occ_view=True)
        assert r["ylt"][0].tolist() == ex["ylt"], name
        assert r["gross"][0].tolist() == ex["gross"], name
        assert r["hits"][0].tolist() == ex["hits"], name
        assert r["occ_view"][0].tolist() == ex["occ_view"], name
        ys, gs, vs = frac_ara(yet, pf)
        assert [float(v) for v in ys[0]] == ex["ylt"], name
        assert [float(v) for v in vs[0]] == ex["occ_view"], name
        n += 1
    assert n == 4


# --------------------------------------------------------------------------
# P2: closed form -- no SU, zero retentions, no limits, unit shares
# --------------------------------------------------------------------------
def test_closed_form_sum_of_means():
    w = config_small(n_trials=400)
    pf = w.portfolio
    pf.su_enabled = False
    for layer in pf.layers:
        layer.occ_retention, layer.occ_limit = 0.0, INF
        layer.agg_retention, layer.agg_limit = 0.0, INF
        for e in layer.elts:
            e.retention, e.limit, e.share = 0.0, INF, 1.0
    r = O.run_ara(w.yet, pf)
    dense = np.zeros(w.yet.n_catalogue, np.float64)
    for e in pf.layers[0].elts:
        np.add.at(dense, e.event_ids, e.mean.astype(np.float64))
    per_occ = dense[w.yet.event_ids]
    expect = np.add.reduceat(np.append(per_occ, 0.0), w.yet.offsets[:-1])
    expect[np.diff(w.yet.offsets) == 0] = 0.0
    np.testing.assert_allclose(r["ylt"][0], expect, rtol=1e-13, atol=0)
    np.testing.assert_allclose(r["gross"][0], expect, rtol=1e-13, atol=0)


# --------------------------------------------------------------------------
# P3: exact rational brute force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(8))
def test_fraction_brute_force_dyadic_exact(seed):
    rng = np.random.default_rng(seed)
    yet, pf = random_tiny_case(rng, dyadic=True)
    r = O.run_ara(yet, pf, occ_view=True)
    ys, gs, vs = frac_ara(yet, pf)
    for l in range(len(pf.layers)):
        assert [Fraction(v) for v in r["ylt"][l]] == ys[l]
        assert [Fraction(v) for v in r["gross"][l]] == gs[l]
        assert [Fraction(v) for v in r["occ_view"][l]] == vs[l]
    tot = [sum(ys[l][i] for l in range(len(pf.layers))) for i in range(yet.n_trials)]
    assert [Fraction(v) for v in r["ylt_pf"]] == tot


@pytest.mark.parametrize("seed", range(8))
def test_fraction_brute_force_general(seed):
    rng = np.random.default_rng(100 + seed)
    yet, pf = random_tiny_case(rng, dyadic=False)
    r = O.run_ara(yet, pf)
    ys, gs, _ = frac_ara(yet, pf)
    for l in range(len(pf.layers)):
        exp_g = np.array([float(g) for g in gs[l]])
        exp_y = np.array([float(y) for y in ys[l]])
        # FP64 rounding enters at the gross scale (every clamp is 1-Lipschitz)
        assert np.all(np.abs(r["ylt"][l] - exp_y) <= 1e-14 * exp_g + 1e-300)
        np.testing.assert_allclose(r["gross"][l], exp_g, rtol=1e-14)


# --------------------------------------------------------------------------
# SU brute force: rocRAND Philox + mpmath Beta quantile + exact terms
# --------------------------------------------------------------------------
def _mp_quantile(a, b, z):
    """40-digit root of I_x(a,b) = z (bracketed; solved on the side where the
    root is small, through I_{1-x}(b,a) = 1 - z when z > 1/2)."""
    mp.mp.dps = 40
    a, b, z = mp.mpf(a), mp.mpf(b), mp.mpf(z)
    if z > mp.mpf(1) / 2:
        return 1 - _mp_quantile(b, a, 1 - z)
    y0 = float(sp.betaincinv(float(a), float(b), float(z)))
    f = lambda x: mp.betainc(a, b, 0, x, regularized=True) - z   # noqa: E731
    lo, hi = mp.mpf(y0) * (1 - mp.mpf("1e-6")), mp.mpf(y0) * (1 + mp.mpf("1e-6"))
    hi = min(hi, mp.mpf(1) - mp.mpf(10) ** -30)
    assert f(lo) < 0 < f(hi)
    return mp.findroot(f, (lo, hi), solver="anderson", tol=mp.mpf(10) ** -35)


def _mp_fit(mu, sigma, mx):
    mp.mp.dps = 40
    mu_b = mp.mpf(mu) / mp.mpf(mx)
    s_b = mp.mpf(sigma) / mp.mpf(mx)
    s_max = mp.sqrt(mu_b * (1 - mu_b))
    if s_b >= s_max:
        s_b = (1 - mp.mpf("1e-6")) * s_max
    kappa = (s_max / s_b) ** 2 - 1
    return mu_b * kappa, (1 - mu_b) * kappa


def _mp_u(word):
    return mp.mpf(int((int(word) >> 8) | 1)) / mp.mpf(2) ** 24


@pytest.mark.parametrize("corr,keying", [(False, 0), (True, 0), (False, 1), (True, 1)])
def test_su_brute_force_mpmath(rocrand_philox, corr, keying):
    rng = np.random.default_rng(7 + corr)
    yet, pf = random_tiny_case(rng, n_cat=10, n_layers=2, max_elts=3, max_occ=5, n_trials=6,
                               dyadic=False, su=True, corr=corr)
    pf.keying = keying
    program = {}
    for li, layer in enumerate(pf.layers):
        layer.program_id = 11 + li
        for e in layer.elts:
            program[e.elt_id] = layer.program_id
    # keep every row away from the sigma cap so the mpmath root solve is tame
    for layer in pf.layers:
        for e in layer.elts:
            e.max_loss = (e.mean * np.float32(4.0)).astype(np.float32)
            e.sigma_i = np.minimum(e.sigma_i, e.mean * np.float32(0.6)).astype(np.float32)
            e.sigma_c = np.minimum(e.sigma_c, e.mean * np.float32(0.3)).astype(np.float32)
    seed = pf.seed
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)

    def word(k, i, c2, s):
        return int(rocrand_philox(np.array([[k, i, c2, s]], np.uint32), key)[0, 0])

    def loss_fn(elt, r, k, i):
        mu, si, sc, mx = (float(elt.mean[r]), float(elt.sigma_i[r]), float(elt.sigma_c[r]),
                          float(elt.max_loss[r]))
        if si + sc == 0.0:
            return Fraction(mu)
        mp.mp.dps = 40
        # section 3.1 (i) / (ii): the independent and the correlated uniform
        if keying == 0:
            cI, cC = (k, i, elt.elt_id, 0), (k, i, 0, 1)
        else:
            cI, cC = (k, i, program[elt.elt_id], 2), (int(elt.event_ids[r]), 0, 0, 3)
        if sc == 0.0:
            z = _mp_u(word(*cI))
        elif si == 0.0:
            z = _mp_u(word(*cC))
        else:
            u1, u2 = _mp_u(word(*cI)), _mp_u(word(*cC))
            v1 = mp.sqrt(2) * mp.erfinv(2 * u1 - 1)
            v2 = mp.sqrt(2) * mp.erfinv(2 * u2 - 1)
            s = mp.mpf(si) + mp.mpf(sc)
            wi, wc = mp.mpf(si) / s, mp.mpf(sc) / s
            v = (v1 * wi + v2 * wc) / mp.sqrt(wi ** 2 + wc ** 2)
            z = mp.ncdf(v)
        a, b = _mp_fit(mu, si + sc, mx)
        x = _mp_quantile(a, b, z)
        return Fraction(str(mp.nstr(mp.mpf(mx) * x, 30)))

    r = O.run_ara(yet, pf)
    ys, gs, _ = frac_ara(yet, pf, loss_fn)
    for l in range(len(pf.layers)):
        exp_y = np.array([float(y) for y in ys[l]])
        exp_g = np.array([float(g) for g in gs[l]])
        assert np.all(np.abs(r["ylt"][l] - exp_y) <= 1e-11 * exp_g + 1e-300), (r["ylt"][l], exp_y)
        np.testing.assert_allclose(r["gross"][l], exp_g, rtol=1e-11)


# --------------------------------------------------------------------------
# P4: invariants
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_su():
    w = config_small(n_trials=600)
    return w, O.run_ara(w.yet, w.portfolio, occ_view=True)


def test_invariants_bounds(small_su):
    w, r = small_su
    layer = w.portfolio.layers[0]
    y, g = r["ylt"][0], r["gross"][0]
    assert np.all(y >= 0) and np.all(y <= layer.agg_limit)
    assert np.all(y <= g + 1e-6)
    # Y = 0 when the occurrence losses never exceed the aggregate retention
    d = r["occ_view"][0]
    sums = np.add.reduceat(np.append(d, 0.0), w.yet.offsets[:-1])
    sums[np.diff(w.yet.offsets) == 0] = 0.0
    np.testing.assert_allclose(sums, y, rtol=1e-12, atol=1e-6)        # sum_k d_k = Y
    assert np.all(d >= 0) and np.all(d <= layer.agg_limit)


def test_invariants_monotone_in_terms(small_su):
    w, r = small_su
    base = r["ylt"][0]
    layer = w.portfolio.layers[0]
    for attr, factor, sign in [("occ_retention", 2.0, -1), ("agg_retention", 2.0, -1),
                               ("occ_limit", 0.1, -1), ("agg_limit", 0.05, -1)]:
        old = getattr(layer, attr)
        setattr(layer, attr, old * factor)
        y2 = O.run_ara(w.yet, w.portfolio)["ylt"][0]
        setattr(layer, attr, old)
        assert np.all(sign * (y2 - base) >= -1e-6), attr
        assert np.any(y2 != base), attr
    e0 = layer.elts[0]
    for attr, factor in [("retention", 3.0), ("limit", 0.3), ("share", 0.5)]:
        old = getattr(e0, attr)
        setattr(e0, attr, old * factor)
        y2 = O.run_ara(w.yet, w.portfolio)["ylt"][0]
        setattr(e0, attr, old)
        assert np.all(y2 <= base + 1e-6), attr


def test_invariants_permutations_and_slices(small_su):
    w, r = small_su
    yet, pf = w.yet, w.portfolio
    # slicing is bit-for-bit: trial results depend on the absolute index only
    a = O.run_ara(yet, pf, 0, 250)
    b = O.run_ara(yet, pf, 250, 350)
    assert np.array_equal(np.concatenate([a["ylt"], b["ylt"]], axis=1), r["ylt"])
    sel = [599, 3, 77, 3]
    c = O.run_ara(yet, pf, trials=sel)
    assert np.array_equal(c["ylt"][0], r["ylt"][0][sel])
    # permuting the ELT list changes only the rounding of the cross-ELT sum
    pf2 = Portfolio(layers=[Layer(elts=pf.layers[0].elts[::-1],
                                  occ_retention=pf.layers[0].occ_retention,
                                  occ_limit=pf.layers[0].occ_limit,
                                  agg_retention=pf.layers[0].agg_retention,
                                  agg_limit=pf.layers[0].agg_limit)],
                    seed=pf.seed, su_enabled=True)
    y2 = O.run_ara(yet, pf2)["ylt"][0]
    assert np.all(np.abs(y2 - r["ylt"][0]) <= 1e-12 * r["gross"][0] + 1e-9)
    # an ELT with no rows is a no-op
    empty = elt_from_dict(99, {})
    pf3 = Portfolio(layers=[Layer(elts=pf.layers[0].elts + [empty],
                                  occ_retention=pf.layers[0].occ_retention,
                                  occ_limit=pf.layers[0].occ_limit,
                                  agg_retention=pf.layers[0].agg_retention,
                                  agg_limit=pf.layers[0].agg_limit)],
                    seed=pf.seed, su_enabled=True)
    assert np.array_equal(O.run_ara(yet, pf3)["ylt"][0], r["ylt"][0])


def test_invariants_occurrence_order_pu():
    # without secondary uncertainty, re-ordering the occurrences of a trial
    # leaves the trial loss unchanged up to rounding (the occurrence losses
    # are non-negative and the aggregate clamp is monotone)
    rng = np.random.default_rng(5)
    yet, pf = random_tiny_case(rng, dyadic=True, n_trials=30)
    r1 = O.run_ara(yet, pf)
    trials = [list(yet.event_ids[yet.offsets[i]:yet.offsets[i + 1]])[::-1]
              for i in range(yet.n_trials)]
    r2 = O.run_ara(yet_from_lists(trials, yet.n_catalogue), pf)
    assert np.array_equal(r1["ylt"], r2["ylt"])


# --------------------------------------------------------------------------
# P5 / P6 / P7 / P13: the Beta quantile and the normal functions
# --------------------------------------------------------------------------
GRID_U = (np.array([1, 3, 1001, 2 ** 20 + 1, 2 ** 22 + 5, 2 ** 23 - 1, 2 ** 23 + 1,
                    2 ** 24 - 2 ** 21 + 1, 2 ** 24 - 1001, 2 ** 24 - 3, 2 ** 24 - 1],
                   np.float64) / 2.0 ** 24)


@pytest.mark.parametrize("mu_b,var_b,exact", [
    (0.5, 1.0 / 12.0, lambda z: z),                                   # Beta(1,1)
    (1.0 / 3.0, 1.0 / 18.0, lambda z: z / (1.0 + np.sqrt(1.0 - z))),  # Beta(1,2): 1-sqrt(1-z)
    (2.0 / 3.0, 1.0 / 18.0, lambda z: np.sqrt(z)),                    # Beta(2,1)
    (0.5, 1.0 / 8.0, lambda z: np.sin(np.pi * z / 2.0) ** 2),         # Beta(1/2,1/2)
])
def test_beta_closed_forms_via_moment_fit(mu_b, var_b, exact):
    a, b = O.beta_fit(mu_b, math.sqrt(var_b), 1.0)
    x = O.betaincinv(a, b, GRID_U)
    np.testing.assert_allclose(x, exact(GRID_U), rtol=1e-12, atol=1e-300)


def test_uniform_shape_whole_chain():
    # (mu_b, var_b) = (1/2, 1/12) fits Beta(1,1): the loss is max_l * u exactly
    # for the draw u of the hit, which pins draw -> fit -> quantile -> scale.
    n = 2000
    k = np.arange(n, dtype=np.uint32)
    i = (np.arange(n, dtype=np.uint32) * 7 + 3).astype(np.uint32)
    e = np.full(n, 5, np.uint32)
    seed = 424242
    mx = 4.0
    loss = O.su_loss(2.0, 4.0 * math.sqrt(1 / 12.0), 0.0, mx, k, i, e, seed)
    u = O.draw_u(np.stack([k, i, e, np.zeros(n, np.uint32)], 1), seed)
    np.testing.assert_allclose(loss, mx * u, rtol=1e-12)


def test_beta_symmetry_on_grid():
    for a, b in [(2.75, 8.25), (0.3, 4.0), (40.0, 3.5), (0.5, 0.5)]:
        x1 = O.betaincinv(a, b, GRID_U)
        x2 = O.betaincinv(b, a, 1.0 - GRID_U)
        np.testing.assert_allclose(x1, 1.0 - x2, rtol=1e-13, atol=1e-16)


SHAPES = [(2.75, 8.25), (1.0, 1.0), (0.5, 0.5), (0.1, 0.3), (0.7, 5.0), (5.0, 0.7),
          (30.0, 70.0), (300.0, 100.0), (1.5, 1500.0), (1e-3, 2e-3)]


@pytest.mark.parametrize("a,b", SHAPES)
def test_betaincinv_vs_scipy(a, b):
    z = np.concatenate([GRID_U, np.linspace(0.01, 0.99, 41)])
    x = O.betaincinv(a, b, z)
    ref = sp.betaincinv(a, b, z)
    ok = ref > 1e-290
    np.testing.assert_allclose(x[ok], ref[ok], rtol=5e-12)
    # re-evaluating I at the root: only where x carries full relative precision
    low = ok & (z <= 0.5)
    I = O.betainc(a, b, x)
    np.testing.assert_allclose(I[low], z[low], rtol=1e-11)
    np.testing.assert_allclose(O.betainc(a, b, np.linspace(0.001, 0.999, 50)),
                               sp.betainc(a, b, np.linspace(0.001, 0.999, 50)), rtol=1e-12,
                               atol=1e-300)


@pytest.mark.parametrize("a,b", [(2.75, 8.25), (0.5, 0.5), (0.7, 5.0), (30.0, 70.0)])
def test_betaincinv_vs_mpmath_paper_criterion(a, b):
    """Section 5.1 states convergence at relative error < 1e-6; the oracle is
    held to 1e-12 against 40-digit mpmath (which also meets the paper's)."""
    zs = [2.0 ** -24, 0.001, 0.05, 0.3, 0.5, 0.7, 0.95, 0.999, 1 - 2.0 ** -24]
    for z in zs:
        ref = _mp_quantile(a, b, z)
        x = O.betaincinv(a, b, z)[0]
        rel = abs(mp.mpf(x) - ref) / ref
        assert rel < 1e-12, (a, b, z, rel)


def test_normal_functions_vs_libraries():
    assert abs(O.norm_quantile([0.975])[0] - 1.959963984540054) < 1e-15
    p = np.concatenate([GRID_U, np.linspace(0.001, 0.999, 99)])
    np.testing.assert_allclose(O.norm_quantile(p), sp.ndtri(p), rtol=1e-13, atol=1e-15)
    nd = statistics.NormalDist()
    for q in [1e-7, 0.01, 0.3, 0.8, 0.9999]:
        assert abs(O.norm_quantile([q])[0] - nd.inv_cdf(q)) < 1e-12
    x = np.linspace(-8, 8, 161)
    # deep-tail erfc amplifies the rounding of -x/sqrt(2) by ~x^2: 5e-14 at |x| = 8
    np.testing.assert_allclose(O.norm_cdf(x), sp.ndtr(x), rtol=5e-14, atol=0)


# --------------------------------------------------------------------------
# P8: the moment fit reproduces the row's mean and variance
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mu,sigma,mx", [(1.0, 0.5, 4.0), (3.0, 0.4, 5.0), (0.2, 0.15, 1.0)])
def test_moment_fit_statistics(mu, sigma, mx):
    n = 200_000
    k = (np.arange(n) % 1000).astype(np.uint32)
    i = (np.arange(n) // 1000).astype(np.uint32)
    loss = O.su_loss(mu, sigma, 0.0, mx, k, i, np.full(n, 11, np.uint32), 99)
    se = sigma / math.sqrt(n)
    assert abs(loss.mean() - mu) < 4.0 * se
    # sample variance within a 4-sigma band of its sampling distribution
    m4 = np.mean((loss - mu) ** 4)
    se_var = math.sqrt((m4 - sigma ** 4) / n)
    assert abs(loss.var() - sigma ** 2) < 4.0 * se_var
    assert loss.min() >= 0 and loss.max() <= mx


# --------------------------------------------------------------------------
# P9 / P10: the two extreme cases and the correlation structure
# --------------------------------------------------------------------------
def test_extreme_cases_short_circuit():
    n = 500
    k = np.arange(n, dtype=np.uint32)
    i = np.full(n, 17, np.uint32)
    e = np.full(n, 3, np.uint32)
    seed = 5
    a, b = O.beta_fit(1.0, 0.5, 4.0)
    uI = O.draw_u(np.stack([k, i, e, np.zeros(n, np.uint32)], 1), seed)
    uC = O.draw_u(np.stack([k, i, np.zeros(n, np.uint32), np.ones(n, np.uint32)], 1), seed)
    l1 = O.su_loss(1.0, 0.5, 0.0, 4.0, k, i, e, seed)          # sigma_C = 0: z = u_I
    assert np.array_equal(l1, 4.0 * O.betaincinv(a, b, uI))
    l2 = O.su_loss(1.0, 0.0, 0.5, 4.0, k, i, e, seed)          # sigma_I = 0: z = u_C
    assert np.array_equal(l2, 4.0 * O.betaincinv(a, b, uC))
    l3 = O.su_loss(1.0, 0.0, 0.0, 4.0, k, i, e, seed)          # sigma = 0: the mean
    assert np.all(l3 == 1.0)


def test_paper_keying_draws(rocrand_philox):
    """Section 3.1 keying: z_(Prog,E) is shared by every ELT of a program for
    one occurrence and differs across programs; z_(E) is fixed per event.
    With the Beta(1,1) moment fit the loss is max_l * z, so each hit's loss
    shows its draw; the draws come from rocRAND's Philox."""
    seed = 987654321
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)

    def u(c):
        w = int(rocrand_philox(np.array([c], np.uint32), key)[0, 0])
        return ((w >> 8) | 1) * 2.0 ** -24

    s1 = 4.0 * math.sqrt(1 / 12.0)          # (mu, sigma, max) = (2, s1, 4) fits Beta(1, 1)
    for k, i, ev in [(0, 0, 3), (5, 17, 3), (2, 99, 41)]:
        for prog in (0, 7, 8):
            ref = 4.0 * u((k, i, prog, 2))
            for elt in (1, 5, 900):
                got = O.su_loss_keyed(2.0, s1, 0.0, 4.0, k, i, elt, prog, ev, 1, seed)
                assert abs(got - ref) <= 1e-12 * ref
        # the correlated-only draw depends on the event alone
        refc = 4.0 * u((ev, 0, 0, 3))
        for kk, ii, elt, prog in [(k, i, 1, 0), (k + 1, i + 3, 9, 4)]:
            got = O.su_loss_keyed(2.0, 0.0, s1, 4.0, kk, ii, elt, prog, ev, 1, seed)
            assert abs(got - refc) <= 1e-12 * refc
    # the default keying ignores program and event
    a = O.su_loss_keyed(2.0, s1, 0.0, 4.0, 3, 4, 5, 0, 0, 0, seed)
    b = O.su_loss_keyed(2.0, s1, 0.0, 4.0, 3, 4, 5, 9, 77, 0, seed)
    assert a == b and abs(a - 4.0 * u((3, 4, 5, 0))) <= 1e-12 * a


def test_correlation_structure():
    n = 100_000
    k = (np.arange(n) % 1000).astype(np.uint32)
    i = (np.arange(n) // 1000).astype(np.uint32)
    mu, s, mx = 1.0, 0.25, 4.0       # sigma_I = sigma_C = 0.25: sigma = 0.5
    a, b = O.beta_fit(mu, 2 * s, mx)
    l1 = O.su_loss(mu, s, s, mx, k, i, np.full(n, 1, np.uint32), 8)
    l2 = O.su_loss(mu, s, s, mx, k, i, np.full(n, 2, np.uint32), 8)
    z1 = sp.betainc(a, b, l1 / mx)
    z2 = sp.betainc(a, b, l2 / mx)
    assert st.kstest(z1, "uniform").pvalue > 1e-4
    v1, v2 = sp.ndtri(z1), sp.ndtri(z2)
    rho = np.corrcoef(v1, v2)[0, 1]
    # corr = sigma_C^2 / (sigma_I^2 + sigma_C^2) = 1/2, standard error ~ 1/sqrt(n)
    assert abs(rho - 0.5) < 5.0 / math.sqrt(n)
    assert abs(v1.std() - 1.0) < 0.02


# --------------------------------------------------------------------------
# P11: Philox against rocRAND, uniformity of u
# --------------------------------------------------------------------------
def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2 ** 32, size=(200_000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1000] = 0
    ctr[:1000, 0] = np.arange(1000)
    for key in ([0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [150106326, 0], [0x12345678, 0x9ABCDEF0]):
        key = np.array(key, np.uint32)
        assert np.array_equal(O.philox4x32_10(ctr, key), rocrand_philox(ctr, key))


def test_uniform_mapping_and_chi2():
    assert O.u01(0) == 2.0 ** -24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert O.u01(0x100) == 2.0 ** -24 and O.u01(0x200) == 3.0 * 2.0 ** -24
    n = 1_000_000
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n) % 1000
    ctr[:, 1] = np.arange(n) // 1000
    u = O.draw_u(ctr, 150106326)
    assert np.all((u > 0) & (u < 1))
    hist = np.bincount(np.minimum((u * 256).astype(int), 255), minlength=256)
    chi2 = ((hist - n / 256) ** 2 / (n / 256)).sum()
    assert st.chi2.sf(chi2, 255) > 1e-4
    # the grid is symmetric: 1 - u is again an odd multiple of 2^-24
    assert np.all(((1.0 - u) * 2 ** 24) % 2 == 1)


# --------------------------------------------------------------------------
# P12: PML / TVaR brute force
# --------------------------------------------------------------------------
def _bf_pml_tvar(y, rp):
    s = sorted(y, reverse=True)
    k = max(1, int(math.floor(len(y) / rp)))
    return s[k - 1], math.fsum(s[:k]) / k


@pytest.mark.parametrize("case", ["random", "ties", "zeros", "small_n"])
def test_pml_tvar_brute_force(case):
    rng = np.random.default_rng(3)
    if case == "random":
        y = rng.lognormal(14, 2, size=10_000)
    elif case == "ties":
        y = np.repeat(rng.lognormal(14, 2, size=50), 200)
    elif case == "zeros":
        y = np.zeros(1000)
    else:
        y = rng.lognormal(14, 2, size=57)
    rps = [100.0, 250.0, 2.0, 1.0, 1e9]
    pml, tvar = O.pml_tvar(y, rps)
    for j, rp in enumerate(rps):
        p, t = _bf_pml_tvar(list(y), rp)
        assert pml[j] == p
        assert abs(tvar[j] - t) <= 1e-15 * abs(t)


@pytest.mark.parametrize("case", ["random", "ties", "zeros", "tiny"])
def test_ep_curve_exact(case):
    """EP curve: descending order and running means against exact rational
    arithmetic, and agreement with the independent C PML / TVaR."""
    from fractions import Fraction
    rng = np.random.default_rng(4)
    if case == "random":
        y = rng.lognormal(14, 2, size=3000)
    elif case == "ties":
        y = np.repeat(rng.lognormal(14, 2, size=30), 40)
    elif case == "zeros":
        y = np.array([0.0, -0.0, 0.0, 5.0])
    else:
        y = rng.lognormal(3, 1, size=7)
    srt, tm = O.ep_curve(y)
    ref = sorted([float(v) for v in y], reverse=True)
    assert [float(v) for v in srt] == ref
    assert np.all(np.signbit(srt) == False)          # noqa: E712  (-0.0 folded)
    run = Fraction(0)
    for j, v in enumerate(ref):
        run += Fraction(v)
        exact = run / (j + 1)
        assert abs(Fraction(float(tm[j])) - exact) <= Fraction(1, 10 ** 15) * abs(exact)
    assert np.all(np.diff(srt) <= 0) and np.all(tm[:-1] >= tm[1:] - 1e-9 * tm[1:])
    rps = [1.0, 2.0, 10.0, 100.0, 1e9]
    pml, tvar = O.pml_tvar(y, rps)
    for j, rp in enumerate(rps):
        k = max(1, int(math.floor(len(y) / rp)))
        assert pml[j] == srt[k - 1]
        assert abs(tvar[j] - tm[k - 1]) <= 1e-15 * abs(tvar[j])


# --------------------------------------------------------------------------
# P14: hit counts of the direct-access lookups
# --------------------------------------------------------------------------
def test_hit_counts_and_checksum():
    w = config_small(n_trials=300)
    r = O.run_ara(w.yet, w.portfolio)
    member = np.zeros((3, w.yet.n_catalogue), bool)
    for j, e in enumerate(w.portfolio.layers[0].elts):
        member[j, e.event_ids] = True
    hits = np.zeros(w.yet.n_trials, np.int64)
    chk = np.zeros(w.yet.n_trials, np.uint64)
    for i in range(w.yet.n_trials):
        ev = w.yet.event_ids[w.yet.offsets[i]:w.yet.offsets[i + 1]]
        for j, e in enumerate(w.portfolio.layers[0].elts):
            ks = np.nonzero(member[j, ev])[0].astype(np.uint64)
            hits[i] += ks.size
            chk[i] += np.sum((ks + np.uint64(1)) * np.uint64(2654435761) + np.uint64(e.elt_id),
                             dtype=np.uint64)
    assert np.array_equal(r["hits"][0], hits)
    assert np.array_equal(r["hit_chk"][0], chk)


# --------------------------------------------------------------------------
# input generator properties (shared by both sides)
# --------------------------------------------------------------------------
def test_generator_properties():
    y1 = make_yet(20_000, 100.0, 10_000, 1501, threads=1)
    y2 = make_yet(20_000, 100.0, 10_000, 1501, threads=4)
    assert np.array_equal(y1.event_ids, y2.event_ids) and np.array_equal(y1.times, y2.times)
    assert y1.offsets[0] == 0 and np.all(np.diff(y1.offsets) >= 0)
    assert y1.event_ids.min() >= 0 and y1.event_ids.max() < 10_000
    for i in range(0, 20_000, 997):
        t = y1.times[y1.offsets[i]:y1.offsets[i + 1]]
        assert np.all(np.diff(t) >= 0) and (t.size == 0 or (t[0] >= 0 and t[-1] < 365))
    c = np.diff(y1.offsets)
    assert abs(c.mean() - 100) < 0.5 and abs(c.var() - 100) < 5
    w = config_small(n_trials=10)
    e = w.portfolio.layers[0].elts[0]
    assert e.n_rows == 2000 and np.unique(e.event_ids).size == 2000
    assert np.all(e.sigma_i == e.mean * np.float32(0.5))
    assert np.all(e.max_loss == e.mean * np.float32(4.0))
    assert abs(np.log(e.mean).mean() - 12) < 0.1 and abs(np.log(e.mean).std() - 1.5) < 0.1


# --------------------------------------------------------------------------
# regression guard (not a pin): the oracle's stored results on the small
# workload, written by tests/golden/make_oracle_small.py.  A change to the
# oracle's arithmetic shows here and must be justified before the file is
# rewritten.
# --------------------------------------------------------------------------
def test_oracle_matches_its_stored_small_results():
    with open(GOLDEN / "oracle_small.json") as f:
        doc = json.load(f)
    for case in doc["cases"]:
        w = config_small(corr=case["workload"].endswith("_corr"))
        assert w.name == case["workload"]
        r = O.run_ara(w.yet, w.portfolio)
        pml, tvar = O.pml_tvar(r["ylt_pf"], case["return_periods"])
        assert int(r["hits"].sum()) == case["hits"]
        assert int((r["ylt_pf"] > 0).sum()) == case["positive_trials"]
        np.testing.assert_allclose(pml, case["pml"], rtol=1e-12)
        np.testing.assert_allclose(tvar, case["tvar"], rtol=1e-12)
        np.testing.assert_allclose(r["ylt_pf"][:16], case["ylt_head"], rtol=1e-12)
        assert math.isclose(float(r["ylt_pf"].sum()), case["ylt_sum"], rel_tol=1e-12)


# --------------------------------------------------------------------------
# The sigma cap of section 3.3 and the near-Bernoulli shapes it produces
# --------------------------------------------------------------------------
# When sigma_b >= sigma_b,max = sqrt(mu_b (1 - mu_b)) the fit uses
# (1 - eps) sigma_b,max instead (eps = 1e-6, the reading of "a value very close
# to sigma_b,max").  Then (sigma_b,max / sigma_b)^2 - 1 = (1 - eps)^-2 - 1 for
# every capped row, so the fit is alpha = mu_b k, beta = (1 - mu_b) k with the
# single constant k below, whatever the row's mean, sigma or exposure; and a
# Beta(alpha, beta) has variance mu_b (1 - mu_b) / (alpha + beta + 1), which
# must equal the capped sigma_b squared.  Neither fact retypes the oracle's
# branch: the first is the cap's algebra done once in 50 digits, the second
# is the Beta distribution's variance.
def _kappa_eps():
    mp.mp.dps = 50
    return (1 - mp.mpf("1e-6")) ** -2 - 1


@pytest.mark.parametrize("mu,sigma,mx", [
    (2.0, 2.0, 4.0),          # sigma_b = sigma_b,max exactly (mu_b = 1/2): the cap applies
    (1.0, 3.0, 4.0),          # the sigma-capped test rows: sigma_I = 3 mean, max = 4 mean
    (0.1, 0.9, 1.0), (9.0, 5.0, 10.0), (1e6, 2.5e6, 3e6), (0.25, 2.0, 0.5)])
def test_sigma_cap_fit_closed_form(mu, sigma, mx):
    a, b = O.beta_fit(mu, sigma, mx)
    k = _kappa_eps()
    mu_b = mp.mpf(mu) / mp.mpf(mx)
    # FP64 forms k as the difference of (sigma_b,max / sigma_b)^2 ~ 1 + 2e-6 and
    # 1, which leaves about 1e-16 / 2e-6 = 5e-11 of relative precision; a slip
    # (the cap on sigma_b^2, '>' for '>=', another eps) moves k by O(1)
    tol = 1e-9
    assert abs(mp.mpf(a) - mu_b * k) <= tol * mu_b * k, (a, mu_b * k)
    assert abs(mp.mpf(b) - (1 - mu_b) * k) <= tol * (1 - mu_b) * k, (b, (1 - mu_b) * k)
    # the fitted Beta's standard deviation is the capped sigma_b
    var = mu_b * (1 - mu_b) / (mp.mpf(a) + mp.mpf(b) + 1)
    s_max = mp.sqrt(mu_b * (1 - mu_b))
    assert abs(mp.sqrt(var) / ((1 - mp.mpf("1e-6")) * s_max) - 1) < 1e-12


@pytest.mark.parametrize("mu,mx,below", [(2.0, 4.0, 1e-3), (1.0, 4.0, 1e-9), (0.3, 1.0, 0.25),
                                         (7.0, 8.0, 1e-5)])
def test_sigma_below_cap_keeps_moments(mu, mx, below):
    """Just below sigma_b,max no cap applies: the fit reproduces the row's
    mean and standard deviation (Beta mean alpha/(alpha+beta), variance
    mu_b (1-mu_b)/(alpha+beta+1))."""
    mp.mp.dps = 50
    mu_b = mp.mpf(mu) / mp.mpf(mx)
    s_max = mp.sqrt(mu_b * (1 - mu_b))
    sigma = float(s_max * (1 - mp.mpf(below)) * mp.mpf(mx))
    a, b = O.beta_fit(mu, sigma, mx)
    A_, B_ = mp.mpf(a), mp.mpf(b)
    assert abs(A_ / (A_ + B_) - mu_b) < 1e-12 * mu_b
    s_b = mp.mpf(sigma) / mp.mpf(mx)
    sd = mp.sqrt(mu_b * (1 - mu_b) / (A_ + B_ + 1))
    # the moment fit loses ~ eps / (1 - s_b/s_max) of relative precision
    assert abs(sd / s_b - 1) < 1e-15 / float(below) + 1e-13, (sd / s_b - 1)


def _near_bernoulli_shapes():
    k = float(_kappa_eps())
    out = [(mu_b * k, (1 - mu_b) * k) for mu_b in (0.25, 0.5, 0.1, 0.9)]
    return out + [(1e-3, 1e-3), (5e-4, 2e-3), (1e-3, 1e-2), (3e-3, 1e-4)]


def _grid_points(a, b):
    """Draw-grid values of z (odd multiples of 2^-24): spread over (0, 1),
    plus the narrow bands next to the mass split I_(1/2)(a, b) where the
    roots are representable doubles."""
    mp.mp.dps = 50
    ih = mp.betainc(a, b, 0, mp.mpf("0.5"), regularized=True)
    j = [1, 3, 101, 2 ** 20 + 1, 2 ** 22 + 1, 2 ** 23 - 1, 2 ** 23 + 1, 3 * 2 ** 22 + 1,
         2 ** 24 - 101, 2 ** 24 - 3, 2 ** 24 - 1]
    c = int(ih * 2 ** 24) | 1
    for d in (-40001, -4001, -401, -41, -5, -1, 1, 5, 41, 401, 4001, 40001):
        jj = c + 2 * d
        if 0 < jj < 2 ** 24:
            j.append(jj)
    return sorted(set(j))


@pytest.mark.parametrize("a,b", _near_bernoulli_shapes())
def test_betaincinv_near_bernoulli_brackets(a, b):
    """The oracle's Beta inverse at the near-Bernoulli shapes the cap makes
    (alpha, beta ~ 1e-6) and at alpha, beta ~ 1e-3, on the draw grid, against
    mpmath's 50-digit regularized incomplete beta, on the side where the root
    is at most 1/2 (the other side through I_(1-x)(b, a) = 1 - z).  Near 0,
    I_x ~ x^a / (a B(a, b)), so a relative change d of the root changes I by
    a d: the root itself is conditioned like 1/a (2e6 here) and FP64 cannot
    hold it to 1e-12.  What FP64 can hold is the backward error: I at the
    returned root must equal z to 1e-13 relative (the forward error is then
    at most 1e-13 / a).  Where the oracle returns an exact 0 the true root
    must lie below 1e-300 (I at 1e-300 already exceeds z)."""
    mp.mp.dps = 50
    js = np.array(_grid_points(a, b), np.float64)
    z = js / 2 ** 24
    zc = (2 ** 24 - js) / 2 ** 24
    x, xc = O.betaincinv(np.full(z.size, a), np.full(z.size, b), z, zc, complement=True)
    A_, B_ = mp.mpf(a), mp.mpf(b)
    n_inner = 0
    for zi, zci, xi, xci, ji in zip(z, zc, x, xc, js):
        Z, ZC = mp.mpf(int(ji)) / 2 ** 24, mp.mpf(2 ** 24 - int(ji)) / 2 ** 24
        if xi <= 0.5:
            s, t, S, T = A_, B_, Z, mp.mpf(xi)
        else:
            s, t, S, T = B_, A_, ZC, mp.mpf(xci)
        if T == 0:
            # below the smallest double: the root must be under 1e-300
            assert mp.betainc(s, t, 0, mp.mpf("1e-300"), regularized=True) >= S, (a, b, ji)
        else:
            back = abs(mp.betainc(s, t, 0, T, regularized=True) / S - 1)
            assert back < 1e-13, (a, b, ji, float(T), float(back))
            n_inner += 1
        assert abs(xi + xci - 1.0) <= 2.3e-16
    # the bands next to the mass split give roots inside the double range
    assert n_inner >= 4


def test_oracle_matches_its_stored_full_results():
    """tests/golden/oracle_full.json (written by make_oracle_full.py from the
    oracle and the input generators) still matches the oracle: a sample of
    its stored trials recomputed here, at 1e-12 of the trial's gross loss."""
    from pathlib import Path
    from workloads import config_full, full_portfolio
    gold = json.loads((Path(__file__).parent / "golden" / "oracle_full.json").read_text())
    w = config_full(n_trials=gold["n_trials"], with_times=False)
    assert w.yet.n_occ == gold["n_occurrences"]
    assert int(w.yet.event_ids.sum(dtype=np.int64)) == gold["event_id_sum"]
    for case, pf in (("su", w.portfolio), ("pu", full_portfolio(su=False))):
        g = gold["cases"][case]
        idx = g["top_index"][:40] + g["sample_index"][::100]
        ref_y = np.array(g["top_y"][:40] + g["sample_y"][::100])
        ref_g = np.array(g["top_gross"][:40] + g["sample_gross"][::100])
        r = O.run_ara(w.yet, pf, trials=idx)
        assert np.all(np.abs(r["ylt_pf"] - ref_y) <= 1e-12 * np.maximum(ref_g, 1.0))
        assert np.allclose(r["gross"][0], ref_g, rtol=1e-9)
    # the primary-uncertainty case looks up the same rows: equal lookup counts
    assert gold["cases"]["su"]["hits_total"] == gold["cases"]["pu"]["hits_total"]
    assert gold["cases"]["su"]["hit_chk_total"] == gold["cases"]["pu"]["hit_chk_total"]
