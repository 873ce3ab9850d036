"""FP64 CPU oracle for Aggregate Risk Analysis -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``ara_oracle.c`` (plain C, FP64, OpenMP over trials),
which follows the paper's definitions step by step and shares no code with the
GPU library.  See the header of ``ara_oracle.c`` for the readings it takes where
the paper is silent.

Parity is pinned by the tests in ``tests/test_oracle_*.py`` (closed forms,
exact rational brute force, library special functions, invariants and an
independent Philox implementation).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

from . import build as _build

_LIB = None

_i64 = C.c_int64
_i32 = C.c_int32
_u64 = C.c_uint64
_u32 = C.c_uint32
_dbl = C.c_double
_p = C.c_void_p


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_philox4x32_10.argtypes = [_p, _p, _p]
        L.orc_u01.argtypes = [_u32]
        L.orc_u01.restype = _dbl
        L.orc_norm_cdf.argtypes = [_dbl]
        L.orc_norm_cdf.restype = _dbl
        L.orc_norm_quantile.argtypes = [_dbl]
        L.orc_norm_quantile.restype = _dbl
        L.orc_betainc.argtypes = [_dbl, _dbl, _dbl]
        L.orc_betainc.restype = _dbl
        L.orc_betaincinv.argtypes = [_dbl, _dbl, _dbl]
        L.orc_betaincinv.restype = _dbl
        L.orc_beta_fit.argtypes = [_dbl, _dbl, _dbl, _p, _p]
        L.orc_su_loss.argtypes = [_dbl, _dbl, _dbl, _dbl, _u32, _u32, _u32, _u64]
        L.orc_su_loss.restype = _dbl
        L.orc_su_loss_keyed.argtypes = [_dbl, _dbl, _dbl, _dbl, _u32, _u32, _u32, _u32, _u32,
                                        _i32, _u64]
        L.orc_su_loss_keyed.restype = _dbl
        L.orc_ara_run.argtypes = [_i64, _i64, _p, _p, _i32, _i32, _p, _i32, _p, _p, _p, _p,
                                  _p, _p, _p, _p, _p, _u64, _i32, _i32, _p, _i32,
                                  _p, _p, _p, _p, _p, _p]
        L.orc_ara_run.restype = _i32
        L.orc_pml_tvar.argtypes = [_p, _i64, _p, _i32, _p, _p]
        L.orc_pml_tvar.restype = _i32
        L.orc_philox_batch.argtypes = [_i64, _p, _p, _p]
        L.orc_draw_u_batch.argtypes = [_i64, _p, _u64, _p]
        L.orc_betaincinv_batch.argtypes = [_i64, _p, _p, _p, _p, _p, _p]
        L.orc_betainc_batch.argtypes = [_i64, _p, _p, _p, _p, _p]
        L.orc_norm_batch.argtypes = [_i64, _p, _p, _p]
        L.orc_su_loss_batch.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _u64, _p]
        _LIB = L
    return _LIB


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# scalar / array special functions
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    key = _c(key, np.uint32).reshape(2)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def draw_u(ctr, seed: int) -> np.ndarray:
    """u = ((x0 >> 8) | 1) * 2^-24 of Philox(ctr, key = seed)."""
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    out = np.empty(ctr.shape[0], dtype=np.float64)
    lib().orc_draw_u_batch(ctr.shape[0], _ptr(ctr), int(seed), _ptr(out))
    return out


def u01(w: int) -> float:
    return lib().orc_u01(int(w))


def norm_cdf(x) -> np.ndarray:
    x = _c(x, np.float64).reshape(-1)
    out = np.empty_like(x)
    lib().orc_norm_batch(x.shape[0], _ptr(x), _ptr(out), None)
    return out


def norm_quantile(p) -> np.ndarray:
    p = _c(p, np.float64).reshape(-1)
    out = np.empty_like(p)
    lib().orc_norm_batch(p.shape[0], _ptr(p), None, _ptr(out))
    return out


def betainc(a, b, x, complement: bool = False):
    a, b, x = np.broadcast_arrays(np.asarray(a, np.float64), np.asarray(b, np.float64),
                                  np.asarray(x, np.float64))
    a, b, x = (_c(v, np.float64).reshape(-1) for v in (a, b, x))
    I = np.empty_like(x)
    Ic = np.empty_like(x)
    lib().orc_betainc_batch(x.shape[0], _ptr(a), _ptr(b), _ptr(x), _ptr(I), _ptr(Ic))
    return (I, Ic) if complement else I


def betaincinv(a, b, z, zc=None, complement: bool = False):
    a, b, z = np.broadcast_arrays(np.asarray(a, np.float64), np.asarray(b, np.float64),
                                  np.asarray(z, np.float64))
    a, b, z = (_c(v, np.float64).reshape(-1) for v in (a, b, z))
    zc = (1.0 - z) if zc is None else _c(np.broadcast_to(np.asarray(zc, np.float64), z.shape),
                                         np.float64)
    x = np.empty_like(z)
    xc = np.empty_like(z)
    lib().orc_betaincinv_batch(z.shape[0], _ptr(a), _ptr(b), _ptr(z), _ptr(zc), _ptr(x), _ptr(xc))
    return (x, xc) if complement else x


def beta_fit(mu: float, sigma: float, max_l: float):
    a = C.c_double()
    b = C.c_double()
    lib().orc_beta_fit(float(mu), float(sigma), float(max_l), C.byref(a), C.byref(b))
    return a.value, b.value


def su_loss_keyed(mu, s_i, s_c, max_l, k, i, elt_id, program, event, keying, seed: int):
    """One hit's loss under either keying (scalar arguments)."""
    return lib().orc_su_loss_keyed(float(mu), float(s_i), float(s_c), float(max_l), int(k),
                                   int(i), int(elt_id), int(program), int(event), int(keying),
                                   int(seed) & 0xFFFFFFFFFFFFFFFF)


def su_loss(mu, s_i, s_c, max_l, k, i, elt_id, seed: int) -> np.ndarray:
    arrs = np.broadcast_arrays(*(np.asarray(v) for v in (mu, s_i, s_c, max_l, k, i, elt_id)))
    mu, s_i, s_c, max_l = (_c(v, np.float64).reshape(-1) for v in arrs[:4])
    k, i, e = (_c(v, np.uint32).reshape(-1) for v in arrs[4:])
    out = np.empty_like(mu)
    lib().orc_su_loss_batch(mu.shape[0], _ptr(mu), _ptr(s_i), _ptr(s_c), _ptr(max_l),
                            _ptr(k), _ptr(i), _ptr(e), int(seed), _ptr(out))
    return out


# --------------------------------------------------------------------------
# ARA run and risk metrics
# --------------------------------------------------------------------------
def _flatten_portfolio(pf):
    layer_terms, layer_program = [], []
    elt_layer, elt_id, elt_terms, row_off = [], [], [], [0]
    ev, mu, si, sc, mx = [], [], [], [], []
    for li, layer in enumerate(pf.layers):
        layer_terms += [layer.occ_retention, layer.occ_limit,
                        layer.agg_retention, layer.agg_limit]
        layer_program.append(int(getattr(layer, "program_id", 0)) & 0xFFFFFFFF)
        for elt in layer.elts:
            elt_layer.append(li)
            elt_id.append(elt.elt_id)
            elt_terms += [elt.retention, elt.limit, elt.share]
            n = len(elt.event_ids)
            row_off.append(row_off[-1] + n)
            ev.append(np.asarray(elt.event_ids, np.int32))
            mu.append(np.asarray(elt.mean, np.float32))
            si.append(np.asarray(elt.sigma_i, np.float32))
            sc.append(np.asarray(elt.sigma_c, np.float32))
            mx.append(np.asarray(elt.max_loss, np.float32))

    def cat(lst, dt):
        return np.ascontiguousarray(np.concatenate(lst) if lst else np.zeros(0, dt), dtype=dt)

    return dict(
        layer_terms=np.asarray(layer_terms, np.float64),
        layer_program=np.asarray(layer_program, np.uint32),
        elt_layer=np.asarray(elt_layer, np.int32),
        elt_id=np.asarray(elt_id, np.uint32),
        elt_terms=np.asarray(elt_terms, np.float64),
        row_off=np.asarray(row_off, np.int64),
        ev=cat(ev, np.int32), mu=cat(mu, np.float32), si=cat(si, np.float32),
        sc=cat(sc, np.float32), mx=cat(mx, np.float32))


def run_ara(yet, pf, trial_begin: int = 0, trial_count: Optional[int] = None,
            threads: Optional[int] = None, occ_view: bool = False,
            trials: Optional[Sequence[int]] = None) -> Dict[str, np.ndarray]:
    """Run the oracle over trials [trial_begin, trial_begin + trial_count) of
    ``yet`` (or over the explicit list ``trials``) for portfolio ``pf``.

    Returns ``ylt`` [n_layers, n], ``ylt_pf`` [n], ``gross`` [n_layers, n],
    ``hits`` and ``hit_chk`` [n_layers, n] and, on request, ``occ_view``
    [n_layers, n_occ of the selected trials]."""
    if trials is not None:
        outs = [run_ara(yet, pf, int(t), 1, threads=threads, occ_view=occ_view) for t in trials]
        res = {}
        for key in outs[0] if outs else []:
            axis = 0 if key == "ylt_pf" else 1
            res[key] = np.concatenate([o[key] for o in outs], axis=axis)
        return res
    n_total = yet.n_trials
    if trial_count is None:
        trial_count = n_total - trial_begin
    assert 0 <= trial_begin and trial_begin + trial_count <= n_total
    off = np.ascontiguousarray(yet.offsets[trial_begin:trial_begin + trial_count + 1], np.int64)
    ids = np.ascontiguousarray(yet.event_ids, np.int32)
    f = _flatten_portfolio(pf)
    L = len(pf.layers)
    n = trial_count
    ylt = np.zeros((L, n), np.float64)
    ylt_pf = np.zeros(n, np.float64)
    gross = np.zeros((L, n), np.float64)
    hits = np.zeros((L, n), np.int64)
    chk = np.zeros((L, n), np.uint64)
    n_occ = int(off[-1] - off[0]) if n > 0 else 0
    ov = np.zeros((L, n_occ), np.float64) if occ_view else None
    nthr = threads if threads else len(os.sched_getaffinity(0))
    rc = lib().orc_ara_run(
        n, trial_begin, _ptr(off), _ptr(ids), int(yet.n_catalogue), L, _ptr(f["layer_terms"]),
        len(f["elt_layer"]), _ptr(f["elt_layer"]), _ptr(f["elt_id"]), _ptr(f["row_off"]),
        _ptr(f["elt_terms"]), _ptr(f["ev"]), _ptr(f["mu"]), _ptr(f["si"]), _ptr(f["sc"]),
        _ptr(f["mx"]), int(pf.seed) & 0xFFFFFFFFFFFFFFFF, 1 if pf.su_enabled else 0,
        int(getattr(pf, "keying", 0)), _ptr(f["layer_program"]), int(nthr),
        _ptr(ylt), _ptr(ylt_pf), _ptr(gross), _ptr(hits), _ptr(chk), _ptr(ov))
    if rc != 0:
        raise ValueError(f"oracle rejected the inputs (code {rc})")
    out = dict(ylt=ylt, ylt_pf=ylt_pf, gross=gross, hits=hits, hit_chk=chk)
    if occ_view:
        out["occ_view"] = ov
    return out


def pml_tvar(ylt, return_periods):
    y = _c(ylt, np.float64).reshape(-1)
    rp = _c(return_periods, np.float64).reshape(-1)
    pml = np.empty(rp.shape[0], np.float64)
    tvar = np.empty(rp.shape[0], np.float64)
    rc = lib().orc_pml_tvar(_ptr(y), y.shape[0], _ptr(rp), rp.shape[0], _ptr(pml), _ptr(tvar))
    if rc != 0:
        raise ValueError("oracle pml_tvar: empty input")
    return pml, tvar


def ep_curve(ylt):
    """Exceedance-probability curve of a YLT (the return-period-loss report
    of section 2.3): the losses in descending order (-0.0 taken as +0.0), so
    entry j is the loss equalled or exceeded in a fraction (j+1)/N of the
    trials, and the running means of the sorted losses (the TVaR at each
    point), accumulated in extended precision.  At k = max(1, floor(N/RP))
    entry k-1 is the PML / TVaR of ``pml_tvar``."""
    y = np.asarray(ylt, np.float64).reshape(-1)
    y = np.where(y == 0.0, 0.0, y)
    srt = -np.sort(-y, kind="stable")
    if srt.shape[0] == 0:
        return srt, srt.copy()
    cs = np.cumsum(srt.astype(np.longdouble))
    tm = (cs / np.arange(1, srt.shape[0] + 1, dtype=np.longdouble)).astype(np.float64)
    return srt, tm

