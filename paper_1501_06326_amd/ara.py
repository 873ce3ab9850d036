"""Python binding of the gfx950 ARA library (``libara.so``).

The functions named ``ara_*`` mirror the C-ABI of ``include/ara.h`` one to one
(argument marshalling only).  :class:`Ara` is a small convenience layer for
the tests and the benchmark: it keeps device memory in torch tensors, passes
their pointers and the current torch stream to the library, and checks every
status.  Every computation runs in the library's HIP kernels; nothing here
computes a loss or a risk metric.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libara.so")

ARA_OK = 0
ARA_E_INVALID_ARG = -1
ARA_E_NO_DEVICE = -2
ARA_E_HIP = -3
ARA_E_EVENT_ID_RANGE = -4
ARA_E_OFFSETS_NOT_MONOTONE = -5
ARA_E_TIMES_UNSORTED = -6
ARA_E_BAD_ELT_ROW = -7
ARA_E_WORKSPACE_TOO_SMALL = -8
ARA_E_NUMERIC = -9
ARA_E_UNSUPPORTED = -10

ARA_SUM_KAHAN32, ARA_SUM_NAIVE32, ARA_SUM_F64 = 0, 1, 2
ARA_DEBUG_QUANTILE_ONE_STEP = 1
ARA_F32, ARA_F64 = 0, 1
SUM_MODES = {"naive32": ARA_SUM_NAIVE32, "kahan32": ARA_SUM_KAHAN32, "f64": ARA_SUM_F64}

EXPORTS = ["ara_create", "ara_destroy", "ara_status_string", "ara_last_error", "ara_load_yet",
           "ara_free_yet", "ara_portfolio_workspace_size", "ara_load_portfolio",
           "ara_free_portfolio", "ara_run", "ara_run_scratch_size", "ara_sync_status",
           "ara_pml_tvar_scratch_size", "ara_pml_tvar", "ara_debug_philox",
           "ara_debug_beta_quantile", "ara_batch_scratch_size", "ara_run_batch",
           "ara_batch_autotune", "ara_batch_graph_create", "ara_graph_launch",
           "ara_graph_destroy", "ara_server_create", "ara_server_submit", "ara_server_poll",
           "ara_server_release", "ara_server_destroy", "ara_server_last_error",
           "ara_ep_curve_scratch_size", "ara_ep_curve", "ara_probe_stream_read",
           "ara_probe_valu_lanes", "ara_probe_valu", "ara_probe_draws",
           "ara_debug_beta_quantile_shape", "ara_run_static"]

PROBE_KINDS = {"fma_f32": 0, "mul_f32": 1, "xad_u32": 2, "mulhi_u32": 3, "mad_u64_u32": 4,
               "exp2_f32": 5, "fma_f64": 6}

SERVER_MAX_RP = 16


class AraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class ara_elt_desc(C.Structure):
    _fields_ = [("elt_id", C.c_uint32), ("n_rows", C.c_int32),
                ("event_ids", C.c_void_p), ("mean", C.c_void_p), ("sigma_i", C.c_void_p),
                ("sigma_c", C.c_void_p), ("max_loss", C.c_void_p),
                ("retention", C.c_double), ("limit", C.c_double), ("share", C.c_double)]


class ara_layer_desc(C.Structure):
    _fields_ = [("n_elts", C.c_int32), ("elts", C.POINTER(ara_elt_desc)),
                ("occ_retention", C.c_double), ("occ_limit", C.c_double),
                ("agg_retention", C.c_double), ("agg_limit", C.c_double),
                ("program_id", C.c_uint32)]


class ara_portfolio_desc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("layers", C.POINTER(ara_layer_desc)),
                ("seed", C.c_uint64), ("su_enabled", C.c_int32), ("keying", C.c_int32)]


ARA_KEYING_OCCURRENCE, ARA_KEYING_PAPER = 0, 1


ARA_BATCH_PORTFOLIO_MAJOR, ARA_BATCH_TRIAL_MAJOR = 0, 1


class ara_batch_config(C.Structure):
    _fields_ = [("trial_tile", C.c_int32), ("waves_per_cu", C.c_int32), ("order", C.c_int32)]


def _batch_cfg(cfg):
    """(trial_tile, waves_per_cu[, order]) -> ara_batch_config; None -> None."""
    if cfg is None:
        return None
    t = tuple(cfg) + ((ARA_BATCH_PORTFOLIO_MAJOR,) if len(cfg) == 2 else ())
    return ara_batch_config(*t)


class ara_server_config(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("max_batch", C.c_int32), ("sum_mode", C.c_int32),
                ("reserved", C.c_int32), ("d_pool", C.c_void_p), ("pool_bytes", C.c_size_t)]


class ara_server_result(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("status", C.c_int32), ("n_rp", C.c_int32),
                ("pml", C.c_double * 16), ("tvar", C.c_double * 16), ("queue_s", C.c_double),
                ("latency_s", C.c_double), ("ylt", C.POINTER(C.c_float)),
                ("ylt_count", C.c_int64)]


class ara_run_opts(C.Structure):
    _fields_ = [("trial_begin", C.c_int64), ("trial_count", C.c_int64),
                ("sum_mode", C.c_int32), ("ylt_dtype", C.c_int32),
                ("tail_band", C.c_float), ("debug_flags", C.c_int32),
                ("d_hits", C.c_void_p), ("d_hit_chk", C.c_void_p),
                ("d_scratch", C.c_void_p), ("scratch_bytes", C.c_size_t),
                ("d_occ_view", C.c_void_p), ("occ_view_stride", C.c_int64)]


_lib = None


def lib():
    """Load ``libara.so``; fail loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
        L.ara_create.argtypes = [C.c_int, C.POINTER(p)]
        L.ara_destroy.argtypes = [p]
        L.ara_destroy.restype = None
        L.ara_status_string.argtypes = [i32]
        L.ara_status_string.restype = C.c_char_p
        L.ara_last_error.argtypes = [p]
        L.ara_last_error.restype = C.c_char_p
        L.ara_load_yet.argtypes = [p, i64, i32, p, p, p, p, C.POINTER(p)]
        L.ara_free_yet.argtypes = [p, p]
        L.ara_portfolio_workspace_size.argtypes = [C.POINTER(ara_portfolio_desc), i32,
                                                   C.POINTER(sz)]
        L.ara_load_portfolio.argtypes = [p, C.POINTER(ara_portfolio_desc), i32, p, sz, p,
                                         C.POINTER(p)]
        L.ara_free_portfolio.argtypes = [p, p]
        L.ara_run.argtypes = [p, p, p, C.POINTER(ara_run_opts), p, p, p]
        L.ara_run_static.argtypes = [p, p, p, C.POINTER(ara_run_opts), p, p, p]
        L.ara_run_scratch_size.argtypes = [i64, C.POINTER(sz)]
        L.ara_sync_status.argtypes = [p, p]
        L.ara_pml_tvar_scratch_size.argtypes = [i64, C.POINTER(sz)]
        L.ara_pml_tvar.argtypes = [p, p, i32, i64, p, i32, p, p, p, sz, p]
        L.ara_debug_philox.argtypes = [p, i64, p, u64, p, p]
        L.ara_debug_beta_quantile.argtypes = [p, i64, p, p, p, p, C.c_float, p, p, p]
        pp = C.POINTER(C.c_void_p)
        L.ara_batch_scratch_size.argtypes = [i32, i64, C.POINTER(sz)]
        L.ara_run_batch.argtypes = [p, p, i32, pp, C.POINTER(ara_run_opts),
                                    C.POINTER(ara_batch_config), pp, pp, p, sz, p]
        L.ara_batch_autotune.argtypes = [p, p, i32, pp, C.POINTER(ara_run_opts), pp, pp, p, sz, p,
                                         C.POINTER(ara_batch_config), C.POINTER(C.c_double)]
        L.ara_batch_graph_create.argtypes = [p, p, i32, pp, C.POINTER(ara_run_opts),
                                             C.POINTER(ara_batch_config), pp, pp, p, sz,
                                             C.POINTER(p)]
        L.ara_graph_launch.argtypes = [p, p, p]
        L.ara_graph_destroy.argtypes = [p, p]
        L.ara_server_create.argtypes = [C.c_int, i64, i32, p, p, C.POINTER(ara_server_config),
                                        C.POINTER(p)]
        L.ara_server_submit.argtypes = [p, C.POINTER(ara_portfolio_desc), i64, i64, p, i32, i32,
                                        C.POINTER(C.c_uint64)]
        L.ara_server_poll.argtypes = [p, C.POINTER(ara_server_result), i32, C.c_double,
                                      C.POINTER(i32)]
        L.ara_server_release.argtypes = [p, C.c_uint64]
        L.ara_server_destroy.argtypes = [p]
        L.ara_server_last_error.argtypes = [p]
        L.ara_server_last_error.restype = C.c_char_p
        L.ara_ep_curve_scratch_size.argtypes = [i64, i32, C.POINTER(sz)]
        L.ara_ep_curve.argtypes = [p, p, i32, i64, p, p, p, sz, p]
        L.ara_probe_stream_read.argtypes = [p, p, sz, p, p]
        L.ara_probe_valu_lanes.argtypes = [p, i32, C.POINTER(i64)]
        L.ara_probe_valu.argtypes = [p, i32, i32, i32, p, C.POINTER(u64), p]
        L.ara_probe_draws.argtypes = [p, i64, u64, C.c_uint32, C.c_float, C.c_float, i32, p, p]
        L.ara_debug_beta_quantile_shape.argtypes = [p, i64, C.c_float, C.c_float, p, p, p, p, p]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is C.c_int:       # default
                f.restype = i32
        _lib = L
    return _lib


# ---- thin C-ABI mirrors ------------------------------------------------------
def ara_create(device: int = 0):
    h = C.c_void_p()
    rc = lib().ara_create(int(device), C.byref(h))
    if rc != ARA_OK:
        raise AraError(rc, "ara_create: " + lib().ara_status_string(rc).decode())
    return h


def ara_destroy(ctx) -> None:
    lib().ara_destroy(ctx)


def ara_status_string(code: int) -> str:
    return lib().ara_status_string(int(code)).decode()


def ara_last_error(ctx) -> str:
    return lib().ara_last_error(ctx).decode()


def _check(ctx, rc: int, what: str):
    if rc != ARA_OK:
        raise AraError(rc, f"{what}: {ara_last_error(ctx)}")


def ara_load_yet(ctx, n_trials: int, n_catalogue: int, d_offsets: int, d_event_ids: int,
                 d_times: Optional[int], stream: Optional[int]):
    h = C.c_void_p()
    _check(ctx, lib().ara_load_yet(ctx, int(n_trials), int(n_catalogue), d_offsets, d_event_ids,
                                   d_times, stream, C.byref(h)), "ara_load_yet")
    return h


def ara_free_yet(ctx, yet) -> None:
    _check(ctx, lib().ara_free_yet(ctx, yet), "ara_free_yet")


def ara_portfolio_workspace_size(desc: "ara_portfolio_desc", n_catalogue: int) -> int:
    n = C.c_size_t()
    rc = lib().ara_portfolio_workspace_size(C.byref(desc), int(n_catalogue), C.byref(n))
    if rc != ARA_OK:
        raise AraError(rc, "ara_portfolio_workspace_size: " + ara_status_string(rc))
    return int(n.value)


def ara_load_portfolio(ctx, desc: "ara_portfolio_desc", n_catalogue: int, d_workspace: int,
                       nbytes: int, stream: Optional[int]):
    h = C.c_void_p()
    _check(ctx, lib().ara_load_portfolio(ctx, C.byref(desc), int(n_catalogue), d_workspace,
                                         int(nbytes), stream, C.byref(h)), "ara_load_portfolio")
    return h


def ara_free_portfolio(ctx, pf) -> None:
    _check(ctx, lib().ara_free_portfolio(ctx, pf), "ara_free_portfolio")


def ara_run(ctx, yet, pf, opts: "ara_run_opts", d_ylt_layers: Optional[int],
            d_ylt_portfolio: Optional[int], stream: Optional[int]) -> None:
    _check(ctx, lib().ara_run(ctx, yet, pf, C.byref(opts), d_ylt_layers, d_ylt_portfolio, stream),
           "ara_run")


ARA_STATIC_MAX_TRIALS = 1 << 22


def ara_run_static(ctx, yet, pf, opts: "ara_run_opts", d_ylt_layers: Optional[int],
                   d_ylt_portfolio: Optional[int], stream: Optional[int]) -> None:
    _check(ctx, lib().ara_run_static(ctx, yet, pf, C.byref(opts), d_ylt_layers, d_ylt_portfolio,
                                     stream), "ara_run_static")


def ara_run_scratch_size(trial_count: int) -> int:
    n = C.c_size_t()
    rc = lib().ara_run_scratch_size(int(trial_count), C.byref(n))
    if rc != ARA_OK:
        raise AraError(rc, "ara_run_scratch_size")
    return int(n.value)


def ara_sync_status(ctx, stream: Optional[int]) -> None:
    _check(ctx, lib().ara_sync_status(ctx, stream), "ara_run")


def ara_pml_tvar_scratch_size(n: int) -> int:
    sz = C.c_size_t()
    rc = lib().ara_pml_tvar_scratch_size(int(n), C.byref(sz))
    if rc != ARA_OK:
        raise AraError(rc, "ara_pml_tvar_scratch_size")
    return int(sz.value)


def ara_pml_tvar(ctx, d_ylt: int, ylt_dtype: int, n: int, return_periods, d_scratch: int,
                 scratch_bytes: int, stream: Optional[int]):
    rp = np.ascontiguousarray(return_periods, np.float64)
    pml = np.empty(rp.shape[0], np.float64)
    tvar = np.empty(rp.shape[0], np.float64)
    _check(ctx, lib().ara_pml_tvar(ctx, d_ylt, int(ylt_dtype), int(n), rp.ctypes.data,
                                   rp.shape[0], pml.ctypes.data, tvar.ctypes.data, d_scratch,
                                   int(scratch_bytes), stream), "ara_pml_tvar")
    return pml, tvar


def ara_debug_philox(ctx, n: int, d_ctr: int, key: int, d_out: int, stream: Optional[int]):
    _check(ctx, lib().ara_debug_philox(ctx, int(n), d_ctr, int(key) & 0xFFFFFFFFFFFFFFFF, d_out,
                                       stream), "ara_debug_philox")


def ara_debug_beta_quantile(ctx, n: int, d_a: int, d_b: int, d_z: int, d_zc: int,
                            tail_band: float, d_x: int, d_path: Optional[int],
                            stream: Optional[int]):
    _check(ctx, lib().ara_debug_beta_quantile(ctx, int(n), d_a, d_b, d_z, d_zc, float(tail_band),
                                              d_x, d_path, stream), "ara_debug_beta_quantile")


def _ptr_array(vals):
    arr = (C.c_void_p * max(1, len(vals)))()
    for i, v in enumerate(vals):
        arr[i] = v
    return arr


def ara_batch_scratch_size(n_portfolios: int, trial_count: int) -> int:
    n = C.c_size_t()
    rc = lib().ara_batch_scratch_size(int(n_portfolios), int(trial_count), C.byref(n))
    if rc != ARA_OK:
        raise AraError(rc, "ara_batch_scratch_size")
    return int(n.value)


def ara_run_batch(ctx, yet, pfs, opts: "ara_run_opts", cfg: Optional["ara_batch_config"],
                  d_ylt_layers, d_ylt_portfolio, d_scratch: int, scratch_bytes: int,
                  stream: Optional[int]) -> None:
    _check(ctx, lib().ara_run_batch(ctx, yet, len(pfs), _ptr_array(pfs), C.byref(opts),
                                    C.byref(cfg) if cfg is not None else None,
                                    _ptr_array(d_ylt_layers), _ptr_array(d_ylt_portfolio),
                                    d_scratch, int(scratch_bytes), stream), "ara_run_batch")


def ara_batch_autotune(ctx, yet, pfs, opts: "ara_run_opts", d_ylt_layers, d_ylt_portfolio,
                       d_scratch: int, scratch_bytes: int, stream: Optional[int]):
    best = ara_batch_config()
    ms = C.c_double()
    _check(ctx, lib().ara_batch_autotune(ctx, yet, len(pfs), _ptr_array(pfs), C.byref(opts),
                                         _ptr_array(d_ylt_layers), _ptr_array(d_ylt_portfolio),
                                         d_scratch, int(scratch_bytes), stream, C.byref(best),
                                         C.byref(ms)), "ara_batch_autotune")
    return best, float(ms.value)


def ara_batch_graph_create(ctx, yet, pfs, opts: "ara_run_opts", cfg: Optional["ara_batch_config"],
                           d_ylt_layers, d_ylt_portfolio, d_scratch: int, scratch_bytes: int):
    h = C.c_void_p()
    _check(ctx, lib().ara_batch_graph_create(ctx, yet, len(pfs), _ptr_array(pfs), C.byref(opts),
                                             C.byref(cfg) if cfg is not None else None,
                                             _ptr_array(d_ylt_layers),
                                             _ptr_array(d_ylt_portfolio), d_scratch,
                                             int(scratch_bytes), C.byref(h)),
           "ara_batch_graph_create")
    return h


def ara_graph_launch(ctx, graph, stream: Optional[int]) -> None:
    _check(ctx, lib().ara_graph_launch(ctx, graph, stream), "ara_graph_launch")


def ara_graph_destroy(ctx, graph) -> None:
    _check(ctx, lib().ara_graph_destroy(ctx, graph), "ara_graph_destroy")


def ara_ep_curve_scratch_size(n: int, dtype: int) -> int:
    b = C.c_size_t()
    rc = lib().ara_ep_curve_scratch_size(int(n), int(dtype), C.byref(b))
    if rc != ARA_OK:
        raise AraError(rc, "ara_ep_curve_scratch_size")
    return int(b.value)


def ara_ep_curve(ctx, d_ylt, dtype, n, d_sorted, d_tail_mean, d_scratch, nbytes, stream):
    _check(ctx, lib().ara_ep_curve(ctx, d_ylt, int(dtype), int(n), d_sorted, d_tail_mean,
                                   d_scratch, nbytes, stream), "ara_ep_curve")


def ara_probe_stream_read(ctx, d_src: int, nbytes: int, d_sink: int, stream) -> None:
    _check(ctx, lib().ara_probe_stream_read(ctx, d_src, int(nbytes), d_sink, stream),
           "ara_probe_stream_read")


def ara_probe_valu_lanes(ctx, waves_per_simd: int) -> int:
    n = C.c_int64()
    _check(ctx, lib().ara_probe_valu_lanes(ctx, int(waves_per_simd), C.byref(n)),
           "ara_probe_valu_lanes")
    return int(n.value)


def ara_probe_valu(ctx, kind: int, waves_per_simd: int, iters: int, d_out: int, stream) -> int:
    n = C.c_uint64()
    _check(ctx, lib().ara_probe_valu(ctx, int(kind), int(waves_per_simd), int(iters), d_out,
                                     C.byref(n), stream), "ara_probe_valu")
    return int(n.value)


def ara_probe_draws(ctx, n: int, seed: int, elt_id: int, a: float, b: float,
                    use_shape_table: bool, d_x: int, stream) -> None:
    _check(ctx, lib().ara_probe_draws(ctx, int(n), int(seed) & 0xFFFFFFFFFFFFFFFF, int(elt_id),
                                      float(a), float(b), 1 if use_shape_table else 0, d_x,
                                      stream), "ara_probe_draws")


def ara_debug_beta_quantile_shape(ctx, n: int, a: float, b: float, d_z: int, d_zc: int, d_x: int,
                                  d_path: Optional[int], stream) -> None:
    _check(ctx, lib().ara_debug_beta_quantile_shape(ctx, int(n), float(a), float(b), d_z, d_zc,
                                                    d_x, d_path, stream),
           "ara_debug_beta_quantile_shape")


def ara_server_create(device: int, n_trials: int, n_catalogue: int, d_offsets: int,
                      d_event_ids: int, cfg: "ara_server_config"):
    h = C.c_void_p()
    rc = lib().ara_server_create(int(device), int(n_trials), int(n_catalogue), d_offsets,
                                 d_event_ids, C.byref(cfg), C.byref(h))
    if rc != ARA_OK:
        raise AraError(rc, "ara_server_create: " + ara_status_string(rc))
    return h


ARA_SUBMIT_WANT_YLT, ARA_SUBMIT_BORROW = 1, 2


def ara_server_submit(srv, desc: "ara_portfolio_desc", trial_begin: int, trial_count: int,
                      return_periods, flags: int) -> int:
    rp = np.ascontiguousarray(return_periods, np.float64)
    rid = C.c_uint64()
    rc = lib().ara_server_submit(srv, C.byref(desc), int(trial_begin), int(trial_count),
                                 rp.ctypes.data, rp.shape[0], int(flags), C.byref(rid))
    if rc != ARA_OK:
        raise AraError(rc, "ara_server_submit: " + ara_status_string(rc))
    return int(rid.value)


def ara_server_poll(srv, max_results: int, wait_s: float):
    out = (ara_server_result * max_results)()
    n = C.c_int32()
    rc = lib().ara_server_poll(srv, out, int(max_results), float(wait_s), C.byref(n))
    if rc != ARA_OK:
        raise AraError(rc, "ara_server_poll")
    return [out[i] for i in range(n.value)]


def ara_server_release(srv, request_id: int) -> None:
    rc = lib().ara_server_release(srv, int(request_id))
    if rc != ARA_OK:
        raise AraError(rc, "ara_server_release")


def ara_server_destroy(srv) -> None:
    lib().ara_server_destroy(srv)


def ara_server_last_error(srv) -> str:
    return lib().ara_server_last_error(srv).decode()


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def _on(stream):
    """Context in which the convenience layer allocates the device tensors of
    a call enqueued on ``stream``: torch's caching allocator then hands a
    freed block of them out again only to later work of that same stream, so
    a scratch tensor dropped on return is not reused by a call on another
    stream while this call's kernels still run."""
    import contextlib
    import torch
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


# ---- convenience layer -------------------------------------------------------
class _Desc:
    """Holds a portfolio description and the host arrays it points into."""

    def __init__(self, pf):
        self.keep = []
        self.elt_arrays = []
        layers = (ara_layer_desc * max(1, len(pf.layers)))()
        for li, layer in enumerate(pf.layers):
            elts = (ara_elt_desc * max(1, len(layer.elts)))()
            self.elt_arrays.append(elts)
            for j, e in enumerate(layer.elts):
                ev = np.ascontiguousarray(e.event_ids, np.int32)
                mu = np.ascontiguousarray(e.mean, np.float32)
                si = np.ascontiguousarray(e.sigma_i, np.float32)
                sc = np.ascontiguousarray(e.sigma_c, np.float32)
                mx = np.ascontiguousarray(e.max_loss, np.float32)
                self.keep += [ev, mu, si, sc, mx]
                d = elts[j]
                d.elt_id = int(e.elt_id) & 0xFFFFFFFF
                d.n_rows = int(ev.shape[0])
                d.event_ids, d.mean, d.sigma_i = ev.ctypes.data, mu.ctypes.data, si.ctypes.data
                d.sigma_c, d.max_loss = sc.ctypes.data, mx.ctypes.data
                d.retention, d.limit, d.share = float(e.retention), float(e.limit), float(e.share)
            L = layers[li]
            L.n_elts = len(layer.elts)
            L.elts = C.cast(elts, C.POINTER(ara_elt_desc))
            L.occ_retention, L.occ_limit = float(layer.occ_retention), float(layer.occ_limit)
            L.agg_retention, L.agg_limit = float(layer.agg_retention), float(layer.agg_limit)
            L.program_id = int(getattr(layer, "program_id", 0))
        self.layers = layers
        self.desc = ara_portfolio_desc(n_layers=len(pf.layers),
                                       layers=C.cast(layers, C.POINTER(ara_layer_desc)),
                                       seed=int(pf.seed) & 0xFFFFFFFFFFFFFFFF,
                                       su_enabled=1 if pf.su_enabled else 0,
                                       keying=int(getattr(pf, "keying", 0)))


class DeviceYET:
    def __init__(self, handle, offsets, event_ids, times, n_trials, n_catalogue,
                 offsets_host=None):
        self.handle = handle
        self.offsets, self.event_ids, self.times = offsets, event_ids, times
        self.offsets_host = offsets_host
        self.n_trials, self.n_catalogue = n_trials, n_catalogue


class DevicePortfolio:
    def __init__(self, handle, workspace, n_layers, n_elts, su):
        self.handle = handle
        self.workspace = workspace
        self.n_layers, self.n_elts, self.su = n_layers, n_elts, su


class Ara:
    """One library context on ``cuda:device``; tensors are torch (HIP) tensors."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the ARA library needs a ROCm GPU (torch.cuda is not available)")
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = ara_create(device)

    def close(self):
        if self.ctx is not None:
            ara_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- YET --------------------------------------------------------------------
    def load_yet(self, yet, device_arrays=None, stream=None) -> DeviceYET:
        """Copy a host YET (workloads.YET) to the device (or take already
        resident tensors ``device_arrays=(offsets, event_ids, times)``) and
        validate it with ``ara_load_yet``."""
        t = self.torch
        if device_arrays is None:
            off = t.from_numpy(np.ascontiguousarray(yet.offsets, np.int64)).to(self.device)
            ev = t.from_numpy(np.ascontiguousarray(yet.event_ids, np.int32)).to(self.device)
            tm = (None if yet.times is None else
                  t.from_numpy(np.ascontiguousarray(yet.times, np.float32)).to(self.device))
        else:
            off, ev, tm = device_arrays
        n_trials = int(off.shape[0] - 1)
        h = ara_load_yet(self.ctx, n_trials, int(yet.n_catalogue), _ptr(off), _ptr(ev), _ptr(tm),
                         _stream_handle(stream))
        return DeviceYET(h, off, ev, tm, n_trials, int(yet.n_catalogue),
                         np.asarray(yet.offsets, np.int64))

    def free_yet(self, y: DeviceYET):
        ara_free_yet(self.ctx, y.handle)

    # -- portfolio --------------------------------------------------------------
    def workspace_size(self, pf, n_catalogue: int) -> int:
        return ara_portfolio_workspace_size(_Desc(pf).desc, n_catalogue)

    def load_portfolio(self, pf, n_catalogue: int, stream=None) -> DevicePortfolio:
        d = _Desc(pf)
        n = ara_portfolio_workspace_size(d.desc, n_catalogue)
        ws = self.torch.empty(max(1, n), dtype=self.torch.uint8, device=self.device)
        h = ara_load_portfolio(self.ctx, d.desc, n_catalogue, _ptr(ws), n, _stream_handle(stream))
        return DevicePortfolio(h, ws, len(pf.layers), pf.n_elts, bool(pf.su_enabled))

    def free_portfolio(self, p: DevicePortfolio):
        ara_free_portfolio(self.ctx, p.handle)

    def sync_status(self, stream=None):
        """Wait for the stream and raise on a device-side error of its runs."""
        ara_sync_status(self.ctx, _stream_handle(stream))

    # -- analysis ---------------------------------------------------------------
    def run(self, y: DeviceYET, p: DevicePortfolio, trial_begin: int = 0,
            trial_count: Optional[int] = None, sum_mode: str = "kahan32",
            ylt_dtype: str = "f32", tail_band: float = 0.0, diagnostics: bool = False,
            out_layers=None, out_pf=None, stream=None, sync: bool = True,
            layers: bool = True, scratch=None, occ_view: bool = False,
            occ_view_stride: Optional[int] = None, debug_flags: int = 0):
        """``ara_run``; returns dict of device tensors ``ylt`` [n_layers, n]
        and ``ylt_pf`` [n] (plus ``hits``/``hit_chk`` with diagnostics, and
        ``occ_view`` [n_layers, occurrences of the run] on request).  The run's
        scratch is a fresh tensor unless ``scratch`` is given (runs that may
        overlap on the device need scratch of their own)."""
        with _on(stream):
            return self._run(y, p, trial_begin, trial_count, sum_mode, ylt_dtype, tail_band,
                             diagnostics, out_layers, out_pf, stream, sync, layers, scratch,
                             occ_view, occ_view_stride, debug_flags)

    def _run(self, y, p, trial_begin, trial_count, sum_mode, ylt_dtype, tail_band, diagnostics,
             out_layers, out_pf, stream, sync, layers, scratch, occ_view, occ_view_stride,
             debug_flags):
        t = self.torch
        if trial_count is None:
            trial_count = y.n_trials - trial_begin
        if scratch is None and p.su:
            scratch = t.empty(ara_run_scratch_size(trial_count), dtype=t.uint8,
                              device=self.device)
        dt = t.float64 if ylt_dtype == "f64" else t.float32
        if layers and out_layers is None:
            out_layers = t.empty((p.n_layers, trial_count), dtype=dt, device=self.device)
        if out_pf is None:
            out_pf = t.empty(trial_count, dtype=dt, device=self.device)
        hits = chk = None
        if diagnostics:
            hits = t.empty((p.n_layers, trial_count), dtype=t.int64, device=self.device)
            chk = t.empty((p.n_layers, trial_count), dtype=t.int64, device=self.device)
        ov = None
        if occ_view:
            n_occ = int(y.offsets_host[trial_begin + trial_count] - y.offsets_host[trial_begin])
            stride = max(1, n_occ) if occ_view_stride is None else int(occ_view_stride)
            ov = t.zeros((p.n_layers, max(1, stride)), dtype=dt, device=self.device)
        o = ara_run_opts(trial_begin=int(trial_begin), trial_count=int(trial_count),
                         sum_mode=SUM_MODES[sum_mode],
                         ylt_dtype=ARA_F64 if ylt_dtype == "f64" else ARA_F32,
                         tail_band=float(tail_band), debug_flags=int(debug_flags),
                         d_hits=_ptr(hits),
                         d_hit_chk=_ptr(chk), d_scratch=_ptr(scratch),
                         scratch_bytes=0 if scratch is None else scratch.numel(),
                         d_occ_view=_ptr(ov),
                         occ_view_stride=0 if ov is None else int(ov.shape[1]))
        s = _stream_handle(stream)
        ara_run(self.ctx, y.handle, p.handle, o, _ptr(out_layers), _ptr(out_pf), s)
        if sync:
            ara_sync_status(self.ctx, s)
        res = {"ylt": out_layers, "ylt_pf": out_pf}
        if diagnostics:
            res["hits"], res["hit_chk"] = hits, chk
        if ov is not None:
            res["occ_view"] = ov
        return res

    def ep_curve(self, ylt, tail_mean: bool = True, stream=None):
        """``ara_ep_curve``: (losses in descending order, FP64 running means or
        None) as device tensors."""
        t = self.torch
        with _on(stream):
            y = ylt.contiguous()
            n = int(y.numel())
            dtype = ARA_F64 if y.dtype == t.float64 else ARA_F32
            srt = t.empty(n, dtype=y.dtype, device=self.device)
            tm = t.empty(n, dtype=t.float64, device=self.device) if tail_mean else None
            sz = ara_ep_curve_scratch_size(n, dtype)
            sc = t.empty(max(1, sz), dtype=t.uint8, device=self.device)
            ara_ep_curve(self.ctx, _ptr(y), dtype, n, _ptr(srt), _ptr(tm), _ptr(sc), sz,
                         _stream_handle(stream))
        return srt, tm

    def run_scratch_size(self, trial_count: int) -> int:
        return ara_run_scratch_size(trial_count)

    def pml_tvar(self, ylt, return_periods: Sequence[float], stream=None):
        t = self.torch
        n = int(ylt.numel())
        sz = ara_pml_tvar_scratch_size(n)
        scratch = t.empty(sz, dtype=t.uint8, device=self.device)
        y = ylt.contiguous()
        dtype = ARA_F64 if y.dtype == t.float64 else ARA_F32
        return ara_pml_tvar(self.ctx, _ptr(y), dtype, n, return_periods, _ptr(scratch), sz,
                            _stream_handle(stream))

    # -- batched portfolios -----------------------------------------------------
    def _batch_setup(self, y, pfs, trial_begin, trial_count, sum_mode, ylt_dtype, tail_band,
                     outs):
        t = self.torch
        if trial_count is None:
            trial_count = y.n_trials - trial_begin
        dt = t.float64 if ylt_dtype == "f64" else t.float32
        if outs is None:
            outs = [{"ylt": t.empty((p.n_layers, trial_count), dtype=dt, device=self.device),
                     "ylt_pf": t.empty(trial_count, dtype=dt, device=self.device)} for p in pfs]
        n = ara_batch_scratch_size(len(pfs), trial_count)
        scratch = t.empty(n, dtype=t.uint8, device=self.device)
        o = ara_run_opts(trial_begin=int(trial_begin), trial_count=int(trial_count),
                         sum_mode=SUM_MODES[sum_mode],
                         ylt_dtype=ARA_F64 if ylt_dtype == "f64" else ARA_F32,
                         tail_band=float(tail_band), debug_flags=0, d_hits=None, d_hit_chk=None,
                         d_scratch=None, scratch_bytes=0)
        return o, outs, scratch

    def run_batch(self, y, pfs, trial_begin=0, trial_count=None, sum_mode="kahan32",
                  ylt_dtype="f32", tail_band=0.0, cfg=None, outs=None, stream=None, sync=True,
                  scratch=None):
        """One persistent launch over several DevicePortfolio; returns a list of
        {"ylt", "ylt_pf"} device tensors, one per portfolio."""
        with _on(stream):
            o, outs, sc = self._batch_setup(y, pfs, trial_begin, trial_count, sum_mode,
                                            ylt_dtype, tail_band, outs)
            if scratch is not None:
                sc = scratch
            c = _batch_cfg(cfg)
            s = _stream_handle(stream)
            ara_run_batch(self.ctx, y.handle, [p.handle.value for p in pfs], o, c,
                          [_ptr(r["ylt"]) for r in outs], [_ptr(r["ylt_pf"]) for r in outs],
                          _ptr(sc), sc.numel(), s)
        if sync:
            ara_sync_status(self.ctx, s)
        return outs

    def batch_autotune(self, y, pfs, trial_begin=0, trial_count=4096, stream=None):
        o, outs, sc = self._batch_setup(y, pfs, trial_begin, trial_count, "kahan32", "f32", 0.0,
                                        None)
        best, ms = ara_batch_autotune(self.ctx, y.handle, [p.handle.value for p in pfs], o,
                                      [_ptr(r["ylt"]) for r in outs],
                                      [_ptr(r["ylt_pf"]) for r in outs], _ptr(sc), sc.numel(),
                                      _stream_handle(stream))
        return (best.trial_tile, best.waves_per_cu, best.order), ms

    def batch_graph(self, y, pfs, trial_begin=0, trial_count=None, sum_mode="kahan32",
                    ylt_dtype="f32", cfg=None):
        """Capture the batched run in a HIP graph; returns (graph handle, outs,
        scratch); keep outs and scratch alive while the graph exists."""
        o, outs, sc = self._batch_setup(y, pfs, trial_begin, trial_count, sum_mode, ylt_dtype,
                                        0.0, None)
        c = _batch_cfg(cfg)
        g = ara_batch_graph_create(self.ctx, y.handle, [p.handle.value for p in pfs], o, c,
                                   [_ptr(r["ylt"]) for r in outs],
                                   [_ptr(r["ylt_pf"]) for r in outs], _ptr(sc), sc.numel())
        return g, outs, sc

    def graph_launch(self, g, stream=None):
        ara_graph_launch(self.ctx, g, _stream_handle(stream))

    def graph_destroy(self, g):
        ara_graph_destroy(self.ctx, g)

    # -- diagnostics ------------------------------------------------------------
    def debug_philox(self, ctr, key: int, stream=None):
        t = self.torch
        c = t.as_tensor(np.ascontiguousarray(ctr, np.uint32).view(np.int32)).to(self.device)
        out = t.empty_like(c)
        ara_debug_philox(self.ctx, c.numel() // 4, _ptr(c), key, _ptr(out), _stream_handle(stream))
        return out.cpu().numpy().view(np.uint32).reshape(-1, 4)

    def debug_beta_quantile(self, a, b, z, zc, tail_band: float = 0.0, stream=None):
        t = self.torch
        A = t.as_tensor(np.ascontiguousarray(a, np.float32)).to(self.device)
        B = t.as_tensor(np.ascontiguousarray(b, np.float32)).to(self.device)
        Z = t.as_tensor(np.ascontiguousarray(z, np.float64)).to(self.device)
        ZC = t.as_tensor(np.ascontiguousarray(zc, np.float64)).to(self.device)
        x = t.empty(A.numel(), dtype=t.float32, device=self.device)
        path = t.empty(A.numel(), dtype=t.int32, device=self.device)
        ara_debug_beta_quantile(self.ctx, A.numel(), _ptr(A), _ptr(B), _ptr(Z), _ptr(ZC),
                                tail_band, _ptr(x), _ptr(path), _stream_handle(stream))
        return x.cpu().numpy(), path.cpu().numpy()

    def debug_beta_quantile_shape(self, a: float, b: float, z, zc, stream=None):
        """The FP32 quantile of one shape through its shape table."""
        t = self.torch
        Z = t.as_tensor(np.ascontiguousarray(z, np.float64)).to(self.device)
        ZC = t.as_tensor(np.ascontiguousarray(zc, np.float64)).to(self.device)
        x = t.empty(Z.numel(), dtype=t.float32, device=self.device)
        path = t.empty(Z.numel(), dtype=t.int32, device=self.device)
        ara_debug_beta_quantile_shape(self.ctx, Z.numel(), a, b, _ptr(Z), _ptr(ZC), _ptr(x),
                                      _ptr(path), _stream_handle(stream))
        return x.cpu().numpy(), path.cpu().numpy()


def evaluations(yet, pf, trial_begin: int = 0, trial_count: Optional[int] = None) -> int:
    """Trial x event x ELT evaluations of a run (zero lookups included)."""
    if trial_count is None:
        trial_count = yet.n_trials - trial_begin
    occ = int(yet.offsets[trial_begin + trial_count] - yet.offsets[trial_begin])
    return occ * sum(len(l.elts) for l in pf.layers)


__all__ = [n for n in EXPORTS] + ["Ara", "AraError", "Server", "lib", "evaluations",
                                  "SUM_MODES"]


class Server:
    """Serving loop (ara_server_*): a YET resident on the device, requests
    admitted by HBM footprint from a pool tensor, continuous batching on
    max_inflight streams.  Requests are workloads.Portfolio objects."""

    def __init__(self, yet, device: int = 0, pool_bytes: int = 4 << 30, max_inflight: int = 2,
                 max_batch: int = 4, sum_mode: str = "kahan32", device_arrays=None):
        import torch
        self.torch = torch
        dev = torch.device("cuda", device)
        if device_arrays is None:
            self.off = torch.from_numpy(np.ascontiguousarray(yet.offsets, np.int64)).to(dev)
            self.ev = torch.from_numpy(np.ascontiguousarray(yet.event_ids, np.int32)).to(dev)
        else:
            self.off, self.ev = device_arrays[0], device_arrays[1]
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        cfg = ara_server_config(max_inflight=int(max_inflight), max_batch=int(max_batch),
                                sum_mode=SUM_MODES[sum_mode], reserved=0,
                                d_pool=self.pool.data_ptr(), pool_bytes=int(pool_bytes))
        self._lent = {}
        self.h = ara_server_create(device, int(self.off.shape[0] - 1), int(yet.n_catalogue),
                                   _ptr(self.off), _ptr(self.ev), cfg)

    def submit(self, pf, trial_begin: int, trial_count: int, return_periods=(100.0, 250.0),
               want_ylt: bool = False, borrow: bool = False) -> int:
        """Queue a request.  borrow=True lends the row arrays instead of having
        the server copy them; they are kept alive here until the result is
        polled."""
        d = _Desc(pf)
        flags = (ARA_SUBMIT_WANT_YLT if want_ylt else 0) | (ARA_SUBMIT_BORROW if borrow else 0)
        rid = ara_server_submit(self.h, d.desc, trial_begin, trial_count, return_periods, flags)
        if borrow:
            self._lent[rid] = d
        return rid

    def poll(self, max_results: int = 64, wait_s: float = 0.0):
        res = []
        for r in ara_server_poll(self.h, max_results, wait_s):
            item = {"id": int(r.request_id), "status": int(r.status),
                    "pml": np.array(r.pml[:r.n_rp]), "tvar": np.array(r.tvar[:r.n_rp]),
                    "queue_s": float(r.queue_s), "latency_s": float(r.latency_s), "ylt": None}
            if r.ylt_count > 0 and bool(r.ylt):
                item["ylt"] = np.ctypeslib.as_array(r.ylt, shape=(int(r.ylt_count),)).copy()
            ara_server_release(self.h, r.request_id)
            self._lent.pop(int(r.request_id), None)
            res.append(item)
        return res

    def close(self):
        if self.h is not None:
            ara_server_destroy(self.h)      # waits for the queued requests
            self.h = None
            self._lent.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

