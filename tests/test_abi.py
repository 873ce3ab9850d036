"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1501_06326_amd.ara as A
from workloads import config_small

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "ara.h")).read()
    return re.findall(r"^\s*(?:ara_status|void|const char \*)\s*(ara_\w+)\s*\(", hdr, re.M)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 16
    lib = A.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(A.EXPORTS)


def test_status_strings():
    assert A.ara_status_string(0) == "ok"
    assert A.ara_status_string(A.ARA_E_BAD_ELT_ROW) == "bad ELT row"
    assert A.ara_status_string(-999) == "unknown status"


def test_workspace_size_host_side():
    w = config_small(n_trials=10)
    d = A._Desc(w.portfolio)
    n = A.ara_portfolio_workspace_size(d.desc, w.yet.n_catalogue)
    rows = sum(e.n_rows for e in w.portfolio.layers[0].elts)
    # at least: rows x (16 + 4 + 4 + 4 + 8 + 20 bytes) + event offsets + tables
    assert n >= rows * 56 + (w.yet.n_catalogue + 1) * 4
    assert n % 256 == 0


def test_invalid_descriptions_rejected_without_gpu():
    w = config_small(n_trials=10)
    e = w.portfolio.layers[0].elts[0]
    old = e.share
    e.share = 1.5
    with pytest.raises(A.AraError) as ei:
        A.ara_portfolio_workspace_size(A._Desc(w.portfolio).desc, w.yet.n_catalogue)
    assert ei.value.code == A.ARA_E_BAD_ELT_ROW
    e.share = old
    w.portfolio.layers[0].occ_retention = -1.0
    with pytest.raises(A.AraError) as ei:
        A.ara_portfolio_workspace_size(A._Desc(w.portfolio).desc, w.yet.n_catalogue)
    assert ei.value.code == A.ARA_E_BAD_ELT_ROW
    with pytest.raises(A.AraError) as ei:
        A.ara_portfolio_workspace_size(A._Desc(w.portfolio).desc, 0)
    assert ei.value.code == A.ARA_E_INVALID_ARG


def test_layer_row_limit_rejected_without_gpu():
    """A layer's compact row records hold its row index in 27 bits: a layer
    of 2^27 rows or more is refused before any row is read (the row arrays
    are not touched, so their true length does not matter here)."""
    w = config_small(n_trials=10)
    d = A._Desc(w.portfolio)
    elts = d.elt_arrays[0]
    elts[0].n_rows = (1 << 27) - sum(elts[j].n_rows for j in range(1, len(w.portfolio.layers[0].elts)))
    with pytest.raises(A.AraError) as ei:
        A.ara_portfolio_workspace_size(d.desc, w.yet.n_catalogue)
    assert ei.value.code == A.ARA_E_UNSUPPORTED
    elts[0].n_rows -= 1                       # 2^27 - 1 rows: accepted
    assert A.ara_portfolio_workspace_size(d.desc, w.yet.n_catalogue) > 0


def test_scratch_sizes():
    assert A.ara_run_scratch_size(1_000_000) >= 4_000_000
    assert A.ara_pml_tvar_scratch_size(10) > 0
    n = ctypes.c_size_t()
    assert A.lib().ara_run_scratch_size(-1, ctypes.byref(n)) == A.ARA_E_INVALID_ARG


def test_null_context_is_an_error_not_a_crash():
    lib = A.lib()
    assert lib.ara_run(None, None, None, None, None, None, None) == A.ARA_E_INVALID_ARG
    assert lib.ara_sync_status(None, None) == A.ARA_E_INVALID_ARG
    assert math.isfinite(0.0) and np is not None


def test_missing_library_fails_loudly(tmp_path):
    """No fallback: without libara.so the binding refuses to run."""
    code = ("import paper_1501_06326_amd.ara as A\n"
            f"A.LIB_PATH = {str(tmp_path / 'absent' / 'libara.so')!r}\n"
            "A._lib = None\n"
            "try:\n"
            "    A.lib()\n"
            "except ImportError as e:\n"
            "    print('refused:', e)\n"
            "    raise SystemExit(0)\n"
            "raise SystemExit(1)\n")
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "is missing" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
