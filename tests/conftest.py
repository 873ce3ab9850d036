import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def rocrand_philox():
    """rocRAND's Philox4x32-10 engine driven on the host with a raw
    counter/key: an implementation independent of the oracle and of the GPU
    library."""
    import ctypes
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox.cpp")
    out_dir = tempfile.mkdtemp(prefix="rr_philox_")
    so = os.path.join(out_dir, "rr_philox.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.run([hipcc, "-O2", "-fPIC", "-shared", "--offload-arch=gfx950", "-o", so, src],
                   check=True, cwd=out_dir)
    lib = ctypes.CDLL(so)
    lib.rr_philox_batch.argtypes = [ctypes.c_longlong, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]

    def run(ctr, key):
        import numpy as np
        c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
        o = np.empty_like(c)
        lib.rr_philox_batch(c.shape[0], c.ctypes.data, k.ctypes.data, o.ctypes.data)
        return o
    return run
