"""ara_run_static, the entry point for callers that cannot allocate device
memory: its results equal ara_run's (same kernels; the hand-over scratch is
the library's static device array instead of the caller's), on two calls in a
row through the C-ABI, the second with a smaller input, with rows that go
through the FP64-capable second pass; runs beyond its trial limit are refused
before anything is enqueued."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ara():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06326_amd import Ara
    a = Ara(0)
    yield a
    a.close()


def _opts(A, begin, count, scratch=None):
    return A.ara_run_opts(trial_begin=begin, trial_count=count, sum_mode=A.ARA_SUM_KAHAN32,
                          ylt_dtype=A.ARA_F32, tail_band=0.0, debug_flags=0, d_hits=None,
                          d_hit_chk=None,
                          d_scratch=None if scratch is None else scratch.data_ptr(),
                          scratch_bytes=0 if scratch is None else scratch.numel(),
                          d_occ_view=None, occ_view_stride=0)


def test_static_scratch_run_equals_ara_run(ara):
    from paper_1501_06326_amd import ara as A
    from workloads import config_small, varied_shapes
    w = config_small(corr=True, n_trials=6000)
    y = ara.load_yet(w.yet)
    pfs = [ara.load_portfolio(w.portfolio, w.yet.n_catalogue),
           ara.load_portfolio(varied_shapes(config_small(n_trials=10).portfolio),
                              w.yet.n_catalogue)]
    dev = ara.device
    for p in pfs:
        for begin, count in ((0, 6000), (1234, 777)):     # second call: a smaller input
            print("static scratch run", begin, count, flush=True)
            out_l = torch.full((p.n_layers, count), -1.0, dtype=torch.float32, device=dev)
            out_p = torch.full((count,), -1.0, dtype=torch.float32, device=dev)
            A.ara_run_static(ara.ctx, y.handle, p.handle, _opts(A, begin, count),
                             out_l.data_ptr(), out_p.data_ptr(), None)
            A.ara_sync_status(ara.ctx, None)
            ref_l = torch.empty_like(out_l)
            ref_p = torch.empty_like(out_p)
            sc = torch.empty(A.ara_run_scratch_size(count), dtype=torch.uint8, device=dev)
            A.ara_run(ara.ctx, y.handle, p.handle, _opts(A, begin, count, sc), ref_l.data_ptr(),
                      ref_p.data_ptr(), None)
            A.ara_sync_status(ara.ctx, None)
            assert torch.equal(out_l, ref_l)
            assert torch.equal(out_p, ref_p)


def test_static_scratch_limit(ara):
    from paper_1501_06326_amd import ara as A
    from workloads import config_small
    w = config_small(n_trials=100)
    y = ara.load_yet(w.yet)
    p = ara.load_portfolio(w.portfolio, w.yet.n_catalogue)
    out = torch.empty(100, dtype=torch.float32, device=ara.device)
    o = _opts(A, 0, A.ARA_STATIC_MAX_TRIALS + 1)
    rc = A.lib().ara_run_static(ara.ctx, y.handle, p.handle, o, None, out.data_ptr(), None)
    assert rc == A.ARA_E_WORKSPACE_TOO_SMALL
