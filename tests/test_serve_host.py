"""Host-side logic of the serving loop (no device): the per-window memory
footprint used for admission and the latency summary."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_0909_4969_amd import mach as M
from paper_0909_4969_amd import serve


def _footprint(shape, cfg=None):
    return serve.Engine.footprint(SimpleNamespace(cfg=cfg or serve.ServeConfig()), shape)


def test_footprint_is_the_sum_of_the_library_size_queries():
    cfg = serve.ServeConfig()
    shape = (64, 16, 4096)
    cap = M.nnz_capacity(shape, cfg.p)
    want = (4 * 64 * 16 * 4096 + M.sample_workspace_bytes(shape, cap)
            + M.solver_workspace_bytes(shape, cfg.ranks, cap)
            + 8 * (64 * 8 + 16 * 4 + 4096 * 16) + 8 * 8 * 4 * 16 + 64)
    assert _footprint(shape, cfg) == want


def test_footprint_grows_with_the_window_and_with_p():
    small, large = _footprint((32, 16, 1024)), _footprint((32, 16, 16384))
    assert 0 < small < large
    assert large >= 4 * 32 * 16 * 16384          # at least the dense window
    dense = serve.ServeConfig(p=0.5)
    assert _footprint((32, 16, 4096), dense) > _footprint((32, 16, 4096))


def test_latency_summary():
    rs = []
    for k in range(100):
        rs.append(serve.WindowResult(req_id=k, stream_id=k % 4, window_id=k // 4, warm=k >= 4,
                                     nnz=10, fit=0.5, factors=[], core=None,
                                     arrival_s=0.01 * k, admit_s=0.01 * k, done_s=0.01 * k + 0.001 * (k + 1),
                                     footprint=1))
    s = serve.latency_summary(rs)
    lat = np.array([1.0 * (k + 1) for k in range(100)])
    assert s["windows"] == 100
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert s["max_ms"] == pytest.approx(100.0)
    assert s["span_s"] == pytest.approx(0.99 + 0.1)
