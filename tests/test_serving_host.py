"""Host-side accounting of the serving loop: latency statistics from the
per-request records (no device needed)."""
import numpy as np

from paper_2505_14372_amd import serving


def _result(rid, finished_at, lat):
    z = np.zeros(1)
    return serving.Result(rid=rid, probe=z, obj=z, positions=z, losses=[], iter_latency_s=lat, admitted_at=0.0,
                          finished_at=finished_at)


def test_request_latency_is_arrival_to_completion():
    z = np.zeros(1)
    reqs = [serving.ReconRequest(rid=i, N=64, M=1, S=1, probe=z, obj=z, positions=z, patterns=z, dz=[], arrival=a)
            for i, a in enumerate([0.0, 1.0, 2.5])]
    res = {0: _result(0, 2.0, [1.0]), 1: _result(1, 4.0, [1.5]), 2: _result(2, 3.0, [0.5])}
    p50, p99 = serving.request_latency_stats(res, reqs)
    lat = np.array([2.0, 3.0, 0.5])
    assert p50 == np.percentile(lat, 50) == 2.0
    assert abs(p99 - np.percentile(lat, 99)) < 1e-12
    q50, q99 = serving.latency_stats(res)
    assert q50 == 1.0 and abs(q99 - np.percentile([1.0, 1.5, 0.5], 99)) < 1e-12
