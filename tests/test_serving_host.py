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


def test_object_error_is_relative_to_the_scanned_region():
    """The accuracy score of a served reconstruction: 0 at the truth, 1 at the
    vacuum start, and only the region the windows cover counts."""
    rng = np.random.default_rng(0)
    N, S, H, W = 8, 2, 30, 26
    truth = np.exp(0.2j * rng.random((S, H, W)))
    pos = np.array([[2.2, 3.0], [10.4, 12.6]])     # windows cover rows 2..18, cols 3..21
    req = serving.ReconRequest(rid=0, N=N, M=1, S=S, probe=np.zeros((1, N, N)), obj=np.ones((S, H, W)),
                               positions=pos, patterns=np.zeros((2, N, N)), dz=[2.0], truth=truth)
    assert serving.object_error(truth, req) == 0.0
    assert abs(serving.object_error(np.ones((S, H, W)), req) - 1.0) < 1e-12
    off = truth.copy()
    off[:, 25:, :] = 5.0                             # outside every window: not scored
    assert serving.object_error(off, req) == 0.0
    half = truth.copy()
    half[:, 2:19, 3:22] = 0.5 * (truth[:, 2:19, 3:22] + 1.0)
    assert abs(serving.object_error(half, req) - 0.5) < 1e-12
