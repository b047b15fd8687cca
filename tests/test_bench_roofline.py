"""The roofline arithmetic of bench.py, pinned to closed forms on the CPU: the
per-launch method counts of the kernel classes add up over one step's
launches to the per-position counts of the step roofline (4 S M 2D FFTs; the
pattern, the object patch read twice and the object-gradient read-modify-write),
and the figures quoted for the 256 x 256, 8-mode, 30-slice group of 512 follow."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _launches(S):
    """Launches of each class in one forward + adjoint step over S slices."""
    return {"col_shift": 1, "row_fwd": S, "col_prop": S - 1, "far_loss": 1, "row_adj": S,
            "col_prop_adj": S - 1, "col_final": 1}


@pytest.mark.parametrize("N,M,S,B", [(256, 8, 30, 512), (192, 6, 20, 256), (128, 4, 8, 1024), (64, 1, 1, 256)])
def test_method_counts_add_up_to_the_step(bench, N, M, S, B):
    flops = sum(n * bench.method_flops_per_launch(k, N, M, B, S) for k, n in _launches(S).items())
    assert flops == pytest.approx(B * 4 * S * M * 5 * N * N * np.log2(N * N), rel=1e-12)
    by = sum(n * bench.method_bytes_per_launch(k, N, B, S) for k, n in _launches(S).items())
    assert by == B * (N * N * 4 + 4 * S * N * N * 8)
    # the LDS-resident chains do the same work in two launches
    res = bench.method_flops_per_launch("res_fwd", N, M, B, S) + bench.method_flops_per_launch("res_adj", N, M, B, S)
    res += sum(bench.method_flops_per_launch(k, N, M, B, S) for k in ("col_shift", "far_loss", "col_final"))
    assert res == pytest.approx(flops, rel=1e-12)


def test_step_roofline_of_the_headline_workload(bench):
    r = bench.step_roofline(256, 8, 30, 1.0 / 5966.1)
    assert r["flops_per_position"] == pytest.approx(5.0331648e9)
    assert r["bytes_per_position"] == 256 * 256 * 4 + 4 * 30 * 256 * 256 * 8 == 63176704
    assert r["bound"] == "alu"
    assert r["t_roof_us_per_position"] == pytest.approx(5.0331648e9 / 157.3e12 * 1e6, abs=1e-3)
    assert r["frac"] == pytest.approx(5.0331648e9 / 157.3e12 * 5966.1, abs=1e-4)
    # a workload with few flops per byte is bound by memory
    assert bench.step_roofline(64, 1, 1, 1e-6)["bound"] == "hbm"


def test_dominant_kernel_counts(bench):
    N, M, B, S = 256, 8, 512, 30
    # the adjoint row pass: the method's two line transforms per tile row
    assert bench.method_flops_per_launch("row_adj", N, M, B) == 2 * B * M * N * 5 * N * 8 == 21474836480
    # its method bytes: object patch read and object-gradient read-modify-write
    assert bench.method_bytes_per_launch("row_adj", N, B) == 3 * B * 8 * N * N == 805306368
    # the band limit at 2/3 of Nyquist keeps |u_x| <= 85 of 256 columns
    phi = bench.live_fraction(N, 2.0 / 3.0, S)
    assert phi == 171 / 256
    assert bench.live_fraction(N, 2.0 / 3.0, 1) == 1.0 and bench.live_fraction(N, 0.0, S) == 1.0
    # the design's tile streaming at an interior slice: B (3 M phi + 3) 8 N^2
    d = bench.kernel_bytes_per_launch("row_adj", N, M, B, S, spectral=True, live=phi)
    assert d == int(B * (3 * M * phi + 3) * 8 * N * N) == 5108662272
