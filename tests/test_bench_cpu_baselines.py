"""The CPU baselines bench.py reports: the structured FP64 baseline (one BLAS
complex GEMM per lateral offset) computes the same A and A^H as the oracle's
direct sum, and its work count equals the algorithmic count of the windowed
sum."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import operator as O  # noqa: E402
from oracle import select as S  # noqa: E402
from paper_2012_04534_amd import workloads as W  # noqa: E402


@pytest.mark.parametrize("per_pos,win,theta", [(True, -1, 0.0), (False, 2, 0.0), (True, 1, 0.5),
                                               (False, -1, 0.3)])
def test_structured_equals_oracle(per_pos, win, theta):
    g = W.geometry(6, 5, 12, 64, win_x=win, win_y=win)
    g["theta"] = theta
    bins = S.select_freqs(g, 7, per_pos, 3)
    offs = bench.window_offsets(g)
    plan = bench.structured_plan(g, bins, offs)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 1)
    y = W.cn((g["ny"], g["nx"], 7), 2)
    yo = O.apply_A(g, bins, x)
    xo = O.apply_AH(g, bins, y)
    np.testing.assert_allclose(bench.structured_forward(plan, x, offs), yo, rtol=0,
                               atol=1e-12 * np.abs(yo).max())
    np.testing.assert_allclose(bench.structured_adjoint(plan, y, offs, g["nz"]), xo, rtol=0,
                               atol=1e-12 * np.abs(xo).max())
    assert bench._offset_terms(g, 7, offs) == bench.window_terms(g, bins, per_pos)


def test_b_scan_offsets():
    """A B-scan (N_y = 1) has only d_y = 0; a window of 1 has three d_x."""
    g = W.geometry(9, 1, 8, 64, win_x=1, win_y=-1)
    assert bench.window_offsets(g) == [(0, -1), (0, 0), (0, 1)]
    bins = S.select_freqs(g, 4, False, 1)
    offs = bench.window_offsets(g)
    x = W.cn((1, 9, 8), 4)
    np.testing.assert_allclose(bench.structured_forward(bench.structured_plan(g, bins, offs), x, offs),
                               O.apply_A(g, bins, x), rtol=1e-12, atol=1e-12)


def test_traffic_entry_needs_the_measured_source(monkeypatch):
    """A counted traffic figure is reported only for the kernel source it was
    measured on (same SHA-256 prefix) and for the same tiling; otherwise null."""
    key = next(iter(bench.TRAFFIC))
    workload, algo, direction, _ = key.split("/")
    entry = bench.TRAFFIC[key]
    info = {"fwd_split": 4, "fwd_zsplit": 8, "fwd_waves": 5, "fwd_tile": 2, "fwd_chunk": 8,
            "adj_split": 12, "adj_tile": 2, "adj_chunk": 16}
    monkeypatch.setattr(bench, "tiling_key", lambda i, d: key.split("/")[3])
    monkeypatch.setattr(bench, "source_sha", lambda rel: entry["sha"])
    assert bench.traffic_bytes(workload, algo, direction, info) == int(entry["bytes"])
    monkeypatch.setattr(bench, "source_sha", lambda rel: "0" * 16)
    assert bench.traffic_bytes(workload, algo, direction, info) is None
    monkeypatch.setattr(bench, "source_sha", lambda rel: entry["sha"])
    monkeypatch.setattr(bench, "tiling_key", lambda i, d: "another-tiling")
    assert bench.traffic_bytes(workload, algo, direction, info) is None
