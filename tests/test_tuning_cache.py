"""The shipped autotuner cache (tilings chosen on MI355X for the benchmarked
workloads) parses, covers every benchmarked workload and precision, and holds
only values that the tiling entry point accepts.  CPU only."""
import json
import os

import numpy as np
import pytest

from paper_2012_04534_amd import ufss
from paper_2012_04534_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIPPED = os.path.join(ROOT, "paper_2012_04534_amd", "tuning_gfx950.json")


def shape_key(name, dtype):
    w = W.workload(name)
    g = w["geom"]
    bins, _ = ufss.ufss_select_freqs(g, w["m"], w["per_position"], w["seed"])
    mu = len(np.unique(bins))
    wx = g["nx"] - 1 if g["win_x"] < 0 else min(g["win_x"], g["nx"] - 1)
    wy = g["ny"] - 1 if g["win_y"] < 0 else min(g["win_y"], g["ny"] - 1)
    return "gfx950/nx%d/ny%d/nz%d/mu%d/m%d/wx%d/wy%d/%s" % (
        g["nx"], g["ny"], g["nz"], mu, w["m"], wx, wy, dtype)


@pytest.mark.parametrize("name,dtype", [("cscan32", "f32"), ("cscan32", "bf16"),
                                        ("cscan64", "f32"), ("cscan64", "bf16")])
def test_shipped_cache_entry(name, dtype):
    cache = json.load(open(SHIPPED))
    e = cache[shape_key(name, dtype)]
    assert len(e) == 14
    fs, as_, tf, ta, nw, zs, npf, npa, rf, ra, zc, kc, bnz, aw = e
    assert 1 <= fs <= 64 and 1 <= as_ <= 64 and tf > 0 and ta > 0
    assert 1 <= nw <= 8 and 1 <= zs <= 64 and npf in (2, 4) and npa in (2, 4)
    assert rf in (1, 2) and ra in (1, 2) and zc in (8, 16) and kc in (8, 16)
    assert bnz in (2, 4)                    # BF16 adjoint depth sub-tiles (4 on FP32 entries)
    assert aw in (4, 8) and (aw == 4 or npa == 2)   # FP32 adjoint waves (8 with 2 sub-tiles only)
    assert fs * zs <= 96                    # the autotuner's bound on forward partials
