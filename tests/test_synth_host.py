"""CPU checks of the host mirror of the device-side synthetic data generator
(workloads.synth_scene / synth_noise): its SplitMix64 stream reproduces the
published reference output, its noise has the CN(0, 1) moments, and its scenes
have the requested structure.  No GPU call is made."""
import numpy as np

from paper_2012_04534_amd import workloads as W


def test_splitmix64_stream_matches_reference(golden):
    want = [int(v) for v in golden("splitmix64_seed1234567.txt")]
    got = [int(v) for v in W.splitmix64_outputs(1234567, 1, len(want))]
    assert got == want
    # any window of the stream is the same stream
    assert [int(v) for v in W.splitmix64_outputs(1234567, 3, 2)] == want[2:4]


def test_noise_is_circular_standard_gaussian():
    n = W.synth_noise(400000, 11)
    assert abs(n.mean()) < 5e-3
    np.testing.assert_allclose(np.mean(np.abs(n) ** 2), 1.0, rtol=1e-2)
    np.testing.assert_allclose(np.mean(n.real ** 2), 0.5, rtol=1e-2)
    assert abs(np.mean(n.real * n.imag)) < 5e-3
    assert abs(np.mean(n * n)) < 5e-3            # circular: E n^2 = 0
    # the radius is Rayleigh: P(|n| > 2) = exp(-4)
    np.testing.assert_allclose(np.mean(np.abs(n) > 2.0), np.exp(-4.0), rtol=5e-2)
    assert not np.array_equal(W.synth_noise(8, 11), W.synth_noise(8, 12))


def test_scene_structure():
    g = W.geometry(9, 7, 40, 128)
    x = W.synth_scene(g, 25, (0.5, 1.0), 30, 35, 5)
    wall = x[:, :, 35]
    assert np.all(wall == 1.0)
    rest = x.copy()
    rest[:, :, 35] = 0
    nz = np.flatnonzero(rest)
    assert nz.size == 25                               # distinct voxels
    iz = np.unravel_index(nz, x.shape)[2]
    assert iz.max() < 30                               # above max_depth
    a = rest.reshape(-1)[nz]
    assert np.all(a.imag == 0) and a.real.min() >= 0.5 and a.real.max() <= 1.0
    # every allowed voxel drawn: the redraw-on-repeat path ends with all of them
    g2 = W.geometry(2, 2, 3, 64)
    x2 = W.synth_scene(g2, 12, (1.0, 1.0), 3, None, 9)
    assert np.all(x2 == 1.0)
