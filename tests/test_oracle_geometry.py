"""Pins of the oracle's geometry and bin selection against closed forms,
hand-computed values and a published generator test vector (CPU only)."""
import math

import numpy as np
import pytest

from oracle import geometry as G
from oracle import select as S
from paper_2012_04534_amd import workloads as W


def test_splitmix64_reference_vector(golden):
    """SplitMix64 reproduces the reference implementation's output."""
    want = [int(v) for v in golden("splitmix64_seed1234567.txt")]
    rng = S.SplitMix64(1234567)
    assert [rng.next() for _ in want] == want


def test_round_trip_delay_closed_forms():
    """Sec. II-A delay: twice the straight-line distance over c."""
    g = W.geometry(4, 4, 4, 64)
    # 3-4-5 triangle: lateral 3 mm, depth 4 mm -> path 5 mm each way.
    assert G.tau(g, 3e-3, 0.0, 4e-3) == pytest.approx(2 * 5e-3 / g["c"], rel=1e-15)
    assert G.tau(g, 0.0, 3e-3, 4e-3) == pytest.approx(2 * 5e-3 / g["c"], rel=1e-15)
    assert G.tau(g, 2e-3, 3e-3, 6e-3) == pytest.approx(2 * 7e-3 / g["c"], rel=1e-15)
    # depth pitch c/(2 fs): one depth step under the transducer is one sample
    steps = np.diff(G.tau(g, 0.0, 0.0, G.depth(g, np.arange(10))))
    np.testing.assert_allclose(steps * g["fs"], 1.0, rtol=1e-9)


def test_band_edges_hand_computed():
    """-40 dB band: |f - fc| <= sigma_f sqrt(2 ln 100), sigma_f = b fc / (2 sqrt(2 ln 2)).

    sigma_f = 0.5 * 4 MHz / 2.35482 = 0.849322 MHz; half-width 2.57746 MHz,
    so f in [1.42254, 6.57746] MHz.  Bin spacing fs/N_t = 40 MHz / N_t.
    """
    half = 0.849321800288 * math.sqrt(2 * math.log(100.0))
    for nt, lo, hi in [(256, 10, 42), (512, 19, 84), (1024, 37, 168), (64, 3, 10)]:
        b = G.band(W.geometry(8, 1, 8, nt))
        assert (b[0], b[-1], len(b)) == (lo, hi, hi - lo + 1)
        df = 40e6 / nt
        assert abs(lo * df - 4e6) <= half * 1e6 < abs((lo - 1) * df - 4e6)
        assert abs(hi * df - 4e6) <= half * 1e6 < abs((hi + 1) * df - 4e6)


def test_pulse_spectrum_matches_numerical_fourier_integral():
    """H_k / f_s equals the continuous Fourier transform of h(t) at f_k,
    integrated numerically (independent of the Gaussian closed form)."""
    g = W.geometry(4, 1, 4, 256)
    _, st = G.pulse_sigmas(g)
    t = np.linspace(-12 * st, 12 * st, 200001)
    h = G.pulse_time(g, t)
    for k in [10, 20, 26, 33, 42, 60]:
        f = k * g["fs"] / g["nt"]
        integrand = h * np.exp(-2j * math.pi * f * t)
        val = np.trapezoid(integrand, t) if hasattr(np, "trapezoid") else np.trapz(integrand, t)
        assert abs(val * g["fs"] - G.pulse_spectrum(g, k)) < 1e-9 * G.pulse_spectrum(g, 26)


def test_pulse_spectrum_peak_and_bandwidth():
    """Peak f_s sqrt(2 pi) sigma_t; the -6 dB full width equals b * fc."""
    g = W.geometry(4, 1, 4, 256)
    sf, st = G.pulse_sigmas(g)
    assert st == pytest.approx(1.0 / (2 * math.pi * sf), rel=1e-15)
    peak = g["fs"] * math.sqrt(2 * math.pi) * st
    assert peak == pytest.approx(18.7886, rel=1e-4)
    # -6 dB (half amplitude) half-width of the envelope equals b fc / 2
    f_half = g["fc"] + 0.5 * g["frac_bw"] * g["fc"]
    env = math.exp(-((f_half - g["fc"]) ** 2) / (2 * sf * sf))
    assert env == pytest.approx(0.5, rel=1e-12)


def test_window_start_contains_every_echo():
    """The centred window holds each in-aperture echo with > 4 sigma_t margin."""
    for name in ["bscan32", "cscan32", "cscan64"]:
        g = W.workload(name)["geom"]
        _, st = G.pulse_sigmas(g)
        wx, wy = G.window(g)
        start = G.t0(g)
        end = start + g["nt"] / g["fs"]
        t_min = G.tau(g, 0.0, 0.0, G.depth(g, 0))
        t_max = G.tau(g, wx * g["dx"], wy * g["dy"], G.depth(g, g["nz"] - 1))
        assert t_min - start > 4 * st and end - t_max > 4 * st
        assert (t_min - start) == pytest.approx(end - t_max, rel=1e-12)
    # explicit t0 is honoured
    g = W.geometry(4, 1, 4, 64, t0=5e-6)
    assert G.t0(g) == 5e-6


def test_select_shared_and_per_position_properties():
    g = W.geometry(6, 5, 8, 256)
    band = G.band(g)
    s = S.select_freqs(g, 20, False, 77)
    assert s.shape == (20,) and np.all(np.diff(s) > 0) and set(s) <= set(band)
    assert np.array_equal(s, S.select_freqs(g, 20, False, 77))
    assert not np.array_equal(s, S.select_freqs(g, 20, False, 78))
    p = S.select_freqs(g, 20, True, 77)
    assert p.shape == (5, 6, 20)
    assert all(np.all(np.diff(p[iy, ix]) > 0) for iy in range(5) for ix in range(6))
    assert len({tuple(p[iy, ix]) for iy in range(5) for ix in range(6)}) > 20
    full = S.select_freqs(g, len(band), False, 3)
    assert np.array_equal(full, band)
    with pytest.raises(ValueError):
        S.select_freqs(g, len(band) + 1, False, 3)


def test_select_is_uniform_over_band():
    """Each band bin is kept with probability m/|band| (chi-square, 2000 draws)."""
    g = W.geometry(8, 1, 8, 256)
    band = G.band(g)
    counts = np.zeros(len(band))
    draws = 2000
    for s in range(draws):
        sel = S.select_freqs(g, 8, False, s)
        counts[np.searchsorted(band, sel)] += 1
    expect = draws * 8 / len(band)
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    # 32 dof: the 99.9% quantile is 62.5
    assert chi2 < 62.5


def test_select_draw_by_hand():
    """First swap partner of the Fisher-Yates draw equals the multiply-high
    bound of the first SplitMix64 output (checked for a 5-element pool)."""
    pool = [10, 11, 12, 13, 14]
    v = S.SplitMix64(1234567).next()
    j = (v * 5) >> 64
    got = S.draw_subset(pool, 1, 1234567)
    assert got == [pool[j]]


def test_sim50_replica_geometry():
    """Table III readings: the Gaussian envelope exp(-alpha t^2) with alpha =
    (0.65 f_c)^2 has the -6 dB bandwidth the workload uses; every delay of the
    full aperture, with three pulse widths on either side, lies inside the
    window [t0, t0 + N_t / f_s); the first voxel sits at the window start
    (t0 = 10 us = 2 z_d / c0 up to 0.1%)."""
    import math
    from paper_2012_04534_amd import workloads as W
    g = W.sim_geometry()
    sigma_f, sigma_t = G.pulse_sigmas(g)
    alpha = (0.65 * g["fc"]) ** 2
    assert 1.0 / (2.0 * sigma_t ** 2) == pytest.approx(alpha, rel=1e-12)
    tmin = float(G.tau(g, 0.0, 0.0, G.depth(g, 0)))
    far = float(G.tau(g, (g["nx"] - 1) * g["dx"], (g["ny"] - 1) * g["dy"],
                      G.depth(g, g["nz"] - 1)))
    assert tmin == pytest.approx(g["t0"], rel=1e-3)
    assert far + 3 * sigma_t < g["t0"] + g["nt"] / g["fs"]
    assert np.count_nonzero(W.sim_line(g)) == 30
    rect = W.sim_rectangle(g)
    assert np.count_nonzero(rect) == 28 * 40
    iy, ix, iz = np.nonzero(rect)
    assert np.all(iz - ix == iz[0] - ix[0])          # 45 degrees in the z-x plane
    assert np.allclose(rect[rect != 0], np.exp(1j * math.pi / 4))


def test_directivity_matches_printed_derivative():
    """Sec. VI prints dg/dx_1 = -2 (x_1 - x_i) / (z_1 tan theta)^2 g for the
    Gaussian beam; a central difference of the oracle's g reproduces it, so
    g = exp(-r^2 / (z tan theta)^2) (the printed g itself is garbled)."""
    g = W.geometry(4, 4, 4, 64)
    g["theta"] = math.radians(30.0)
    z = 31.2e-3
    for ddx, ddy in ((0.0, 0.0), (2.5e-3, 0.0), (-4e-3, 1.5e-3), (9e-3, -7e-3)):
        h = 1e-7
        fd = (G.directivity(g, ddx + h, ddy, z) - G.directivity(g, ddx - h, ddy, z)) / (2 * h)
        printed = -2.0 * ddx / (z * math.tan(g["theta"])) ** 2 * G.directivity(g, ddx, ddy, z)
        assert float(fd) == pytest.approx(float(printed), rel=1e-6, abs=1e-9)


def test_directivity_shape():
    """The beam falls to 1/e at lateral distance z tan theta, is separable in
    x and y, is 1 on axis, and tends to 1 everywhere as theta -> 90 deg; with
    no theta the geometry has no Gaussian factor."""
    g = W.geometry(4, 4, 4, 64)
    g["theta"] = math.radians(30.0)
    z = 40e-3
    r = z * math.tan(g["theta"])
    assert float(G.directivity(g, r, 0.0, z)) == pytest.approx(math.exp(-1.0), rel=1e-14)
    assert float(G.directivity(g, 0.6 * r, 0.8 * r, z)) == pytest.approx(math.exp(-1.0), rel=1e-14)
    a = G.directivity(g, 3e-3, 5e-3, z)
    assert float(a) == pytest.approx(float(G.directivity(g, 3e-3, 0.0, z) *
                                           G.directivity(g, 0.0, 5e-3, z)), rel=1e-14)
    assert float(G.directivity(g, 0.0, 0.0, z)) == 1.0
    g["theta"] = math.radians(89.9999)
    assert float(G.directivity(g, 10e-3, 10e-3, z)) > 1.0 - 1e-9
    g["theta"] = 0.0
    assert float(G.directivity(g, 10e-3, 10e-3, z)) == 1.0
