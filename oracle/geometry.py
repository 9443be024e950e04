"""Oracle geometry: pulse spectrum, band, grids, delays (test infrastructure only).

A geometry is a plain ``dict`` of numbers (SI units):

    nx, ny, nz, nt        scan grid N_x x N_y, depth samples N_z, time samples N_t
    dx, dy, dz, z_start   lateral pitch, depth pitch, depth of the first voxel
    t0                    start of the time window (NaN -> centering rule below)
    c, fs, fc             speed of sound, sampling rate, pulse centre frequency
    frac_bw, band_db      -6 dB fractional bandwidth, band threshold in dB
    win_x, win_y          lateral aperture half-width in voxels (<0 -> full grid)

Sources (paper sections):
  * Sec. II-A, round-trip delay: tau = (2/c) sqrt((x-x_d)^2 + (y-y_d)^2 + z_d^2).
  * Sec. II-A, frequency-domain model: B(w) = sum a_d g H(w) exp(-j w tau).
  * Sec. II-A, grids G2D / G3D: positions n_x dx, n_y dy; voxels on the same
    lateral grid, depth on a uniform grid.
  * Sec. VI, Gabor pulse h(t) = exp(-alpha^2 t^2 + j w_c t).

Readings taken where the paper is silent or garbled:
  * Pulse width.  The printed alpha = (0.65 f_c)^2 has inconsistent units; the
    pulse is parameterised by its -6 dB fractional bandwidth b instead:
    sigma_f = b f_c / (2 sqrt(2 ln 2)), sigma_t = 1 / (2 pi sigma_f),
    h(t) = exp(-t^2 / (2 sigma_t^2)) exp(j 2 pi f_c t)  (complex Gabor, analytic).
  * Spectrum normalisation.  Unnormalised forward DFT with kernel
    exp(-j 2 pi k n / N_t); the DFT of the sampled echo then equals
    H_k exp(-j 2 pi f_k (tau - t0)) with
    H_k = f_s sqrt(2 pi) sigma_t exp(-(f_k - f_c)^2 / (2 sigma_f^2))  (real).
  * Pulse band.  {k in [0, N_t/2] : exp(-(f_k-f_c)^2/(2 sigma_f^2)) >= 10^(-band_db/20)}.
  * Depth pitch.  The printed dz = t_s c is one-way while tau is round trip;
    dz = c / (2 f_s) is used so that depth steps are whole samples.
  * Window start.  Not given; t0 centres the delay span of the aperture:
    t0 = (tau_min + tau_max)/2 - N_t / (2 f_s).
  * Directivity g.  The printed Gaussian of Sec. VI is dimensionally garbled;
    its printed x-derivative, -2 (x_1 - x_i) / (z_1 tan theta)^2 g, fixes it as
    g = exp(-r^2 / (z tan theta)^2), r the lateral distance, theta the beam's
    half-angle (geometry key ``theta``; 0 or absent: no Gaussian, g = 1).  The
    per-axis window |d_x| <= W_x, |d_y| <= W_y applies in both cases.
"""
import math

import numpy as np


def pulse_sigmas(g):
    """(sigma_f, sigma_t) of the Gaussian envelope from the -6 dB bandwidth."""
    sigma_f = g["frac_bw"] * g["fc"] / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    sigma_t = 1.0 / (2.0 * math.pi * sigma_f)
    return sigma_f, sigma_t


def bin_freq(g, k):
    """Frequency f_k = k f_s / N_t of DFT bin k (float64 array or scalar)."""
    return np.asarray(k, dtype=np.float64) * g["fs"] / g["nt"]


def pulse_spectrum(g, k):
    """H_k, the DFT of one sampled echo at zero delay (real, float64)."""
    sigma_f, sigma_t = pulse_sigmas(g)
    f = bin_freq(g, k)
    return g["fs"] * math.sqrt(2.0 * math.pi) * sigma_t * np.exp(
        -((f - g["fc"]) ** 2) / (2.0 * sigma_f ** 2))


def pulse_time(g, t):
    """Complex Gabor pulse h(t) (float64 -> complex128)."""
    _, sigma_t = pulse_sigmas(g)
    t = np.asarray(t, dtype=np.float64)
    return np.exp(-t * t / (2.0 * sigma_t ** 2)) * np.exp(2j * math.pi * g["fc"] * t)


def band(g):
    """Ascending list of DFT bins inside the pulse band (int64 array)."""
    sigma_f, _ = pulse_sigmas(g)
    k = np.arange(0, g["nt"] // 2 + 1)
    env = np.exp(-((bin_freq(g, k) - g["fc"]) ** 2) / (2.0 * sigma_f ** 2))
    return k[env >= 10.0 ** (-g["band_db"] / 20.0)]


def window(g):
    """Effective lateral half-widths (W_x, W_y) in voxels."""
    wx = g["nx"] - 1 if g["win_x"] < 0 else min(g["win_x"], g["nx"] - 1)
    wy = g["ny"] - 1 if g["win_y"] < 0 else min(g["win_y"], g["ny"] - 1)
    return wx, wy


def directivity(g, ddx, ddy, z):
    """Gaussian beam amplitude for lateral offsets (ddx, ddy) in metres at depth z."""
    ddx, ddy, z = (np.asarray(a, dtype=np.float64) for a in (ddx, ddy, z))
    theta = g.get("theta", 0.0)
    if not theta:
        return np.ones(np.broadcast(ddx, ddy, z).shape)
    w = z * math.tan(theta)
    return np.exp(-(ddx * ddx + ddy * ddy) / (w * w))


def depth(g, jz):
    """Depth z_j = z_start + j dz of depth index j (float64)."""
    return g["z_start"] + np.asarray(jz, dtype=np.float64) * g["dz"]


def tau(g, ddx, ddy, z):
    """Round-trip delay for lateral offsets (ddx, ddy) in metres and depth z."""
    ddx = np.asarray(ddx, dtype=np.float64)
    ddy = np.asarray(ddy, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    return (2.0 / g["c"]) * np.sqrt(ddx * ddx + ddy * ddy + z * z)


def t0(g):
    """Start of the recorded time window (given, or the centering rule)."""
    if not math.isnan(g["t0"]):
        return float(g["t0"])
    wx, wy = window(g)
    t_min = float(tau(g, 0.0, 0.0, depth(g, 0)))
    t_max = float(tau(g, wx * g["dx"], wy * g["dy"], depth(g, g["nz"] - 1)))
    return 0.5 * (t_min + t_max) - g["nt"] / (2.0 * g["fs"])
