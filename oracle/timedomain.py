"""Oracle time-domain pulse-echo A-scans (test infrastructure only).

Sec. II-A pulse-echo model: the analytic A-scan at position p is the sum over
reflectors of a_v g h(t - tau) (g: the beam amplitude of the geometry); sampling at t = t0 + n / f_s gives b_p[n].
The DFT of one recorded window equals the frequency-domain operator exactly
when the record is the periodised echo (Poisson summation), so the samples
are summed over whole-window shifts q in {-2..2}; terms further out are below
exp(-100) for every geometry used in the tests.

This module never uses the frequency-domain formula: it is the independent
side of the check "the full set of bins equals the DFT of the time-domain
model".
"""
import numpy as np

from . import geometry


def ascans(g, x, shifts=2):
    """b [ny, nx, nt] complex128: periodised sampled echoes of the scene x."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    wx, wy = geometry.window(g)
    vy, vx, jz = np.meshgrid(np.arange(g["ny"]), np.arange(g["nx"]),
                             np.arange(g["nz"]), indexing="ij")
    vy, vx, jz = vy.reshape(-1), vx.reshape(-1), jz.reshape(-1)
    nz_mask = x != 0
    t_start = geometry.t0(g)
    n = np.arange(g["nt"], dtype=np.float64)
    b = np.zeros((g["ny"], g["nx"], g["nt"]), dtype=np.complex128)
    for py in range(g["ny"]):
        for px in range(g["nx"]):
            sel = nz_mask & (np.abs(px - vx) <= wx) & (np.abs(py - vy) <= wy)
            if not np.any(sel):
                continue
            ddx, ddy = (px - vx[sel]) * g["dx"], (py - vy[sel]) * g["dy"]
            z = geometry.depth(g, jz[sel])
            delay = geometry.tau(g, ddx, ddy, z)
            refl = x[sel] * geometry.directivity(g, ddx, ddy, z)
            acc = np.zeros(g["nt"], dtype=np.complex128)
            for q in range(-shifts, shifts + 1):
                t = t_start + (n[None, :] + q * g["nt"]) / g["fs"] - delay[:, None]
                acc += (refl[:, None] * geometry.pulse_time(g, t)).sum(axis=0)
            b[py, px] = acc
    return b
