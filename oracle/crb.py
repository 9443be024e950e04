"""Oracle Cramer-Rao bound for locating one scatterer (test infrastructure only).

Sec. VI (asymptotic performance): the measurements of one point scatterer at
p = (x_1, y_1, z_1) with complex amplitude a e^{j phi} are, at scan position i
and selected DFT bin k,

    b_{i,k}(u) = a e^{j phi} H_k g_i(p) exp(-j 2 pi f_k (tau_i(p) - t0)),

u = (x_1, y_1, z_1, a, phi), observed in circular white noise of variance
sigma^2.  The Slepian-Bangs Fisher information is
J = (2 / sigma^2) Re{ D^H D } with D the matrix of derivatives d b / d u^T over
every measured (i, k), and the bound on the position is the upper-left 3 x 3
block of J^{-1}; the paper writes that block with the Schur complement of the
nuisance block (a, phi).

Readings (the printed derivatives are partly garbled):
  * tau_i = (2 / c) R_i, R_i = sqrt((x_1 - x_i)^2 + (y_1 - y_i)^2 + z_1^2), so
    d tau / d x_1 = (2 / c)(x_1 - x_i) / R_i (printed with c/2, which has the
    wrong units) and d tau / d z_1 = (2 / c) z_1 / R_i;
  * g_i = exp(-r_i^2 / (z_1 tan theta)^2) (the Gaussian beam of the geometry;
    g = 1 without one): d g / d x_1 = -2 (x_1 - x_i) / (z_1 tan theta)^2 g (as
    printed) and d g / d z_1 = 2 r_i^2 / (z_1^3 tan^2 theta) g (the printed form
    is garbled);
  * the aperture window keeps the positions with |x_1 - x_i| <= W_x dx and
    |y_1 - y_i| <= W_y dy (its edges are not differentiated);
  * scan positions sit at (i_x dx, i_y dy); the measured bins are those of the
    operator, k in [0, N_t / 2], with H_k and f_k as there.
"""
import math

import numpy as np

from . import geometry


def model(g, bins, u):
    """b for parameters u = (x1, y1, z1, a, phi): list of complex128 arrays,
    one per scan position (the bins of that position), in row-major order."""
    x1, y1, z1, a, phi = (float(v) for v in u)
    wx, wy = geometry.window(g)
    out = []
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            k = np.asarray(bins if np.ndim(bins) == 1 else bins[iy, ix])
            dxm, dym = x1 - ix * g["dx"], y1 - iy * g["dy"]
            if abs(dxm) > wx * g["dx"] + 1e-12 or abs(dym) > wy * g["dy"] + 1e-12:
                out.append(np.zeros(len(k), complex))
                continue
            tau = geometry.tau(g, dxm, dym, z1)
            beam = geometry.directivity(g, dxm, dym, z1)
            f = geometry.bin_freq(g, k)
            out.append(a * np.exp(1j * phi) * geometry.pulse_spectrum(g, k) * beam *
                       np.exp(-2j * math.pi * f * (tau - geometry.t0(g))))
    return out


def derivatives(g, bins, u):
    """D = d b / d u^T, complex128 [n_meas, 5], from the closed-form derivatives."""
    x1, y1, z1, a, phi = (float(v) for v in u)
    theta = g.get("theta", 0.0)
    rows = []
    b = model(g, bins, u)
    idx = 0
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            bi = b[idx]
            idx += 1
            k = np.asarray(bins if np.ndim(bins) == 1 else bins[iy, ix])
            dxm, dym = x1 - ix * g["dx"], y1 - iy * g["dy"]
            R = math.sqrt(dxm * dxm + dym * dym + z1 * z1)
            tx, ty, tz = (2.0 / g["c"]) * dxm / R, (2.0 / g["c"]) * dym / R, (2.0 / g["c"]) * z1 / R
            if theta:
                w2 = (z1 * math.tan(theta)) ** 2
                gx, gy = -2.0 * dxm / w2, -2.0 * dym / w2
                gz = 2.0 * (dxm * dxm + dym * dym) / (z1 ** 3 * math.tan(theta) ** 2)
            else:
                gx = gy = gz = 0.0
            om = 2.0 * math.pi * geometry.bin_freq(g, k)
            D = np.stack([bi * (gx - 1j * om * tx), bi * (gy - 1j * om * ty),
                          bi * (gz - 1j * om * tz), bi / a, 1j * bi], axis=1)
            rows.append(D)
    return np.concatenate(rows, axis=0)


def fisher(g, bins, u, sigma2):
    """Slepian-Bangs FIM (2 / sigma^2) Re{D^H D}, float64 [5, 5]."""
    D = derivatives(g, bins, u)
    return (2.0 / sigma2) * np.real(D.conj().T @ D)


def crb_position(J):
    """[C_x, C_y, C_z]: diagonal of the position block of J^{-1}, by the Schur
    complement of the nuisance block as in the paper."""
    Jp, Jpn, Jn = J[:3, :3], J[:3, 3:], J[3:, 3:]
    Jp_inv = np.linalg.inv(Jp)
    Q = Jn - Jpn.T @ Jp_inv @ Jpn
    C = Jp_inv + Jp_inv @ Jpn @ np.linalg.inv(Q) @ Jpn.T @ Jp_inv
    return np.diag(C).copy()


def fisher_mixed(g, bins, signs, u, sigma2):
    """FIM of mixed measurements (Rademacher Sigma, Sec. III-A): position i
    measures M_i B_i with M_i the rows of S_i F Sigma_i F^{-1} over every DFT
    index (signed bins), so the derivative rows are M_i D_i with D_i over all
    N_t signed bins; J = (2 / sigma^2) Re{sum_i (M_i D_i)^H (M_i D_i)}."""
    from . import mixing as X
    nt = g["nt"]
    full = X.signed_bins(nt)
    D = derivatives(g, full, u)                      # [npos * nt, 5], position-major
    J = np.zeros((5, 5))
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            p = iy * g["nx"] + ix
            k = bins if np.ndim(bins) == 1 else bins[iy, ix]
            xi = signs if np.ndim(signs) == 1 else signs[iy, ix]
            MD = X.mixing_rows(g, k, xi) @ D[p * nt:(p + 1) * nt]
            J += np.real(MD.conj().T @ MD)
    return (2.0 / sigma2) * J
