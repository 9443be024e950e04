"""Oracle forward operator A = Phi H and its adjoint (test infrastructure only).

Definition written out (Sec. II-A frequency-domain model discretised on the
G2D / G3D grids; Sec. II-B compression Phi = S F Sigma with Sigma = I, so a
measurement is one selected DFT coefficient of one A-scan):

    A[(p, m), v] = H_{k} * 1[d in W] * exp(-j 2 pi f_k (tau(d, z_v) - t0)),
    k = k_m(p),  d = p - v (lateral),  f_k = k f_s / N_t.

Layouts: x is [ny][nx][nz] (depth fastest), y is [ny][nx][m] (bin fastest);
row index (py*nx + px)*m + mi, column index (vy*nx + vx)*nz + jz.

``bins`` is int [m] (one subset shared by every position, Kronecker form of
Sec. III-A) or int [ny, nx, m] (a subset per A-scan, the "f" strategies of
Table I).  Every entry is evaluated in float64 from the closed form by
``entries``; the dense matrix, the per-position products and the sampled
products all call it, so the modes agree by construction.
"""
import math

import numpy as np

from . import geometry


def _bins_at(bins, py, px):
    bins = np.asarray(bins)
    return bins if bins.ndim == 1 else bins[py, px]


def entries(g, k, px, py, vx, vy, jz, unit_spectrum=False):
    """A entries for one scan position and a list of voxels.

    k: bins of that position [m]; vx, vy, jz: voxel indices [n].
    Returns complex128 [m, n].
    """
    k = np.asarray(k, dtype=np.float64)
    vx, vy, jz = (np.asarray(a) for a in (vx, vy, jz))
    wx, wy = geometry.window(g)
    inside = (np.abs(px - vx) <= wx) & (np.abs(py - vy) <= wy)
    ddx, ddy, z = (px - vx) * g["dx"], (py - vy) * g["dy"], geometry.depth(g, jz)
    delay = geometry.tau(g, ddx, ddy, z) - geometry.t0(g)
    beam = geometry.directivity(g, ddx, ddy, z) * inside
    f = geometry.bin_freq(g, k)
    amp = np.ones_like(f) if unit_spectrum else geometry.pulse_spectrum(g, k)
    phase = np.exp(-2j * math.pi * f[:, None] * delay[None, :])
    return amp[:, None] * phase * beam[None, :]


def _all_voxels(g):
    vy, vx, jz = np.meshgrid(np.arange(g["ny"]), np.arange(g["nx"]),
                             np.arange(g["nz"]), indexing="ij")
    return vx.reshape(-1), vy.reshape(-1), jz.reshape(-1)


def row_block(g, bins, py, px, unit_spectrum=False):
    """Rows of A for scan position (px, py): complex128 [m, ny*nx*nz]."""
    vx, vy, jz = _all_voxels(g)
    return entries(g, _bins_at(bins, py, px), px, py, vx, vy, jz, unit_spectrum)


def dense_A(g, bins, unit_spectrum=False):
    """The whole matrix A (complex128 [ny*nx*m, ny*nx*nz]); tiny grids only."""
    blocks = [row_block(g, bins, py, px, unit_spectrum)
              for py in range(g["ny"]) for px in range(g["nx"])]
    return np.concatenate(blocks, axis=0)


def apply_A(g, bins, x, unit_spectrum=False):
    """y = A x by direct sum over the voxels, one scan position at a time."""
    xv = np.asarray(x, dtype=np.complex128).reshape(-1)
    m = np.asarray(bins).shape[-1]
    y = np.empty((g["ny"], g["nx"], m), dtype=np.complex128)
    for py in range(g["ny"]):
        for px in range(g["nx"]):
            y[py, px] = row_block(g, bins, py, px, unit_spectrum) @ xv
    return y


def apply_AH(g, bins, y, unit_spectrum=False):
    """x = A^H y by direct sum over scan positions."""
    y = np.asarray(y, dtype=np.complex128)
    acc = np.zeros(g["ny"] * g["nx"] * g["nz"], dtype=np.complex128)
    for py in range(g["ny"]):
        for px in range(g["nx"]):
            acc += row_block(g, bins, py, px, unit_spectrum).conj().T @ y[py, px]
    return acc.reshape(g["ny"], g["nx"], g["nz"])


def _window_voxels(g, px, py):
    """Lateral voxels inside the window of position (px, py)."""
    wx, wy = geometry.window(g)
    xs = np.arange(max(px - wx, 0), min(px + wx, g["nx"] - 1) + 1)
    ys = np.arange(max(py - wy, 0), min(py + wy, g["ny"] - 1) + 1)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return xx.reshape(-1), yy.reshape(-1)


def apply_A_at(g, bins, x, py, px, chunk=1 << 16):
    """One row of y = A x, [m], summing only voxels inside the window.

    Used to sample outputs of full-size problems one position at a time.
    """
    x = np.asarray(x)
    k = _bins_at(bins, py, px)
    lx, ly = _window_voxels(g, px, py)
    vx = np.repeat(lx, g["nz"])
    vy = np.repeat(ly, g["nz"])
    jz = np.tile(np.arange(g["nz"]), lx.size)
    xv = x[vy, vx, jz].astype(np.complex128)
    out = np.zeros(len(k), dtype=np.complex128)
    for s in range(0, vx.size, chunk):
        e = entries(g, k, px, py, vx[s:s + chunk], vy[s:s + chunk], jz[s:s + chunk])
        out += e @ xv[s:s + chunk]
    return out


def apply_AH_at(g, bins, y, vy, vx):
    """One depth column of x = A^H y at lateral voxel (vx, vy): [nz]."""
    y = np.asarray(y)
    wx, wy = geometry.window(g)
    jz = np.arange(g["nz"])
    out = np.zeros(g["nz"], dtype=np.complex128)
    for py in range(max(vy - wy, 0), min(vy + wy, g["ny"] - 1) + 1):
        for px in range(max(vx - wx, 0), min(vx + wx, g["nx"] - 1) + 1):
            e = entries(g, _bins_at(bins, py, px), px, py,
                        np.full(g["nz"], vx), np.full(g["nz"], vy), jz)
            out += e.conj().T @ y[py, px].astype(np.complex128)
    return out


def _beam_sq_sums(g):
    """S[|dy|, |dx|] = sum over depths of g(d, z)^2 (N_z without a Gaussian beam)."""
    wx, wy = geometry.window(g)
    ady, adx = np.meshgrid(np.arange(wy + 1), np.arange(wx + 1), indexing="ij")
    z = geometry.depth(g, np.arange(g["nz"]))
    b = geometry.directivity(g, adx[..., None] * g["dx"], ady[..., None] * g["dy"], z)
    return np.sum(b * b, axis=2)


def frobenius_sq(g, bins):
    """||A||_F^2 counted from the structure of the entries.

    A non-zero entry has modulus |H_k| g(d, z), so the squared Frobenius norm
    is the sum over positions p and bins m of |H_{k_m(p)}|^2 times the sum of
    g^2 over the voxels inside the window of p (N_z times their lateral count
    without a Gaussian beam; Sec. IV-C norm bounds).
    """
    wx, wy = geometry.window(g)
    S = _beam_sq_sums(g)
    total = 0.0
    for py in range(g["ny"]):
        ry = np.abs(np.arange(max(py - wy, 0), min(py + wy, g["ny"] - 1) + 1) - py)
        for px in range(g["nx"]):
            rx = np.abs(np.arange(max(px - wx, 0), min(px + wx, g["nx"] - 1) + 1) - px)
            h = geometry.pulse_spectrum(g, _bins_at(bins, py, px))
            total += float(np.sum(h * h)) * float(S[np.ix_(ry, rx)].sum())
    return total


def central_column_sq(g, bins):
    """Squared norms of the columns of the voxel below the grid centre,
    ((N_x - 1) // 2, (N_y - 1) // 2), summed over depth.  Every position p
    whose window holds that voxel contributes sum_m |H_{k_m(p)}|^2 times the
    depth sum of g^2 at its offset."""
    wx, wy = geometry.window(g)
    S = _beam_sq_sums(g)
    vx, vy = (g["nx"] - 1) // 2, (g["ny"] - 1) // 2
    total = 0.0
    for py in range(max(vy - wy, 0), min(vy + wy, g["ny"] - 1) + 1):
        for px in range(max(vx - wx, 0), min(vx + wx, g["nx"] - 1) + 1):
            h = geometry.pulse_spectrum(g, _bins_at(bins, py, px))
            total += float(np.sum(h * h)) * float(S[abs(py - vy), abs(px - vx)])
    return total


def sigma_estimate(g, bins):
    """Sec. IV-C estimate of the largest singular value.

    ||A||_F / sqrt(N) <= sigma_max <= ||A||_F when N bounds the rank; the
    estimate is the geometric mean of the two bounds, ||A||_F / N^(1/4).
    Reading: N = min(rows, columns) = N_x N_y min(M, N_z).  The paper
    approximates ||A||_F^2 by N_x N_y times the squared norms of the central
    columns summed over depth (boundary effects neglected); both versions are
    returned.
    Returns dict(fro_sq, fro_sq_central, n, sigma_hat, sigma_hat_central).
    """
    m = bins.shape[-1]
    npos = g["nx"] * g["ny"]
    n = npos * min(m, g["nz"])
    fro = frobenius_sq(g, bins)
    cen = npos * central_column_sq(g, bins)
    return dict(fro_sq=fro, fro_sq_central=cen, n=n,
                sigma_hat=math.sqrt(fro) / n ** 0.25,
                sigma_hat_central=math.sqrt(cen) / n ** 0.25)
