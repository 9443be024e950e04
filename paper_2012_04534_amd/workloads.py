"""Synthetic workloads: geometry parameters and seeded input generators.

This module holds numbers and random draws only -- none of the method's
arithmetic (no pulse spectrum, no delays, no operator).  Both the HIP path and
the FP64 oracle take their inputs from here.

Geometry parameters follow the simulation setup of the paper (Sec. VII and
its Table III) where it gives them, with these choices where it does not:
  * c = 5900 m/s, f_s = 40 MHz, f_c = 4 MHz, -6 dB fractional bandwidth 0.5;
  * lateral pitch 0.5 mm; depth pitch c / (2 f_s) = 73.75 um (whole samples);
  * first voxel at 29.6 mm depth (the imaging region of Sec. VII);
  * t0 = NaN asks for the window that centres the aperture's delay span;
  * pulse band: bins within 40 dB of the spectral peak.

Workloads (one per measured configuration):
  bscan32   B-scan, 32 positions, 32 x 128 voxels, N_t = 256, 32 shared bins
  cscan32   C-scan, 32 x 32 positions, 32 x 32 x 256 voxels, N_t = 512,
            64 bins drawn per position, full aperture
  cscan64   C-scan, 64 x 64 positions, 64 x 64 x 512 voxels, N_t = 1024,
            128 shared bins, aperture window of +-16 voxels
  sim50     the simulated specimen of Sec. VII / Table III: 50 x 50 positions,
            50 depths, f_c = 3.2 MHz, f_s = 20 MHz, c = 5920 m/s, t0 = 10 us,
            N_t = 256, full aperture with a Gaussian beam of half-angle 30
            degrees; line and tilted-rectangle defects of
            amplitude exp(j pi/4), noise free; n_f in {1, 2, 5, 10}
Scenes are distinct on-grid point scatterers; noise is circular complex
Gaussian scaled to a target SNR over all measured values (the scaling needs
||A x||, which the caller computes with its own operator).
"""
import math

import numpy as np

C_SOUND = 5900.0
FS = 40e6
FC = 4e6
FRAC_BW = 0.5
BAND_DB = 40.0
PITCH = 0.5e-3
DZ = 73.75e-6          # c / (2 f_s) for the values above
Z_START = 29.6e-3

DTYPE_F32 = 0
DTYPE_BF16 = 1


def geometry(nx, ny, nz, nt, win_x=-1, win_y=-1, t0=float("nan"), **over):
    """Geometry dict (SI units) with the common physical constants."""
    g = dict(nx=nx, ny=ny, nz=nz, nt=nt, dx=PITCH, dy=PITCH, dz=DZ,
             z_start=Z_START, t0=t0, c=C_SOUND, fs=FS, fc=FC,
             frac_bw=FRAC_BW, band_db=BAND_DB, win_x=win_x, win_y=win_y, theta=0.0)
    g.update(over)
    return g


WORKLOADS = {
    "bscan32": dict(
        geom=geometry(32, 1, 128, 256), m=32, per_position=False, seed=1001,
        n_scat=3, amp=(1.0, 1.0), snr_db=20.0, iters=200, mu=0.1, back_wall=None),
    "cscan32": dict(
        geom=geometry(32, 32, 256, 512), m=64, per_position=True, seed=1002,
        n_scat=20, amp=(0.5, 1.0), snr_db=10.0, iters=100, mu=0.1, back_wall=240),
    "cscan64": dict(
        geom=geometry(64, 64, 512, 1024, win_x=16, win_y=16), m=128,
        per_position=False, seed=1003, n_scat=50, amp=(0.5, 1.0), snr_db=15.0,
        iters=100, mu=0.1, back_wall=None),
}


# Sec. VII simulation (Table III).  Readings: the garbled "N_z = 20 MHz" entry
# is the sampling rate; alpha = (0.65 f_c)^2 is the envelope exp(-alpha t^2), so
# sigma_t = 1 / (0.65 f_c sqrt(2)) and the -6 dB fractional bandwidth is
# 2 sqrt(2 ln 2) * 0.65 sqrt(2) / (2 pi) = 0.3445; N_t (not given) = 256 covers
# the delays of the whole aperture from t0 = 10 us; depth pitch c / (2 f_s);
# Gaussian beam of half-angle theta = 30 degrees over the full aperture.
SIM_FRAC_BW = 2.0 * math.sqrt(2.0 * math.log(2.0)) * 0.65 * math.sqrt(2.0) / (2.0 * math.pi)
SIM50 = dict(nx=50, ny=50, nz=50, nt=256, c=5920.0, fs=20e6, fc=3.2e6, t0=10e-6,
             z_start=29.6e-3, dx=0.5e-3, dy=0.5e-3, dz=5920.0 / (2 * 20e6),
             frac_bw=SIM_FRAC_BW, band_db=40.0, win_x=-1, win_y=-1,
             theta=math.radians(30.0))
SIM_NF = (1, 2, 5, 10)
SIM_ITERS = 80
SIM_MU = (0.1, 0.6)
SIM_AMP = complex(math.cos(math.pi / 4), math.sin(math.pi / 4))


def sim_geometry():
    return dict(SIM50)


def sim_line(g=None, depth=25, x_span=(10, 40)):
    """Line defect along x at the centre row, one depth (Sec. VII, first scene)."""
    g = g or SIM50
    x = np.zeros((g["ny"], g["nx"], g["nz"]), dtype=np.complex128)
    x[g["ny"] // 2, x_span[0]:x_span[1], depth] = SIM_AMP
    return x


def sim_rectangle(g=None, diag=40, width=40):
    """Rectangle tilted by 45 degrees in the z-x plane: ``diag`` voxels of
    length along the diagonal (diag / sqrt 2 steps in x and z) and ``width``
    voxels along y, centred in the volume (Sec. VII, second scene)."""
    g = g or SIM50
    n = int(round(diag / math.sqrt(2.0)))
    x0 = (g["nx"] - n) // 2
    z0 = (g["nz"] - n) // 2
    y0 = (g["ny"] - width) // 2
    x = np.zeros((g["ny"], g["nx"], g["nz"]), dtype=np.complex128)
    for i in range(n):
        x[y0:y0 + width, x0 + i, z0 + i] = SIM_AMP
    return x


def batch_workload(seed=1004, n=64, max_lateral=64, max_depth=512):
    """Uneven batch of scans: list of dicts like WORKLOADS entries.

    Per scan: B-scan or C-scan with probability 1/2; lateral size U{16..64}
    per side; depth N_z in {128, 192, ..., 512} with N_t = 2 N_z; M = U{32..128}
    (capped by the caller at the band size); shared or per-position bins with
    probability 1/2; aperture window +-16 for C-scans, full for B-scans;
    5-50 scatterers; SNR U[10, 25] dB.  ``max_lateral`` / ``max_depth`` shrink
    the draw for quick tests.
    """
    rng = np.random.default_rng(seed)
    out = []
    depths = [d for d in range(128, 513, 64) if d <= max_depth] or [min(max_depth, 128)]
    for i in range(n):
        three_d = bool(rng.integers(2))
        nx = int(rng.integers(16, max_lateral + 1))
        ny = int(rng.integers(16, max_lateral + 1)) if three_d else 1
        nz = int(depths[rng.integers(len(depths))])
        nt = 2 * nz
        m = int(rng.integers(32, 129))
        per_pos = bool(rng.integers(2))
        win = 16 if three_d else -1
        g = geometry(nx, ny, nz, nt, win_x=win, win_y=win)
        out.append(dict(geom=g, m=m, per_position=per_pos, seed=seed * 1000 + i,
                        n_scat=int(rng.integers(5, 51)), amp=(0.5, 1.0),
                        snr_db=float(rng.uniform(10.0, 25.0)), iters=100, mu=0.1,
                        back_wall=None))
    return out


def workload(name):
    w = dict(WORKLOADS[name])
    w["geom"] = dict(w["geom"])
    return w


def subvolume(g, nx, ny, nz):
    """Smaller grid with the same physics; t0 is pinned by the caller."""
    s = dict(g)
    s.update(nx=nx, ny=ny, nz=nz)
    return s


def scene(g, n_scat, amp=(1.0, 1.0), seed=0, back_wall=None, phase=0.0,
          max_depth=None):
    """Sparse reflectivity [ny, nx, nz] complex128 with distinct voxels.

    Scatterer depths are drawn below ``max_depth`` (default: all depths, or
    24 samples above a back wall).  A back wall sets every lateral voxel at
    depth index ``back_wall`` to amplitude 1.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    if max_depth is None:
        max_depth = nz if back_wall is None else back_wall - 8
    x = np.zeros((ny, nx, nz), dtype=np.complex128)
    flat = rng.choice(ny * nx * max_depth, size=n_scat, replace=False)
    iy, rem = np.divmod(flat, nx * max_depth)
    ix, iz = np.divmod(rem, max_depth)
    a = rng.uniform(amp[0], amp[1], size=n_scat) if amp[0] != amp[1] else np.full(n_scat, amp[0])
    x[iy, ix, iz] = a * np.exp(1j * phase)
    if back_wall is not None:
        x[:, :, back_wall] = 1.0
    return x


# Counter-based generator of the device-side synthetic data (the library's
# ufss_synth_scene / ufss_synth_measure draw the same numbers): SplitMix64
# (Steele, Lea & Flood 2014), whose k-th output of the stream keyed s is
# mix64(s + k gamma).
_SM_MASK = (1 << 64) - 1
_SM_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_outputs(seed, first, count):
    """Outputs first .. first + count - 1 (1-based) of the stream keyed seed (uint64)."""
    k = np.arange(first, first + count, dtype=np.uint64)
    z = (np.uint64(seed & _SM_MASK) + k * np.uint64(_SM_GAMMA))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def synth_scene(g, n_scat, amp, max_depth, back_wall, seed):
    """The scene ufss_synth_scene draws on the device, [ny, nx, nz] complex128:
    n_scat distinct voxels with depth index < max_depth (index j of scatterer j
    = floor(out N / 2^64) over the N = ny nx max_depth allowed voxels, redrawn
    on repeats), then the amplitudes lo + (hi - lo) (out >> 11) 2^-53, plus a
    back wall of amplitude 1 at depth index back_wall (None: none)."""
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    nallow = ny * nx * max_depth
    x = np.zeros((ny, nx, nz), dtype=np.complex128)
    if back_wall is not None:
        x[:, :, back_wall] = 1.0
    k = 1
    chosen = []
    while len(chosen) < n_scat:
        v = (int(splitmix64_outputs(seed, k, 1)[0]) * nallow) >> 64
        k += 1
        if v not in chosen:
            chosen.append(v)
    u = (splitmix64_outputs(seed, k, n_scat) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    for v, uj in zip(chosen, u):
        iy, rem = divmod(v, nx * max_depth)
        ix, iz = divmod(rem, max_depth)
        x[iy, ix, iz] = np.float32(amp[0] + (amp[1] - amp[0]) * uj)
    return x


def synth_noise(count, seed):
    """The CN(0, 1) values ufss_synth_measure scales and adds (complex128 [count]):
    value i from outputs 2i + 1 and 2i + 2 by Box-Muller."""
    o1 = splitmix64_outputs(seed, 1, 2 * count)
    u1 = ((o1[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (o1[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    return r * (np.cos(2.0 * math.pi * u2) + 1j * np.sin(2.0 * math.pi * u2)) / math.sqrt(2.0)


def rademacher(shape, seed):
    """Independent uniform signs in {-1, +1} (int8), for the mixing Sigma of the
    random sampling strategy."""
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, size=shape) - 1).astype(np.int8)


def uniform_subsets(nt, m, lead_shape, seed):
    """m distinct DFT bins of [0, nt) per entry of lead_shape, each subset
    uniform over all such subsets and sorted (int32 [*lead_shape, m])."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(lead_shape)) if len(lead_shape) else 1
    out = np.empty((n, m), dtype=np.int32)
    for i in range(n):
        out[i] = np.sort(rng.choice(nt, size=m, replace=False))
    return out.reshape(tuple(lead_shape) + (m,))


def cn(shape, seed):
    """Circular complex Gaussian CN(0, 1) array (complex128)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def noise_sigma(signal_energy, count, snr_db):
    """Noise std so that E||n||^2 = ||A x||^2 / 10^(snr/10) over ``count`` values."""
    return math.sqrt(signal_energy / (count * 10.0 ** (snr_db / 10.0)))
