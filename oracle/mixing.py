"""Oracle random-mixing operator (test infrastructure only).

Sec. II-B compression Phi_i = S_i F Sigma_i with the random sampling strategy
of Sec. III-A: Sigma_i = Diag(xi_i), xi_i a Rademacher vector in {-1, 1}^N_t,
applied to the sampled A-scan before the DFT; S_i keeps m of the N_t DFT
coefficients (Table I: Phi_rnd with one xi for all positions, Phi_rnd,m with
one per position, Phi_rnd,m,f with per-position subsets as well).

The A-scan's full spectrum is B_i = F b_i, so the measurement is
y_i = S_i (F Sigma_i F^{-1}) B_i, and F Sigma F^{-1} is the circulant matrix
with entries xi_hat[(k - k') mod N_t], xi_hat = F xi / N_t.  Every DFT index
k' of B enters; index k' is the signed bin k' (k' <= N_t/2) or k' - N_t
(above), whose row is the unmixed operator at that (negative) frequency: the
complex Gabor spectrum is small there but not zero, and the sampled echo
carries it.  The signs are inputs (drawn by the caller).
"""
import numpy as np

from . import geometry
from . import operator as O


def xi_hat(xi):
    """F xi / N_t for one sign row (complex128 [N_t])."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.fft.fft(xi) / xi.size


def signed_bins(nt):
    """DFT indices 0 .. N_t-1 as signed bins: k (k <= N_t/2) or k - N_t."""
    k = np.arange(nt)
    return np.where(k <= nt // 2, k, k - nt)


def mixing_rows(g, k_sel, xi):
    """[m, N_t] complex128: rows of S F Sigma F^{-1} (columns in DFT index order)."""
    nt = g["nt"]
    xh = xi_hat(xi)
    kp = np.arange(nt)
    k_sel = np.asarray(k_sel)
    return xh[(k_sel[:, None] - kp[None, :]) % nt]


def _row(arr, iy, ix):
    a = np.asarray(arr)
    return a if a.ndim == 1 else a[iy, ix]


def dense_A_mixed(g, bins, signs):
    """Dense mixed operator [npos*m, nvox] (complex128).

    bins: [m] or [ny, nx, m] in [0, N_t); signs: [N_t] or [ny, nx, N_t] of +-1.
    """
    full = signed_bins(g["nt"])
    rows = []
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            M = mixing_rows(g, _row(bins, iy, ix), _row(signs, iy, ix))
            rows.append(M @ O.row_block(g, full, iy, ix))
    return np.concatenate(rows, axis=0)
