"""Pins of the oracle Cramer-Rao bound (Sec. VI): derivatives against finite
differences of the measurement model, the paper's Schur-complement form
against the plain inverse, the classic delay-estimation bound, and the
ordering that more measurements can only lower the bound."""
import math

import numpy as np
import pytest

from oracle import crb as K
from oracle import geometry as G
from oracle import select as S
from paper_2012_04534_amd import workloads as W


def small(theta_deg=30.0, win=-1):
    g = W.geometry(7, 5, 8, 128, win_x=win, win_y=win)
    g["theta"] = math.radians(theta_deg)
    return g


U = (1.37e-3, 0.91e-3, 31.7e-3, 0.8, 0.4)


@pytest.mark.parametrize("theta_deg,per_pos", [(30.0, False), (30.0, True), (0.0, True)])
def test_derivatives_match_finite_differences(theta_deg, per_pos):
    g = small(theta_deg)
    bins = S.select_freqs(g, 5, per_pos, 3)
    D = K.derivatives(g, bins, U)
    steps = (1e-7, 1e-7, 1e-7, 1e-6, 1e-6)
    for j in range(5):
        up, dn = list(U), list(U)
        up[j] += steps[j]
        dn[j] -= steps[j]
        fd = (np.concatenate(K.model(g, bins, up)) - np.concatenate(K.model(g, bins, dn))) / (2 * steps[j])
        np.testing.assert_allclose(D[:, j], fd, rtol=0, atol=2e-6 * np.abs(D[:, j]).max())


def test_schur_form_equals_inverse_and_scaling():
    g = small()
    bins = S.select_freqs(g, 6, True, 5)
    J = K.fisher(g, bins, U, 0.3)
    c = K.crb_position(J)
    np.testing.assert_allclose(c, np.diag(np.linalg.inv(J))[:3], rtol=1e-9)
    # C scales with sigma^2 and with 1 / a^2
    np.testing.assert_allclose(K.crb_position(K.fisher(g, bins, U, 0.6)), 2 * c, rtol=1e-9)
    u2 = list(U)
    u2[3] *= 2.0
    np.testing.assert_allclose(K.crb_position(K.fisher(g, bins, u2, 0.3)), c / 4, rtol=1e-9)


def test_single_ascan_delay_bound():
    """One A-scan straight above the scatterer, no beam, x and y known: the
    bound on z is (c/2)^2 times the delay bound with unknown phase and
    amplitude, sigma^2 / (2 sum_k |b_k|^2 (w_k - w_bar)^2), w_bar the
    |b|^2-weighted mean angular frequency."""
    g = W.geometry(1, 1, 8, 256)
    bins = np.arange(10, 45)
    u = (0.0, 0.0, 32.1e-3, 1.3, -0.7)
    sigma2 = 0.25
    J = K.fisher(g, bins, u, sigma2)
    sub = J[np.ix_([2, 3, 4], [2, 3, 4])]
    cz = np.linalg.inv(sub)[0, 0]
    b2 = np.abs(np.concatenate(K.model(g, bins, u))) ** 2
    w = 2 * math.pi * G.bin_freq(g, bins)
    wbar = np.sum(b2 * w) / np.sum(b2)
    var_tau = sigma2 / (2 * np.sum(b2 * (w - wbar) ** 2))
    assert cz == pytest.approx((g["c"] / 2) ** 2 * var_tau, rel=1e-9)


def test_more_bins_never_raise_the_bound():
    g = small()
    full = S.sample_bins(g, 20, S.STRATEGY_MAX, 0)
    sub = full[::3]
    Jf = K.fisher(g, full, U, 1.0)
    Js = K.fisher(g, sub, U, 1.0)
    # J_full - J_sub is positive semi-definite, so every bound can only drop
    assert np.linalg.eigvalsh(Jf - Js).min() > -1e-9 * np.abs(Jf).max()
    assert np.all(K.crb_position(Jf) <= K.crb_position(Js) * (1 + 1e-12))


def test_window_drops_far_positions():
    g = small(win=1)
    bins = S.select_freqs(g, 4, False, 2)
    b = K.model(g, bins, U)
    # scatterer near (x, y) = (2.7 dx, 1.8 dy): positions farther than one pitch are empty
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            far = abs(U[0] - ix * g["dx"]) > g["dx"] or abs(U[1] - iy * g["dy"]) > g["dy"]
            assert (np.abs(b[iy * g["nx"] + ix]).max() == 0) == far


def test_mixed_fim_reductions():
    """Mixed measurements: all signs +1 reduce to bin selection; every
    coefficient selected gives the full-band information (F Sigma F^-1 is
    unitary); the mixed model's derivatives match finite differences."""
    from oracle import mixing as X
    g = small()
    nt = g["nt"]
    bins = S.select_freqs(g, 5, True, 9)
    J1 = K.fisher_mixed(g, bins, np.ones(nt), U, 0.2)
    J0 = K.fisher(g, bins, U, 0.2)
    np.testing.assert_allclose(J1, J0, rtol=0, atol=1e-10 * np.abs(J0).max())
    signs = W.rademacher((g["ny"], g["nx"], nt), 3)
    Jm = K.fisher_mixed(g, np.arange(nt), signs, U, 0.2)
    Jf = K.fisher(g, X.signed_bins(nt), U, 0.2)
    np.testing.assert_allclose(Jm, Jf, rtol=0, atol=1e-9 * np.abs(Jf).max())
    # derivatives of the mixed model by central differences
    sub = W.uniform_subsets(nt, 4, (g["ny"], g["nx"]), 4)
    def ymix(uu):
        b = K.model(g, X.signed_bins(nt), uu)
        return np.concatenate([X.mixing_rows(g, sub[iy, ix], signs[iy, ix]) @ b[iy * g["nx"] + ix]
                               for iy in range(g["ny"]) for ix in range(g["nx"])])
    D = K.derivatives(g, X.signed_bins(nt), U)
    MD = np.concatenate([X.mixing_rows(g, sub[iy, ix], signs[iy, ix]) @
                         D[(iy * g["nx"] + ix) * nt:(iy * g["nx"] + ix + 1) * nt]
                         for iy in range(g["ny"]) for ix in range(g["nx"])])
    for j, h in enumerate((1e-7, 1e-7, 1e-7, 1e-6, 1e-6)):
        up, dn = list(U), list(U)
        up[j] += h
        dn[j] -= h
        fd = (ymix(up) - ymix(dn)) / (2 * h)
        np.testing.assert_allclose(MD[:, j], fd, rtol=0, atol=2e-6 * np.abs(MD[:, j]).max())
    Jd = (2 / 0.2) * np.real(MD.conj().T @ MD)
    np.testing.assert_allclose(K.fisher_mixed(g, sub, signs, U, 0.2), Jd, rtol=0,
                               atol=1e-10 * np.abs(Jd).max())
