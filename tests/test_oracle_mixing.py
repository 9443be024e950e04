"""Pins of the oracle random-mixing operator (Sec. II-B compression with the
Rademacher Sigma of Sec. III-A): against the time-domain pulse-echo model
mixed sample by sample, the reduction to plain bin selection when every sign
is +1, and Parseval (the mixing is orthogonal in the time domain)."""
import numpy as np
import pytest

from oracle import mixing as X
from oracle import operator as O
from oracle import select as S
from oracle import timedomain as T
from paper_2012_04534_amd import workloads as W


def geom(win=-1):
    return W.geometry(5, 4, 12, 64, win_x=win, win_y=win)


@pytest.mark.parametrize("per_sign,per_bins,win", [(False, False, -1), (True, False, 2),
                                                   (True, True, -1)])
def test_mixed_operator_equals_mixed_time_domain_samples(per_sign, per_bins, win):
    """y = S F (xi * b) with b the periodised sampled echoes (independent
    time-domain model): every selected coefficient, bins anywhere in [0, N_t)."""
    g = geom(win)
    nt = g["nt"]
    signs = W.rademacher((g["ny"], g["nx"], nt) if per_sign else (nt,), 7)
    bins = W.uniform_subsets(nt, 9, (g["ny"], g["nx"]) if per_bins else (), 8)
    x = W.scene(g, 6, amp=(0.5, 1.0), seed=3, phase=0.4)
    y = X.dense_A_mixed(g, bins, signs) @ x.reshape(-1)
    b = T.ascans(g, x)
    ref = []
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            xi = signs if signs.ndim == 1 else signs[iy, ix]
            k = bins if np.ndim(bins) == 1 else bins[iy, ix]
            ref.append(np.fft.fft(xi * b[iy, ix])[k])
    ref = np.concatenate(ref)
    assert np.abs(y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_all_plus_signs_is_bin_selection():
    g = geom(2)
    bins = S.select_freqs(g, 6, True, 4)
    signs = np.ones(g["nt"])
    np.testing.assert_allclose(X.dense_A_mixed(g, bins, signs), O.dense_A(g, bins),
                               rtol=0, atol=1e-12 * np.abs(O.dense_A(g, bins)).max())


def test_parseval_full_selection():
    """All N_t coefficients selected: ||A_mix x|| = ||A_full x|| (Sigma is
    orthogonal, F / sqrt(N_t) unitary)."""
    g = geom()
    signs = W.rademacher((g["ny"], g["nx"], g["nt"]), 11)
    allk = np.arange(g["nt"])
    x = W.cn((g["ny"], g["nx"], g["nz"]), 12)
    ym = X.dense_A_mixed(g, allk, signs) @ x.reshape(-1)
    yf = O.dense_A(g, X.signed_bins(g["nt"])) @ x.reshape(-1)
    assert np.linalg.norm(ym) == pytest.approx(np.linalg.norm(yf), rel=1e-12)


def test_signs_and_subsets_generators():
    s = W.rademacher((3, 64), 5)
    assert set(np.unique(s)) <= {-1, 1} and s.dtype == np.int8
    assert abs(s.mean()) < 0.2
    b = W.uniform_subsets(64, 9, (4, 3), 6)
    assert b.shape == (4, 3, 9)
    assert all(len(set(r)) == 9 and list(r) == sorted(r) for r in b.reshape(-1, 9))
    assert b.min() >= 0 and b.max() < 64
