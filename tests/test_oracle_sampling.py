"""Pins of the oracle's knowledge-based frequency sampling (Sec. III-A,
maximal and energy-based sampling; Table I for the per-A-scan variant).

Each check comes from outside the oracle's own code: the nearest-frequency
closed form of maximal sampling under a Gaussian spectrum, and the exact draw
probabilities of sampling without replacement, compared with empirical
frequencies over many seeded draws.
"""
import math

import numpy as np
import pytest

from oracle import select as S
from paper_2012_04534_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


def small_geom(nt=64, **over):
    return W.geometry(4, 3, 8, nt, **over)


@pytest.mark.parametrize("nt,m", [(64, 1), (64, 5), (256, 8), (256, 20), (512, 64)])
def test_max_is_the_bins_nearest_fc(nt, m):
    # A Gaussian spectrum is monotone in |f - f_c|, so the m largest |H_k| are
    # the m bins closest in frequency to f_c.
    g = small_geom(nt)
    near = sorted(range(nt // 2 + 1), key=lambda k: (abs(k * g["fs"] / nt - g["fc"]), k))[:m]
    got = S.sample_bins(g, m, S.STRATEGY_MAX, 0)
    assert list(got) == sorted(near)
    # and they form one contiguous run of bins
    assert got[-1] - got[0] == m - 1


def test_max_all_bins_and_too_many():
    g = small_geom(64)
    assert list(S.sample_bins(g, 33, S.STRATEGY_MAX, 0)) == list(range(33))
    with pytest.raises(ValueError):
        S.sample_bins(g, 34, S.STRATEGY_MAX, 0)


def test_energy_weights_are_the_spectrum_shape():
    # w_k must be |H_k| / max |H|, not |H_k|^2 (a plausible slip): at the
    # -6 dB band edge f_c (1 +- b/2) the amplitude is one half.
    g = small_geom(64, fc=4e6, frac_bw=0.5)
    # place f_c + b f_c / 2 = 5 MHz exactly on a bin: f_s / N_t = 0.625 MHz
    w = S.energy_weights(g)
    assert abs(w[8] - 0.5) < 1e-12          # 8 * 0.625 MHz = 5 MHz
    assert abs(max(w) - w[round(4e6 / 0.625e6)]) == 0.0


def _q(g):
    w = np.array(S.energy_weights(g))
    return w / w.sum()


def test_single_draw_distribution():
    # One draw picks bin k with probability q_k = |H_k| / ||H||_1.
    g = small_geom(64)
    q = _q(g)
    n = 20000
    counts = np.zeros(len(q))
    for s in range(n):
        counts[S.draw_energy(S.energy_weights(g), 1, s)[0]] += 1
    keep = q * n >= 5                        # chi-square cells with enough mass
    exp = np.append(q[keep] * n, q[~keep].sum() * n)
    obs = np.append(counts[keep], counts[~keep].sum())
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    dof = len(exp) - 1
    # 99.9% quantile of chi-square, Wilson-Hilferty
    z = 3.09
    crit = dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3
    assert chi2 < crit, (chi2, crit)
    # against the squared-spectrum alternative the statistic explodes
    q2 = q ** 2 / (q ** 2).sum()
    exp2 = np.append(q2[keep] * n, q2[~keep].sum() * n)
    assert float(((obs - exp2) ** 2 / exp2).sum()) > 10 * crit


def test_two_draws_inclusion_probabilities():
    # Without replacement and renormalised after the first draw, bin k is in
    # the pair with probability pi_k = q_k + sum_{i != k} q_i q_k / (1 - q_i).
    g = small_geom(64)
    q = _q(g)
    pi = q + np.array([sum(q[i] * q[k] / (1 - q[i]) for i in range(len(q)) if i != k)
                       for k in range(len(q))])
    assert abs(pi.sum() - 2.0) < 1e-12
    n = 12000
    counts = np.zeros(len(q))
    w = S.energy_weights(g)
    for s in range(n):
        pair = S.draw_energy(w, 2, 1000003 + s)
        assert len(set(pair)) == 2
        counts[pair] += 1
    big = pi * n > 50
    zs = (counts[big] - pi[big] * n) / np.sqrt(n * pi[big] * (1 - pi[big]))
    assert np.max(np.abs(zs)) < 4.5, zs
    # drawing with replacement (no renormalisation) gives 1 - (1 - q)^2 and
    # sometimes one bin twice; the top bins separate the two clearly
    top = int(np.argmax(q))
    alt = 1 - (1 - q[top]) ** 2
    assert abs(pi[top] - alt) * n > 6 * math.sqrt(n * pi[top] * (1 - pi[top]))


def test_energy_all_bins_distinct_sorted():
    g = small_geom(64)
    got = S.sample_bins(g, 33, S.STRATEGY_NRG, 7)
    assert list(got) == list(range(33))
    got = S.sample_bins(g, 12, S.STRATEGY_NRG, 7)
    assert len(set(got)) == 12 and list(got) == sorted(got)


def test_per_position_keys():
    g = small_geom(128)
    per = S.sample_bins(g, 6, S.STRATEGY_NRG_F, 99)
    assert per.shape == (3, 4, 6)
    w = S.energy_weights(g)
    for iy in range(3):
        for ix in range(4):
            p = ix + 4 * iy
            assert list(per[iy, ix]) == S.draw_energy(w, 6, 99 ^ S.mix64(p + 1))
    # positions differ from one another (12 draws of 6 from ~60 bins)
    assert len({tuple(r) for r in per.reshape(-1, 6)}) > 6
    assert list(S.sample_bins(g, 6, S.STRATEGY_RND_F, 99).reshape(-1, 6)[5]) == \
        list(S.select_freqs(g, 6, True, 99).reshape(-1, 6)[5])
