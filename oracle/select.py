"""Oracle frequency-bin selection (test infrastructure only).

Sec. III-A (random sampling strategy, and the per-A-scan variants of
Table I): each A-scan keeps n_f of the DFT coefficients.  The paper draws the
subset uniformly at random but does not fix a generator.  Reading taken here:

  * Generator: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), written from its
    published definition with Python integers.
  * Stream key: ``seed`` for a subset shared by all positions; for the subset
    of position p = i_x + N_x i_y the key is ``seed XOR mix64(p + 1)``, where
    mix64 is the SplitMix64 output function.
  * Draw: a partial Fisher-Yates shuffle of the ascending band list; the j-th
    swap partner is i + floor(next() * (n - i) / 2^64) (multiply-high bound,
    no rejection).  The first m entries are sorted ascending.

The maximal and energy-based strategies follow below (``sample_bins``).
"""
import math

import numpy as np

from . import geometry

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    """SplitMix64 output function applied to a 64-bit integer."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


class SplitMix64:
    """The SplitMix64 generator: state advances by the golden gamma."""

    def __init__(self, seed):
        self.state = seed & _MASK

    def next(self):
        self.state = (self.state + _GAMMA) & _MASK
        return mix64(self.state)


def draw_subset(band_list, m, key):
    """m distinct entries of ``band_list`` (ascending), keyed stream ``key``."""
    pool = [int(b) for b in band_list]
    n = len(pool)
    if m > n:
        raise ValueError("m exceeds the band size")
    rng = SplitMix64(key)
    for i in range(m):
        j = i + ((rng.next() * (n - i)) >> 64)
        pool[i], pool[j] = pool[j], pool[i]
    return sorted(pool[:m])


def select_freqs(g, m, per_position, seed):
    """Selected bins: int64 [m] (shared) or [ny, nx, m] (per position)."""
    b = geometry.band(g)
    if not per_position:
        return np.array(draw_subset(b, m, seed), dtype=np.int64)
    out = np.empty((g["ny"], g["nx"], m), dtype=np.int64)
    for iy in range(g["ny"]):
        for ix in range(g["nx"]):
            p = ix + g["nx"] * iy
            out[iy, ix] = draw_subset(b, m, seed ^ mix64(p + 1))
    return out


# ---------------------------------------------------------------------------
# Knowledge-based strategies of Sec. III-A (maximal and energy-based sampling)
# and their per-A-scan variant (Table I).  Readings taken here:
#
#   * Candidate bins are k = 0 .. N_t/2.  The pulse is the complex (analytic)
#     Gabor, so the bins above N_t/2 (negative frequencies) carry no energy.
#   * The energy weight of bin k is |H_k| up to a constant factor that cancels
#     in the normalisation: w_k = exp(-(f_k - f_c)^2 / (2 sigma_f^2)).
#   * Maximal sampling keeps the m largest weights; equal weights go to the
#     lower bin.
#   * Energy-based sampling draws without replacement: each draw removes the
#     chosen bin and renormalises the rest.  One draw takes u = (next() >> 11)
#     * 2^-53 from the SplitMix64 stream, scales it by the sum of the remaining
#     weights (summed in ascending bin order) and returns the first remaining
#     bin whose running sum exceeds it (the last remaining bin with a positive
#     weight if rounding leaves none).  All of this is FP64.
#   * Per-position subsets use the keys of the random strategy.
# ---------------------------------------------------------------------------
STRATEGY_RND = 0      # uniform over the band, one subset for all positions
STRATEGY_RND_F = 1    # uniform over the band, one subset per position
STRATEGY_MAX = 2      # the m bins of largest |H_k|
STRATEGY_NRG = 3      # drawn with probability proportional to |H_k|, shared
STRATEGY_NRG_F = 4    # the same, one subset per position


def energy_weights(g):
    """w_k for k = 0 .. N_t/2 as a Python list of floats (FP64)."""
    sigma_f = g["frac_bw"] * g["fc"] / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    out = []
    for k in range(g["nt"] // 2 + 1):
        f = k * g["fs"] / g["nt"]
        d = f - g["fc"]
        out.append(math.exp(-(d * d) / (2.0 * sigma_f * sigma_f)))
    return out


def select_max(weights, m):
    """Indices of the m largest weights (ties to the lower index), ascending."""
    if m > len(weights):
        raise ValueError("m exceeds the number of candidate bins")
    order = sorted(range(len(weights)), key=lambda k: (-weights[k], k))
    return sorted(order[:m])


def draw_energy(weights, m, key):
    """m distinct indices drawn with probability proportional to ``weights``,
    renormalised after every draw; ascending."""
    left = [w > 0.0 for w in weights]
    if m > sum(left):
        raise ValueError("m exceeds the number of bins with positive weight")
    rng = SplitMix64(key)
    chosen = []
    for _ in range(m):
        total = 0.0
        for k, w in enumerate(weights):
            if left[k]:
                total += w
        target = (rng.next() >> 11) * (1.0 / 9007199254740992.0) * total
        run = 0.0
        pick = -1
        for k, w in enumerate(weights):
            if not left[k] or w <= 0.0:
                continue
            run += w
            pick = k
            if run > target:
                break
        left[pick] = False
        chosen.append(pick)
    return sorted(chosen)


def sample_bins(g, m, strategy, seed):
    """Bins of one strategy: int64 [m] (shared) or [ny, nx, m] (per position)."""
    if strategy == STRATEGY_RND:
        return select_freqs(g, m, False, seed)
    if strategy == STRATEGY_RND_F:
        return select_freqs(g, m, True, seed)
    w = energy_weights(g)
    if strategy == STRATEGY_MAX:
        return np.array(select_max(w, m), dtype=np.int64)
    if strategy == STRATEGY_NRG:
        return np.array(draw_energy(w, m, seed), dtype=np.int64)
    if strategy == STRATEGY_NRG_F:
        out = np.empty((g["ny"], g["nx"], m), dtype=np.int64)
        for iy in range(g["ny"]):
            for ix in range(g["nx"]):
                p = ix + g["nx"] * iy
                out[iy, ix] = draw_energy(w, m, seed ^ mix64(p + 1))
        return out
    raise ValueError("unknown strategy")
