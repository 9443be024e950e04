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
"""
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
