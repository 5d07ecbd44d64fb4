"""Initial tone phases for a low crest factor, and the crest factor itself.

TEST INFRASTRUCTURE (see the package docstring). The paper controls the peak
(crest) factor of the static waveform with the tone phases theta_j (Theory
section; it cites Schroeder 1970 and gives no formula). Two classical closed
forms, with tones ranked by frequency k = 1..K (ties by input index):

* Schroeder's rule for a given power spectrum p_l = A_l^2 / sum A^2:
  theta_k = theta_1 - 2 pi sum_{l<k} (k - l) p_l, with theta_1 = 0;
  for equal amplitudes this is -pi k (k - 1) / K.
* Newman's phases: theta_k = pi (k - 1)^2 / K.

Phases are returned in turns in [0, 1), computed as exact rationals
(``fractions.Fraction``) from the FP64 amplitudes. The crest factor of a
periodic waveform is max|y| / rms over one period, with rms^2 = G^2 sum A^2 / 2
for tones on distinct bins.
"""
from fractions import Fraction
import math

import numpy as np

SCHROEDER, NEWMAN = 1, 2


def rank_by_frequency(f_hz):
    """Frequency rank (0-based) of every tone; equal frequencies keep input order."""
    order = sorted(range(len(f_hz)), key=lambda i: (float(f_hz[i]), i))
    rank = [0] * len(f_hz)
    for r, i in enumerate(order):
        rank[i] = r
    return rank, order


def phase_plan(method, f_hz, amps):
    """Phases in turns, [0, 1), of every tone (input order)."""
    K = len(f_hz)
    rank, order = rank_by_frequency(f_hz)
    out = [0.0] * K
    if method == NEWMAN:
        for i in range(K):
            k = rank[i] + 1
            t = Fraction((k - 1) ** 2, 2 * K)
            out[i] = float(t - math.floor(t))
        return out
    if method != SCHROEDER:
        raise ValueError("unknown phase method")
    p = [Fraction(float(amps[i])) ** 2 for i in order]
    total = sum(p)
    if total == 0:
        raise ValueError("all amplitudes are zero")
    p = [x / total for x in p]
    # turns: t_k = - sum_{l<k} (k - l) p_l, by rank
    for k in range(1, K + 1):
        t = -sum((k - l) * p[l - 1] for l in range(1, k))
        out[order[k - 1]] = float(t - math.floor(t))
    return out


def crest_factor(y, amps, gain):
    """max|y| / rms, rms^2 = gain^2 sum A^2 / 2 (distinct bins, one full period)."""
    rms = gain * math.sqrt(sum(float(a) ** 2 for a in amps) / 2.0)
    return float(np.max(np.abs(y))) / rms
