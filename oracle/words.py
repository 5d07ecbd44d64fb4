"""Exact phase and frequency words, ramp tables and the piecewise phase law.

TEST INFRASTRUCTURE (see the package docstring). Plain Python big integers and
``fractions.Fraction``; nothing here is fast and nothing is meant to be.

Conventions (the paper works in radians with real-valued phases; the words
below are the same quantities as exact fixed-point numbers):

* A *word* is an integer modulo 2**64; one full turn (2*pi rad) is 2**64.
* Frequency word of a tone at f Hz sampled at fs Hz: the phase advance per
  sample, F = f / fs * 2**64 rounded half-to-even (``tuning_word``). With a
  buffer period L = 2**p the frequency is first snapped to the nearest bin
  j = nint(f L / fs), Eq. (4), and then F = j * 2**(64 - p) exactly.
* Phase word of an initial phase theta (given in turns): P0 = theta * 2**64
  rounded half-to-even, reduced mod 2**64.
* Sample n of a static tone has phase word P0 + F*n (mod 2**64): the sampled
  argument of Eq. (2), 2*pi*j*n/L + theta, written in turns.
* A chirped tone follows Eq. (8): before its ramp window it is static; inside
  the window [a, a+N] its phase is the sampled integral of the frequency
  trajectory; after the window it continues at the end frequency with the phase
  it reached (continuity, the theta' term of Eq. (8)).
"""
from fractions import Fraction
import math

import numpy as np

TWO64 = 1 << 64
MASK64 = TWO64 - 1

RAMP_NONE, RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK = 0, 1, 2, 3
SMOOTH_SHAPES = (RAMP_COSINE, RAMP_MINJERK)
TABLE_SHIFT = 16          # ramp tables hold 2**16 * N * Psi(d/N)
INT16_MIN, INT16_MAX = -32768, 32767


def rne(x):
    """Round a rational to the nearest integer, ties to the even integer.

    The ``nint`` of Eq. (4); the tie rule is not stated in the paper, half-to-even
    is the reading taken here.
    """
    x = Fraction(x)
    fl = x.numerator // x.denominator
    rem = x - fl
    half = Fraction(1, 2)
    if rem > half:
        return fl + 1
    if rem < half:
        return fl
    return fl if fl % 2 == 0 else fl + 1


def to_signed64(w):
    """Two's-complement reading of a word: the phase in turns is this / 2**64."""
    w &= MASK64
    return w - TWO64 if w >= (1 << 63) else w


class WordError(ValueError):
    """A frequency that has no valid word (outside (0, fs/2) after rounding)."""


def tuning_word(f_hz, fs_hz, period_log2=0):
    """Frequency word of ``f_hz`` at sample rate ``fs_hz``.

    period_log2 = p > 0: Eq. (4), j = nint(f L / fs) with L = 2**p, word j*2**(64-p).
    period_log2 = 0: nearest word, nint(f * 2**64 / fs).
    Valid words lie in [1, 2**63 - 1] (0 < f < fs/2); bin j = L/2 (Nyquist, which
    Eq. (4) admits) is excluded because its amplitude depends on its phase.
    """
    f = Fraction(f_hz)
    fs = Fraction(fs_hz)
    if not (0 < f < fs / 2):
        raise WordError("frequency outside (0, fs/2)")
    if period_log2 > 0:
        j = rne(f * (1 << period_log2) / fs)
        if j < 1 or j >= (1 << (period_log2 - 1)):
            raise WordError("bin outside [1, L/2)")
        return j << (64 - period_log2)
    w = rne(f * TWO64 / fs)
    if w < 1 or w >= (1 << 63):
        raise WordError("word outside [1, 2**63)")
    return w


def phase_word(turns):
    """Initial phase word: nint(theta * 2**64) mod 2**64, theta in turns."""
    return rne(Fraction(turns) * TWO64) & MASK64


def default_gain(amplitudes):
    """LSB per unit amplitude when none is given: 32767 / sum|A_k|.

    The paper's Q operator (Eq. (2)) only says "discretisation"; this gain can
    never clip a 16-bit DAC sample. The sum runs in index order in FP64.
    """
    s = 0.0
    for a in amplitudes:
        s += abs(float(a))
    return 32767.0 / s


# ---------------------------------------------------------------- ramp tables

def minjerk_table_entry(N, d):
    """H_N[d] = nint(2**16 * N * Psi(d/N)) for the minimum-jerk ramp, exact.

    Eq. (8) case 1 writes the phase as 2*pi*(i/fs)*(f_start + p[i]) with
    p[i] = df*(5/2 tau^3 - 3 tau^4 + tau^5), tau = i/(T fs). Multiplying out,
    the chirp part of the phase (in units of df*T turns) is
    Psi(tau) = 5/2 tau^4 - 3 tau^5 + tau^6, so N * Psi(d/N) with N = T fs is
    2**15 * d^4 (5 N^2 - 6 d N + 2 d^2) / N^5 after scaling by 2**16.
    """
    num = (d ** 4) * (5 * N * N - 6 * d * N + 2 * d * d) << (TABLE_SHIFT - 1)
    return rne(Fraction(num, N ** 5))


def cosine_table_entry(N, d):
    """H_N[d] for the raised-cosine ramp f = f0 + df*(1 - cos(pi tau))/2.

    Psi(tau) = tau/2 - sin(pi tau)/(2 pi), so 2**16 * N * Psi(d/N) is
    2**15 * d - (2**15 * N / pi) * sin(pi d / N). The paper has no cosine ramp
    (its smooth ramp is minimum-jerk); this shape is taken from the workload
    description. The transcendental part is defined as this FP64 evaluation,
    in this order, with the host C library's sin, rounded half-to-even:
        s = sin((pi * d) / N);  x = ((32768.0 * N) / pi) * s;  H = 2**15 d - nint(x)
    """
    s = math.sin((math.pi * float(d)) / float(N))
    x = ((32768.0 * float(N)) / math.pi) * s
    return (d << (TABLE_SHIFT - 1)) - rne(Fraction(x))


def ramp_table_entries(shape, N, ds):
    """H_N[d] for each d in ``ds`` (0 <= d <= N)."""
    if shape == RAMP_MINJERK:
        return [minjerk_table_entry(N, int(d)) for d in ds]
    if shape == RAMP_COSINE:
        return [cosine_table_entry(N, int(d)) for d in ds]
    raise ValueError("not a table shape")


def ramp_table(shape, N):
    """Whole table H_N[0..N] as uint64 (each entry < 2**47 for N < 2**31)."""
    return np.array(ramp_table_entries(shape, N, range(N + 1)), dtype=np.uint64)


# ------------------------------------------------------------- tone schedules

class Ramp:
    """One chirp of a tone, Eq. (8): window [a, a+N], from word F_from to F_to.

    p_line/f_line: the static line the tone follows before the window,
    phi(n) = p_line + f_line*n. p_after/f_after: the line after it.
    coef: linear -> R = nint(dF / N) (word change per sample per sample);
          smooth -> dF = F_to - F_from (signed).
    """

    def __init__(self, a, N, shape, p_line, f_line, f_to, table=None):
        if not 1 <= N < (1 << 31):
            raise ValueError("ramp length must be in [1, 2**31)")
        self.a, self.N, self.shape = int(a), int(N), int(shape)
        self.p_line, self.f_line, self.f_after = p_line, f_line, f_to
        self.dF = f_to - f_line
        if self.shape == RAMP_LINEAR:
            self.coef = rne(Fraction(self.dF, self.N))
        elif self.shape in SMOOTH_SHAPES:
            self.coef = self.dF
        else:
            raise ValueError("bad ramp shape")
        self.table = table          # optional full H_N table (np.uint64)
        end = self.a + self.N
        phi_end = (self.p_line + self.f_line * end + self.chirp_term(self.N)) & MASK64
        self.p_after = (phi_end - self.f_after * end) & MASK64

    def table_at(self, d):
        if self.table is not None:
            return int(self.table[d])
        return ramp_table_entries(self.shape, self.N, [d])[0]

    def chirp_term(self, d):
        """Extra phase accumulated d samples into the window (exact integer).

        linear: floor(R * d^2 / 2), the sampled integral of a linear frequency ramp.
        smooth: floor(dF * H_N[d] / 2**16).
        """
        if self.shape == RAMP_LINEAR:
            return (self.coef * d * d) >> 1
        return (self.coef * self.table_at(d)) >> TABLE_SHIFT


def amp_shape(shape, tau):
    """Normalised amplitude profile s(tau) on [0, 1], s(0) = 0, s(1) = 1.

    The paper lets every dynamic tone carry a time-dependent amplitude a_j[i]
    (Eq. (5)) without fixing its form; the reading taken here reuses the
    normalised profiles of the frequency ramps: linear tau, raised cosine
    (1 - cos(pi tau)) / 2, and minimum jerk 10 tau^3 - 15 tau^4 + 6 tau^5 (the
    position profile whose integral gives Eq. (8)'s phase).
    """
    tau = float(tau)
    if shape == RAMP_LINEAR:
        return tau
    if shape == RAMP_COSINE:
        return (1.0 - math.cos(math.pi * tau)) / 2.0
    if shape == RAMP_MINJERK:
        return tau ** 3 * (10.0 - 15.0 * tau + 6.0 * tau * tau)
    raise ValueError("bad amplitude ramp shape")


class AmpRamp:
    """One amplitude ramp of a tone: from a_from to a_to over the window [b, b+M]."""

    def __init__(self, b, M, shape, a_from, a_to):
        if not 1 <= M < (1 << 31):
            raise ValueError("amplitude ramp length must be in [1, 2**31)")
        amp_shape(shape, 0.0)                  # validates the shape
        self.b, self.M, self.shape = int(b), int(M), int(shape)
        self.a_from, self.a_to = float(a_from), float(a_to)

    def at(self, d):
        """Amplitude d samples into the window (0 <= d <= M), FP64:
        a_from (1 - s) + a_to s, exact at both ends."""
        s = amp_shape(self.shape, Fraction(d, self.M))
        return self.a_from * (1.0 - s) + self.a_to * s


class ToneWords:
    """All words of one tone: the initial line and its ramps, in time order."""

    def __init__(self, p0, f0, amp):
        self.p0, self.f0, self.amp = p0, f0, float(amp)
        self.ramps = []
        self.amp_ramps = []

    def add_amp_ramp(self, b, M, shape, a_to):
        """Append an amplitude ramp from the tone's current amplitude to a_to."""
        a_from = self.amp_ramps[-1].a_to if self.amp_ramps else self.amp
        free_from = self.amp_ramps[-1].b + self.amp_ramps[-1].M if self.amp_ramps else 0
        if b < free_from:
            raise ValueError("amplitude ramps of one tone must not overlap")
        self.amp_ramps.append(AmpRamp(b, M, shape, a_from, a_to))

    def amp_at(self, n):
        """Amplitude A_k G at absolute sample n (the a_j[i] of Eq. (5))."""
        n = int(n)
        r = None
        for cand in self.amp_ramps:
            if cand.b <= n:
                r = cand
            else:
                break
        if r is None:
            return self.amp
        d = n - r.b
        if d <= r.M:
            return r.at(d)
        return r.a_to

    def current_line(self):
        if self.ramps:
            r = self.ramps[-1]
            return r.p_after, r.f_after, r.a + r.N
        return self.p0, self.f0, 0

    def add_ramp(self, a, N, shape, f_to, table=None):
        p_line, f_line, free_from = self.current_line()
        if a < free_from:
            raise ValueError("ramps of one tone must not overlap")
        self.ramps.append(Ramp(a, N, shape, p_line, f_line, f_to, table))

    def phase_at(self, n):
        """Exact phase word at absolute sample n (the piecewise law of Eq. (8))."""
        n = int(n)
        r = None
        for cand in self.ramps:
            if cand.a <= n:
                r = cand
            else:
                break
        if r is None:
            return (self.p0 + self.f0 * n) & MASK64
        d = n - r.a
        if d <= r.N:
            return (r.p_line + r.f_line * n + r.chirp_term(d)) & MASK64
        return (r.p_after + r.f_after * n) & MASK64


class Plan:
    """Oracle view of a set of tones: words per tone and the gain."""

    def __init__(self, fs_hz, gain_lsb, period_log2, tones, build_tables=False):
        self.fs_hz = float(fs_hz)
        self.period_log2 = int(period_log2)
        amps = [float(t["amplitude"]) for t in tones]
        self.gain = float(gain_lsb) if gain_lsb > 0 else default_gain(amps)
        self.tones = []
        self._tables = {}
        self.build_tables = build_tables
        for t in tones:
            f0 = tuning_word(float(t["f_start_hz"]), self.fs_hz, self.period_log2)
            tw = ToneWords(phase_word(float(t["phase_turns"])), f0, float(t["amplitude"]) * self.gain)
            self.tones.append(tw)
            if int(t["ramp"]) != RAMP_NONE:
                self.add_ramp(len(self.tones) - 1, int(t["ramp_start"]), int(t["ramp_len"]),
                              int(t["ramp"]), float(t["f_end_hz"]))

    def table(self, shape, N):
        if not self.build_tables or shape not in SMOOTH_SHAPES:
            return None
        key = (shape, N)
        if key not in self._tables:
            self._tables[key] = ramp_table(shape, N)
        return self._tables[key]

    def add_ramp(self, k, a, N, shape, f_end_hz):
        """Append a chirp of tone k starting at absolute sample a (retuning)."""
        f_to = tuning_word(f_end_hz, self.fs_hz, self.period_log2)
        self.tones[k].add_ramp(a, N, shape, f_to, self.table(shape, N))

    def add_amp_ramp(self, k, b, M, shape, amplitude_end):
        """Ramp tone k's amplitude to ``amplitude_end`` (in units of the gain, as
        the tone amplitudes) over [b, b+M]; 0 switches the tone off."""
        self.tones[k].add_amp_ramp(b, M, shape, float(amplitude_end) * self.gain)

    def phase_at(self, k, n):
        return self.tones[k].phase_at(n)

    def y_at(self, n):
        """Unquantised sample y[n] = sum_k a_k(n) sin(2 pi phi_k(n) / 2**64), FP64.

        The discretised sum of Eqs. (2)-(3) and (5)-(7), a_k(n) = A_k G unless
        the tone has amplitude ramps; math.fsum makes the sum exactly rounded
        so the tone order does not matter.
        """
        terms = []
        for tw in self.tones:
            t = to_signed64(tw.phase_at(n)) / TWO64
            terms.append(tw.amp_at(n) * math.sin(2.0 * math.pi * t))
        return math.fsum(terms)

    def synth_points(self, ns):
        """(q, y) at the given absolute samples; pure Python, for small cases."""
        ys = np.array([self.y_at(n) for n in ns], dtype=np.float64)
        return quantise(ys), ys


def quantise(y):
    """Q of Eq. (2) for a 16-bit DAC: round half-to-even, saturate to int16."""
    r = np.rint(np.asarray(y, dtype=np.float64))
    return np.clip(r, INT16_MIN, INT16_MAX).astype(np.int16)
