"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle (oracle/words.py and the C sum in oracle/synth.c)
against something other than itself: numbers the paper prints, closed forms
(single tones, the Dirichlet kernel, the continuous chirp phase, Eq. (8) as
printed), invariants (periodicity, mean power, continuity) and brute force on
tiny inputs.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import words, csynth
from paper_2403_15582_amd.abi_types import (make_tones, RAMP_NONE, RAMP_LINEAR, RAMP_COSINE,
                                            RAMP_MINJERK)

TWO64 = 1 << 64
FS = 280e6


def one_tone(f0, phase=0.0, amp=1.0, f1=None, ramp=RAMP_NONE, a=0, N=0):
    t = make_tones(1)
    t["f_start_hz"] = f0
    t["f_end_hz"] = f0 if f1 is None else f1
    t["amplitude"] = amp
    t["phase_turns"] = phase
    t["ramp"] = ramp
    t["ramp_start"] = a
    t["ramp_len"] = N
    return t


def signed_turn_diff(w, turns_exact):
    """(w/2**64 - turns) reduced to [-1/2, 1/2), as a Fraction of a turn."""
    d = Fraction(w, TWO64) - turns_exact
    d -= math.floor(d + Fraction(1, 2))
    return d


# ------------------------------------------------------------------- words

def test_eq4_bin_error_matches_paper():
    g = read_golden("eq4_bin_error.txt")
    L = 1 << g["period_log2"]
    fs = g["fs_hz"]
    bound = fs / (2 * L)
    assert abs(bound - g["max_error_hz"]) < 0.1          # the paper's "534 Hz"
    rng = np.random.default_rng(0)
    worst = 0.0
    for f in rng.uniform(1e6, 139e6, 2000):
        w = words.tuning_word(f, fs, g["period_log2"])
        fq = Fraction(w, TWO64) * Fraction(fs)
        err = abs(float(fq - Fraction(f)))
        worst = max(worst, err)
        assert err <= bound + 1e-9
        assert w % (1 << (64 - g["period_log2"])) == 0    # exact bin word
    assert worst > 0.9 * bound                            # the bound is tight


def test_tuning_word_closed_forms():
    assert words.tuning_word(FS / 4, FS) == 1 << 62
    assert words.tuning_word(FS / 8, FS) == 1 << 61
    assert words.tuning_word(3 * FS / 16, FS) == 3 << 60
    rng = np.random.default_rng(1)
    for m in rng.integers(1, 1 << 19, 50):
        f = float(m) * FS / (1 << 20)        # an exact bin of L = 2**20 ...
        assert words.tuning_word(f, FS, 20) == int(m) << 44
        # ... and as a free frequency it is within half a word of m * 2**44
        assert abs(words.tuning_word(f, FS) - (int(m) << 44)) <= 1 + (1 << 44) * 1e-15 * 4
    with pytest.raises(words.WordError):
        words.tuning_word(FS / 2, FS)        # Nyquist excluded
    with pytest.raises(words.WordError):
        words.tuning_word(0.0, FS)
    with pytest.raises(words.WordError):
        words.tuning_word(FS / 2 - 1.0, FS, 20)   # snaps onto the Nyquist bin


def test_phase_word_closed_forms():
    assert words.phase_word(0.25) == 1 << 62
    assert words.phase_word(-0.25) == 3 << 62
    assert words.phase_word(0.5) == 1 << 63
    assert words.phase_word(1.75) == 3 << 62
    assert words.phase_word(0.0) == 0
    # 2**-65 is half a word: ties go to the even word (0), 3*2**-65 to 2
    assert words.phase_word(2.0 ** -65) == 0
    assert words.phase_word(3 * 2.0 ** -65) == 2


# ------------------------------------------------------------ static tones

def test_quarter_rate_tone_is_exact(oracle_built):
    g = read_golden("quarter_rate_tone.txt")
    p = words.Plan(g["fs_hz"], g["amp_lsb"], 0, one_tone(g["f_hz"]))
    q, y = csynth.synth(p, 0, 8)
    assert [int(v) for v in q] == [g["q%d" % i] for i in range(8)]
    assert np.allclose(y, q, atol=1e-9)
    # a quarter-turn initial phase is a cosine: 1000, 0, -1000, 0
    p = words.Plan(g["fs_hz"], g["amp_lsb"], 0, one_tone(g["f_hz"], phase=0.25))
    q, _ = csynth.synth(p, 0, 4)
    assert list(q) == [1000, 0, -1000, 0]


def _quarter_rate_codes(g, amp):
    """Codes of a quarter-rate tone of amplitude*gain ``amp`` from the C sum and
    from the Python evaluator (samples 0..7)."""
    p = words.Plan(g["fs_hz"], float(amp), 0, one_tone(g["f_hz"]))
    q, y = csynth.synth(p, 0, 8)
    qp, yp = p.synth_points(range(8))
    return q, y, qp, yp


def test_quantiser_ties_go_to_even(oracle_built):
    """Q of Eq. (2): samples exactly halfway between two codes go to the even code
    (2.5 -> 2, -2.5 -> -2, 3.5 -> 4, -3.5 -> -4) in both the C sum and the Python
    evaluator; rounding half away from zero would give 3 / -3."""
    g = read_golden("quantiser_ties_and_saturation.txt")
    for tag in ("tie_a", "tie_b"):
        a = g[tag + "_amp"]
        q, y, qp, yp = _quarter_rate_codes(g, a)
        want = [0, g[tag + "_q1"], 0, g[tag + "_q3"]] * 2
        assert [int(v) for v in q] == want, (tag, list(q))
        assert [int(v) for v in qp] == want, (tag, list(qp))
        assert y[1] == a and y[3] == -a and yp[1] == a and yp[3] == -a   # the ties are exact
    assert [int(v) for v in words.quantise([0.5, 1.5, -0.5, -1.5, 2.5000001])] == [0, 2, 0, -2, 3]


def test_quantiser_saturates_to_int16(oracle_built):
    """Q of Eq. (2) for a 16-bit DAC: values beyond the code range take the end
    codes 32767 and -32768 (no wrap-around); the tie at 32767.5 rounds to 32768
    and saturates, the one at -32767.5 rounds to -32768, which is in range."""
    g = read_golden("quantiser_ties_and_saturation.txt")
    for tag in ("sat", "edge"):
        a = g[tag + "_amp"]
        q, y, qp, _ = _quarter_rate_codes(g, a)
        want = [0, g[tag + "_q1"], 0, g[tag + "_q3"]] * 2
        assert [int(v) for v in q] == want, (tag, list(q))
        assert [int(v) for v in qp] == want, (tag, list(qp))
        assert y[1] == a                                     # y itself is not clipped
    assert [int(v) for v in words.quantise([1e9, -1e9, 32766.5, -32768.4])] == [32767, -32768, 32766, -32768]


def test_eighth_rate_tone(oracle_built):
    p = words.Plan(FS, 20000.0, 0, one_tone(FS / 8))
    _, y = csynth.synth(p, 0, 16)
    r = math.sqrt(0.5) * 20000.0
    ref = np.array([0, r, 20000, r, 0, -r, -20000, -r] * 2)
    assert np.max(np.abs(y - ref)) < 1e-9


def test_static_tones_match_eq2_in_long_double(oracle_built):
    """Eq. (2): V[i] = sum_j a_j sin(2 pi j (i mod L)/L + theta_j), from the bins."""
    rng = np.random.default_rng(2)
    p2 = 12
    L = 1 << p2
    K = 4
    bins = rng.choice(np.arange(1, L // 2), K, replace=False)
    amps = rng.uniform(0.1, 1.0, K)
    phases = rng.random(K)
    t = make_tones(K)
    t["f_start_hz"] = bins * (FS / L)
    t["f_end_hz"] = t["f_start_hz"]
    t["amplitude"] = amps
    t["phase_turns"] = phases
    G = 7000.0
    p = words.Plan(FS, G, p2, t)
    ns = np.arange(0, 3 * L + 17, 5, dtype=np.int64)
    ref = np.zeros(len(ns), dtype=np.longdouble)
    for b, a, th in zip(bins, amps, phases):
        # theta in turns is exact in binary; reduce b*n mod L exactly in integers
        turns = ((int(b) * ns) % L).astype(np.longdouble) / L + np.longdouble(th)
        ref += np.longdouble(a * G) * np.sin(np.longdouble(2) * np.pi * turns)
    for n, r in zip(ns[:40], ref[:40]):
        q, y = csynth.synth(p, int(n), 1)
        assert abs(float(y[0]) - float(r)) < 1e-8
    q, y = csynth.synth(p, 0, int(ns[-1]) + 1)
    assert np.max(np.abs(y[ns] - ref.astype(np.float64))) < 1e-8


def test_dirichlet_kernel(oracle_built):
    """K equal tones on bins b0 + k db with phases th0 + k dth sum to
    A G sin(K beta/2)/sin(beta/2) sin(alpha + (K-1) beta/2)."""
    p2 = 16
    L = 1 << p2
    K, b0, db = 37, 1201, 53
    th0, dth = 0.125, 0.0625
    A, G = 1.0, 800.0
    t = make_tones(K)
    bins = b0 + db * np.arange(K)
    t["f_start_hz"] = bins * (FS / L)
    t["f_end_hz"] = t["f_start_hz"]
    t["amplitude"] = A
    t["phase_turns"] = (th0 + dth * np.arange(K)) % 1.0
    p = words.Plan(FS, G, p2, t)
    count = 3000
    _, y = csynth.synth(p, 0, count)
    n = np.arange(count, dtype=np.float64)
    alpha = 2 * np.pi * (((b0 * np.arange(count)) % L) / L + th0)
    beta = 2 * np.pi * (((db * np.arange(count)) % L) / L + dth)
    with np.errstate(divide="ignore", invalid="ignore"):
        ref = A * G * np.sin(K * beta / 2) / np.sin(beta / 2) * np.sin(alpha + (K - 1) * beta / 2)
    assert np.all(np.isfinite(ref))
    assert np.max(np.abs(y - ref)) < 1e-8 * K * A * G
    assert np.max(np.abs(y)) > 0.5 * K * A * G      # the kernel peaks are present


def test_periodicity_with_bin_frequencies(oracle_built):
    rng = np.random.default_rng(3)
    p2 = 10
    L = 1 << p2
    K = 9
    t = make_tones(K)
    t["f_start_hz"] = rng.choice(np.arange(1, L // 2), K, replace=False) * (FS / L)
    t["f_end_hz"] = t["f_start_hz"]
    t["amplitude"] = rng.uniform(0.2, 1, K)
    t["phase_turns"] = rng.random(K)
    p = words.Plan(FS, 0.0, p2, t)
    q, y = csynth.synth(p, 0, 3 * L)
    assert np.array_equal(q[L:2 * L], q[:L]) and np.array_equal(q[2 * L:], q[:L])
    assert np.max(np.abs(y[L:2 * L] - y[:L])) < 1e-9
    # without snapping the same tones are not periodic
    p = words.Plan(FS, 0.0, 0, t[:1].copy())
    t1 = t[:1].copy()
    t1["f_start_hz"] += 1000.0
    p = words.Plan(FS, 0.0, 0, t1)
    q, _ = csynth.synth(p, 0, 2 * L)
    assert not np.array_equal(q[L:], q[:L])


def test_mean_power_and_default_gain(oracle_built):
    rng = np.random.default_rng(4)
    p2 = 11
    L = 1 << p2
    K = 25
    t = make_tones(K)
    t["f_start_hz"] = rng.choice(np.arange(1, L // 2), K, replace=False) * (FS / L)
    t["f_end_hz"] = t["f_start_hz"]
    amps = rng.uniform(0.2, 1, K)
    t["amplitude"] = amps
    t["phase_turns"] = rng.random(K)
    p = words.Plan(FS, 0.0, p2, t)
    G = 32767.0 / amps.sum()
    assert p.gain == pytest.approx(G, rel=1e-15)
    q, y = csynth.synth(p, 0, L)
    expect = G * G * float(np.sum(amps ** 2)) / 2
    assert np.mean(y * y) == pytest.approx(expect, rel=1e-9)
    # int16 adds uniform rounding noise of variance 1/12 LSB^2
    assert abs(np.mean(q.astype(np.float64) ** 2) - expect - 1 / 12) < 0.02 * expect ** 0.5 + 0.05
    # all tones at a quarter turn: y[0] = sum A G = 32767 exactly, no clipping
    t["phase_turns"] = 0.25
    p = words.Plan(FS, 0.0, p2, t)
    q, y = csynth.synth(p, 0, 1)
    assert int(q[0]) == 32767 and y[0] == pytest.approx(32767.0, abs=1e-8)


# ----------------------------------------------------------------- chirps

def _exact_freq(w, fs):
    return Fraction(w, TWO64) * Fraction(fs)


def test_linear_chirp_matches_continuous_phase():
    """A linear sweep f0 -> f1 over T has phase theta + f0 t + df t^2/(2T) turns."""
    f0, f1, N, a, th = 101.3e6, 97.9e6, 1_000_003, 777, 0.3
    p = words.Plan(FS, 1.0, 0, one_tone(f0, th, 1.0, f1, RAMP_LINEAR, a, N))
    tw = p.tones[0]
    r = tw.ramps[0]
    F0, F1 = r.f_line, r.f_after
    fq0, fq1 = _exact_freq(F0, FS), _exact_freq(F1, FS)
    T = Fraction(N) / Fraction(FS)
    theta = Fraction(tw.p0, TWO64)
    for d in [0, 1, 2, 3, 1000, N // 2, N - 1, N]:
        n = a + d
        t = Fraction(n) / Fraction(FS)
        tau_t = Fraction(d) / Fraction(FS)
        cont = theta + fq0 * t + (fq1 - fq0) * tau_t * tau_t / (2 * T)
        diff = abs(signed_turn_diff(p.phase_at(0, n), cont)) * TWO64
        assert diff <= Fraction(d * d, 4) + 2, d
    # after the window the tone runs at f1 from the phase it reached
    for d in [N + 1, N + 2, N + 12345]:
        assert (p.phase_at(0, a + d) - p.phase_at(0, a + d - 1)) % TWO64 == F1
    # before it, at f0
    assert (p.phase_at(0, a) - p.phase_at(0, a - 1)) % TWO64 == F0
    assert p.phase_at(0, 5) == (tw.p0 + F0 * 5) % TWO64


def test_minjerk_matches_eq8_as_printed():
    """Eq. (8) with ramp start 0: case 1 (i <= T fs) phase 2 pi (i/fs)(f_start + p[i]),
    case 2 (i > T fs) 2 pi f_finish i/fs + pi T (f_start - f_finish)."""
    fs_, fa, fb, N = FS, 88.8e6, 92.1e6, 280_000
    p = words.Plan(fs_, 1.0, 0, one_tone(fa, 0.0, 1.0, fb, RAMP_MINJERK, 0, N))
    r = p.tones[0].ramps[0]
    fA, fB = _exact_freq(r.f_line, fs_), _exact_freq(r.f_after, fs_)
    T = Fraction(N) / Fraction(fs_)
    tol = abs(r.dF) / Fraction(1 << 17) + 3
    for i in [0, 1, 2, 17, 1000, N // 3, N // 2, N - 5, N]:
        tau = Fraction(i, N)
        pp = (fB - fA) * (Fraction(5, 2) * tau ** 3 - 3 * tau ** 4 + tau ** 5)
        case1 = Fraction(i) / Fraction(fs_) * (fA + pp)
        assert abs(signed_turn_diff(p.phase_at(0, i), case1)) * TWO64 <= tol, i
    for i in [N + 1, N + 2, 3 * N]:
        case2 = fB * Fraction(i) / Fraction(fs_) + T * (fA - fB) / 2
        assert abs(signed_turn_diff(p.phase_at(0, i), case2)) * TWO64 <= tol, i


def test_minjerk_end_phase_golden():
    g = read_golden("eq8_minjerk_end_phase.txt")
    N = int(round(g["T_s"] * g["fs_hz"]))
    p = words.Plan(g["fs_hz"], 1.0, 0, one_tone(g["f_start_hz"], 0.0, 1.0, g["f_finish_hz"],
                                                RAMP_MINJERK, 0, N))
    w = p.phase_at(0, N)
    d = signed_turn_diff(w, Fraction(g["end_phase_turns"]))
    # only word rounding separates the two: F0, F1 to 1/2 word, H to 1/2 unit
    assert abs(d) < 1e-6


def test_cosine_ramp_matches_continuous_phase():
    """f = f0 + df (1 - cos(pi t/T))/2 has phase theta + f0 t + df (t/2 - T sin(pi t/T)/(2 pi))."""
    f0, f1, N, a, th = 77.7e6, 81.0e6, 123_457, 1000, 0.6
    p = words.Plan(FS, 1.0, 0, one_tone(f0, th, 1.0, f1, RAMP_COSINE, a, N))
    tw = p.tones[0]
    r = tw.ramps[0]
    fA, fB = _exact_freq(r.f_line, FS), _exact_freq(r.f_after, FS)
    T = Fraction(N) / Fraction(FS)
    theta = Fraction(tw.p0, TWO64)
    for d in [0, 1, 5, 999, N // 4, N // 2, N - 1, N]:
        n = a + d
        t = Fraction(n) / Fraction(FS)
        tl = Fraction(d) / Fraction(FS)
        sin_part = Fraction(float(T) * math.sin(math.pi * d / N) / (2 * math.pi))
        cont = theta + fA * t + (fB - fA) * (tl / 2 - sin_part)
        diff = abs(signed_turn_diff(p.phase_at(0, n), cont)) * TWO64
        assert diff <= abs(r.dF) / Fraction(1 << 17) + 1e8, d


@pytest.mark.parametrize("shape", [RAMP_COSINE, RAMP_MINJERK])
def test_ramp_table_invariants(shape):
    for N in [1, 2, 3, 7, 64, 1000, 4099]:
        H = [int(v) for v in words.ramp_table(shape, N)]
        assert H[0] == 0 and H[N] == N << 15                # Psi(0) = 0, Psi(1) = 1/2
        assert all(H[i + 1] >= H[i] for i in range(N))      # frequency never below f0
        for d in range(N + 1):
            # s(1 - tau) = 1 - s(tau)  =>  Psi(1 - tau) - Psi(tau) = 1/2 - tau
            assert abs(H[N - d] - H[d] - ((N << 15) - (d << 16))) <= 1


def test_all_shapes_share_end_phase():
    f0, f1, N = 99e6, 104e6, 50_000
    ends = []
    for shape in (RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK):
        p = words.Plan(FS, 1.0, 0, one_tone(f0, 0.1, 1.0, f1, shape, 10, N))
        ends.append(p.phase_at(0, 10 + N))
        assert (p.phase_at(0, 11 + N) - ends[-1]) % TWO64 == p.tones[0].ramps[0].f_after
    dF = abs(p.tones[0].ramps[0].dF)
    for e in ends[1:]:
        d = (e - ends[0]) % TWO64
        d = min(d, TWO64 - d)
        assert d <= N * N / 4 + dF / (1 << 17) + 4


def test_held_tone_is_periodic_after_ramp(oracle_built):
    """Eq. (8) case 3: past the window the tone is a bin tone again, period L."""
    p2 = 12
    L = 1 << p2
    t = make_tones(2)
    t["f_start_hz"] = [1000 * FS / L, 1500 * FS / L]
    t["f_end_hz"] = [1100.3 * FS / L, 1399.6 * FS / L]
    t["amplitude"] = [0.7, 0.4]
    t["phase_turns"] = [0.2, 0.9]
    t["ramp"] = [RAMP_MINJERK, RAMP_LINEAR]
    t["ramp_start"] = [100, 333]
    t["ramp_len"] = [3000, 2500]
    p = words.Plan(FS, 0.0, p2, t, build_tables=True)
    start = 4000
    q, y = csynth.synth(p, start, 2 * L)
    assert np.array_equal(q[L:], q[:L])
    assert not np.array_equal(*csynth.synth(p, 0, 2 * L)[0].reshape(2, L))


def test_retune_chain_is_continuous():
    p = words.Plan(FS, 1.0, 0, one_tone(90e6, 0.4, 1.0))
    p.add_ramp(0, 100, 50, RAMP_LINEAR, 91e6)
    p.add_ramp(0, 150, 70, RAMP_COSINE, 89e6)      # starts exactly where the first ends
    p.add_ramp(0, 400, 30, RAMP_MINJERK, 93e6)
    tw = p.tones[0]
    r1, r2, r3 = tw.ramps
    assert r2.f_line == r1.f_after and r2.p_line == r1.p_after
    assert r3.f_line == r2.f_after and r3.p_line == r2.p_after
    # the chirp term vanishes at d = 0, so each window opens on the previous line
    for r in (r1, r2, r3):
        assert p.phase_at(0, r.a) == (r.p_line + r.f_line * r.a) % TWO64
    for n in range(220, 400):
        assert (p.phase_at(0, n + 1) - p.phase_at(0, n)) % TWO64 == r2.f_after
    with pytest.raises(ValueError):
        p.add_ramp(0, 420, 10, RAMP_LINEAR, 90e6)   # overlaps the last window


# -------------------------------------------------- two oracle paths agree

def _tiny_cases():
    rng = np.random.default_rng(5)
    cases = []
    for seed in range(6):
        K = int(rng.integers(1, 5))
        t = make_tones(K)
        t["f_start_hz"] = rng.uniform(1e6, 139e6, K)
        t["f_end_hz"] = np.clip(t["f_start_hz"] + rng.uniform(-5e6, 5e6, K), 1e6, 139e6)
        t["amplitude"] = rng.uniform(0.1, 1, K)
        t["phase_turns"] = rng.random(K)
        t["ramp"] = rng.integers(0, 4, K)
        t["ramp_start"] = rng.integers(0, 30, K)
        t["ramp_len"] = rng.integers(1, 40, K)
        cases.append(t)
    return cases


@pytest.mark.parametrize("case", range(6))
def test_c_sum_equals_python_bigint(oracle_built, case):
    t = _tiny_cases()[case]
    p = words.Plan(FS, 0.0, 0, t, build_tables=True)
    q, y = csynth.synth(p, 0, 64)
    qp, yp = p.synth_points(range(64))
    assert np.array_equal(q, qp)
    assert np.max(np.abs(y - yp)) < 1e-9
    for k in range(len(t)):
        ph = csynth.phases(p, k, 0, 64)
        assert [int(v) for v in ph] == [p.phase_at(k, n) for n in range(64)]


def test_brute_force_long_double(oracle_built):
    """K <= 4, n < 64: the int16 samples from the physical definition evaluated in
    80-bit long double (phases as exact rationals of the bin tones) match."""
    rng = np.random.default_rng(6)
    p2 = 9
    L = 1 << p2
    for _ in range(5):
        K = int(rng.integers(1, 5))
        bins = rng.choice(np.arange(1, L // 2), K, replace=False)
        th = rng.integers(0, 1 << 20, K) / float(1 << 20)
        amps = rng.uniform(0.1, 1, K)
        t = make_tones(K)
        t["f_start_hz"] = bins * (FS / L)
        t["f_end_hz"] = t["f_start_hz"]
        t["amplitude"] = amps
        t["phase_turns"] = th
        p = words.Plan(FS, 0.0, p2, t)
        q, y = csynth.synth(p, 0, 64)
        G = np.longdouble(32767) / np.sum(amps.astype(np.longdouble))
        n = np.arange(64)
        ref = np.zeros(64, dtype=np.longdouble)
        for b, a, h in zip(bins, amps, th):
            turns = ((int(b) * n) % L).astype(np.longdouble) / L + np.longdouble(h)
            ref += np.longdouble(a) * G * np.sin(2 * np.pi * turns)
        assert np.max(np.abs(y - ref.astype(np.float64))) < 1e-9
        rq = np.clip(np.rint(ref), -32768, 32767).astype(np.int16)
        assert np.array_equal(q, rq)


# ------------------------------------------------------- amplitude ramps (Eq. (5) a_j[i])

def test_amp_ramp_quarter_rate_closed_form(oracle_built):
    """A quarter-rate cosine (samples 1, 0, -1, 0) of 1000 LSB ramped linearly to 0
    over [4, 12]: every sample is a hand-computed multiple of 125."""
    p = words.Plan(FS, 1000.0, 0, one_tone(FS / 4, phase=0.25))
    p.add_amp_ramp(0, 4, 8, RAMP_LINEAR, 0.0)
    _, y = csynth.synth(p, 0, 16)
    want = [1000, 0, -1000, 0, 1000, 0, -750, 0, 500, 0, -250, 0, 0, 0, 0, 0]
    assert np.max(np.abs(y - np.array(want, dtype=float))) < 1e-9
    _, yp = p.synth_points(range(16))
    assert np.max(np.abs(yp - np.array(want, dtype=float))) < 1e-9


@pytest.mark.parametrize("shape,M,d,frac", [
    (RAMP_LINEAR, 1024, 512, Fraction(1, 2)),
    (RAMP_COSINE, 768, 256, Fraction(1, 4)),        # (1 - cos(pi/3)) / 2
    (RAMP_COSINE, 1024, 512, Fraction(1, 2)),
    (RAMP_MINJERK, 1024, 256, Fraction(106, 1024)),  # 10/64 - 15/256 + 6/1024
    (RAMP_MINJERK, 1024, 512, Fraction(1, 2)),
    (RAMP_MINJERK, 1024, 768, Fraction(918, 1024)),
])
def test_amp_profile_values(oracle_built, shape, M, d, frac):
    """From 1000 to 0: amplitude 1000 (1 - s); s at these points fixed by hand."""
    p = words.Plan(FS, 1000.0, 0, one_tone(30e6))
    p.add_amp_ramp(0, 100, M, shape, 0.0)
    want = float(1000 * (1 - frac))
    assert abs(p.tones[0].amp_at(100 + d) - want) < 1e-9
    assert abs(csynth.amps_at(p, 0, [100 + d])[0] - want) < 1e-9


@pytest.mark.parametrize("shape", [RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK])
def test_amp_profile_invariants(oracle_built, shape):
    """Ends exact, s(1 - t) = 1 - s(t), monotone; minimum jerk starts and ends flat."""
    M = 1000
    p = words.Plan(FS, 1.0, 0, one_tone(30e6, amp=2.0))
    p.add_amp_ramp(0, 50, M, shape, 0.5)
    tw = p.tones[0]
    ns = np.arange(0, 50 + M + 60)
    a = csynth.amps_at(p, 0, ns)
    assert a[0] == 2.0 and a[50] == 2.0 and a[50 + M] == 0.5 and a[-1] == 0.5
    d = np.arange(M + 1)
    s = (2.0 - a[50 + d]) / 1.5
    assert np.max(np.abs(s + s[::-1] - 1.0)) < 1e-12
    assert np.all(np.diff(s) >= -1e-15)
    if shape == RAMP_MINJERK:
        assert s[1] < 1e-7 and 1.0 - s[M - 1] < 1e-7          # s ~ 10 t^3 near the ends
    else:
        assert s[1] > 1e-6
    assert abs(tw.amp_at(50 + M // 2) - csynth.amps_at(p, 0, [50 + M // 2])[0]) < 1e-12


def test_switched_off_tone_leaves_the_others(oracle_built):
    """Ramping a tone to 0 (the rearrangement demo's tones turned off): afterwards the
    sum is exactly that of the other tones; before the ramp, that of all three."""
    t = make_tones(3)
    t["f_start_hz"] = [31e6, 47e6, 88e6]
    t["f_end_hz"] = t["f_start_hz"]
    t["amplitude"] = [0.5, 0.9, 0.7]
    t["phase_turns"] = [0.1, 0.6, 0.3]
    p = words.Plan(FS, 1000.0, 0, t)
    p.add_amp_ramp(1, 100, 64, RAMP_COSINE, 0.0)
    keep = words.Plan(FS, 1000.0, 0, t[[0, 2]])
    full = words.Plan(FS, 1000.0, 0, t)
    _, y = csynth.synth(p, 0, 300)
    _, yk = csynth.synth(keep, 0, 300)
    _, yf = csynth.synth(full, 0, 300)
    assert np.array_equal(y[165:], yk[165:])
    assert np.array_equal(y[:101], yf[:101])
    assert not np.array_equal(y[101:164], yk[101:164])


def test_amp_ramp_chain_is_continuous():
    p = words.Plan(FS, 10.0, 0, one_tone(30e6, amp=1.0))
    p.add_amp_ramp(0, 10, 10, RAMP_LINEAR, 0.5)
    p.add_amp_ramp(0, 20, 20, RAMP_MINJERK, 1.5)        # starts where the first ends
    tw = p.tones[0]
    assert tw.amp_at(9) == 10.0 and tw.amp_at(20) == 5.0 and tw.amp_at(40) == 15.0
    assert tw.amp_at(1000) == 15.0
    assert abs(tw.amp_at(15) - 7.5) < 1e-12
    with pytest.raises(ValueError):
        p.add_amp_ramp(0, 39, 5, RAMP_LINEAR, 0.0)       # overlaps the last window
    with pytest.raises(ValueError):
        p.add_amp_ramp(0, 50, 0, RAMP_LINEAR, 0.0)       # empty window


@pytest.mark.parametrize("case", range(6))
def test_c_sum_equals_python_with_amp_ramps(oracle_built, case):
    """The C and the Python evaluators agree with amplitude and frequency ramps mixed."""
    t = _tiny_cases()[case]
    p = words.Plan(FS, 0.0, 0, t, build_tables=True)
    rng = np.random.default_rng(100 + case)
    for k in range(len(t)):
        b = int(rng.integers(0, 20))
        p.add_amp_ramp(k, b, int(rng.integers(1, 30)), int(rng.integers(1, 4)), float(rng.uniform(0, 1)))
        if rng.random() < 0.5:
            p.add_amp_ramp(k, 52, int(rng.integers(1, 10)), int(rng.integers(1, 4)), 0.0)
    q, y = csynth.synth(p, 0, 64)
    qp, yp = p.synth_points(range(64))
    assert np.array_equal(q, qp)
    assert np.max(np.abs(y - yp)) < 1e-9


# ------------------------------------------------ crest-factor phases (Theory section)

from oracle import phases as PH   # noqa: E402


def test_schroeder_equal_amplitudes_reduce_to_textbook_form():
    """For equal amplitudes Schroeder's rule is -pi k (k - 1) / K, i.e. -k(k-1)/(2K) turns."""
    K = 37
    f = np.linspace(10e6, 50e6, K)[::-1]            # ranks are by frequency, not input order
    got = PH.phase_plan(PH.SCHROEDER, f, np.ones(K))
    for i in range(K):
        k = K - i                                  # rank of input i (frequencies descend)
        t = Fraction(-k * (k - 1), 2 * K)
        assert abs(got[i] - float(t - math.floor(t))) < 1e-15


def test_schroeder_unequal_amplitudes_by_hand():
    """K = 3, A = 1, 2, 3: Schroeder's rule weights each tone by its power share
    A^2 / sum A^2 (tests/golden/schroeder_unequal_k3.txt works it by hand);
    frequencies are given out of order to check the ranking."""
    g = read_golden("schroeder_unequal_k3.txt")
    f = [3e6, 1e6, 2e6]
    amps = [3.0, 1.0, 2.0]                          # rank 3, 1, 2
    got = PH.phase_plan(PH.SCHROEDER, f, amps)
    want = [Fraction(g["theta%d_num" % r], g["theta%d_den" % r]) for r in (3, 1, 2)]
    for x, w in zip(got, want):
        assert abs(x - float(w)) < 1e-15, (got, want)


def test_schroeder_sweep_spends_time_by_power():
    """Schroeder's construction: the phase slope between neighbouring tones is
    minus the power fraction accumulated so far, so the waveform's frequency
    sweep dwells on each tone for a share of the period equal to its power
    share. With p_k = A_k^2 / sum A^2 and P_k = p_1 + ... + p_k (turns):
    theta_{k+1} - theta_k = -P_k (mod 1). Two amplitude levels, 1 and 3, make the
    weighting by power (not by amplitude) visible."""
    rng = np.random.default_rng(11)
    K = 40
    amps = np.where(rng.random(K) < 0.5, 1.0, 3.0)
    f = rng.permutation(np.arange(K) + 1.0) * 1e6
    got = PH.phase_plan(PH.SCHROEDER, f, amps)
    order = np.argsort(f, kind="stable")
    power = amps[order] ** 2 / np.sum(amps ** 2)
    P = np.cumsum(power)
    th = np.array(got)[order]
    for k in range(K - 1):
        d = (th[k + 1] - th[k] + P[k]) % 1.0
        assert min(d, 1.0 - d) < 1e-12, k


def test_newman_phases_by_hand():
    """K = 4: (k-1)^2 / 8 turns = 0, 1/8, 4/8, 9/8 -> 1/8."""
    got = PH.phase_plan(PH.NEWMAN, [4e6, 1e6, 3e6, 2e6], None)
    assert got == [0.125, 0.0, 0.5, 0.125]


def test_crest_factor_of_aligned_cosines_is_exact(oracle_built):
    """All tones in cosine phase meet at n = 0: peak = G sum A, so the crest factor is
    sum A / sqrt(sum A^2 / 2) exactly (|y| can never exceed G sum A)."""
    p2 = 12
    L = 1 << p2
    rng = np.random.default_rng(7)
    K = 9
    t = make_tones(K)
    t["f_start_hz"] = rng.choice(np.arange(1, L // 2), K, replace=False) * (FS / L)
    t["f_end_hz"] = t["f_start_hz"]
    t["amplitude"] = rng.uniform(0.2, 1.0, K)
    t["phase_turns"] = 0.25
    p = words.Plan(FS, 100.0, p2, t)
    _, y = csynth.synth(p, 0, L)
    want = np.sum(t["amplitude"]) / math.sqrt(np.sum(t["amplitude"] ** 2) / 2)
    assert abs(PH.crest_factor(y, t["amplitude"], 100.0) - want) < 1e-9


def test_schroeder_phases_lower_the_crest_factor(oracle_built):
    """64 equal tones on consecutive bins: aligned cosines give sqrt(2K) = 11.3;
    Schroeder's phases bring the peak within 2x the rms (about 1.7 is the
    classical figure for such multisines)."""
    p2, K = 12, 64
    L = 1 << p2
    t = make_tones(K)
    t["f_start_hz"] = (np.arange(K) + 100) * (FS / L)
    t["f_end_hz"] = t["f_start_hz"]
    t["amplitude"] = 1.0
    t["phase_turns"] = PH.phase_plan(PH.SCHROEDER, t["f_start_hz"], t["amplitude"])
    _, y = csynth.synth(words.Plan(FS, 100.0, p2, t), 0, L)
    cf = PH.crest_factor(y, t["amplitude"], 100.0)
    assert 1.41 < cf < 2.0, cf
    t["phase_turns"] = 0.25
    _, y0 = csynth.synth(words.Plan(FS, 100.0, p2, t), 0, L)
    assert abs(PH.crest_factor(y0, t["amplitude"], 100.0) - math.sqrt(2 * K)) < 1e-9
