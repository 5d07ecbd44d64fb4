"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each case patches one piece of oracle/words.py (a dropped term, a wrong sign or
index, a swapped operand, a wrong rounding) or compiles a mutated copy of
oracle/synth.c, then runs the pin tests that should notice and asserts that at
least one of them fails. Nothing here touches the library or a GPU.
"""
import math
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import words, csynth

WORD_PINS = [pins.test_eq4_bin_error_matches_paper, pins.test_tuning_word_closed_forms,
             pins.test_phase_word_closed_forms]
CHIRP_PINS = [pins.test_linear_chirp_matches_continuous_phase, pins.test_minjerk_matches_eq8_as_printed,
              pins.test_minjerk_end_phase_golden, pins.test_cosine_ramp_matches_continuous_phase,
              pins.test_all_shapes_share_end_phase, pins.test_retune_chain_is_continuous]
AMP_PINS = [pins.test_amp_ramp_quarter_rate_closed_form, pins.test_amp_profile_values,
            pins.test_amp_profile_invariants, pins.test_switched_off_tone_leaves_the_others,
            pins.test_amp_ramp_chain_is_continuous]
SUM_PINS = [pins.test_quarter_rate_tone_is_exact, pins.test_eighth_rate_tone,
            pins.test_static_tones_match_eq2_in_long_double, pins.test_dirichlet_kernel,
            pins.test_periodicity_with_bin_frequencies, pins.test_mean_power_and_default_gain,
            pins.test_held_tone_is_periodic_after_ramp, pins.test_brute_force_long_double,
            pins.test_c_sum_equals_python_bigint]
QUANT_PINS = [pins.test_quantiser_ties_go_to_even, pins.test_quantiser_saturates_to_int16]


AMP_CASES = [(words.RAMP_LINEAR, 1024, 512, Fraction(1, 2)), (words.RAMP_COSINE, 768, 256, Fraction(1, 4)),
             (words.RAMP_MINJERK, 1024, 256, Fraction(106, 1024))]


def some_pin_fails(tests):
    for t in tests:
        try:
            names = t.__code__.co_varnames[:t.__code__.co_argcount]
            if "frac" in names:
                for c in AMP_CASES:
                    t(True, *c)
            elif names == ("oracle_built", "shape"):
                for s in (words.RAMP_LINEAR, words.RAMP_COSINE, words.RAMP_MINJERK):
                    t(True, s)
            elif "case" in names:
                for c in range(6):
                    t(True, c)
            elif t.__code__.co_argcount == 1:
                t(True)
            elif t.__code__.co_argcount == 0:
                t()
            else:
                t(words.RAMP_COSINE)
                t(words.RAMP_MINJERK)
        except Exception:
            return True
    return False


def test_unmutated_oracle_passes_every_pin_used_here(oracle_built):
    """Control: the harness itself reports no failure on the real oracle."""
    assert not some_pin_fails(WORD_PINS)
    assert not some_pin_fails(CHIRP_PINS)
    assert not some_pin_fails(SUM_PINS)
    assert not some_pin_fails(AMP_PINS)
    assert not some_pin_fails(QUANT_PINS)
    assert not some_pin_fails(PHASE_PINS)


def _floor_round(x):
    x = Fraction(x)
    return x.numerator // x.denominator


def _tuning_word_truncating(f_hz, fs_hz, period_log2=0):
    f, fs = Fraction(f_hz), Fraction(fs_hz)
    if period_log2 > 0:
        return _floor_round(f * (1 << period_log2) / fs) << (64 - period_log2)
    return _floor_round(f * words.TWO64 / fs)


def _quantise_half_away(y):
    y = np.asarray(y, dtype=np.float64)
    r = np.sign(y) * np.floor(np.abs(y) + 0.5)                      # ties away from zero
    return np.clip(r, words.INT16_MIN, words.INT16_MAX).astype(np.int16)


def _quantise_no_clamp(y):
    return np.rint(np.asarray(y, dtype=np.float64)).astype(np.int64).astype(np.int16)   # wraps


QUANT_MUTANTS = {
    "quantiser rounds ties away from zero": _quantise_half_away,
    "quantiser does not saturate": _quantise_no_clamp,
}


@pytest.mark.parametrize("name", sorted(QUANT_MUTANTS))
def test_python_quantiser_mutants_are_caught(monkeypatch, oracle_built, name):
    monkeypatch.setattr(words, "quantise", QUANT_MUTANTS[name])
    assert some_pin_fails(QUANT_PINS), name


WORD_MUTANTS = {
    "bin snapping truncates instead of rounding": ("tuning_word", _tuning_word_truncating),
    "phase word has the wrong sign": ("phase_word", lambda t: (-words.rne(Fraction(t) * words.TWO64)) & words.MASK64),
}


@pytest.mark.parametrize("name", sorted(WORD_MUTANTS))
def test_word_mutants_are_caught(monkeypatch, oracle_built, name):
    attr, fn = WORD_MUTANTS[name]
    monkeypatch.setattr(words, attr, fn)
    assert some_pin_fails(WORD_PINS + SUM_PINS), name


def _minjerk_wrong_coefficient(N, d):
    num = (d ** 4) * (5 * N * N - 5 * d * N + 2 * d * d) << 15      # 6 -> 5
    return words.rne(Fraction(num, N ** 5))


def _cosine_missing_pi(N, d):
    import math
    s = math.sin((math.pi * float(d)) / float(N))
    x = ((32768.0 * float(N)) / 1.0) * s                            # dropped 1/pi
    return (d << 15) - words.rne(Fraction(x))


def _linear_term_no_half(self, d):
    if self.shape == words.RAMP_LINEAR:
        return self.coef * d * d                                    # dropped the /2
    return (self.coef * self.table_at(d)) >> words.TABLE_SHIFT


def _linear_term_plus_sign(self, d):
    if self.shape == words.RAMP_LINEAR:
        return -((self.coef * d * d) >> 1)                          # wrong sign
    return (self.coef * self.table_at(d)) >> words.TABLE_SHIFT


def _smooth_term_wrong_shift(self, d):
    if self.shape == words.RAMP_LINEAR:
        return (self.coef * d * d) >> 1
    return (self.coef * self.table_at(d)) >> (words.TABLE_SHIFT - 1)


CHIRP_MUTANTS = {
    "min-jerk table coefficient": ("minjerk_table_entry", _minjerk_wrong_coefficient, words),
    "cosine table without 1/pi": ("cosine_table_entry", _cosine_missing_pi, words),
    "linear chirp term without 1/2": ("chirp_term", _linear_term_no_half, words.Ramp),
    "linear chirp term with the wrong sign": ("chirp_term", _linear_term_plus_sign, words.Ramp),
    "smooth chirp term scaled by 2": ("chirp_term", _smooth_term_wrong_shift, words.Ramp),
}


@pytest.mark.parametrize("name", sorted(CHIRP_MUTANTS))
def test_chirp_mutants_are_caught(monkeypatch, oracle_built, name):
    attr, fn, owner = CHIRP_MUTANTS[name]
    monkeypatch.setattr(owner, attr, fn)
    assert some_pin_fails(CHIRP_PINS), name


def test_post_window_line_mutant_is_caught(monkeypatch, oracle_built):
    orig = words.Ramp.__init__

    def init(self, a, N, shape, p_line, f_line, f_to, table=None):
        orig(self, a, N, shape, p_line, f_line, f_to, table)
        end = self.a + self.N
        phi_end = (self.p_line + self.f_line * end + self.chirp_term(self.N)) & words.MASK64
        self.p_after = (phi_end - self.f_line * end) & words.MASK64     # start frequency after the window

    monkeypatch.setattr(words.Ramp, "__init__", init)
    assert some_pin_fails(CHIRP_PINS)


def _minjerk_amp_wrong(shape, tau):
    tau = float(tau)
    if shape == words.RAMP_MINJERK:
        return tau ** 3 * (10.0 - 15.0 * tau + 5.0 * tau * tau)     # 6 -> 5
    return ORIG_AMP_SHAPE(shape, tau)


def _cosine_amp_wrong(shape, tau):
    tau = float(tau)
    if shape == words.RAMP_COSINE:
        return (1.0 - math.cos(math.pi * tau))                        # dropped / 2
    return ORIG_AMP_SHAPE(shape, tau)


def _amp_ramp_reversed(self, d):
    s = words.amp_shape(self.shape, Fraction(d, self.M))
    return self.a_to * (1.0 - s) + self.a_from * s


ORIG_AMP_SHAPE = words.amp_shape
AMP_MUTANTS = {
    "min-jerk amplitude profile coefficient": ("amp_shape", _minjerk_amp_wrong, words),
    "raised-cosine amplitude profile without 1/2": ("amp_shape", _cosine_amp_wrong, words),
    "amplitude ramp runs backwards": ("at", _amp_ramp_reversed, words.AmpRamp),
}


@pytest.mark.parametrize("name", sorted(AMP_MUTANTS))
def test_amp_mutants_are_caught(monkeypatch, oracle_built, name):
    attr, fn, owner = AMP_MUTANTS[name]
    monkeypatch.setattr(owner, attr, fn)
    assert some_pin_fails(AMP_PINS), name


def _schroeder_sign_flipped(method, f_hz, amps):
    return [(1.0 - x) % 1.0 for x in ORIG_PHASE_PLAN(method, f_hz, amps)]


def _newman_off_by_one(method, f_hz, amps):
    if method != PH.NEWMAN:
        return ORIG_PHASE_PLAN(method, f_hz, amps)
    K = len(f_hz)
    rank, _ = PH.rank_by_frequency(f_hz)
    return [float(Fraction(rank[i] + 1, 1) ** 2 / (2 * K) % 1) for i in range(K)]


from oracle import phases as PH   # noqa: E402
ORIG_PHASE_PLAN = PH.phase_plan
PHASE_PINS = [pins.test_schroeder_equal_amplitudes_reduce_to_textbook_form, pins.test_newman_phases_by_hand,
              pins.test_schroeder_phases_lower_the_crest_factor, pins.test_schroeder_unequal_amplitudes_by_hand,
              pins.test_schroeder_sweep_spends_time_by_power]


def _schroeder_amplitude_weighted(method, f_hz, amps):
    if method != PH.SCHROEDER:
        return ORIG_PHASE_PLAN(method, f_hz, amps)
    K = len(f_hz)
    _, order = PH.rank_by_frequency(f_hz)
    p = [Fraction(float(amps[i])) for i in order]                   # A_l instead of A_l^2
    total = sum(p)
    p = [x / total for x in p]
    out = [0.0] * K
    for k in range(1, K + 1):
        t = -sum((k - l) * p[l - 1] for l in range(1, k))
        out[order[k - 1]] = float(t - math.floor(t))
    return out


@pytest.mark.parametrize("name,fn", [("Schroeder phases with the wrong sign", _schroeder_sign_flipped),
                                     ("Newman phases with k^2 for (k-1)^2", _newman_off_by_one),
                                     ("Schroeder weights amplitudes instead of powers",
                                      _schroeder_amplitude_weighted)])
def test_phase_plan_mutants_are_caught(monkeypatch, oracle_built, name, fn):
    monkeypatch.setattr(PH, "phase_plan", fn)
    assert some_pin_fails(PHASE_PINS), name


def test_default_gain_mutant_is_caught(monkeypatch, oracle_built):
    monkeypatch.setattr(words, "default_gain", lambda amps: 32767.0 / sum(float(a) ** 2 for a in amps))
    assert some_pin_fails([pins.test_mean_power_and_default_gain])


C_MUTANTS = {
    "sum uses cosine": ("acc += oracle_amp_at(&tones[k], amps, n) * sin(two_pi * turns);",
                        "acc += oracle_amp_at(&tones[k], amps, n) * cos(two_pi * turns);"),
    "turn scale off by 2": ("double turns = (double)(int64_t)w * 0x1p-64;", "double turns = (double)(int64_t)w * 0x1p-63;"),
    "linear term without 1/2": ("return (uint64_t)(prod >> 1);", "return (uint64_t)(prod);"),
    "post-window line uses the start frequency": ("return r->p_after + r->f_after * n;", "return r->p_after + r->f_line * n;"),
    "rounding truncates": ("double r = nearbyint(acc);", "double r = trunc(acc);"),
    "rounding takes ties away from zero": ("double r = nearbyint(acc);", "double r = round(acc);"),
    "no saturation": ("        if (r > 32767.0) r = 32767.0;\n        if (r < -32768.0) r = -32768.0;\n", ""),
    "amplitude held at its start after the ramp": ("if (d > r->m) return r->a_to;", "if (d > r->m) return r->a_from;"),
    "min-jerk amplitude profile coefficient": ("(10.0 - 15.0 * tau + 6.0 * tau * tau)", "(10.0 - 15.0 * tau + 5.0 * tau * tau)"),
}


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_c_oracle_mutants_are_caught(monkeypatch, tmp_path, oracle_built, name):
    old, new = C_MUTANTS[name]
    src = open(csynth._SRC).read()
    assert src.count(old) >= 1, name
    mutated = tmp_path / "synth_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "synth_mut.so"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           str(mutated), "-o", str(lib), "-lm"])
    monkeypatch.setattr(csynth, "_LIB", str(lib))
    monkeypatch.setattr(csynth, "_lib", None)
    monkeypatch.setattr(csynth, "build", lambda force=True: str(lib))
    try:
        assert some_pin_fails(SUM_PINS + AMP_PINS + QUANT_PINS), name
    finally:
        csynth._lib = None
