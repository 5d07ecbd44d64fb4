"""Randomised argument checks of awg_plan_tones on host-only plans (no GPU).

Inputs mix plausible values with the edges of every documented rule (NaN and
infinite fields, negative amplitudes, frequencies at 0, fs/2 and the bins next
to them, ramp lengths 0, 1 and 2^31, windows ending at 2^63, unknown ramp
shapes, reserved fields). The status must be the one the rules in awg.h give,
checked in the order the header lists them, and an accepted plan must carry
exactly the oracle's words."""
import math

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st, HealthCheck

import paper_2403_15582_amd as awg
from paper_2403_15582_amd.abi_types import TONE_DTYPE
from oracle import words

NAN, INF = float("nan"), float("inf")


def _mostly(valid, edges, one_in=8):
    """valid values, and an edge value about once in ``one_in`` draws"""
    return st.integers(min_value=0, max_value=one_in - 1).flatmap(lambda i: edges if i == 0 else valid)


# frequencies as fractions u of fs/2 (f = u fs / 2), so they suit every sample rate
frac_st = _mostly(st.floats(min_value=1e-6, max_value=0.999999, allow_nan=False),
                  st.sampled_from([0.0, 1.0, -0.1, 1.5, NAN, INF, 1e-12, 0.5, 0.9999999999]))

tone_st = st.fixed_dictionaries({
    "u_start": frac_st,
    "u_end": frac_st,
    "amplitude": _mostly(st.floats(min_value=0.0, max_value=2.0, allow_nan=False),
                         st.sampled_from([0.0, -0.5, NAN, INF]), 16),
    "phase_turns": _mostly(st.floats(min_value=-3.0, max_value=3.0, allow_nan=False),
                           st.sampled_from([NAN, -INF, 1e300]), 16),
    "ramp_start": _mostly(st.integers(min_value=0, max_value=1 << 40),
                          st.sampled_from([(1 << 63) - 2, (1 << 63) - 1, (1 << 64) - 1])),
    "ramp_len": _mostly(st.integers(min_value=1, max_value=1 << 20),
                        st.sampled_from([0, 1, (1 << 31) - 1, 1 << 31])),
    "ramp": _mostly(st.sampled_from([0, 0, 1, 2, 3]), st.sampled_from([-1, 4]), 16),
    "reserved": _mostly(st.just(0), st.just(1), 32),
})

params_st = st.fixed_dictionaries({
    "fs": _mostly(st.sampled_from([280e6, 50e6, 1.0]), st.sampled_from([0.0, -1.0, NAN, INF]), 16),
    "gain": _mostly(st.sampled_from([0.0, 100.0, 0.25]), st.sampled_from([-1.0, NAN, INF]), 16),
    "p": _mostly(st.sampled_from([0, 16, 20, 24, 2, 63]), st.sampled_from([1, 64]), 16),
    "flags": _mostly(st.sampled_from([0, 1, 2]), st.sampled_from([3, 4]), 16),
})


def _tone_fields(t, fs):
    """awg_tone fields of a drawn tone at sample rate fs."""
    d = {k: v for k, v in t.items() if k not in ("u_start", "u_end")}
    d["f_start_hz"] = t["u_start"] * fs * 0.5 if math.isfinite(fs) else t["u_start"]
    d["f_end_hz"] = t["u_end"] * fs * 0.5 if math.isfinite(fs) else t["u_end"]
    return d


def _word_status(f, fs, p):
    """Status of a frequency's word: None when it has one."""
    if not (0.0 < f < fs * 0.5):
        return awg.AWG_E_INVALID
    try:
        words.tuning_word(f, fs, p)
    except words.WordError:
        return awg.AWG_E_RANGE
    return None


def expected_status(prm, tones):
    fs, gain, p, flags = prm["fs"], prm["gain"], prm["p"], prm["flags"]
    if not (math.isfinite(fs) and fs > 0) or not (math.isfinite(gain) and gain >= 0):
        return awg.AWG_E_INVALID
    if p == 1 or p > 63 or flags not in (0, 1, 2):
        return awg.AWG_E_INVALID
    for t in tones:
        if not all(math.isfinite(t[k]) for k in ("f_start_hz", "amplitude", "phase_turns")):
            return awg.AWG_E_INVALID
        if not t["amplitude"] >= 0 or t["reserved"] != 0 or not 0 <= t["ramp"] <= 3:
            return awg.AWG_E_INVALID
        if t["ramp"] != 0 and not math.isfinite(t["f_end_hz"]):
            return awg.AWG_E_INVALID
    if gain == 0 and not sum(abs(t["amplitude"]) for t in tones) > 0:
        return awg.AWG_E_INVALID
    for t in tones:
        s = _word_status(t["f_start_hz"], fs, p)
        if s is not None:
            return s
        if t["ramp"] != 0:
            a, n = t["ramp_start"], t["ramp_len"]
            if n == 0 or n >= 1 << 31 or a >= 1 << 63 or n >= (1 << 63) - a:
                return awg.AWG_E_RANGE
            s = _word_status(t["f_end_hz"], fs, p)
            if s is not None:
                return s
    return awg.AWG_OK


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(prm=params_st, drawn=st.lists(tone_st, min_size=1, max_size=4))
def test_plan_status_and_words(prm, drawn):
    tones = [_tone_fields(t, prm["fs"]) for t in drawn]
    arr = np.zeros(len(tones), dtype=TONE_DTYPE)
    for i, t in enumerate(tones):
        for k, v in t.items():
            arr[i][k] = v
    want = expected_status(prm, tones)
    try:
        plan, fq = awg.awg_plan_tones(None, prm["fs"], prm["gain"], prm["p"], prm["flags"], arr)
    except awg.AwgError as e:
        assert e.status == want, (e.status, want, prm, tones)
        return
    try:
        assert want == awg.AWG_OK, (want, prm, tones)
        lw = awg.awg_plan_words(plan, len(tones))
    finally:
        awg.awg_plan_destroy(plan)
    op = words.Plan(prm["fs"], prm["gain"], prm["p"], arr)
    for k, tw in enumerate(op.tones):
        assert int(lw["f0"][k]) == tw.f0
        if tw.ramps:
            r = tw.ramps[0]
            assert (int(lw["p0"][k]), int(lw["f1"][k]), int(lw["coef"][k])) == (r.p_line, r.f_after, r.coef)
        else:
            assert (int(lw["p0"][k]), int(lw["f1"][k]), int(lw["coef"][k])) == (tw.p0, tw.f0, 0)
        assert fq[k] == tw.f0 * prm["fs"] / 2.0 ** 64 or fq[k] == pytest.approx(tw.f0 * prm["fs"] / 2.0 ** 64,
                                                                               rel=1e-15)
