"""CPU tests of the library's host side: exported symbols, exact plan words,
ramp tables and argument validation, each compared with the oracle or with the
rules stated in include/awg.h. No GPU call is made here (host-only plans)."""
import os
import re

import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "awg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(awg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 17
    L = awg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(awg.EXPORTED), sorted(set(names) ^ set(awg.EXPORTED))
    assert awg.awg_version() >= 100
    assert awg.awg_strerror(awg.AWG_E_RANGE) == "value out of range"


def _host_plan(w, flags=0):
    return awg.awg_plan_tones(None, w.fs_hz, w.gain_lsb, w.period_log2, flags, w.tones)


def _compare_words(w):
    plan, fq = _host_plan(w)
    try:
        lw = awg.awg_plan_words(plan, len(w.tones))
        info = awg.awg_plan_info_get(plan)
    finally:
        awg.awg_plan_destroy(plan)
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones)
    assert info["gain_lsb"] == op.gain
    for k, tw in enumerate(op.tones):
        assert int(lw["f0"][k]) == tw.f0
        if tw.ramps:
            r = tw.ramps[0]
            assert int(lw["p0"][k]) == r.p_line
            assert int(lw["f1"][k]) == r.f_after
            assert int(lw["coef"][k]) == r.coef
        else:
            assert int(lw["p0"][k]) == tw.p0
            assert int(lw["f1"][k]) == tw.f0
            assert int(lw["coef"][k]) == 0
        assert fq[k] == pytest.approx(tw.f0 * w.fs_hz / 2.0 ** 64, rel=1e-15)


@pytest.mark.parametrize("maker", [W.static_100tone_chunk, W.static_period, lambda: W.chirp_35ms(shape="mixed"),
                                   lambda: W.chirp_35ms(shape="minjerk", K=50),
                                   lambda: W.small_mixed(), lambda: W.small_mixed(seed=3, period_log2=16),
                                   lambda: W.array_group_chirps(K=5000, seconds=0.01)])
def test_plan_words_equal_oracle(maker):
    _compare_words(maker())


def test_plan_words_random_extremes():
    rng = np.random.default_rng(7)
    for fs in (1.0, 3.0, 280e6, 1e12, 2.0 ** 40 + 1):
        t = awg.make_tones(64)
        t["f_start_hz"] = rng.uniform(1e-9, 0.4999, 64) * fs
        t["f_end_hz"] = rng.uniform(1e-9, 0.4999, 64) * fs
        t["amplitude"] = rng.random(64)
        t["phase_turns"] = rng.normal(0, 1e3, 64)
        t["phase_turns"][:4] = [0.0, -0.5, 2.0 ** -65, -3 * 2.0 ** -66]
        t["ramp"] = rng.integers(0, 4, 64)
        t["ramp_start"] = rng.integers(0, 1 << 40, 64)
        t["ramp_len"] = rng.integers(1, 1 << 20, 64)
        _compare_words(W.Workload("rand", fs, 0.0, 0, t))
        _compare_words(W.Workload("rand", fs, 1.5, 40, t))


@pytest.mark.parametrize("period_log2", [0, 10, 20, 24])
def test_frequency_words_at_exact_ties(period_log2):
    """Frequencies whose word is exactly half-way between two integers (fs a
    power of two, f = (k + 1/2) fs / 2^s with s the word's shift), and the
    doubles either side of them: the rounding to nearest, ties to even, of
    Eq. (4) for both parities of k, against the oracle's tuning word."""
    fs = 2.0 ** 28
    s = period_log2 if period_log2 else 64
    top = (1 << (period_log2 - 1)) - 2 if period_log2 else (1 << 52)
    rng = np.random.default_rng(period_log2 + 1)
    ks = np.concatenate([[1, 2, 3, top - 1, top], rng.integers(1, top, 27)])
    f = []
    for k in ks.tolist():
        x = (k + 0.5) * 2.0 ** (28 - s)
        f += [x, np.nextafter(x, 0.0), np.nextafter(x, np.inf)]
    t = awg.make_tones(len(f))
    t["f_start_hz"] = f
    t["f_end_hz"] = f
    t["amplitude"] = 1.0
    w = W.Workload("ties", fs, 0.0, period_log2, t)
    _compare_words(w)
    plan, _ = _host_plan(w)
    try:
        lw = awg.awg_plan_words(plan, len(f))
    finally:
        awg.awg_plan_destroy(plan)
    shift = 64 - s
    for j, k in enumerate(ks.tolist()):           # the tie itself goes to the even neighbour
        even = k if k % 2 == 0 else k + 1
        assert int(lw["f0"][3 * j]) >> shift == even, (k, period_log2)


@pytest.mark.parametrize("shape", [awg.RAMP_COSINE, awg.RAMP_MINJERK])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 100, 4097, 65537])
def test_ramp_tables_equal_oracle(shape, n):
    lt = awg.awg_ramp_table(shape, n)
    if n <= 5000:
        ot = words.ramp_table(shape, n)
        assert np.array_equal(lt, ot)
    else:
        ds = list(range(0, n + 1, 997)) + [n - 1, n]
        assert [int(lt[d]) for d in ds] == words.ramp_table_entries(shape, n, ds)


@pytest.mark.parametrize("shape", [awg.RAMP_COSINE, awg.RAMP_MINJERK])
def test_ramp_table_full_size_samples(shape):
    n = W.RAMP_35MS
    lt = awg.awg_ramp_table(shape, n)
    rng = np.random.default_rng(8)
    ds = sorted(set(rng.integers(0, n + 1, 300).tolist()) | {0, 1, n // 2, n - 1, n})
    assert [int(lt[d]) for d in ds] == words.ramp_table_entries(shape, n, ds)


def _status(tones, fs=280e6, gain=0.0, p=0, flags=0):
    try:
        plan, _ = awg.awg_plan_tones(None, fs, gain, p, flags, tones)
    except awg.AwgError as e:
        return e.status
    awg.awg_plan_destroy(plan)
    return awg.AWG_OK


def test_validation_codes():
    good = W.small_mixed().tones
    assert _status(good) == awg.AWG_OK
    assert _status(good[:0]) == awg.AWG_E_INVALID
    assert _status(good, fs=0.0) == awg.AWG_E_INVALID
    assert _status(good, fs=float("nan")) == awg.AWG_E_INVALID
    assert _status(good, gain=-1.0) == awg.AWG_E_INVALID
    assert _status(good, p=1) == awg.AWG_E_INVALID
    assert _status(good, p=64) == awg.AWG_E_INVALID
    assert _status(good, flags=3) == awg.AWG_E_INVALID
    for field, val, code in [("f_start_hz", 140e6, awg.AWG_E_INVALID),
                             ("f_start_hz", 0.0, awg.AWG_E_INVALID),
                             ("f_start_hz", float("inf"), awg.AWG_E_INVALID),
                             ("amplitude", -0.1, awg.AWG_E_INVALID),
                             ("phase_turns", float("nan"), awg.AWG_E_INVALID),
                             ("ramp", 7, awg.AWG_E_INVALID),
                             ("reserved", 1, awg.AWG_E_INVALID)]:
        t = good.copy()
        t[1][field] = val
        assert _status(t) == code, field
    t = good.copy()
    t[1]["ramp"] = awg.RAMP_LINEAR
    t[1]["ramp_len"] = 0
    assert _status(t) == awg.AWG_E_RANGE
    t[1]["ramp_len"] = 1 << 31
    assert _status(t) == awg.AWG_E_RANGE
    t[1]["ramp_len"] = 10
    t[1]["ramp_start"] = (1 << 63) - 5
    assert _status(t) == awg.AWG_E_RANGE
    t[1]["ramp_start"] = 0
    t[1]["f_end_hz"] = 150e6
    assert _status(t) == awg.AWG_E_INVALID
    # bins: 140 MHz - 1 Hz snaps onto the Nyquist bin of L = 2**20; 1 Hz onto bin 0
    t = good.copy()
    t[0]["f_start_hz"] = 140e6 - 1.0
    assert _status(t, p=20) == awg.AWG_E_RANGE
    t[0]["f_start_hz"] = 1.0
    assert _status(t, p=20) == awg.AWG_E_RANGE
    # all amplitudes zero with the default gain
    t = good.copy()
    t["amplitude"] = 0.0
    assert _status(t) == awg.AWG_E_INVALID
    assert _status(t, gain=5.0) == awg.AWG_OK


def test_host_only_plan_rejects_synthesis():
    plan, _ = awg.awg_plan_tones(None, 280e6, 0.0, 0, 0, W.small_mixed().tones)
    try:
        with pytest.raises(awg.AwgError) as e:
            awg.awg_synth_chirp(plan, 0, 16, 1234)
        assert e.value.status == awg.AWG_E_INVALID
        awg.awg_stream_seek(plan, 77)
        assert awg.awg_stream_tell(plan) == 77
        with pytest.raises(awg.AwgError):
            awg.awg_stream_seek(plan, 1 << 63)
    finally:
        awg.awg_plan_destroy(plan)


def test_retune_words_follow_oracle_chain():
    w = W.array_group_chirps(K=300, seconds=0.004, group=100)
    plan, _ = _host_plan(w)
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones)
    try:
        for (k, a, n, shape, f) in w.retunes:
            awg.awg_plan_retune(plan, [(k, shape, a, n, f)])
            op.add_ramp(k, a, n, shape, f)
        lw = awg.awg_plan_words(plan, len(w.tones))
        for k, tw in enumerate(op.tones):
            r = tw.ramps[-1]
            assert int(lw["p0"][k]) == r.p_line and int(lw["f1"][k]) == r.f_after
            assert int(lw["coef"][k]) == r.coef
        # a window may not open before the previous one closes, nor twice per call
        k, a, n, shape, f = w.retunes[-1]
        with pytest.raises(awg.AwgError) as e:
            awg.awg_plan_retune(plan, [(k, shape, a + 1, n, f)])
        assert e.value.status == awg.AWG_E_RANGE
        with pytest.raises(awg.AwgError) as e:
            awg.awg_plan_retune(plan, [(0, shape, 1 << 40, 5, 70e6), (0, shape, 1 << 41, 5, 71e6)])
        assert e.value.status == awg.AWG_E_UNSUPPORTED
    finally:
        awg.awg_plan_destroy(plan)


def test_amplitude_ramp_validation_and_counts():
    """awg_plan_amplitude on a host-only plan: argument checks, chaining rules, and the
    plan counts a tone with an amplitude window as dynamic (no static fast path)."""
    w = W.static_100tone_chunk()
    plan, _ = _host_plan(w)
    try:
        assert awg.awg_plan_info_get(plan)["n_ramped"] == 0
        L, C, M = awg.RAMP_LINEAR, awg.RAMP_COSINE, awg.RAMP_MINJERK
        awg.awg_plan_amplitude(plan, [(0, L, 100, 50, 0.0), (1, C, 0, 1, 2.0), (2, M, 5, 1000, 0.5)])
        assert awg.awg_plan_info_get(plan)["n_ramped"] == 3
        awg.awg_plan_amplitude(plan, [(0, M, 150, 10, 1.0)])          # starts where the last ended
        assert awg.awg_plan_info_get(plan)["n_ramped"] == 3
        bad = [
            ([(len(w.tones), L, 0, 10, 0.0)], awg.AWG_E_INVALID),      # no such tone
            ([(5, awg.RAMP_NONE, 0, 10, 0.0)], awg.AWG_E_INVALID),     # no profile
            ([(5, L, 0, 10, -0.1)], awg.AWG_E_INVALID),                # negative amplitude
            ([(5, L, 0, 10, float("nan"))], awg.AWG_E_INVALID),
            ([(5, L, 0, 0, 0.0)], awg.AWG_E_RANGE),                    # empty window
            ([(5, L, 0, 1 << 31, 0.0)], awg.AWG_E_RANGE),              # too long
            ([(5, L, (1 << 63) - 5, 10, 0.0)], awg.AWG_E_RANGE),       # past the last sample
            ([(0, L, 159, 10, 0.0)], awg.AWG_E_RANGE),                 # before the previous end
            ([(6, L, 0, 10, 0.0), (6, L, 100, 10, 0.0)], awg.AWG_E_UNSUPPORTED),
        ]
        for events, status in bad:
            with pytest.raises(awg.AwgError) as e:
                awg.awg_plan_amplitude(plan, events)
            assert e.value.status == status, events
        assert awg.awg_plan_info_get(plan)["n_ramped"] == 3            # failed calls change nothing
        # a tone named twice in a failed call can be named once in the next one,
        # and a duplicate at the end of a long list is still found
        awg.awg_plan_amplitude(plan, [(6, L, 0, 10, 0.0)])
        many = [(k, L, 1000, 10, 0.5) for k in range(7, len(w.tones))]
        with pytest.raises(awg.AwgError) as e:
            awg.awg_plan_amplitude(plan, many + [(len(w.tones) - 1, L, 5000, 10, 0.5)])
        assert e.value.status == awg.AWG_E_UNSUPPORTED
        awg.awg_plan_amplitude(plan, many)
        assert awg.awg_plan_info_get(plan)["n_ramped"] == 4 + len(many)
        with pytest.raises(awg.AwgError) as e:
            awg.awg_synth_static(plan, 0, 16, 1234)                     # host-only, and no longer static
        assert e.value.status == awg.AWG_E_INVALID
    finally:
        awg.awg_plan_destroy(plan)


def test_phase_plan_matches_oracle():
    from oracle import phases as PH
    rng = np.random.default_rng(8)
    for K in (1, 2, 7, 100, 300):
        f = rng.uniform(1e6, 100e6, K)
        f[:K // 3] = f[0]                                      # ties keep input order
        a = rng.uniform(0.0, 1.0, K)
        for m in (awg.AWG_PHASES_SCHROEDER, awg.AWG_PHASES_NEWMAN):
            got = awg.awg_phase_plan(m, f, a)
            want = np.array(PH.phase_plan(m, f, a))
            d = np.abs(got - want)
            d = np.minimum(d, 1.0 - d)                         # distance on the circle
            assert np.all((got >= 0) & (got < 1)) and d.max() < 1e-12, (K, m, d.max())
    for bad in [(3, [1e6], [1.0]), (awg.AWG_PHASES_SCHROEDER, [1e6, 2e6], [0.0, 0.0]),
                (awg.AWG_PHASES_SCHROEDER, [1e6], [-1.0]), (awg.AWG_PHASES_NEWMAN, [float("inf")], None)]:
        with pytest.raises(awg.AwgError) as e:
            awg.awg_phase_plan(*bad)
        assert e.value.status == awg.AWG_E_INVALID


def test_smooth_table_limit():
    """A plan holds at most 1024 distinct smooth ramp tables (shape, length):
    1024 distinct lengths plan, 1025 are refused with AWG_E_UNSUPPORTED; linear
    ramps need no table and are not counted."""
    def tones(n_smooth, n_linear=0):
        K = n_smooth + n_linear
        t = np.zeros(K, dtype=awg.abi_types.TONE_DTYPE)
        t["f_start_hz"] = 50e6
        t["f_end_hz"] = 51e6
        t["amplitude"] = 1.0
        t["ramp"] = [awg.RAMP_COSINE] * n_smooth + [awg.RAMP_LINEAR] * n_linear
        t["ramp_len"] = np.arange(1, K + 1)
        return t
    plan, _ = awg.awg_plan_tones(None, 280e6, 0.0, 0, 0, tones(1024, 50))
    awg.awg_plan_destroy(plan)
    with pytest.raises(awg.AwgError) as e:
        awg.awg_plan_tones(None, 280e6, 0.0, 0, 0, tones(1025))
    assert e.value.status == awg.AWG_E_UNSUPPORTED


def test_reserve_on_host_only_plan_is_invalid():
    w = W.static_100tone_chunk()
    plan, _ = _host_plan(w)
    try:
        with pytest.raises(awg.AwgError) as e:
            awg.awg_plan_reserve(plan, awg.AWG_F_METHOD_DIRECT, 1 << 20)
        assert e.value.status == awg.AWG_E_INVALID
    finally:
        awg.awg_plan_destroy(plan)
