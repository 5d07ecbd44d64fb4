"""The direct kernel's per-sample phase-word rules, replayed in Python integers
and checked against the oracle's exact words (Eq. (8); words mod 2^64).

The kernel never forms a chirp word in closed form per sample: inside a
window and in the tiles where a window's edge falls it steps a lane's 16
words by exact increments (linear windows), by table steps times dF / 2^16
(smooth windows with dF a multiple of 2^16), or by a closed form in the
lane's table rise (smooth windows with any dF, whose sine needs only the
word's high half). A wrong carry or index in those rules moves a word by a
unit of 2^-32 turn, which no comparison of samples can see (about 2e-4 LSB),
so the rules themselves are pinned here: each function below mirrors one
loop of the kernel operation for operation (64-bit wraparound, 24-bit signed
multiplies, 16-bit fraction carries, the 2^40 rounding bias the device words
carry), and every word it yields must equal the oracle's. CPU only.
"""
import numpy as np
import pytest

from oracle import words as OW

M64 = (1 << 64) - 1
M32 = (1 << 32) - 1
BIAS = 1 << 40
S = 16


def s64(x):
    x &= M64
    return x - (1 << 64) if x >> 63 else x


def s32(x):
    x &= M32
    return x - (1 << 32) if x >> 31 else x


def mul24(a, b):
    """__mul24: low 32 bits of the product of two signed 24-bit values."""
    assert -(1 << 23) <= a < (1 << 23) and -(1 << 23) <= b < (1 << 23)
    return (a * b) & M32


# --------------------------------------------------------------- kernel rules

def lin_term(R, d):
    d &= M64
    dd = (d * d) & M64
    return (R * (dd >> 1) + ((R >> 1) if d & 1 else 0)) & M64


def smooth_term(dF, H):
    hh, hl = H >> 16, H & 0xFFFF
    t1 = dF * hh
    lo = (dF & M32) * hl
    hi = s32(dF >> 32) * hl
    return (t1 + (hi << 16) + (lo >> 16)) & M64


def phase_general(t, n):
    if n < t["a"]:
        return (t["p0"] + t["f0"] * n) & M64
    d = n - t["a"]
    if d <= t["N"]:
        base = t["p0"] + t["f0"] * n
        if t["shape"] == OW.RAMP_LINEAR:
            return (base + lin_term(t["coef"], d)) & M64
        return (base + smooth_term(t["coef"], int(t["H"][d]))) & M64
    return (t["p1"] + t["f1"] * n) & M64


def linear_in_window(t, tile0, j):
    R, dt = t["coef"], tile0 - t["a"]
    h, r = R >> 1, R & 1
    W = t["p0"] + t["f0"] * tile0 + lin_term(R, dt)
    V = t["f0"] + R * dt
    I = V + h + (r if dt & 1 else 0)
    Dp = R + (-r if dt & 1 else r)
    Dq = R + (r if dt & 1 else -r)
    ph = (W + V * j + R * (j * j // 2)) & M64
    inc = (I + R * j) & M64
    out = []
    for s in range(S):
        out.append(ph)
        ph = (ph + inc) & M64
        inc = (inc + (Dq if s & 1 else Dp)) & M64
    return out


def linear_edge(t, n):
    d, N, R = n - t["a"], t["N"], t["coef"]
    s_lo = 0 if d >= 0 else (S if -d >= S else -d)
    s_hi = 0 if d >= N else (S if N - d >= S else N - d)
    h, r = R >> 1, R & 1
    inc = (t["f0"] + R * d + ((R - h) if d & 1 else h)) & M64
    De, Do = R + r, R - r
    D0, D1 = (Do, De) if d & 1 else (De, Do)
    ph = phase_general(t, n)
    out = []
    for s in range(S):
        out.append(ph)
        if s + 1 < S:
            ph = (ph + (t["f0"] if s < s_lo else (inc if s < s_hi else t["f1"]))) & M64
            inc = (inc + (D1 if s & 1 else D0)) & M64
    return out


def split_m(dF):
    m = (dF >> 16) & M64
    return m, m & M32, s32(m >> 32)


def smooth_step16_in_window(t, tile0, j):
    H, dF, f0 = t["H"], t["coef"], t["f0"]
    d0 = tile0 - t["a"] + j
    hv = [int(H[d0 + s]) for s in range(S)]
    m, m_lo, m_hi = split_m(dF)
    ph = (t["p0"] + f0 * tile0 + f0 * j + m * hv[0]) & M64
    out = []
    for s in range(S):
        out.append(ph)
        if s + 1 < S:
            dh = hv[s + 1] - hv[s]
            lo = (m_lo * dh + f0) & M64
            hi = ((lo >> 32) + mul24(m_hi, dh)) & M32
            ph = (ph + ((hi << 32) | (lo & M32))) & M64
    return out


def clamp_table(t, d):
    return int(t["H"][0 if d < 0 else (d if d < t["N"] else t["N"])])


def smooth_step16_edge(t, n):
    dF, f0, f1, N = t["coef"], t["f0"], t["f1"], t["N"]
    d0 = n - t["a"]
    s_hi = 0 if d0 >= N else (S if N - d0 >= S else N - d0)
    hv = [clamp_table(t, d0 + s) for s in range(S)]
    m, m_lo, m_hi = split_m(dF)
    line = t["p0"] + f0 * n if d0 < N else t["p0"] + f0 * (t["a"] + N) + f1 * (d0 - N)
    ph = (line + m * hv[0]) & M64
    out = []
    for s in range(S):
        out.append(ph)
        if s + 1 < S:
            dh = hv[s + 1] - hv[s]
            lo = (m_lo * dh + (f0 if s < s_hi else f1)) & M64
            hi = ((lo >> 32) + mul24(m_hi, dh)) & M32
            ph = (ph + ((hi << 32) | (lo & M32))) & M64
    return out


def any_df_high_words(t, hv, ps0, steps):
    """High halves of P + m dH_s + floor((A_lo + r dH_s) / 2^16) along the
    lane (the any-dF loops): ps0 is the line part at the lane's first sample,
    steps[s] what it moves by after sample s."""
    dF = t["coef"]
    m, m_lo, m_hi = split_m(dF)
    rr = dF & 0xFFFF
    A = rr * hv[0]
    assert A < (1 << 63)
    ps = (ps0 + m * hv[0] + (A >> 16)) & M64
    a_lo = A & 0xFFFF
    out, carries = [], 0
    for s in range(S):
        dH = hv[s] - hv[0]
        assert 0 <= dH < (1 << 23)
        lo = (m_lo * dH + ps) & M64
        tt = rr * dH + a_lo
        assert tt < (1 << 40)
        c = (tt >> 16) & M32
        cy0 = ((lo & M32) + c) >> 32
        carries += cy0
        whi = ((lo >> 32) + mul24(m_hi, dH) + cy0) & M32
        out.append(whi)
        ps = (ps + steps[s]) & M64
    return out, carries


def smooth_anydf_in_window(t, tile0, j):
    d0 = tile0 - t["a"] + j
    hv = [int(t["H"][d0 + s]) for s in range(S)]
    f0 = t["f0"]
    return any_df_high_words(t, hv, t["p0"] + f0 * tile0 + f0 * j, [f0] * S)


def smooth_anydf_edge(t, n):
    f0, f1, N = t["f0"], t["f1"], t["N"]
    d0 = n - t["a"]
    s_hi = 0 if d0 >= N else (S if N - d0 >= S else N - d0)
    hv = [clamp_table(t, d0 + s) for s in range(S)]
    line = t["p0"] + f0 * n if d0 < N else t["p0"] + f0 * (t["a"] + N) + f1 * (d0 - N)
    return any_df_high_words(t, hv, line, [f0 if s < s_hi else f1 for s in range(S)])


# --------------------------------------------------------------- random tones

_TABLES = {}


def table(shape, N):
    key = (shape, N)
    if key not in _TABLES:
        _TABLES[key] = OW.ramp_table(shape, N)
    return _TABLES[key]


def random_tone(r, shape, N, free=True, df_max=1 << 58, p0_shift=0):
    """A tone whose words the oracle's Ramp defines; device words carry +2^40."""
    p0 = (int(r.integers(0, 1 << 63)) * 2 + int(r.integers(0, 2)) + p0_shift) & M64
    f0 = int(r.integers(1 << 60, 1 << 63))
    dF = int(r.integers(-df_max, df_max))
    if not free:
        dF &= ~0xFFFF                           # a multiple of 2^16 (bin frequencies)
    f1 = f0 + dF
    a = int(r.integers(1 << 20, 1 << 24))
    return make_tone(shape, N, p0, f0, f1, a)


def make_tone(shape, N, p0, f0, f1, a):
    H = table(shape, N) if shape != OW.RAMP_LINEAR else None
    ramp = OW.Ramp(a, N, shape, p0, f0, f1, H)
    tw = OW.ToneWords(p0, f0, 1.0)
    tw.ramps.append(ramp)
    t = {"p0": (p0 + BIAS) & M64, "f0": f0, "p1": (ramp.p_after + BIAS) & M64, "f1": f1, "a": a, "N": N,
         "coef": ramp.coef, "shape": shape, "H": H}
    return t, tw


def exact(tw, n):
    return tw.phase_at(n)


SMOOTH = [OW.RAMP_COSINE, OW.RAMP_MINJERK]
LENS = [1, 2, 15, 16, 17, 33, 1000, 4097]


def test_smooth_tables_step_below_2_19():
    """The kernels' smooth paths assume never-decreasing tables with steps
    below 2^19 (so a lane's rise stays below 2^23): true of both shapes."""
    for shape in SMOOTH:
        for N in LENS + [70000]:
            d = np.diff(table(shape, N).astype(np.int64))
            assert d.min() >= 0 and d.max() < (1 << 19), (shape, N, d.max())


@pytest.mark.parametrize("shape", [OW.RAMP_LINEAR] + SMOOTH)
def test_closed_form_at_a_lane_start(shape):
    r = np.random.default_rng(1 + shape)
    for _ in range(300):
        N = int(r.choice(LENS))
        t, tw = random_tone(r, shape, N)
        for n in t["a"] + r.integers(-40, N + 40, 4):
            assert (phase_general(t, int(n)) - BIAS) & M64 == exact(tw, int(n))


def test_linear_in_window_steps():
    r = np.random.default_rng(2)
    for _ in range(400):
        N = int(r.choice([1100, 4097, 20000]))
        t, tw = random_tone(r, OW.RAMP_LINEAR, N)
        tile0 = t["a"] + int(r.integers(0, N - 1024 + 1))
        j = 16 * int(r.integers(0, 64))
        got = linear_in_window(t, tile0, j)
        want = [exact(tw, tile0 + j + s) for s in range(S)]
        assert [(g - BIAS) & M64 for g in got] == want


def test_linear_edge_steps():
    r = np.random.default_rng(3)
    for _ in range(800):
        N = int(r.choice(LENS))
        t, tw = random_tone(r, OW.RAMP_LINEAR, N)
        n = t["a"] + int(r.integers(-20, N + 20))
        got = linear_edge(t, n)
        want = [exact(tw, n + s) for s in range(S)]
        assert [(g - BIAS) & M64 for g in got] == want


@pytest.mark.parametrize("shape", SMOOTH)
def test_smooth_step16_rules(shape):
    """dF a multiple of 2^16: full words, in the window and at its edges."""
    r = np.random.default_rng(4 + shape)
    for _ in range(300):
        N = int(r.choice(LENS))
        t, tw = random_tone(r, shape, N, free=False)
        n = t["a"] + int(r.integers(-20, N + 20))
        got = smooth_step16_edge(t, n)
        assert [(g - BIAS) & M64 for g in got] == [exact(tw, n + s) for s in range(S)]
        if N >= 1100:
            tile0 = t["a"] + int(r.integers(0, N - 1024 + 1))
            j = 16 * int(r.integers(0, 64))
            got = smooth_step16_in_window(t, tile0, j)
            assert [(g - BIAS) & M64 for g in got] == [exact(tw, tile0 + j + s) for s in range(S)]


def near_wrap(t, tw, r, n):
    """The same tone with p0 moved so that at the lane's last sample n + 15 the
    exact word's low half lies below c = floor((A_lo + r dH_15) / 2^16), the
    term the any-dF rule adds to the low half there (c does not depend on p0):
    the low half then wraps, and the rule must carry into the high half."""
    d0 = n - t["a"]
    hv = [clamp_table(t, d0 + s) for s in range(S)]
    rr = t["coef"] & 0xFFFF
    c = ((rr * hv[0]) % (1 << 16) + rr * (hv[S - 1] - hv[0])) >> 16
    if c == 0:
        return t, tw
    lo = (exact(tw, n + S - 1) + BIAS) & M32
    shift = (int(r.integers(0, c)) - lo) & M32
    return make_tone(t["shape"], t["N"], (t["p0"] - BIAS + shift) & M64, t["f0"], t["f1"], t["a"])


@pytest.mark.parametrize("shape", SMOOTH)
def test_smooth_any_df_rules(shape):
    """Any dF (free frequencies): the high halves the sine reads, in the window
    and at its edges, including the largest |dF| of a 5 MHz step at 280 MS/s;
    half the lanes start just below a wrap of the low half, so the carry into
    the high half is taken (and counted) many times."""
    r = np.random.default_rng(6 + shape)
    carries = 0
    for i in range(400):
        N = int(r.choice(LENS))
        t, tw = random_tone(r, shape, N, df_max=(1 << 58) if i % 2 else (1 << 40))
        n = t["a"] + int(r.integers(-20, N + 20))
        if i % 4 < 2:
            t, tw = near_wrap(t, tw, r, n)
        got, c = smooth_anydf_edge(t, n)
        carries += c
        assert got == [((exact(tw, n + s) + BIAS) & M64) >> 32 for s in range(S)]
        if N >= 1100:
            tile0 = t["a"] + int(r.integers(0, N - 1024 + 1))
            j = 16 * int(r.integers(0, 64))
            if i % 4 < 2:
                t, tw = near_wrap(t, tw, r, tile0 + j)
            got, c = smooth_anydf_in_window(t, tile0, j)
            carries += c
            assert got == [((exact(tw, tile0 + j + s) + BIAS) & M64) >> 32 for s in range(S)]
    assert carries > 50


def test_a_planted_carry_mistake_fails():
    """Control: the any-dF rule with the low half's carry dropped (the mistake
    the rule guards against) gives wrong high words on lanes near a wrap."""
    r = np.random.default_rng(9)
    bad = 0
    for _ in range(100):
        t, tw = random_tone(r, OW.RAMP_COSINE, 4097)
        tile0 = t["a"] + int(r.integers(0, 4097 - 1024 + 1))
        t, tw = near_wrap(t, tw, r, tile0)
        d0 = tile0 - t["a"]
        hv = [int(t["H"][d0 + s]) for s in range(S)]
        dF = t["coef"]
        m, m_lo, m_hi = split_m(dF)
        rr = dF & 0xFFFF
        A = rr * hv[0]
        ps = (t["p0"] + t["f0"] * tile0 + m * hv[0] + (A >> 16)) & M64
        for s in range(S):
            dH = hv[s] - hv[0]
            lo = (m_lo * dH + ps) & M64
            whi = ((lo >> 32) + mul24(m_hi, dH)) & M32            # carry of lo + c left out
            bad += whi != ((exact(tw, tile0 + s) + BIAS) & M64) >> 32
            ps = (ps + t["f0"]) & M64
    assert bad > 0
