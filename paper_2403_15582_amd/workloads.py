"""Seeded synthetic inputs: tone lists, retune schedules and job streams.

This module only draws random numbers and lays them out as ``awg_tone``
records; it holds none of the synthesis arithmetic (no words, no sines, no
sums). Tests, the benchmark and the smoke check all take their inputs from
here, so the library and the oracle see identical tone lists.

The paper measures on no public dataset; these recipes reproduce the shapes of
its workloads (Performance section: defect-free multi-tone arrays, rearrangement
chirps, large arrays chirped in groups, a 280 MS/s sample clock, 2**20-sample
chunks) with numpy's PCG64 generator.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .abi_types import (TONE_DTYPE, RAMP_NONE, RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK)

FS_280 = 280e6
CHUNK = 1 << 20
RAMP_35MS = 9_800_000          # 35 ms at 280 MS/s
RAMP_1MS = 280_000            # 1 ms at 280 MS/s


@dataclass
class Workload:
    """Inputs of one synthesis problem plus the sample range it covers."""
    name: str
    fs_hz: float
    gain_lsb: float            # 0 = default (32767 / sum|A|)
    period_log2: int           # 0 = no bin snapping
    tones: np.ndarray          # TONE_DTYPE records
    n0: int = 0
    count: int = 0
    chunk: int = CHUNK
    retunes: list = field(default_factory=list)   # (k, ramp_start, ramp_len, shape, f_end_hz)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def schroeder_turns(K):
    """Schroeder's low-crest-factor phases for K equal tones, in turns.

    theta_k = -pi k (k-1) / K for rank k = 1..K (Schroeder 1970, cited by the
    paper for crest-factor control); in turns that is -k(k-1)/(2K) mod 1, taken
    here from exact integers.
    """
    k = np.arange(1, K + 1, dtype=np.int64)
    num = (-(k * (k - 1))) % (2 * K)
    return num.astype(np.float64) / float(2 * K)


def bins_to_hz(bins, fs_hz, period_log2):
    """Centre frequency of each bin: b * fs / L (float64)."""
    return np.asarray(bins, dtype=np.float64) * (fs_hz / float(1 << period_log2))


def static_tones(f_hz, amps, phases):
    t = np.zeros(len(f_hz), dtype=TONE_DTYPE)
    t["f_start_hz"] = f_hz
    t["f_end_hz"] = f_hz
    t["amplitude"] = amps
    t["phase_turns"] = phases
    t["ramp"] = RAMP_NONE
    return t


def static_100tone_chunk(seed=1):
    """100 static tones, bins of L=2**20 in 75-125 MHz, A=1/100, one 2**20 chunk."""
    r = _rng(seed)
    lo, hi = 280869, 468114
    bins = np.sort(r.choice(np.arange(lo, hi + 1), size=100, replace=False))
    tones = static_tones(bins_to_hz(bins, FS_280, 20), np.full(100, 0.01), r.random(100))
    return Workload("static-100tone-2^20", FS_280, 32767.0, 20, tones, 0, CHUNK)


def static_period(seed=2, K=1000):
    """Static periodic buffer: K tones, bins of L=2**24 in 60-140 MHz (Nyquist bin
    excluded), A ~ U[0.5, 1], Schroeder phases by frequency rank, one period."""
    r = _rng(seed)
    lo, hi = 3595118, 8388607
    bins = np.sort(r.choice(np.arange(lo, hi + 1), size=K, replace=False))
    amps = r.uniform(0.5, 1.0, K)
    tones = static_tones(bins_to_hz(bins, FS_280, 24), amps, schroeder_turns(K))
    return Workload("static-%dtone-2^24" % K, FS_280, 0.0, 24, tones, 0, 1 << 24)


def _chirp_ends(r, n, lo, hi, max_step):
    f0 = r.uniform(lo, hi, n)
    f1 = f0 + r.uniform(-max_step, max_step, n)
    bad = (f1 < lo) | (f1 > hi)
    while bad.any():
        f1[bad] = f0[bad] + r.uniform(-max_step, max_step, int(bad.sum()))
        bad = (f1 < lo) | (f1 > hi)
    return f0, f1


def chirp_35ms(seed=3, shape="linear", K=1000, ramp_len=RAMP_35MS, n_chunks=10):
    """K tones chirped from f_start ~ U[75,125] MHz by U[-5,5] MHz over 35 ms.

    shape: 'linear', 'cosine', 'minjerk', or 'mixed' (seeded coin per tone between
    linear and cosine). Ramps start at sample 0; tones hold f_end afterwards.
    Frequencies snap to bins of L=2**20 so the held tones are periodic.
    """
    r = _rng(seed)
    f0, f1 = _chirp_ends(r, K, 75e6, 125e6, 5e6)
    amps = r.uniform(0.5, 1.0, K)
    phases = r.random(K)
    coin = r.random(K) < 0.5
    t = static_tones(f0, amps, phases)
    t["f_end_hz"] = f1
    t["ramp_start"] = 0
    t["ramp_len"] = ramp_len
    shapes = {"linear": RAMP_LINEAR, "cosine": RAMP_COSINE, "minjerk": RAMP_MINJERK}
    if shape == "mixed":
        t["ramp"] = np.where(coin, RAMP_LINEAR, RAMP_COSINE)
    else:
        t["ramp"] = shapes[shape]
    return Workload("chirp-%dtone-%s-35ms" % (K, shape), FS_280, 0.0, 20, t, 0,
                    n_chunks * CHUNK)


def array_group_chirps(seed=4, K=5000, seconds=1.0, group=100, ramp_len=RAMP_1MS):
    """Large array: K tones on an even grid over 60-140 MHz, A ~ U[0.5,1],
    Schroeder phases; groups of ``group`` consecutive tones (cycling) chirp one
    after another, each by a seeded 0-2 MHz offset of seeded sign over 1 ms
    (reflected back into the band), linear. The first group starts at 0.
    Each entry of ``retunes`` is one chirp: (tone, start, length, shape, f_end).
    """
    r = _rng(seed)
    f = 60e6 + (np.arange(K) + 0.5) * (80e6 / K)
    amps = r.uniform(0.5, 1.0, K)
    tones = static_tones(f, amps, schroeder_turns(K))
    total = int(round(seconds * FS_280))
    n_groups_total = (total + ramp_len - 1) // ramp_len
    cur = f.copy()
    retunes = []
    for j in range(n_groups_total):
        start = j * ramp_len
        ks = (np.arange(group) + j * group) % K
        off = r.uniform(0.0, 2e6, group) * np.where(r.random(group) < 0.5, -1.0, 1.0)
        tgt = cur[ks] + off
        # reflect into the band; the top stays clear of the Nyquist bin
        tgt = np.where(tgt < 60e6, 2 * 60e6 - tgt, tgt)
        tgt = np.where(tgt > 139.99e6, 2 * 139.99e6 - tgt, tgt)
        for kk, ft in zip(ks.tolist(), tgt.tolist()):
            retunes.append((kk, start, ramp_len, RAMP_LINEAR, ft))
        cur[ks] = tgt
    n_chunks = (total + CHUNK - 1) // CHUNK
    return Workload("array-%dtone-groups%d" % (K, group), FS_280, 0.0, 20, tones, 0,
                    n_chunks * CHUNK, CHUNK, retunes)


@dataclass
class Job:
    """One rearrangement request of the serving workload."""
    job_id: int
    arrival_s: float
    fs_hz: float
    n_samples: int
    tones: np.ndarray
    gain_lsb: float = 0.0      # 0 = default (32767 / sum|A|)


def poisson_jobs(seed=5, rate_hz=2000.0, seconds=2.0, kmin=50, kmax=2000,
            dmin_ms=0.1, dmax_ms=35.0, max_jobs=None):
    """Poisson stream of chirp jobs: K ~ round(exp U[ln kmin, ln kmax]), duration
    ~ U[dmin, dmax] ms, fs 50 or 280 MS/s (fair coin), per-tone linear chirps over
    the whole job in the band [75, 125] * fs/280 MHz with |df| <= 5 * fs/280 MHz.
    """
    r = _rng(seed)
    jobs = []
    t = 0.0
    while True:
        t += r.exponential(1.0 / rate_hz)
        if t >= seconds or (max_jobs is not None and len(jobs) >= max_jobs):
            break
        K = int(round(math.exp(r.uniform(math.log(kmin), math.log(kmax)))))
        dur = r.uniform(dmin_ms, dmax_ms) * 1e-3
        fs = 50e6 if r.random() < 0.5 else FS_280
        scale = fs / FS_280
        f0, f1 = _chirp_ends(r, K, 75e6 * scale, 125e6 * scale, 5e6 * scale)
        n = max(1, int(round(dur * fs)))
        tn = static_tones(f0, r.uniform(0.5, 1.0, K), r.random(K))
        tn["f_end_hz"] = f1
        tn["ramp"] = RAMP_LINEAR
        tn["ramp_start"] = 0
        tn["ramp_len"] = n
        jobs.append(Job(len(jobs), t, fs, n, tn))
    return jobs


def row_edges(seed=12, n0=3 * CHUNK + 12345, rows=70, tail=37, K_static=192, per=6, fs_hz=FS_280):
    """Ramped tones whose windows sit on the edges of the 1024-sample rows that
    start at n0 (a window opening on a row's last sample or the next one,
    closing on a row's first sample or the one before, inside one row, before
    n0, past the range, over the whole range, entirely before / after it), each
    edge case carried by ``per`` tones of cycling shapes, plus ``K_static``
    static tones. The range is n0 .. n0 + 1024 rows + tail (ragged)."""
    R = 1024
    count = rows * R + tail
    specs = [
        (n0 + 5 * R + R - 1, 10 * R),            # opens on row 5's last sample
        (n0 + 6 * R, 10 * R - 1),                # opens on row 6's first, closes on row 16's first - 1
        (n0 + 20 * R - 1, 3 * R + 1),            # closes on row 23's first sample
        (n0 + 30 * R + 100, 500),                # inside one row
        (n0 - 5000, 8 * R),                      # opened before the range
        (n0 + count - 3000, 40000),              # still open after the range
        (n0 - 10, count + 100),                  # covers the whole range
        (n0 + 2 * R, count - 3 * R),             # few line rows: direct only
        (n0 - 30000, 20000),                     # closed before the range
        (n0 + count + 10, 5000),                 # opens after the range
        (n0 + 40 * R + 1, 1),                    # one-sample window
    ]
    r = _rng(seed)
    K = K_static + per * len(specs)
    f0, f1 = _chirp_ends(r, K, 0.05 * fs_hz, 0.45 * fs_hz, 0.02 * fs_hz)
    t = static_tones(f0, r.uniform(0.2, 1.0, K), r.random(K))
    shapes = [RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK]
    for i, (a, n) in enumerate(specs):
        for j in range(per):
            k = K_static + i * per + j
            t[k]["f_end_hz"] = f1[k]
            t[k]["ramp"] = shapes[(i + j) % 3]
            t[k]["ramp_start"] = a
            t[k]["ramp_len"] = n
    # interleave the ramped tones among the static ones (device order is sorted anyway)
    t = t[r.permutation(K)]
    return Workload("row-edges", fs_hz, 0.0, 0, t, n0, count)


def rearrangement(seed=14, K=100, off_frac=0.5, fs_hz=FS_280, f_lo=75e6, f_hi=125e6,
                  t_off=20000, off_len=2800, t_move=30000, move_len=280000, tail=60000):
    """The rearrangement of the paper's dynamic-pathway demonstration (a
    stochastically loaded array made defect-free), in the rf domain: K tones on
    an even grid over [f_lo, f_hi] with Schroeder phases; a seeded off_frac of
    them are switched off (amplitude ramped to 0, minimum-jerk profile) over
    [t_off, t_off + off_len]; the remaining tones are then chirped (minimum
    jerk) over [t_move, t_move + move_len] onto the first grid positions, in
    order. ``amp_events`` holds (tone, ramp, start, length, amplitude_end),
    ``retunes`` (tone, start, length, shape, f_end_hz)."""
    r = _rng(seed)
    f = f_lo + (np.arange(K) + 0.5) * ((f_hi - f_lo) / K)
    tones = static_tones(f, np.full(K, 1.0), schroeder_turns(K))
    off = np.sort(r.choice(K, int(round(off_frac * K)), replace=False))
    keep = np.setdiff1d(np.arange(K), off)
    amp_events = [(int(k), RAMP_MINJERK, t_off, off_len, 0.0) for k in off]
    retunes = [(int(k), t_move, move_len, RAMP_MINJERK, float(f[i])) for i, k in enumerate(keep)]
    w = Workload("rearrange-%dtone" % K, fs_hz, 0.0, 20, tones, 0, t_move + move_len + tail,
                 retunes=retunes)
    w.amp_events = amp_events
    return w


def edge_blocks(seed=15, group=8, fs_hz=FS_280, period_log2=20):
    """Groups of ``group`` tones sharing one window and shape (so the kernels
    take a group's regime once per 1024-sample tile), with window edges at
    chosen offsets inside tiles (first sample, second, just before and after a
    lane's 16 samples, the last sample) and windows of 1 sample up to several
    tiles; each (offset, length) pair is carried by one linear, one
    raised-cosine and one minimum-jerk group. With bin frequencies (L = 2^20,
    the default) every frequency step is a multiple of 2^16 of the word;
    period_log2 = 0 gives free frequencies (any step)."""
    offsets = [0, 1, 7, 15, 16, 17, 500, 1023]
    lens = [1, 2, 5, 15, 16, 17, 1000, 3000]
    specs = [(1024 * (2 + 3 * i) + off, n) for i, (off, n) in enumerate(zip(offsets, lens))]
    shapes = [RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK]
    r = _rng(seed)
    K = len(specs) * len(shapes) * group
    f0, f1 = _chirp_ends(r, K, 0.05 * fs_hz, 0.45 * fs_hz, 0.02 * fs_hz)
    t = static_tones(f0, r.uniform(0.2, 1.0, K), r.random(K))
    t["f_end_hz"] = f1
    k = 0
    for a, n in specs:
        for sh in shapes:
            for _ in range(group):
                t[k]["ramp"] = sh
                t[k]["ramp_start"] = a
                t[k]["ramp_len"] = n
                k += 1
    return Workload("edge-blocks" if period_log2 else "edge-blocks-free", fs_hz, 0.0, period_log2, t, 0,
                    1024 * (2 + 3 * len(specs)) + 333)


def small_mixed(seed=11, K=24, fs_hz=FS_280, n_total=5000, period_log2=0):
    """Small tone set covering every ramp shape and regime (pre / in / post
    window, windows straddling tile edges, rising and falling chirps), for
    parity tests the oracle finishes in well under a second."""
    r = _rng(seed)
    f0, f1 = _chirp_ends(r, K, 0.05 * fs_hz, 0.45 * fs_hz, 0.02 * fs_hz)
    t = static_tones(f0, r.uniform(0.2, 1.0, K), r.random(K))
    t["f_end_hz"] = f1
    shapes = [RAMP_NONE, RAMP_LINEAR, RAMP_COSINE, RAMP_MINJERK]
    t["ramp"] = [shapes[i % 4] for i in range(K)]
    t["ramp_start"] = r.integers(0, n_total // 2, K)
    t["ramp_len"] = r.integers(1, n_total // 2, K)
    return Workload("small-mixed", fs_hz, 0.0, period_log2, t, 0, n_total)
