"""GPU parity of amplitude ramps (the time-dependent amplitude a_j[i] of Eq. (5)):
tones faded in and out with every profile, windows on tile edges and inside one
tile, chained ramps, combined with chirps; and the paper's rearrangement (half
the tones switched off, the rest chirped onto a defect-free grid) streamed,
with the direct method and with the hybrid path. Every sample is compared with
the oracle."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words, csynth

from gpu_common import need_gpu, say, to_np, compare

pytestmark = pytest.mark.gpu

LIN, COS, MJ = awg.RAMP_LINEAR, awg.RAMP_COSINE, awg.RAMP_MINJERK
GAIN = 700.0


def _faded_plan():
    """small_mixed tones (every chirp shape) with amplitude ramps on most of them."""
    w = W.small_mixed(seed=21, K=24, n_total=20000)
    t = w.tones.copy()
    t["amplitude"][3] = 0.0                        # planned silent, switched on below
    first = [  # (tone, profile, start, length, amplitude_end)
        (0, LIN, 0, 5000, 0.0),                    # fade out from the first sample
        (1, COS, 1023, 2, 0.2),                    # window across a tile edge
        (2, MJ, 2100, 300, 0.0),                   # inside one tile
        (3, MJ, 4096, 4096, 0.9),                  # switched on, window on tile edges
        (4, LIN, 7000, 1, 1.0),                    # one-sample window (a step)
        (5, COS, 100, 19000, 0.05),                # long window over the whole range
        (6, LIN, 30000, 100, 0.0),                 # opens after the range
        (7, MJ, 1500, 2500, 1.2),
        (9, COS, 8000, 3000, 0.0),
        (10, LIN, 9000, 7000, 0.4),
        (12, MJ, 12345, 678, 0.0),
        (13, LIN, 0, 1, 0.3),
    ]
    second = [(0, MJ, 6000, 4000, 0.8), (2, LIN, 2400, 10, 0.5), (9, MJ, 11000, 3000, 0.6),
              (7, COS, 4000, 12000, 0.0)]
    return w, t, first, second


def _oracle(w, t, events):
    op = words.Plan(w.fs_hz, GAIN, w.period_log2, t, build_tables=True)
    for k, sh, b, m, amp in events:
        op.add_amp_ramp(k, b, m, sh, amp)
    return op


@pytest.mark.parametrize("method", [awg.AWG_F_METHOD_DIRECT, awg.AWG_F_METHOD_MFMA_F16X3])
def test_amplitude_ramps_every_sample(method):
    """One ramp per tone, every sample of the range against the oracle."""
    torch = need_gpu()
    w, t, first, _ = _faded_plan()
    p = awg.Plan(t, w.fs_hz, GAIN, w.period_log2, method)
    p.amplitude(first)
    count = w.count if method == awg.AWG_F_METHOD_DIRECT else 1 << 16
    say("amplitude ramps method=%d: %d events, 0..%d" % (method, len(first), count))
    q = to_np(p.synth_chirp(0, count))
    y = to_np(p.synth_f32(0, count, method=method))
    torch.cuda.synchronize()
    qo, yo = csynth.synth(_oracle(w, t, first), 0, count)
    compare(q, y, qo, yo, "amplitude ramps method=%d" % method)
    if method == awg.AWG_F_METHOD_DIRECT:
        # chunked == one-shot, bit for bit
        parts = [p.synth_chirp(n0, c) for n0, c in [(0, 777), (777, 4096), (4873, 15127)]]
        torch.cuda.synchronize()
        assert np.array_equal(np.concatenate([to_np(x) for x in parts]), q)


def test_chained_amplitude_ramps_streamed():
    """Second ramps of some tones, each applied when the stream reaches its start
    (the device keeps one amplitude window per tone, like retuning)."""
    torch = need_gpu()
    w, t, first, second = _faded_plan()
    p = awg.Plan(t, w.fs_hz, GAIN, w.period_log2)
    p.amplitude(first)
    parts = []
    for ev in sorted(second, key=lambda e: e[2]):
        parts.append(p.stream_next(ev[2] - p.tell())[1])
        p.amplitude([ev])
    parts.append(p.stream_next(w.count - p.tell())[1])
    torch.cuda.synchronize()
    q = np.concatenate([to_np(x) for x in parts])
    qo, yo = csynth.synth(_oracle(w, t, first + second), 0, w.count)
    compare(q, None, qo, yo, "chained amplitude ramps, streamed")


def test_switched_off_tones_leave_the_rest():
    """After a tone's fade-out ends the samples equal those of the plan without it."""
    torch = need_gpu()
    w, t, _, _ = _faded_plan()
    p = awg.Plan(t, w.fs_hz, GAIN, w.period_log2)
    p.amplitude([(k, MJ, 100 + 37 * k, 500, 0.0) for k in (2, 5, 11)])
    keep = np.setdiff1d(np.arange(len(t)), [2, 5, 11])
    p2 = awg.Plan(t[keep], w.fs_hz, GAIN, w.period_log2)
    a = to_np(p.synth_f32(1000, 5000))
    b = to_np(p2.synth_f32(1000, 5000))
    torch.cuda.synchronize()
    # different tone lists sum in different orders: equal to FP32 rounding
    assert np.max(np.abs(a - b)) < 0.01


@pytest.mark.parametrize("method", [awg.AWG_F_METHOD_DIRECT, awg.AWG_F_METHOD_MFMA_F16X3])
def test_rearrangement_stream_against_oracle(method):
    torch = need_gpu()
    w = W.rearrangement()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method)
    p.amplitude(w.amp_events)
    p.retune([(k, sh, a, n, f) for k, a, n, sh, f in w.retunes])
    say("rearrangement method=%d: %d tones, %d off, %d chirped, %d samples"
        % (method, len(w.tones), len(w.amp_events), len(w.retunes), w.count))
    chunk = 1 << 16
    parts = []
    while p.tell() < w.count:
        parts.append(p.stream_next(min(chunk, w.count - p.tell()))[1])
    y = to_np(p.synth_f32(0, w.count, method=method)) if method == awg.AWG_F_METHOD_DIRECT else None
    torch.cuda.synchronize()
    q = np.concatenate([to_np(x) for x in parts])
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    for k, sh, b, m, amp in w.amp_events:
        op.add_amp_ramp(k, b, m, sh, amp)
    for k, a, n, sh, f in w.retunes:
        op.add_ramp(k, a, n, sh, f)
    ns = np.arange(w.count, dtype=np.int64)
    csynth.sparse_tables(op, ns)
    qo, yo = csynth.synth(op, 0, w.count)
    compare(q, y, qo, yo, "rearrangement method=%d" % method)
