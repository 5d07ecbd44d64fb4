"""GPU parity of the matrix-core (angle addition) static path against the oracle.

FP16 and BF16 hi/lo x3 must both meet the int16 bar (<= 1 LSB) and the FP32-sum
bar on the unquantised output (<= 0.25 LSB), at the default gain and at the gain
that puts the Schroeder buffer at 90% of full scale.
"""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words, csynth

from gpu_common import need_gpu, say, to_np, compare

pytestmark = pytest.mark.gpu

F16 = awg.AWG_F_METHOD_MFMA_F16X3
BF16 = awg.AWG_F_METHOD_MFMA_BF16X3


def _pts(rng, n0, count, extra=()):
    ns = set(rng.integers(n0, n0 + count, 3000).tolist())
    ns |= set(range(n0, n0 + 300)) | set(range(n0 + count - 300, n0 + count))
    ns |= set(int(e) for e in extra)
    return np.array(sorted(n for n in ns if n0 <= n < n0 + count), dtype=np.int64)


@pytest.fixture(scope="module")
def static_period_oracle():
    """The oracle over the whole 2^24-sample period of the 1000-tone buffer
    (1.7e10 tone-samples of FP64 direct sum on the host's cores)."""
    w = W.static_period()
    say("oracle: static period 1000 tones x 2^24 samples, every sample")
    qo, yo = csynth.synth(words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones), 0, w.count)
    return w, qo, yo


@pytest.mark.parametrize("method", [BF16, F16, awg.AWG_F_METHOD_DIRECT])
def test_static_period_every_sample(static_period_oracle, method):
    """The benchmark's static buffer, one call over the whole period, compared
    with the oracle element by element (codes and unquantised sum)."""
    torch = need_gpu()
    w, qo, yo = static_period_oracle
    lp = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method)
    say("static-period full 2^24 x 1000 method=%d, every sample" % method)
    q = to_np(lp.synth_static(0, w.count))
    y = to_np(lp.synth_f32(0, w.count, method=method))
    torch.cuda.synchronize()
    compare(q, y, qo, yo, "static-period method=%d (all %d samples)" % (method, w.count))
    dy = np.abs(y.astype(np.float64) - yo)
    say("static-period method=%d unquantised rms|dy| = %.5f LSB" % (method, np.sqrt(np.mean(dy ** 2))))
    lp.close()


@pytest.mark.parametrize("n0,count", [(12345, (1 << 20) + 777), (3, 1 << 16), (2 ** 41 + 9, 300000),
                                      (0, 5000), (5, (1 << 24) + 1234)])
def test_mfma_ragged_ranges(n0, count):
    torch = need_gpu()
    w = W.static_period(K=333)
    lp = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, F16)
    say("mfma ragged n0=%d count=%d K=333" % (n0, count))
    q = to_np(lp.synth_static(n0, count))
    y = to_np(lp.synth_f32(n0, count, method=F16))
    torch.cuda.synchronize()
    ns = _pts(np.random.default_rng(52), n0, count)
    qo, yo = csynth.synth_at(words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones), ns)
    compare(q[ns - n0], y[ns - n0], qo, yo, "mfma ragged n0=%d count=%d" % (n0, count))


def test_mfma_peak_gain():
    """Gain raised so the buffer peaks near 90% of full scale (Schroeder phases)."""
    torch = need_gpu()
    w = W.static_period()
    op1 = words.Plan(w.fs_hz, 1.0, w.period_log2, w.tones)
    _, y1 = csynth.synth(op1, 0, 1 << 16)
    gain = 0.9 * 32767.0 / float(np.max(np.abs(y1)))
    say("peak gain %.2f LSB per unit amplitude" % gain)
    ns = _pts(np.random.default_rng(53), 0, w.count)
    qo, yo = csynth.synth_at(words.Plan(w.fs_hz, gain, w.period_log2, w.tones), ns)
    for method in (F16, BF16, awg.AWG_F_METHOD_DIRECT):
        lp = awg.Plan(w.tones, w.fs_hz, gain, w.period_log2, method)
        q = to_np(lp.synth_static(0, w.count))
        y = to_np(lp.synth_f32(0, w.count, method=method))
        torch.cuda.synchronize()
        dq = np.abs(q[ns].astype(np.int32) - qo.astype(np.int32))
        dy = np.abs(y[ns].astype(np.float64) - yo)
        say("peak gain method=%d: max|dq|=%d max|dy|=%.4f rms|dy|=%.5f LSB"
            % (method, dq.max(), dy.max(), np.sqrt(np.mean(dy ** 2))))
        assert dq.max() <= 1 and dy.max() <= 0.25, method


def test_mfma_equals_direct_within_one_lsb_everywhere():
    torch = need_gpu()
    w = W.static_100tone_chunk()
    a = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, F16)
    b = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, awg.AWG_F_METHOD_DIRECT)
    qa = to_np(a.synth_static(0, w.count))
    qb = to_np(b.synth_static(0, w.count))
    torch.cuda.synchronize()
    qo, _ = csynth.synth(words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones), 0, w.count)
    compare(qa, None, qo, None, "static-100tone-chunk mfma vs oracle (all samples)")
    assert np.max(np.abs(qa.astype(np.int32) - qb.astype(np.int32))) <= 2


@pytest.mark.parametrize("ramped", [False, True])
def test_two_streams_on_one_plan(ramped):
    """Synthesis calls on one plan from two streams at once (the matrix-core
    workspace is shared and ordered between them) equal the same calls run one
    after the other."""
    torch = need_gpu()
    w = W.array_group_chirps(K=600, seconds=0.01) if ramped else W.static_100tone_chunk()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16)
    if ramped:
        p.retune([(k, sh, a, n, f) for k, a, n, sh, f in sorted(w.retunes, key=lambda e: e[1])[:100]])
    calls = [(0, 1 << 20), (12345, 3 << 18), (1 << 20, 1 << 20), (777, 1 << 19)]
    say("two streams, ramped=%s" % ramped)
    ref = [to_np(p.synth_chirp(n0, c)) for n0, c in calls]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [torch.empty(c, dtype=torch.int16, device="cuda") for _, c in calls]
    torch.cuda.synchronize()
    for rep in range(3):
        for i, (n0, c) in enumerate(calls):
            st = s1 if i % 2 == 0 else s2
            with torch.cuda.stream(st):
                p.synth_chirp(n0, c, out=outs[i], stream=st)
        torch.cuda.synchronize()
        for i in range(len(calls)):
            assert np.array_equal(to_np(outs[i]), ref[i]), (rep, i)


def test_mfma_more_groups_than_one_launch():
    """270,000 tones: the A operand's 67,500 tone groups exceed one launch's grid
    (65,535 in y), so it is generated in two launches; sampled outputs against
    the oracle."""
    torch = need_gpu()
    K, fs = 270_000, 280e6
    rng = np.random.default_rng(54)
    t = W.static_tones(rng.uniform(0.05 * fs, 0.45 * fs, K), rng.uniform(0.5, 1.0, K), rng.random(K))
    lp = awg.Plan(t, fs, 0.0, 0, F16)
    n0, count = 7, 1 << 16
    say("mfma %d tones n0=%d count=%d" % (K, n0, count))
    y = to_np(lp.synth_f32(n0, count, method=F16))
    q = to_np(lp.synth_static(n0, count))
    torch.cuda.synchronize()
    ns = np.unique(np.concatenate([np.arange(n0, n0 + 40), rng.integers(n0, n0 + count, 300),
                                   np.arange(n0 + count - 40, n0 + count)]))
    qo, yo = csynth.synth_at(words.Plan(fs, 0.0, 0, t), ns)
    compare(q[ns - n0], y[ns - n0], qo, yo, "mfma %d tones (sampled %d)" % (K, len(ns)))
    lp.close()


@pytest.mark.parametrize("method", [F16, BF16])
@pytest.mark.parametrize("n0,count", [(7, 1 << 16), (1 << 33, (1 << 18) + 3), (99, (1 << 20) + 5),
                                      (0, 1 << 22)])
def test_mfma_short_requests_split_k(method, n0, count):
    """Requests with fewer output tiles than compute units sum their tones in
    slices (FP32 planes added in order): same bar as the one-slice product."""
    torch = need_gpu()
    w = W.static_period()
    lp = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method)
    say("mfma split-K n0=%d count=%d method=%d" % (n0, count, method))
    q = to_np(lp.synth_static(n0, count))
    y = to_np(lp.synth_f32(n0, count, method=method))
    q2 = to_np(lp.synth_static(n0, count))
    torch.cuda.synchronize()
    assert np.array_equal(q, q2), "repeated call differs"
    ns = _pts(np.random.default_rng(53), n0, count)
    qo, yo = csynth.synth_at(words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones), ns)
    compare(q[ns - n0], y[ns - n0], qo, yo, "mfma split-K n0=%d count=%d method=%d" % (n0, count, method))


def test_mfma_request_longer_than_one_piece():
    """2^28 + 4097 samples: the static matrix-core path runs in pieces of 2^28
    samples; sampled codes on both sides of the piece boundary and at the ends."""
    torch = need_gpu()
    w = W.static_period(K=333)
    lp = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16)
    n0, count = 1000, (1 << 28) + 4097
    say("mfma two pieces n0=%d count=%d" % (n0, count))
    q = lp.synth_static(n0, count)
    torch.cuda.synchronize()
    edge = n0 + (1 << 28)
    ns = np.unique(np.concatenate([np.arange(n0, n0 + 200), np.arange(edge - 300, edge + 300),
                                   np.arange(n0 + count - 200, n0 + count),
                                   np.random.default_rng(55).integers(n0, n0 + count, 2000)]))
    qs = q[torch.from_numpy(ns - n0).to(q.device)].cpu().numpy()
    del q
    qo, yo = csynth.synth_at(words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones), ns)
    compare(qs, None, qo, yo, "mfma two pieces (sampled %d)" % len(ns))


def test_calls_from_several_host_threads():
    """Four host threads, each on its own stream, call the same plan (static
    matrix-core path and its shared workspace; hybrid path on a ramped plan) at
    once; every output equals the same call made alone."""
    import threading
    torch = need_gpu()
    ws = W.static_100tone_chunk()
    wr = W.array_group_chirps(K=600, seconds=0.01)
    ps = awg.Plan(ws.tones, ws.fs_hz, ws.gain_lsb, ws.period_log2, BF16)
    pr = awg.Plan(wr.tones, wr.fs_hz, wr.gain_lsb, wr.period_log2, BF16)
    pr.retune([(k, sh, a, n, f) for k, a, n, sh, f in sorted(wr.retunes, key=lambda e: e[1])[:100]])
    calls = [(ps, 0, 1 << 20), (ps, 777, 3 << 18), (pr, 0, 1 << 20), (pr, 4096, 1 << 19)]
    say("4 host threads x 6 calls on shared plans")
    ref = [to_np(p.synth_chirp(n0, c)) for p, n0, c in calls]
    torch.cuda.synchronize()
    errors = []

    def work(i):
        try:
            p, n0, c = calls[i]
            st = torch.cuda.Stream()
            out = torch.empty(c, dtype=torch.int16, device="cuda")
            for _ in range(6):
                with torch.cuda.stream(st):
                    p.synth_chirp(n0, c, out=out, stream=st)
                st.synchronize()
                if not np.array_equal(to_np(out), ref[i]):
                    errors.append(i)
        except Exception as e:           # reported below
            errors.append(repr(e))

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(calls))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in th)
    assert not errors, errors
    ps.close()
    pr.close()
