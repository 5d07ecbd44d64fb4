"""GPU parity of the hybrid path (ramped plans with a matrix-core method): the
tones on a line over a 1024-sample row go through the angle-addition product,
the ramping ones through the direct kernel, and the direct epilogue adds both.

Checked against the oracle element by element on a small plan whose windows sit
on every row-edge case, against the direct method over whole 2^20-sample chunks
of the large-array stream (10,000 tones, groups retuned every 1 ms), and for
exact identity with the direct method where the product has nothing to do.
"""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words, csynth

from gpu_common import need_gpu, say, to_np, compare, TOL_Q

pytestmark = pytest.mark.gpu

F16 = awg.AWG_F_METHOD_MFMA_F16X3
BF16 = awg.AWG_F_METHOD_MFMA_BF16X3


def _plans(w, method):
    return (awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method),
            awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, awg.AWG_F_METHOD_DIRECT))


@pytest.mark.parametrize("method", [F16, BF16])
def test_row_edges_every_sample_against_oracle(method):
    torch = need_gpu()
    w = W.row_edges()
    hp, dp = _plans(w, method)
    say("row-edges hybrid method=%d: %d tones, n0=%d count=%d" % (method, len(w.tones), w.n0, w.count))
    q = to_np(hp.synth_chirp(w.n0, w.count))
    y = to_np(hp.synth_f32(w.n0, w.count, method=method))
    qd = to_np(dp.synth_chirp(w.n0, w.count))
    torch.cuda.synchronize()
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    ns = np.arange(w.n0, w.n0 + w.count, dtype=np.int64)
    csynth.sparse_tables(op, ns)
    qo, yo = csynth.synth_at(op, ns)
    compare(q, y, qo, yo, "row-edges hybrid method=%d" % method)
    assert int(np.abs(q.astype(np.int32) - qd).max()) <= TOL_Q
    # the same call again gives the same samples
    q2 = to_np(hp.synth_chirp(w.n0, w.count))
    torch.cuda.synchronize()
    assert np.array_equal(q, q2)


@pytest.mark.parametrize("method", [F16, BF16])
def test_edge_blocks_hybrid_every_sample(method):
    """Groups of tones sharing a window (linear, raised cosine, minimum jerk; bin
    frequencies) with edges at every awkward offset inside a row: the ramping
    rows on the direct kernel's block-wise edge steps, the rest on the product."""
    torch = need_gpu()
    w = W.edge_blocks()
    hp, dp = _plans(w, method)
    n0, count = 5, 80000
    say("edge-blocks hybrid method=%d n0=%d count=%d" % (method, n0, count))
    q = to_np(hp.synth_chirp(n0, count))
    y = to_np(hp.synth_f32(n0, count, method=method))
    qd = to_np(dp.synth_chirp(n0, count))
    torch.cuda.synchronize()
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones)
    qo, yo = csynth.synth(op, n0, count)
    compare(q, y, qo, yo, "edge-blocks hybrid method=%d" % method)
    assert int(np.abs(q.astype(np.int32) - qd).max()) <= TOL_Q


def test_short_request_is_the_direct_kernel():
    torch = need_gpu()
    w = W.row_edges()
    hp, dp = _plans(w, F16)
    for n0, count in [(w.n0, 65535), (w.n0 + 7, 1000), (w.n0, 1)]:
        say("short hybrid-plan request n0=%d count=%d" % (n0, count))
        a = hp.synth_chirp(n0, count)
        b = dp.synth_chirp(n0, count)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("shape", ["linear", "mixed"])
def test_chirp_35ms_inside_windows_identical_to_direct(shape):
    """While every tone ramps over the whole chunk the product has no entries and
    the hybrid launch is the direct kernel on the same list: bit-identical. The
    chunk where the windows close is split and stays within 1 LSB."""
    torch = need_gpu()
    w = W.chirp_35ms(shape=shape)
    hp, dp = _plans(w, F16)
    N = W.RAMP_35MS
    for c in (0, 4, N // w.chunk):
        n0 = c * w.chunk
        say("chirp-35ms/%s chunk %d hybrid vs direct" % (shape, c))
        a = to_np(hp.synth_chirp(n0, w.chunk))
        b = to_np(dp.synth_chirp(n0, w.chunk))
        torch.cuda.synchronize()
        if n0 + w.chunk <= N:
            assert np.array_equal(a, b), c
        else:
            dq = np.abs(a.astype(np.int32) - b)
            say("closing chunk: max|dq| vs direct = %d (%d samples differ)" % (dq.max(), (dq > 0).sum()))
            assert dq.max() <= TOL_Q
            op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
            ns = np.unique(np.concatenate([np.arange(N - 2000, N + 2000),
                                           np.random.default_rng(c).integers(n0, n0 + w.chunk, 1500)]))
            ns = ns[(ns >= n0) & (ns < n0 + w.chunk)]
            csynth.sparse_tables(op, ns)
            y = to_np(hp.synth_f32(n0, w.chunk, method=F16))
            torch.cuda.synchronize()
            qo, yo = csynth.synth_at(op, ns)
            compare(a[ns - n0], y[ns - n0], qo, yo, "chirp-35ms/%s closing chunk hybrid (sampled %d)" % (shape, len(ns)))


@pytest.mark.parametrize("method", [F16, BF16])
def test_array_group_chirps_stream_against_direct_and_oracle(method):
    """10,000 tones, a group of 100 retuned every 1 ms: 14 chunks of 2^20 streamed
    with the hybrid and the direct method side by side, every sample compared;
    two chunks also against the oracle, with the unquantised sum."""
    torch = need_gpu()
    K = 10000
    w = W.array_group_chirps(K=K, seconds=0.05)
    hp, dp = _plans(w, method)
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    events = sorted(w.retunes, key=lambda e: e[1])
    n_chunks = w.count // w.chunk
    say("array K=%d hybrid method=%d: %d chunks, %d retunes" % (K, method, n_chunks, len(events)))
    i = 0
    checks = {3, n_chunks - 1}
    for c in range(n_chunks):
        end = (c + 1) * w.chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            op.add_ramp(k, a, n, shape, f)
            i += 1
        if batch:
            hp.retune(batch)
            dp.retune(batch)
        n0, qh = hp.stream_next(w.chunk)
        _, qd = dp.stream_next(w.chunk)
        yh = hp.synth_f32(n0, w.chunk, method=method) if c in checks else None
        torch.cuda.synchronize()
        a, b = to_np(qh), to_np(qd)
        dq = np.abs(a.astype(np.int32) - b)
        assert dq.max() <= TOL_Q, (c, int(dq.max()))
        if c in checks:
            rng = np.random.default_rng(c)
            ns = np.unique(np.concatenate([rng.integers(0, w.chunk, 600), [0, 1, w.chunk - 1],
                                           [e[1] - n0 + d for e in events[:: 25] for d in (-1, 0, 1, e[2], e[2] + 1)
                                            if 0 <= e[1] - n0 + d < w.chunk]]))
            qo, yo = csynth.synth_at(op, ns + n0)
            compare(a[ns], to_np(yh)[ns], qo, yo, "array hybrid chunk %d (sampled %d)" % (c, len(ns)))
    say("array hybrid: all %d chunks within %d LSB of the direct method" % (n_chunks, TOL_Q))


def test_array_full_second_line_buffer_against_direct_and_oracle():
    """The benchmark's headline workload for one whole second: 10,000 tones, a
    group of 100 retuned every 1 ms, 268 chunks of 2^20 on the BF16 line buffer
    (the configuration the benchmark times) beside the direct method, every
    sample of every chunk within 1 LSB of it, and five chunks sampled against
    the oracle with the unquantised sum."""
    torch = need_gpu()
    w = W.array_group_chirps(K=10000)
    hp, dp = _plans(w, BF16)
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    events = sorted(w.retunes, key=lambda e: e[1])
    n_chunks = w.count // w.chunk
    picks = {1, 67, 133, 200, n_chunks - 1}
    say("array K=10000 line buffer, %d chunks, %d retunes" % (n_chunks, len(events)))
    worst, differ, i = 0, 0, 0
    for c in range(n_chunks):
        end = (c + 1) * w.chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            op.add_ramp(k, a, n, shape, f)
            i += 1
        if batch:
            hp.retune(batch)
            dp.retune(batch)
        n0, qh = hp.stream_next(w.chunk)
        _, qd = dp.stream_next(w.chunk)
        yh = hp.synth_f32(n0, w.chunk, method=BF16) if c in picks else None
        torch.cuda.synchronize()
        a, b = to_np(qh), to_np(qd)
        dq = np.abs(a.astype(np.int32) - b)
        worst = max(worst, int(dq.max()))
        differ += int((dq > 0).sum())
        assert worst <= TOL_Q, c
        if c in picks:
            rng = np.random.default_rng(c)
            ns = np.unique(np.concatenate([rng.integers(0, w.chunk, 400), [0, w.chunk - 1],
                                           [e[1] - n0 + d for e in events for d in (-1, 0, 1, e[2])
                                            if 0 <= e[1] - n0 + d < w.chunk][:200]]))
            qo, yo = csynth.synth_at(op, ns + n0)
            compare(a[ns], to_np(yh)[ns], qo, yo, "array line buffer chunk %d (sampled %d)" % (c, len(ns)))
    say("array line buffer: %d chunks within %d LSB of the direct method (%d samples differ)"
        % (n_chunks, worst, differ))


def test_array_stream_period_longer_than_chunk():
    """The array stream on bins of 2^22 streamed in 2^20-sample chunks: each
    call covers a quarter of the period (S folded by its own launch), group
    sums that only segments need are made on their tile rows of the period
    alone, and the stream wraps round the period after four chunks: every
    sample against the direct method, two chunks sampled against the oracle."""
    import dataclasses
    torch = need_gpu()
    w = dataclasses.replace(W.array_group_chirps(K=3000, seconds=0.026), period_log2=22)
    hp, dp = _plans(w, BF16)
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    events = sorted(w.retunes, key=lambda e: e[1])
    n_chunks = 7
    i = 0
    for c in range(n_chunks):
        end = (c + 1) * w.chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            op.add_ramp(k, a, n, shape, f)
            i += 1
        if batch:
            hp.retune(batch)
            dp.retune(batch)
        say("array period 2^22 chunk %d" % c)
        n0, qh = hp.stream_next(w.chunk)
        _, qd = dp.stream_next(w.chunk)
        yh = hp.synth_f32(n0, w.chunk, method=BF16) if c in (3, 5) else None
        torch.cuda.synchronize()
        a, b = to_np(qh), to_np(qd)
        assert int(np.abs(a.astype(np.int32) - b).max()) <= TOL_Q, c
        if yh is not None:
            ns = np.unique(np.concatenate([np.random.default_rng(c).integers(0, w.chunk, 500), [0, w.chunk - 1]]))
            qo, yo = csynth.synth_at(op, ns + n0)
            compare(a[ns], to_np(yh)[ns], qo, yo, "array period 2^22 chunk %d (sampled %d)" % (c, len(ns)))


@pytest.mark.parametrize("method", [F16, BF16])
def test_one_period_calls_at_odd_offsets(method):
    """Calls of exactly one period (2^20 samples) that start off a row and off a
    multiple of four, so that the folds of S run in the kernels that read it on
    the per-sample path, and the call wraps round m = L - 1: every sample against
    the direct method, a sample of each against the oracle, and the first call
    repeated after the second (S and the cache brought back) gives the same codes."""
    torch = need_gpu()
    w = W.array_group_chirps(K=2000, seconds=0.012)
    L = 1 << w.period_log2
    hp, dp = _plans(w, method)
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    starts = [12345, 12345 + L + 999]
    batch = []
    for k, a, n, shape, f in sorted(w.retunes, key=lambda e: e[1]):
        if a < starts[-1] + L:
            batch.append((k, shape, a, n, f))
            op.add_ramp(k, a, n, shape, f)
    hp.retune(batch)
    dp.retune(batch)
    first = None
    for j, n0 in enumerate(starts + starts[:1]):
        say("one-period hybrid call method=%d n0=%d count=%d" % (method, n0, L))
        q = to_np(hp.synth_chirp(n0, L))
        y = to_np(hp.synth_f32(n0, L, method=method))
        qd = to_np(dp.synth_chirp(n0, L))
        torch.cuda.synchronize()
        assert int(np.abs(q.astype(np.int32) - qd).max()) <= TOL_Q, n0
        if j == 0:
            first = q
        elif j == len(starts):
            assert np.array_equal(q, first)
            continue
        rng = np.random.default_rng(n0)
        wrap = L - (n0 % L)                    # the sample at m = 0
        ns = np.unique(np.concatenate([rng.integers(0, L, 500), [0, 1, 2, 3, L - 1, wrap - 1, wrap]]))
        qo, yo = csynth.synth_at(op, ns + n0)
        compare(q[ns], y[ns], qo, yo, "one-period call at n0=%d (sampled %d)" % (n0, len(ns)))


def test_retune_records_reach_every_reader():
    """A plan on the line buffer leaves a retune's records to the next call that
    reads its device tone table: the line buffer's own pass applies them in its
    first launch, and every other reader (direct method, peak, phase words,
    multiplexed output) applies them first. After each retune the plan's output
    through that reader equals a direct-method plan retuned the same way."""
    torch = need_gpu()
    w = W.array_group_chirps(K=2000, seconds=0.02)
    hp, dp = _plans(w, BF16)
    C = w.chunk
    events = sorted(w.retunes, key=lambda e: e[1])
    i = 0

    def retune_upto(end):
        nonlocal i
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            i += 1
        if batch:
            hp.retune(batch)
            dp.retune(batch)
        return len(batch)

    retune_upto(C)
    a, b = hp.stream_next(C)[1], dp.stream_next(C)[1]          # the line buffer now exists
    torch.cuda.synchronize()
    assert int(np.abs(to_np(a).astype(np.int32) - to_np(b)).max()) <= TOL_Q
    # direct method on the line-buffer plan
    assert retune_upto(2 * C) > 0
    say("pending records: direct-method call")
    ya = hp.synth_f32(C, C, method=awg.AWG_F_METHOD_DIRECT)
    yb = dp.synth_f32(C, C, method=awg.AWG_F_METHOD_DIRECT)
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
    # peak
    assert retune_upto(3 * C) > 0
    say("pending records: peak")
    scr = torch.empty(C, dtype=torch.float32, device="cuda")
    pk = torch.zeros(2, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    awg.awg_peak(hp.handle, 2 * C, C, scr.data_ptr(), pk.data_ptr(), s)
    awg.awg_peak(dp.handle, 2 * C, C, scr.data_ptr(), pk.data_ptr() + 4, s)
    torch.cuda.synchronize()
    assert pk[0].item() == pk[1].item()
    # phase words of a retuned tone
    assert retune_upto(4 * C) > 0
    k = events[i - 1][0]
    say("pending records: phase words of tone %d" % k)
    wa, wb = hp.phase_dump(k, 3 * C, C), dp.phase_dump(k, 3 * C, C)
    torch.cuda.synchronize()
    assert torch.equal(wa, wb)
    # multiplexed output
    assert retune_upto(5 * C) > 0
    say("pending records: multiplexed channels")
    m = awg.multiplex([hp, dp], 4 * C, C)
    torch.cuda.synchronize()
    assert torch.equal(m[:, 0], m[:, 1])
    # and the line buffer's own pass, after a retune and after none
    for c in (5, 6):
        retune_upto((c + 1) * C)
        say("pending records: line-buffer chunk %d" % c)
        hp.seek(c * C)
        dp.seek(c * C)
        a, b = hp.stream_next(C)[1], dp.stream_next(C)[1]
        torch.cuda.synchronize()
        assert int(np.abs(to_np(a).astype(np.int32) - to_np(b)).max()) <= TOL_Q, c


def test_static_plan_chirp_call_uses_matrix_cores():
    torch = need_gpu()
    w = W.static_100tone_chunk()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, F16)
    a = p.synth_chirp(0, w.count)
    b = p.synth_static(0, w.count)
    n0, c = p.stream_next(w.count)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_line_buffer_output_at_unaligned_addresses():
    """The line buffer writes a thread's four codes in one 8-byte store where the
    destination allows it, else one code at a time: streams into an int16 view
    two bytes off an 8-byte boundary and into one on it give the aligned
    stream's codes chunk by chunk, and leave the elements around them alone."""
    torch = need_gpu()
    w = W.array_group_chirps(K=1000, seconds=0.012)
    plans = [awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16) for _ in range(3)]
    events = sorted(w.retunes, key=lambda e: e[1])
    big = [torch.full((w.chunk + 8,), 7, dtype=torch.int16, device="cuda") for _ in range(2)]
    views = [big[0][1:1 + w.chunk], big[1][4:4 + w.chunk]]
    i = 0
    for c in range(3):
        end = (c + 1) * w.chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            i += 1
        for p in plans:
            if batch:
                p.retune(batch)
        say("line buffer, chunk %d into offsets 0, 1 and 4 elements" % c)
        _, q = plans[0].stream_next(w.chunk)
        plans[1].stream_next(w.chunk, out=views[0])
        plans[2].stream_next(w.chunk, out=views[1])
        torch.cuda.synchronize()
        ref = to_np(q)
        for v in views:
            assert np.array_equal(to_np(v), ref), c
        b0, b1 = to_np(big[0]), to_np(big[1])
        assert b0[0] == 7 and (b0[1 + w.chunk:] == 7).all()
        assert (b1[:4] == 7).all() and (b1[4 + w.chunk:] == 7).all()
    for p in plans:
        p.close()
