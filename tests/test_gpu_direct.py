"""GPU parity of the direct kernel against the CPU oracle (through the C ABI).

Phase words must match bit for bit; int16 codes within 1 LSB; the unquantised
FP32 sum within 0.25 LSB. Sizes: small cases compared element by element over
several tiles with ragged tails, and the full configurations (2^20 x 100,
2^24 x 1000, 10 x 2^20 x 1000 chirped) on sampled outputs.
"""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words, csynth

from gpu_common import need_gpu, say, to_np, compare

pytestmark = pytest.mark.gpu


def oracle_plan(w, tables=True):
    return words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=tables)


def lib_plan(w, method=awg.AWG_F_METHOD_DIRECT):
    return awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method)


def test_phase_words_bit_exact_small_mixed():
    torch = need_gpu()
    w = W.small_mixed()
    op = oracle_plan(w)
    pk = csynth.Packed(op)
    lp = lib_plan(w)
    for n0, count in [(0, w.count), (3, 1234), (2 ** 40 + 7, 3000), (4095, 1)]:
        say("phase dump small_mixed n0=%d count=%d" % (n0, count))
        for k in range(len(w.tones)):
            got = to_np(lp.phase_dump(k, n0, count)).view(np.uint64)
            torch.cuda.synchronize()
            want = csynth.phases(op, k, n0, count, packed=pk)
            assert np.array_equal(got, want), (k, n0, int(np.sum(got != want)))


def test_phase_words_bit_exact_long_ramps():
    """35 ms ramps of every shape, with bin frequencies (dF a multiple of 2^16)
    and with free ones (any dF: the smooth loops carry the fraction of r H)."""
    torch = need_gpu()
    for shape, free in [(s, f) for s in ("linear", "cosine", "minjerk") for f in (False, True)]:
        w = W.chirp_35ms(shape=shape, K=8)
        if free:
            w.period_log2 = 0
            shape += "-free"
        op = oracle_plan(w, tables=False)
        lp = lib_plan(w)
        N = W.RAMP_35MS
        for n0 in [0, 12345, N // 2 - 3, N - 700, N - 1, N + 5, 3 * N]:
            count = 1500
            ns = np.arange(n0, n0 + count)
            csynth.sparse_tables(op, ns)
            pk = csynth.Packed(op)
            say("phase dump chirp-35ms/%s n0=%d" % (shape, n0))
            for k in range(len(w.tones)):
                got = to_np(lp.phase_dump(k, n0, count)).view(np.uint64)
                torch.cuda.synchronize()
                want = csynth.phases(op, k, n0, count, packed=pk)
                assert np.array_equal(got, want), (shape, k, n0)


@pytest.mark.parametrize("n0,count", [(0, 5000), (1, 1), (7, 511), (100, 513), (2 ** 33 + 5, 4099),
                                      (2 ** 62, 700)])
def test_small_mixed_int16_and_f32(n0, count):
    torch = need_gpu()
    w = W.small_mixed()
    op = oracle_plan(w)
    lp = lib_plan(w)
    say("small_mixed int16/f32 n0=%d count=%d" % (n0, count))
    q = to_np(lp.synth_chirp(n0, count))
    y = to_np(lp.synth_f32(n0, count))
    torch.cuda.synchronize()
    qo, yo = csynth.synth(op, n0, count)
    compare(q, y, qo, yo, "small_mixed n0=%d count=%d" % (n0, count))


@pytest.mark.parametrize("period_log2", [20, 0])
@pytest.mark.parametrize("n0,count", [(0, None), (2000, 9000), (1024 * 7 + 15, 1024 * 5 + 3)])
def test_window_edges_in_shared_blocks(n0, count, period_log2):
    """Groups of tones sharing a window whose edges fall at every awkward
    offset inside a tile (linear, raised-cosine and minimum-jerk groups), with
    bin frequencies (smooth steps a multiple of 2^16 of the word) and free ones
    (any step), every sample against the oracle."""
    torch = need_gpu()
    w = W.edge_blocks(period_log2=period_log2)
    count = w.count - n0 if count is None else count
    op = oracle_plan(w)
    lp = lib_plan(w)
    say("edge_blocks int16/f32 n0=%d count=%d" % (n0, count))
    q = to_np(lp.synth_chirp(n0, count))
    y = to_np(lp.synth_f32(n0, count))
    torch.cuda.synchronize()
    qo, yo = csynth.synth(op, n0, count)
    compare(q, y, qo, yo, "edge_blocks n0=%d count=%d" % (n0, count))


def test_output_buffer_checks():
    """Synthesis into pinned host memory is refused before any launch (were it
    not, the kernel would only write mapped host memory), and a device buffer
    passes at any offset inside its allocation."""
    torch = need_gpu()
    w = W.small_mixed()
    lp = lib_plan(w)
    host = torch.zeros(4096, dtype=torch.int16).pin_memory()
    for call in (lambda: awg.awg_synth_chirp(lp.handle, 0, 4096, host.data_ptr()),
                 lambda: awg.awg_stream_next(lp.handle, 4096, host.data_ptr())):
        with pytest.raises(awg.AwgError) as e:
            call()
        assert e.value.status == awg.AWG_E_INVALID
    torch.cuda.synchronize()
    assert int(host.abs().max()) == 0
    dev = torch.zeros(8192, dtype=torch.int16, device="cuda")
    awg.awg_synth_chirp(lp.handle, 0, 4096, dev.data_ptr() + 2 * 4096)
    q = to_np(lp.synth_chirp(0, 4096))
    torch.cuda.synchronize()
    assert np.array_equal(to_np(dev[4096:]), q) and int(dev[:4096].abs().max()) == 0


def test_count_zero_and_errors():
    torch = need_gpu()
    w = W.small_mixed()
    lp = lib_plan(w)
    out = torch.full((16,), 77, dtype=torch.int16, device="cuda")
    awg.awg_synth_chirp(lp.handle, 0, 0, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(out[0]) == 77
    with pytest.raises(awg.AwgError) as e:
        awg.awg_synth_chirp(lp.handle, 2 ** 63 - 4, 8, out.data_ptr())
    assert e.value.status == awg.AWG_E_RANGE
    with pytest.raises(awg.AwgError) as e:
        awg.awg_synth_static(lp.handle, 0, 8, out.data_ptr())      # plan has ramps
    assert e.value.status == awg.AWG_E_UNSUPPORTED
    with pytest.raises(awg.AwgError) as e:
        awg.awg_phase_dump(lp.handle, len(w.tones), 0, 8, out.data_ptr())
    assert e.value.status == awg.AWG_E_INVALID


def test_single_tone_and_quarter_rate():
    torch = need_gpu()
    t = awg.make_tones(1)
    t["f_start_hz"] = 70e6
    t["amplitude"] = 1.0
    lp = awg.Plan(t, 280e6, 1000.0, 0)
    q = to_np(lp.synth_chirp(0, 4096))
    torch.cuda.synchronize()
    assert np.array_equal(q, np.tile(np.array([0, 1000, 0, -1000], dtype=np.int16), 1024))


def test_static_100tone_chunk_full():
    torch = need_gpu()
    w = W.static_100tone_chunk()
    lp = lib_plan(w)
    say("static-100tone-chunk full 2^20 x 100")
    q = to_np(lp.synth_static(0, w.count))
    y = to_np(lp.synth_f32(0, w.count))
    torch.cuda.synchronize()
    qo, yo = csynth.synth(oracle_plan(w), 0, w.count)
    compare(q, y, qo, yo, "static-100tone-chunk")


def _sample_points(rng, total, extra=()):
    ns = set(rng.integers(0, total, 3000).tolist())
    ns |= set(range(0, 600)) | set(range(total - 600, total))
    ns |= set(int(e) for e in extra)
    return np.array(sorted(n for n in ns if 0 <= n < total), dtype=np.int64)


def test_static_period_full_direct_sampled_and_periodic():
    torch = need_gpu()
    w = W.static_period()
    lp = lib_plan(w)
    say("static-period full 2^24 x 1000 direct")
    qd = lp.synth_static(0, w.count)
    yd = lp.synth_f32(0, w.count)
    tail = lp.synth_static(w.count, 1 << 16)          # the next period starts over
    torch.cuda.synchronize()
    q, y = to_np(qd), to_np(yd)
    assert np.array_equal(to_np(tail), q[:1 << 16])
    ns = _sample_points(np.random.default_rng(21), w.count)
    qo, yo = csynth.synth_at(oracle_plan(w), ns)
    compare(q[ns], y[ns], qo, yo, "static-period direct (sampled %d)" % len(ns))


@pytest.mark.parametrize("shape", ["linear", "cosine", "minjerk", "mixed", "cosine-free", "mixed-free"])
def test_chirp_35ms_streamed_equals_oneshot_and_oracle(shape):
    """Config 3: 1000 tones chirped over 35 ms, streamed in 10 chunks of 2^20;
    "-free": frequencies not snapped to bins (any dF), as the config states them."""
    torch = need_gpu()
    w = W.chirp_35ms(shape=shape.split("-")[0])
    if shape.endswith("-free"):
        w.period_log2 = 0
    lp = lib_plan(w)
    say("chirp-35ms/%s streamed 10 x 2^20 x 1000" % shape)
    chunks = []
    for c in range(w.count // w.chunk):
        n0, out = lp.stream_next(w.chunk)
        assert n0 == c * w.chunk
        chunks.append(out)
    streamed = torch.cat(chunks)
    oneshot = lp.synth_chirp(0, w.count)
    y = lp.synth_f32(0, w.count)
    torch.cuda.synchronize()
    assert torch.equal(streamed, oneshot)
    q, yv = to_np(oneshot), to_np(y)
    N = W.RAMP_35MS
    ns = _sample_points(np.random.default_rng(31), w.count, range(N - 300, N + 300))
    op = oracle_plan(w, tables=False)
    csynth.sparse_tables(op, ns)
    qo, yo = csynth.synth_at(op, ns)
    compare(q[ns], yv[ns], qo, yo, "chirp-35ms/%s (sampled %d)" % (shape, len(ns)))


def test_irregular_chunks_and_resume_bit_identical():
    torch = need_gpu()
    w = W.small_mixed(n_total=20000)
    lp = lib_plan(w)
    ref = lp.synth_chirp(0, 20000)
    sizes = [1, 2, 511, 512, 513, 3, 4096, 777, 5000]
    parts = []
    for s in sizes:
        parts.append(lp.stream_next(s)[1])
    pos = lp.tell()
    # checkpoint: a fresh plan from the same inputs resumes at the cursor
    lp2 = lib_plan(w)
    lp2.seek(pos)
    parts.append(lp2.stream_next(20000 - pos)[1])
    torch.cuda.synchronize()
    assert torch.equal(torch.cat(parts), ref)


def test_retune_stream_matches_oracle():
    torch = need_gpu()
    w = W.array_group_chirps(K=1000, seconds=0.02, group=100)
    lp = lib_plan(w)
    op = oracle_plan(w, tables=False)
    events = sorted(w.retunes, key=lambda e: e[1])
    say("array-small retuned stream: %d retunes" % len(events))
    outs = []
    i = 0
    n_chunks = w.count // w.chunk
    for c in range(n_chunks):
        end = (c + 1) * w.chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            op.add_ramp(k, a, n, shape, f)
            i += 1
        # one event per tone per call: split when a tone repeats
        seen, cur = set(), []
        for e in batch:
            if e[0] in seen:
                lp.retune(cur)
                seen, cur = set(), []
            seen.add(e[0])
            cur.append(e)
        if cur:
            lp.retune(cur)
        outs.append(lp.stream_next(w.chunk)[1])
    q = to_np(torch.cat(outs))
    torch.cuda.synchronize()
    ns = _sample_points(np.random.default_rng(41), n_chunks * w.chunk,
                        [e[1] + d for e in events[::37] for d in (-1, 0, 1, 2, 140000, W.RAMP_1MS)])
    qo, yo = csynth.synth_at(op, ns)
    compare(q[ns], None, qo, yo, "array-small (sampled %d)" % len(ns))



def test_retune_largest_batch():
    """One retune call of the largest batch (16384 events, a full staging slot that
    the scatter kernel reads in place) on a 20,000-tone static plan, mixed shapes;
    the direct and hybrid methods streamed across the windows against the oracle."""
    torch = need_gpu()
    K, fs = 20_000, 280e6
    rng = np.random.default_rng(61)
    bins = rng.choice(np.arange(60 * 2 ** 20 // 280, 130 * 2 ** 20 // 280), K, replace=False)
    t = W.static_tones(bins * fs / 2 ** 20, rng.uniform(0.5, 1.0, K), rng.random(K))
    ks = rng.choice(K, 16384, replace=False)
    shapes = [awg.RAMP_LINEAR, awg.RAMP_COSINE, awg.RAMP_MINJERK]
    events = [(int(k), shapes[i % 3], 70_000 + 13 * (i % 997), 50_000 + 7 * (i % 311),
               float(t["f_start_hz"][k] + rng.uniform(-1e6, 1e6))) for i, k in enumerate(ks)]
    count = 3 * (1 << 16) + 333
    op = words.Plan(fs, 0.0, 20, t, build_tables=False)
    for k, sh, a, n, f in events:
        op.add_ramp(k, a, n, sh, f)
    ns = np.unique(np.concatenate([np.arange(0, 50), rng.integers(0, count, 400),
                                   np.array([70_000, 120_000, 140_000, 160_000, count - 1])]))
    csynth.sparse_tables(op, ns)
    qo, yo = csynth.synth_at(op, ns)
    for method in (awg.AWG_F_METHOD_DIRECT, awg.AWG_F_METHOD_MFMA_BF16X3):
        lp = awg.Plan(t, fs, 0.0, 20, method)
        say("retune 16384 events on %d tones, method %d" % (K, method))
        lp.retune(events)
        parts = [lp.stream_next(c)[1] for c in (1 << 16, 1 << 16, (1 << 16) + 333)]
        q = np.concatenate([to_np(x) for x in parts])
        torch.cuda.synchronize()
        compare(q[ns], None, qo, yo, "retune 16384 events method %d (sampled %d)" % (method, len(ns)))
        lp.close()

@pytest.mark.parametrize("K", [5000, 10000])
def test_array_group_chirps_full_second_streamed(K):
    """Large array: 1 s at 280 MS/s (268 chunks), groups of 100 tones retuned in turn."""
    torch = need_gpu()
    w = W.array_group_chirps(K=K)
    lp = lib_plan(w)
    op = oracle_plan(w, tables=False)
    events = sorted(w.retunes, key=lambda e: e[1])
    n_chunks = w.count // w.chunk
    say("array K=%d: %d chunks, %d retunes" % (K, n_chunks, len(events)))
    rng = np.random.default_rng(K)
    picks = sorted(set([0, 1, 2, n_chunks // 2, n_chunks - 1]) | set(rng.integers(0, n_chunks, 4).tolist()))
    kept = {}
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
            lp.retune(batch)
        n0, out = lp.stream_next(w.chunk)
        if c in picks:
            kept[c] = out
    torch.cuda.synchronize()
    pk = csynth.Packed(op)
    for c in picks:
        q = to_np(kept[c])
        base = c * w.chunk
        ns = np.unique(np.concatenate([rng.integers(0, w.chunk, 400), [0, 1, w.chunk - 1]]))
        ramp_edges = [e[1] - base + d for e in events for d in (-1, 0, 1, W.RAMP_1MS)
                      if 0 <= e[1] - base + d < w.chunk]
        ns = np.unique(np.concatenate([ns, np.array(ramp_edges[:200], dtype=np.int64)]))
        qo, yo = csynth.synth_at(op, ns + base, packed=pk)
        compare(q[ns], None, qo, yo, "array K=%d chunk %d (sampled %d)" % (K, c, len(ns)))


def test_direct_many_tones_mixed_windows():
    """120,000 tones (a tenth of them chirped, windows of seeded starts and 40
    lengths with every shape) through the direct kernel over a ragged range:
    sampled codes and sums against the oracle, and the range split in two calls
    gives the same codes."""
    torch = need_gpu()
    K, fs = 120_000, 280e6
    rng = np.random.default_rng(56)
    f0 = rng.uniform(0.05 * fs, 0.45 * fs, K)
    t = W.static_tones(f0, rng.uniform(0.2, 1.0, K), rng.random(K))
    ramped = rng.random(K) < 0.1
    t["f_end_hz"] = np.where(ramped, np.clip(f0 + rng.uniform(-1e6, 1e6, K), 0.05 * fs, 0.45 * fs), f0)
    t["ramp"] = np.where(ramped, rng.integers(1, 4, K), 0)
    t["ramp_start"] = np.where(ramped, rng.integers(0, 6000, K), 0)
    lens = rng.integers(1, 5000, 40)                      # 40 lengths: at most 80 smooth tables
    t["ramp_len"] = np.where(ramped, lens[rng.integers(0, 40, K)], 0)
    lp = awg.Plan(t, fs, 0.0, 20)
    n0, count = 1234, 9000 + 77
    say("direct %d tones n0=%d count=%d" % (K, n0, count))
    q = to_np(lp.synth_chirp(n0, count))
    y = to_np(lp.synth_f32(n0, count))
    a = to_np(lp.synth_chirp(n0, 4096))
    b = to_np(lp.synth_chirp(n0 + 4096, count - 4096))
    torch.cuda.synchronize()
    assert np.array_equal(np.concatenate([a, b]), q)
    ns = np.unique(np.concatenate([np.arange(n0, n0 + 50), np.arange(n0 + count - 50, n0 + count),
                                   rng.integers(n0, n0 + count, 150)]))
    op = words.Plan(fs, 0.0, 20, t, build_tables=False)
    csynth.sparse_tables(op, ns)
    qo, yo = csynth.synth_at(op, ns)
    compare(q[ns - n0], y[ns - n0], qo, yo, "direct %d tones (sampled %d)" % (K, len(ns)))
