"""Multiplexed multi-channel output (the paper's wavetable multiplexer fused
into synthesis): channel c's sample n0 + i lands at out[n_channels * i + c],
and every channel is bit-identical to awg_synth_chirp of its plan."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words, csynth

from gpu_common import need_gpu, say, to_np, compare

pytestmark = pytest.mark.gpu


def _channel_plans():
    ws = [W.small_mixed(seed=11, n_total=20000), W.static_100tone_chunk(), W.small_mixed(seed=13, K=40, n_total=20000)]
    return ws, [awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2) for w in ws]


@pytest.mark.parametrize("n0,count", [(0, 5000), (7, 4099), (2 ** 40 + 3, 3000), (5, 1), (0, 1 << 18)])
def test_four_channels_equal_their_plans(n0, count):
    torch = need_gpu()
    ws, plans = _channel_plans()
    chans = [plans[0], plans[1], plans[2], plans[0]]          # a plan may appear twice
    say("multiplex 4 channels n0=%d count=%d" % (n0, count))
    out = awg.multiplex(chans, n0, count)
    solo = [p.synth_chirp(n0, count) for p in chans]
    torch.cuda.synchronize()
    o = to_np(out)
    assert o.shape == (count, 4)
    for c, s in enumerate(solo):
        assert np.array_equal(o[:, c], to_np(s)), c


@pytest.mark.parametrize("n", [1, 2, 3])
def test_fewer_channels_and_oracle(n):
    torch = need_gpu()
    ws, plans = _channel_plans()
    n0, count = 12345, 3000
    out = to_np(awg.multiplex(plans[:n], n0, count))
    torch.cuda.synchronize()
    for c in range(n):
        w = ws[c]
        op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones)
        qo, yo = csynth.synth_at(op, np.arange(n0, n0 + count, dtype=np.int64))
        compare(out[:, c], None, qo, yo, "multiplex %d channels, channel %d" % (n, c))


def test_streamed_multiplex_equals_one_shot():
    torch = need_gpu()
    ws, plans = _channel_plans()
    chans = plans[:3]
    ref = to_np(awg.multiplex(chans, 0, 20000))
    parts = []
    for size in [1, 1023, 1024, 1025, 4096, 7000, 20000 - (1 + 1023 + 1024 + 1025 + 4096 + 7000)]:
        buf = torch.empty((size, 3), dtype=torch.int16, device="cuda")
        n0 = awg.awg_stream_next_multiplex([p.handle for p in chans], size, buf.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
        assert n0 == sum(x.shape[0] for x in parts)
        parts.append(buf)
    torch.cuda.synchronize()
    assert np.array_equal(np.concatenate([to_np(x) for x in parts]), ref)
    assert all(p.tell() == 20000 for p in chans)


def test_multiplex_errors():
    torch = need_gpu()
    ws, plans = _channel_plans()
    buf = torch.empty(64, dtype=torch.int16, device="cuda")
    for bad in ([], [plans[0]] * 5):
        with pytest.raises(awg.AwgError) as e:
            awg.awg_synth_multiplex([p.handle for p in bad], 0, 8, buf.data_ptr())
        assert e.value.status == awg.AWG_E_INVALID
    host = awg.Plan(ws[0].tones, ws[0].fs_hz, 0.0, 0, host_only=True)
    with pytest.raises(awg.AwgError) as e:
        awg.awg_synth_multiplex([plans[0].handle, host.handle], 0, 8, buf.data_ptr())
    assert e.value.status == awg.AWG_E_INVALID
    plans[1].seek(5)
    with pytest.raises(awg.AwgError) as e:
        awg.awg_stream_next_multiplex([plans[0].handle, plans[1].handle], 8, buf.data_ptr())
    assert e.value.status == awg.AWG_E_INVALID
    with pytest.raises(awg.AwgError) as e:
        awg.awg_synth_multiplex([plans[0].handle], 2 ** 63 - 4, 8, buf.data_ptr())
    assert e.value.status == awg.AWG_E_RANGE
