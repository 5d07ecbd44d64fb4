"""awg_plan_reserve: the workspaces and staging a stream would allocate on first
use are set up ahead; later calls within the reserved sizes allocate no more
device memory and give the same codes as a plan without the set-up."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W

from gpu_common import need_gpu, say, to_np

pytestmark = pytest.mark.gpu

BF16 = awg.AWG_F_METHOD_MFMA_BF16X3


def test_reserve_static_matrix_core():
    torch = need_gpu()
    w = W.static_period()
    a = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16)
    b = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16)
    a.reserve(w.count)
    held = a.info["device_bytes"]
    say("static reserve: %d bytes held" % held)
    for n0, count in [(0, w.count), (5, 1 << 20), (9, (1 << 16) + 3), (77, 1 << 22)]:
        qa = to_np(a.synth_static(n0, count))
        qb = to_np(b.synth_static(n0, count))
        torch.cuda.synchronize()
        assert a.info["device_bytes"] == held, (n0, count)
        assert np.array_equal(qa, qb), (n0, count)
    a.close()
    b.close()


def test_reserve_hybrid_stream():
    torch = need_gpu()
    w = W.array_group_chirps(K=600, seconds=0.02)
    events = sorted(w.retunes, key=lambda e: e[1])
    a = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16)
    b = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, BF16)
    first = [(k, sh, st, n, f) for k, st, n, sh, f in events if st < w.chunk]
    a.retune(first)
    b.retune(first)
    a.reserve(w.chunk)
    held = a.info["device_bytes"]
    say("hybrid reserve: %d bytes held" % held)
    done = len(first)
    for c in range(4):
        end = (c + 1) * w.chunk
        batch = [(k, sh, st, n, f) for k, st, n, sh, f in events[done:] if st < end]
        done += len(batch)
        if c > 0 and batch:
            a.retune(batch)
            b.retune(batch)
        _, qa = a.stream_next(w.chunk)
        _, qb = b.stream_next(w.chunk)
        torch.cuda.synchronize()
        assert a.info["device_bytes"] == held, c
        assert np.array_equal(to_np(qa), to_np(qb)), c
    a.close()
    b.close()


def test_reserve_direct_and_errors():
    need_gpu()
    w = W.small_mixed()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
    p.reserve(1 << 20)                                   # retune staging only
    with pytest.raises(awg.AwgError) as e:
        awg.awg_plan_reserve(p.handle, 3, 1 << 20)
    assert e.value.status == awg.AWG_E_INVALID
    p.close()
