"""Kernel timing through the C ABI: every launch or one launch in n of each
kernel is timed with events recorded by the dispatch; reading resets on request;
the product's output does not change with timing on."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W

from gpu_common import need_gpu, say, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("every,calls,timed", [(1, 5, 5), (3, 7, 3), (8, 8, 1)])
def test_sampled_kernel_timing(every, calls, timed):
    torch = need_gpu()
    w = W.static_100tone_chunk()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, awg.AWG_F_METHOD_MFMA_BF16X3)
    ctx = awg.context(0)
    awg.awg_profile_read(ctx, reset=True)
    ref = to_np(p.synth_static(0, w.count))
    say("profile every=%d calls=%d" % (every, calls))
    awg.awg_profile_enable(ctx, every)
    outs = [p.synth_static(0, w.count) for _ in range(calls)]
    awg.awg_profile_enable(ctx, False)
    torch.cuda.synchronize()
    st = awg.awg_profile_read(ctx, reset=True)
    for o in outs:
        assert np.array_equal(to_np(o), ref)
    for name in ("gen_a_kernel_bf16", "angle_gemm_kernel_bf16"):
        launches, total_ms, max_ms, work = st[name]
        assert launches == timed, (name, st)
        assert 0.0 < total_ms / launches <= max_ms < 100.0
    # the product's algorithmic work: every tone at every sample of the timed calls
    assert st["angle_gemm_kernel_bf16"][3] == timed * len(w.tones) * w.count
    assert st["gen_a_kernel_bf16"][3] == 0.0
    assert awg.awg_profile_read(ctx) == {}
    p.close()


def test_repeated_timing_cycles_agree():
    """Each read cycle times its launches with events of its own: a later cycle's
    launches of the same kernel on the same input read about what the first
    cycle's did, and the stream's output does not change."""
    torch = need_gpu()
    w = W.static_100tone_chunk()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, awg.AWG_F_METHOD_MFMA_BF16X3)
    ctx = awg.context(0)
    awg.awg_profile_read(ctx, reset=True)
    ref = to_np(p.synth_static(0, w.count))
    means = []
    for cycle in range(4):
        say("timing cycle %d" % cycle)
        awg.awg_profile_enable(ctx, 1)
        outs = [p.synth_static(0, w.count) for _ in range(6)]
        awg.awg_profile_enable(ctx, False)
        torch.cuda.synchronize()
        st = awg.awg_profile_read(ctx, reset=True)
        for o in outs:
            assert np.array_equal(to_np(o), ref)
        launches, total_ms, max_ms, _ = st["angle_gemm_kernel_bf16"]
        assert launches == 6
        means.append(total_ms / launches)
    say("mean ms per cycle: %s" % means)
    for m in means[1:]:
        assert m < 3.0 * means[0], means
    p.close()


def test_profile_enable_rejects_negative():
    need_gpu()
    with pytest.raises(awg.AwgError):
        awg.awg_profile_enable(awg.context(0), -1)
