"""The allocation-free peak call (awg_peak_noalloc) against awg_peak on the GPU:
same kernels, the samples in the library's per-device scratch array instead of
the caller's buffer, so the peak must be bit-identical. Two calls in a row, the
second on a smaller, ragged range (the array keeps the first call's samples),
on a chirped plan, plus the size limit and the oracle's FP64 peak."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from oracle import words, csynth

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _peak(torch, plan, n0, count):
    stream = torch.cuda.current_stream().cuda_stream
    scratch = torch.empty(count, dtype=torch.float32, device="cuda")
    ref = torch.empty(1, dtype=torch.float32, device="cuda")
    got = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    say("awg_peak n0=%d count=%d" % (n0, count))
    awg.awg_peak(plan.handle, n0, count, scratch.data_ptr(), ref.data_ptr(), stream)
    say("awg_peak_noalloc n0=%d count=%d" % (n0, count))
    awg.awg_peak_noalloc(plan.handle, n0, count, got.data_ptr(), stream)
    torch.cuda.synchronize()
    return float(ref.item()), float(got.item())


def test_noalloc_peak_equals_peak_two_calls():
    torch = need_gpu()
    w = W.small_mixed(n_total=awg.AWG_PEAK_NOALLOC_MAX)
    plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
    try:
        # the largest request the array holds, then a smaller ragged one
        for n0, count in ((0, awg.AWG_PEAK_NOALLOC_MAX), (12345, 300001)):
            ref, got = _peak(torch, plan, n0, count)
            say("peak %.6f noalloc %.6f" % (ref, got))
            assert got == ref
        # the second range against the oracle's FP64 peak (FP32 path: 0.25 LSB)
        _, y = csynth.synth(words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=True),
                            12345, 300001)
        assert abs(got - float(np.max(np.abs(y)))) < 0.25
    finally:
        plan.close()


def test_noalloc_peak_rejects_oversize_and_bad_args():
    torch = need_gpu()
    w = W.small_mixed(n_total=4096)
    plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
    try:
        peak = torch.empty(1, dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        with pytest.raises(awg.AwgError) as e:
            awg.awg_peak_noalloc(plan.handle, 0, awg.AWG_PEAK_NOALLOC_MAX + 1, peak.data_ptr(), stream)
        assert e.value.status == awg.AWG_E_UNSUPPORTED
        with pytest.raises(awg.AwgError) as e:
            awg.awg_peak_noalloc(plan.handle, 0, 0, peak.data_ptr(), stream)
        assert e.value.status == awg.AWG_E_INVALID
        with pytest.raises(awg.AwgError) as e:
            awg.awg_peak_noalloc(plan.handle, 0, 4096, None, stream)
        assert e.value.status == awg.AWG_E_INVALID
    finally:
        plan.close()
