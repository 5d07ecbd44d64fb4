"""Saturation of the Q operator (Eq. (2)): with a gain that drives the sum past
the int16 code range, every path must clip exactly where the oracle clips and
stay within 1 LSB elsewhere. Compared with the oracle on every sample of the
range: the direct kernel, the matrix-core static path (FP16 and BF16 hi/lo x3),
the hybrid path of a ramped plan, and the batched serving kernel."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W
from paper_2403_15582_amd.serving import Server
from oracle import words, csynth

from gpu_common import need_gpu, say, to_np, compare

pytestmark = pytest.mark.gpu

F16 = awg.AWG_F_METHOD_MFMA_F16X3
BF16 = awg.AWG_F_METHOD_MFMA_BF16X3
DIRECT = awg.AWG_F_METHOD_DIRECT
# peak of the unit-gain sum mapped to 1.8 x full scale: a good share of the
# samples clips on both sides
OVERDRIVE = 1.8


def _oracle(w, gain, n0, count, tables=True):
    op = words.Plan(w.fs_hz, gain, w.period_log2, w.tones, build_tables=tables)
    if not tables:
        csynth.sparse_tables(op, np.arange(n0, n0 + count, dtype=np.int64))
    return csynth.synth(op, n0, count)


def _check_clipped(q, y, qo, yo, what, tol_y):
    """Every sample within the bar; where the oracle's sum is clearly beyond the
    code range the GPU code is exactly the end code."""
    hi, lo = yo > 32768.5, yo < -32769.5
    say("%s: %d samples above, %d below the code range" % (what, int(hi.sum()), int(lo.sum())))
    assert hi.sum() > 100 and lo.sum() > 100, "the gain does not clip"
    compare(q, y, qo, yo, what, tol_y=tol_y)
    assert np.all(q[hi] == 32767) and np.all(q[lo] == -32768), what


@pytest.fixture(scope="module")
def static_clip():
    w = W.static_period()
    _, y1 = _oracle(w, 1.0, 0, 1 << 16)
    gain = OVERDRIVE * 32767.0 / float(np.max(np.abs(y1)))
    count = 1 << 20
    qo, yo = _oracle(w, gain, 0, count)
    return w, gain, count, qo, yo


@pytest.mark.parametrize("method", [DIRECT, F16, BF16])
def test_static_saturation_every_sample(static_clip, method):
    torch = need_gpu()
    w, gain, count, qo, yo = static_clip
    say("static saturation method=%d gain=%.2f: 1000 tones x %d samples" % (method, gain, count))
    p = awg.Plan(w.tones, w.fs_hz, gain, w.period_log2, method)
    q = to_np(p.synth_static(0, count))
    y = to_np(p.synth_f32(0, count, method=method))
    torch.cuda.synchronize()
    # the gain is 2x the 90%-full-scale one, so the FP32 / hi-lo error bar doubles too
    _check_clipped(q, y, qo, yo, "static saturation method=%d" % method, tol_y=0.5)
    p.close()


@pytest.mark.parametrize("method", [F16, BF16])
def test_hybrid_saturation_every_sample(method):
    torch = need_gpu()
    w = W.row_edges()
    _, y1 = _oracle(w, 1.0, w.n0, 1 << 16, tables=False)
    gain = OVERDRIVE * 32767.0 / float(np.max(np.abs(y1)))
    say("hybrid saturation method=%d gain=%.2f: %d tones n0=%d count=%d"
        % (method, gain, len(w.tones), w.n0, w.count))
    p = awg.Plan(w.tones, w.fs_hz, gain, w.period_log2, method)
    q = to_np(p.synth_chirp(w.n0, w.count))
    y = to_np(p.synth_f32(w.n0, w.count, method=method))
    torch.cuda.synchronize()
    qo, yo = _oracle(w, gain, w.n0, w.count, tables=False)
    _check_clipped(q, y, qo, yo, "hybrid saturation method=%d" % method, tol_y=0.5)
    p.close()


def test_serving_saturation_every_sample():
    """Jobs submitted with an overdriving gain through the batched kernel."""
    torch = need_gpu()
    jobs = W.poisson_jobs(seed=21, max_jobs=6, dmax_ms=1.5, kmax=300)
    for j in jobs:
        op1 = words.Plan(j.fs_hz, 1.0, 0, j.tones)
        _, y1 = csynth.synth(op1, 0, j.n_samples)
        j.gain_lsb = OVERDRIVE * 32767.0 / float(np.max(np.abs(y1)))
    say("serving saturation: %d jobs, K %s" % (len(jobs), [len(j.tones) for j in jobs]))
    with Server(max_jobs=8, ring_slots=8) as srv:
        out = srv.run_trace(jobs, collect=range(len(jobs)), time_scale=0.05)
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        qo, yo = csynth.synth(words.Plan(j.fs_hz, j.gain_lsb, 0, j.tones), 0, j.n_samples)
        hi, lo = yo > 32768.5, yo < -32769.5
        compare(out[k], None, qo, yo, "served job %d at gain %.2f (K=%d, %d samples, %d clipped)"
                % (k, j.gain_lsb, len(j.tones), j.n_samples, int(hi.sum() + lo.sum())))
        assert hi.sum() + lo.sum() > 0
        assert np.all(out[k][hi] == 32767) and np.all(out[k][lo] == -32768), k
