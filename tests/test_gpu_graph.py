"""Synthesis calls captured into a HIP graph (torch.cuda.graph) and replayed:
every replay, with eager work and synchronisations between replays, must give
the eager call's codes. The direct method launches kernels only; the static
matrix-core path also orders its workspace with an event, which is recorded
into the graph."""
import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd import workloads as W

from gpu_common import need_gpu, say, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", [awg.AWG_F_METHOD_DIRECT, awg.AWG_F_METHOD_MFMA_BF16X3])
def test_captured_static_synthesis_replays(method):
    torch = need_gpu()
    w = W.static_100tone_chunk()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method)
    n0, count = 777, w.count
    say("graph capture of awg_synth_static, method=%d" % method)
    ref = to_np(p.synth_static(n0, count))          # eager call (also sets up the workspace)
    out = torch.zeros(count, dtype=torch.int16, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.synth_static(n0, count, out=out, stream=s)
    torch.cuda.synchronize()
    other = torch.empty(count, dtype=torch.int16, device="cuda")
    for rep in range(4):
        out.zero_()
        p.synth_static(12345 + rep, count, out=other)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_np(out), ref), rep
    del g
    p.close()


def test_captured_chirp_synthesis_replays():
    torch = need_gpu()
    w = W.small_mixed(n_total=20000)
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
    n0, count = 3, 20000
    say("graph capture of awg_synth_chirp (direct), ramped plan")
    ref = to_np(p.synth_chirp(n0, count))
    out = torch.zeros(count, dtype=torch.int16, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.synth_chirp(n0, count, out=out, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        p.synth_chirp(500 + rep, count)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_np(out), ref), rep
    del g
    p.close()


def test_calls_follow_the_current_stream():
    """With no stream given, a call goes on torch's current stream of the plan's
    device (the binding's raw query names the same handle as torch's Stream
    object, inside and outside a stream context), and its result is ordered on
    that stream."""
    torch = need_gpu()
    w = W.static_100tone_chunk()
    p = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, awg.AWG_F_METHOD_DIRECT)
    ref = to_np(p.synth_static(0, w.count))
    assert awg.current_stream_handle(p.device) == torch.cuda.current_stream(p.device).cuda_stream
    s = torch.cuda.Stream()
    say("synthesis inside a stream context")
    with torch.cuda.stream(s):
        assert awg.current_stream_handle(p.device) == s.cuda_stream
        assert awg.current_stream_handle(p.device, s) == s.cuda_stream
        out = p.synth_static(0, w.count)
        q = out.to(torch.int32)                       # a consumer on the same stream, no synchronisation
    s.synchronize()
    assert np.array_equal(q.cpu().numpy().astype(np.int16), ref)
    assert awg.current_stream_handle(p.device) == torch.cuda.current_stream(p.device).cuda_stream
    p.close()
