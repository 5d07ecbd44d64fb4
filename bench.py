"""Benchmark of the synthesis hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--method auto|direct|mfma-f16|mfma-bf16]

Headline workload: the large-array stream at 280 MS/s, 10,000 tones on an even
grid over 60-140 MHz (amplitudes U[0.5, 1], Schroeder phases, bins of 2^20),
groups of 100 consecutive tones chirped in turn by 0-2 MHz over 1 ms (linear),
streamed in 2^20-sample int16 chunks (seeded, synthetic). A step is one chunk of
that stream: the retune call for the chirps that start in the chunk, then
awg_stream_next of 2^20 samples into a resident int16 buffer (exact phase words,
sinusoids, weighted sum, int16 epilogue). W chunks run untimed, then K chunks
are timed between device synchronisations; value = tones * samples / time, with
per-chunk latency (HIP events around each step of a second stretch of chunks) and the real-time factor.

Also reported (one JSON line):
  roofline      the dominant kernel of the timed steps: its algorithmic rate
                (the library's per-launch work count over its event-timed duration)
                against the MI355X peak, and its HBM bytes per launch when the
                committed counter summary matches the kernel's source
  cpu_baseline  the CPU oracle (FP64 direct sum) on a bounded contiguous stretch
                of the last timed chunk, on this host's cores; its codes also give
                the int16 error of the GPU chunk there
  static_period the 1000-tone 2^24-sample periodic buffer on each method
  static_chunk  100 static tones, one 2^20-sample chunk
  playback      1000 tones chirped over 35 ms, one call over all 9.8M samples
                (bin and free frequencies)
  streaming     the same chirps streamed in 2^20-sample chunks (bin and free frequencies)
  large_arrays  the 5000-tone array stream, and the 10,000-tone one on the direct method
  serving       the Poisson chirp-job trace through the batched server
  short_requests  static calls of 2^16 .. 2^22 samples on each method
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tone-samples/s + real-time factor at 280 MS/s (int16, <=1 LSB); p99 chunk latency"
PEAK_FP32_TFLOPS = 157.3
PEAK_MFMA16_TFLOPS = 2500.0         # dense FP16 and BF16 matrix peak of MI355X
ALL_LEGS = "static,chunk,playback,stream,arrays,serve,short"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256, help="timed chunks of the headline stream")
    ap.add_argument("--warmup", type=int, default=12, help="untimed chunks before them")
    ap.add_argument("--method", default="auto", choices=["auto", "direct", "mfma-f16", "mfma-bf16"])
    ap.add_argument("--tones", type=int, default=10000, help="tones of the headline array stream")
    ap.add_argument("--time-every", type=int, default=16,
                    help="time one launch in N of each kernel with HIP events inside the timed steps "
                         "(a timed launch costs the stream a few microseconds: about 2%% of the "
                         "headline stream's rate at N = 8, none measurable at 16)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default=ALL_LEGS, help="comma list of extra legs: " + ALL_LEGS)
    ap.add_argument("--no-stream", action="store_true", help="run no extra legs")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="seconds of Poisson arrivals of the serving leg")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="job arrivals per second of the serving leg")
    ap.add_argument("--static-tones", type=int, default=1000, help="tones of the static 2^24-sample period")
    ap.add_argument("--stream-shape", default="mixed", choices=["mixed", "linear", "cosine", "minjerk"],
                    help="ramp shape of the chirped stream and playback legs")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def method_codes(awg):
    return {"direct": awg.AWG_F_METHOD_DIRECT, "mfma-f16": awg.AWG_F_METHOD_MFMA_F16X3,
            "mfma-bf16": awg.AWG_F_METHOD_MFMA_BF16X3}


def dtype_of(method):
    return {"direct": "f32", "mfma-f16": "f16x3", "mfma-bf16": "bf16x3"}[method]


def timed_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/traffic.json), or None when it is missing or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[kernel]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec["sha256_16"]:
        return None
    return rec["bytes_per_launch"]


def is_matrix_kernel(name):
    return name.startswith("angle_gemm") or name.startswith("hyb_gemm") or name.startswith("plb_gemm")


def roofline_for(stats):
    """Dominant kernel (largest event-timed total) and its algorithmic rate
    against the MI355X peak. stats: {name: (launches, total_ms, max_ms, work)}
    with work = the algorithmic tone-samples of the timed launches. A matrix
    kernel does 4 flop per tone-sample (two MACs of angle addition; the hi/lo
    split issues 3x that), a direct kernel 2 (one weighting FMA; it is bound by
    VALU issue including one v_sin_f32 per tone-sample)."""
    name, (launches, total_ms, _, work) = max(stats.items(), key=lambda kv: kv[1][1])
    avg_ms = total_ms / launches
    sec = total_ms * 1e-3
    if is_matrix_kernel(name):
        ach = 4.0 * work / sec / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": PEAK_MFMA16_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_MFMA16_TFLOPS, "traffic": traffic_for(name), "avg_kernel_ms": avg_ms,
                "work_per_launch": work / launches,
                "issued_tflops_min": 3 * ach, "issued_frac_min": 3 * ach / PEAK_MFMA16_TFLOPS,
                "note": "achieved: 4 algorithmic flop per tone-sample covered by the product; the hi/lo "
                        "split issues at least 3x that (more with the zero padding of tone blocks)"}
    ach = 2.0 * work / sec / 1e12
    return {"bound": "alu", "kernel": name, "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP32_TFLOPS, "traffic": traffic_for(name), "avg_kernel_ms": avg_ms,
            "work_per_launch": work / launches,
            "note": "2 algorithmic flop per tone-sample over the FP32 vector peak; the kernel is bound "
                    "by VALU issue including one v_sin_f32 per tone-sample"}


def kernel_table(stats):
    return {k: {"launches": v[0], "avg_ms": v[1] / max(1, v[0]), "work_per_launch": v[3] / max(1, v[0])}
            for k, v in stats.items()}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()


# ----------------------------------------------------------------- headline

class StepTicks:
    """Start and end events of each timed step, recorded through the HIP runtime
    directly (two calls per step with no Python object per event): the
    per-chunk latency of the stream at a lower host cost than torch's events."""

    def __init__(self, n):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so.7", mode=ctypes.RTLD_GLOBAL)
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(2 * n):
            e = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(e.value)
        self.record = self.hip.hipEventRecord

    def ms(self, j):
        t = self.ct.c_float()
        if self.hip.hipEventElapsedTime(self.ct.byref(t), self.ev[2 * j], self.ev[2 * j + 1]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return t.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)
        self.ev = []


def array_stream(torch, awg, W, K, method, steps, warmup, time_every):
    """The large-array stream: K tones, groups of 100 retuned in turn (1 ms linear
    chirps), 2^20-sample chunks. warmup chunks untimed, then `steps` chunks timed
    as one stretch (one launch in time_every of each kernel timed by the library
    for the roofline), then one untimed chunk (the queue refills after the
    profiler's read synchronised the device), then `steps` more chunks with HIP
    events around each step for the per-chunk latency (those events hold the
    stream at each step's edges, so they stay out of the timed stretch)."""
    fs = W.FS_280
    chunk = W.CHUNK
    n_total = warmup + 2 * steps + 1
    seconds = max(1.0, n_total * chunk / fs + 1e-3)
    w = W.array_group_chirps(K=K, seconds=seconds)
    plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method_codes(awg)[method])
    plan.reserve(chunk)                              # workspaces and staging before the stream starts
    events = sorted(w.retunes, key=lambda e: e[1])
    # the retune schedule as ready-made C arrays, one per chunk (the controller's
    # side of the stream; building them is not part of the synthesis)
    batches, per_chunk_events = [], []
    i = 0
    for c in range(n_total):
        end = (c + 1) * chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            i += 1
        batches.append(awg.retune_array(batch) if batch else None)
        per_chunk_events.append(len(batch))
    buf = [torch.empty(chunk, dtype=torch.int16, device="cuda") for _ in range(2)]
    s = torch.cuda.current_stream()

    def step(c):
        if batches[c] is not None:
            plan.retune(batches[c])
        plan.stream_next(chunk, out=buf[c % 2])

    for c in range(warmup):
        step(c)
    torch.cuda.synchronize()
    ctx = awg.context(0)
    awg.awg_profile_read(ctx, reset=True)
    awg.awg_profile_enable(ctx, max(1, time_every))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(steps):
        step(warmup + j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    awg.awg_profile_enable(ctx, False)
    stats = awg.awg_profile_read(ctx, reset=True)
    # per-chunk latency on the `steps` chunks after one untimed chunk
    ticks = StepTicks(steps)
    ev, rec, sh = ticks.ev, ticks.record, s.cuda_stream
    step(warmup + steps)
    for j in range(steps):
        rec(ev[2 * j], sh)
        step(warmup + steps + 1 + j)
        rec(ev[2 * j + 1], sh)
    torch.cuda.synchronize()
    lat = np.array([ticks.ms(j) for j in range(steps)])
    ticks.close()
    last = n_total - 1
    q_last = buf[last % 2].cpu().numpy()
    retunes_timed = sum(per_chunk_events[warmup:warmup + steps])
    plan.close()
    return {"w": w, "wall": wall, "lat": lat, "stats": stats, "q_last": q_last, "last_chunk": last,
            "retunes_timed": retunes_timed, "events": events}


def array_cpu_baseline(r, seconds):
    """The oracle on a contiguous stretch of the last timed chunk (all tones, every
    retune up to that chunk), on this host's cores: rate and the GPU codes' error there."""
    from oracle import words, csynth
    w = r["w"]
    n0 = r["last_chunk"] * w.chunk
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones, build_tables=False)
    for k, a, n, shape, f in r["events"]:
        if a < n0 + w.chunk:
            op.add_ramp(k, a, n, shape, f)
    pk = csynth.Packed(op)
    threads = oracle_threads()
    probe = 2048
    t0 = time.perf_counter()
    csynth.synth(op, n0, probe, threads=threads, packed=pk)
    dt = time.perf_counter() - t0
    count = int(min(w.chunk, max(probe, probe * seconds / max(dt, 1e-6))))
    start = n0 + int(np.random.default_rng(99).integers(0, w.chunk - count + 1))
    t0 = time.perf_counter()
    qo, _ = csynth.synth(op, start, count, threads=threads, packed=pk)
    dt = time.perf_counter() - t0
    K = len(w.tones)
    dq = int(np.max(np.abs(r["q_last"][start - n0:start - n0 + count].astype(np.int32) - qo.astype(np.int32))))
    one = int(min(count, max(256, count * 2.0 / max(dt * threads, 1e-6))))
    t0 = time.perf_counter()
    csynth.synth(op, start, one, threads=1, packed=pk)
    dt1 = time.perf_counter() - t0
    return {"value": K * count / dt, "unit": "tone-samples/s", "cores": threads, "kind": "oracle",
            "sample": "samples [%d, %d) of chunk %d of the %d-tone array stream (%d retunes applied), "
                      "all tones (%.1f s)" % (start, start + count, r["last_chunk"], K,
                                             sum(1 for e in r["events"] if e[1] < n0 + w.chunk), dt),
            "max_dq_lsb_vs_gpu": dq, "value_one_core": K * one / dt1,
            "one_core_sample": "samples [%d, %d) (%.1f s)" % (start, start + one, dt1), "host_cpu": host_cpu()}


# -------------------------------------------------------------------- legs

def static_period_leg(torch, awg, W, K, steps, time_every, cpu_seconds):
    """The static 2^24-sample periodic buffer (K tones) on each method: one
    awg_synth_static over the whole period per step; roofline of the BF16
    product; the oracle on a bounded stretch of the buffer."""
    w = W.static_period(K=K)
    L = w.count
    codes = method_codes(awg)
    ctx = awg.context(0)
    out = torch.empty(L, dtype=torch.int16, device="cuda")
    res = {"workload": w.name, "tones": K, "samples": L, "methods": {}}
    q_bf16 = None
    for m in ("mfma-bf16", "mfma-f16", "direct"):
        plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, codes[m])

        def step():
            plan.synth_static(0, L, out=out)

        t0 = time.perf_counter()
        n = 0
        while n < 3 or time.perf_counter() - t0 < 0.3:    # bring the clocks up
            step()
            n += 1
            if n % 8 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        awg.awg_profile_read(ctx, reset=True)
        awg.awg_profile_enable(ctx, max(1, time_every))
        ms, _ = timed_steps(torch, step, steps if m != "direct" else max(3, steps // 4), 0)
        awg.awg_profile_enable(ctx, False)
        stats = awg.awg_profile_read(ctx, reset=True)
        res["methods"][m] = {"ms_per_step": ms, "tone_samples_per_s": K * L / (ms * 1e-3),
                             "rtf": (L / w.fs_hz) / (ms * 1e-3), "roofline": roofline_for(stats),
                             "kernels": kernel_table(stats)}
        log("static %-9s ms/step %.3f  tone-samples/s %.3e" % (m, ms, K * L / (ms * 1e-3)))
        if m == "mfma-bf16":
            q_bf16 = out.cpu().numpy()
        plan.close()
    if cpu_seconds > 0:
        from oracle import words, csynth
        op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones)
        pk = csynth.Packed(op)
        threads = oracle_threads()
        t0 = time.perf_counter()
        csynth.synth(op, 0, 4096, threads=threads, packed=pk)
        dt = time.perf_counter() - t0
        count = int(min(L, max(4096, 4096 * cpu_seconds / max(dt, 1e-6))))
        start = int(np.random.default_rng(99).integers(0, L - count + 1))
        t0 = time.perf_counter()
        qo, _ = csynth.synth(op, start, count, threads=threads, packed=pk)
        dt = time.perf_counter() - t0
        dq = int(np.max(np.abs(q_bf16[start:start + count].astype(np.int32) - qo.astype(np.int32))))
        res["cpu_oracle"] = {"value": K * count / dt, "unit": "tone-samples/s", "cores": threads,
                             "sample": "samples [%d, %d) of the period (%.1f s)" % (start, start + count, dt),
                             "max_dq_lsb_bf16_vs_oracle": dq}
    return res


def static_chunk_leg(torch, awg, W, reps=50):
    """100 static tones, one 2^20-sample chunk (the small static case), direct and BF16."""
    w = W.static_100tone_chunk()
    K, n = len(w.tones), w.count
    out = torch.empty(n, dtype=torch.int16, device="cuda")
    res = {"workload": w.name, "tones": K, "samples": n}
    for m in ("direct", "mfma-bf16"):
        plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method_codes(awg)[m])
        ms, _ = timed_steps(torch, lambda: plan.synth_static(0, n, out=out), reps, 5)
        res[m] = {"ms_per_call": ms, "tone_samples_per_s": K * n / (ms * 1e-3)}
        plan.close()
    log("chunk 100 tones: direct %.4f ms, bf16 %.4f ms" % (res["direct"]["ms_per_call"], res["mfma-bf16"]["ms_per_call"]))
    return res


def _chirp_workload(W, shape, free):
    w = W.chirp_35ms(shape=shape)
    if free:
        w.period_log2 = 0
        w.name += "-free"
    return w


def playback_leg(torch, awg, W, shape, reps=5):
    """1000 tones chirped over 35 ms (9.8M samples): one awg_synth_chirp over the
    whole ramp, direct method (the paper's Playback comparison: 610 ms for this
    job on its GPU); with bin frequencies and with free ones."""
    rows = []
    for free in (False, True):
        w = _chirp_workload(W, shape, free)
        n = W.RAMP_35MS
        plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
        out = torch.empty(n, dtype=torch.int16, device="cuda")
        ms, _ = timed_steps(torch, lambda: plan.synth_chirp(0, n, out=out), reps, 1)
        rows.append({"workload": w.name, "tones": len(w.tones), "samples": n, "ms_per_call": ms,
                     "tone_samples_per_s": len(w.tones) * n / (ms * 1e-3),
                     "rtf": (n / w.fs_hz) / (ms * 1e-3)})
        log("playback %s: %.3f ms (RTF %.1f)" % (w.name, ms, rows[-1]["rtf"]))
        plan.close()
    return {"rows": rows, "paper_context": "610 ms for 1000 tones x 35 ms at 280 MS/s on a Quadro RTX 6000 "
                                           "(its own figure, other hardware)"}


def streaming_leg(torch, awg, W, shape, free, reps=3):
    """1000 tones chirped over 35 ms, streamed in 2^20-sample chunks: per-chunk
    device time, real-time factor."""
    w = _chirp_workload(W, shape, free)
    plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
    s = torch.cuda.current_stream()
    n_chunks = w.count // w.chunk
    buf = [torch.empty(w.chunk, dtype=torch.int16, device="cuda") for _ in range(2)]
    for c in range(2):
        plan.stream_next(w.chunk, out=buf[c % 2])
    lat = []
    for _ in range(reps):
        plan.seek(0)
        evs = []
        for c in range(n_chunks):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            plan.stream_next(w.chunk, out=buf[c % 2])
            e1.record(s)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        lat += [a.elapsed_time(b) for a, b in evs]
    lat = np.array(lat)
    chunk_s = w.chunk / w.fs_hz
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    plan.close()
    log("stream %s: p50 %.3f ms p99 %.3f ms" % (w.name, p50, p99))
    return {"workload": w.name, "tones": len(w.tones), "chunk": w.chunk, "chunks": int(len(lat)),
            "p50_chunk_ms": p50, "p99_chunk_ms": p99,
            "tone_samples_per_s": len(w.tones) * w.chunk / (float(np.mean(lat)) * 1e-3),
            "rtf_p99": chunk_s / (p99 * 1e-3), "rtf_mean": chunk_s / (float(np.mean(lat)) * 1e-3),
            "latency_note": "device time per 2^20-sample chunk (hipEvents on the launch stream)"}


def serving_leg(W, seconds, rate_hz=2000.0):
    """Serving trace in real time: Poisson arrivals of chirp jobs, batched by the
    library's server; latency, throughput and deadline misses."""
    from paper_2403_15582_amd.serving import Server
    jobs = W.poisson_jobs(seconds=seconds, rate_hz=rate_hz)
    with Server(mem_budget_bytes=1 << 30, max_jobs=512, ring_slots=256, playout_delay_ms=5.0) as srv:
        t0 = time.perf_counter()
        srv.run_trace(jobs, time_scale=1.0, timeout_s=300.0)
        wall = time.perf_counter() - t0
        st = srv.stats()
    offered = sum(len(j.tones) * j.n_samples for j in jobs) / seconds
    return {"workload": "poisson-chirp-jobs-%g/s" % rate_hz, "jobs": len(jobs), "arrival_seconds": seconds,
            "offered_tone_samples_per_s": offered,
            "tone_samples_per_s": st["tone_samples"] / (st["wall_ms"] * 1e-3),
            "device_busy_frac": st["device_busy_ms"] / st["wall_ms"],
            "output_seconds_per_second": st["audio_seconds"] / (st["wall_ms"] * 1e-3),
            "p50_chunk_ms": st["chunk_latency_p50_ms"], "p99_chunk_ms": st["chunk_latency_p99_ms"],
            "p50_first_chunk_ms": st["first_chunk_latency_p50_ms"],
            "p99_first_chunk_ms": st["first_chunk_latency_p99_ms"],
            "deadline_misses": st["deadline_misses"], "p99_lateness_ms": st["lateness_p99_ms"],
            "chunks": st["chunks_done"], "mean_batch": st["mean_batch"], "max_batch": st["max_batch"],
            "steps": st["steps"], "wall_s": wall,
            "latency_note": "chunk latency = chunk ready - job arrival (host clock); deadline = "
                            "arrival + 5 ms + chunk start / fs"}


def array_leg(torch, awg, W, K, method):
    """A whole second (268 chunks) of the K-tone array stream: per-chunk device
    time and the per-kernel split."""
    r = array_stream(torch, awg, W, K, method, steps=267, warmup=1, time_every=1)
    lat = r["lat"]
    chunk_s = W.CHUNK / W.FS_280
    return {"workload": r["w"].name, "method": method, "tones": K, "chunks": 2 * len(lat) + 2,
            "retunes": len(r["events"]), "kernels": kernel_table(r["stats"]),
            "p50_chunk_ms": float(np.percentile(lat, 50)), "p99_chunk_ms": float(np.percentile(lat, 99)),
            "max_chunk_ms": float(np.max(lat)),
            "tone_samples_per_s": K * W.CHUNK / (float(np.mean(lat)) * 1e-3),
            "rtf_mean": chunk_s / (float(np.mean(lat)) * 1e-3), "rtf_p99": chunk_s / (float(np.percentile(lat, 99)) * 1e-3),
            "note": "kernels: chunks 1..267, every launch event-timed (a few us added per kernel); per-chunk "
                    "latency: chunks 269..535 after one untimed chunk, HIP events around each step"}


def short_requests_leg(torch, awg, W, reps=20):
    """Static requests shorter than the 2^24-sample period (2^16 .. 2^22 samples from
    a moving n0) on each method: wall clock per call, streams of back-to-back calls."""
    w = W.static_period()
    codes = method_codes(awg)
    K = len(w.tones)
    rows = []
    for lg in (16, 18, 20, 22):
        count = 1 << lg
        out = torch.empty(count, dtype=torch.int16, device="cuda")
        row = {"samples": count}
        for m in ("direct", "mfma-bf16", "mfma-f16"):
            plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, codes[m])
            for i in range(5):
                plan.synth_static(i * count, count, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(reps):
                plan.synth_static((5 + i) * count, count, out=out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            row[m] = {"ms_per_call": ms, "tone_samples_per_s": K * count / (ms * 1e-3)}
            plan.close()
        rows.append(row)
    return {"tones": K, "timing": "host wall clock over %d back-to-back calls per size" % reps, "rows": rows}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the synthesis runs on a single MI355X; "
              "--gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2403_15582_amd as awg
    from paper_2403_15582_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if a.copy_probe_mib:
        n = a.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "copies": 3}), flush=True)
        return
    steps, warmup = max(1, a.steps), max(0, a.warmup)
    method = "mfma-bf16" if a.method == "auto" else a.method
    K = a.tones
    log("headline: %d-tone array stream, %s, %d warm-up + %d timed chunks" % (K, method, warmup, steps))
    r = array_stream(torch, awg, W, K, method, steps, warmup, a.time_every)
    w = r["w"]
    chunk_s = w.chunk / w.fs_hz
    ms = r["wall"] * 1e3 / steps
    lat = r["lat"]
    value = K * w.chunk * steps / r["wall"]
    res = {"metric": METRIC, "value": value, "unit": "tone-samples/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype_of(method), "data": "synthetic",
           "config": {"workload": w.name, "tones": K, "chunk_samples": w.chunk, "fs_hz": w.fs_hz,
                      "group": 100, "chirp_ms": 1.0, "method": method, "output": "int16",
                      "step": "retune of the chirps starting in the chunk + awg_stream_next of one chunk"},
           "rtf": chunk_s / (ms * 1e-3),
           "p50_chunk_ms": float(np.percentile(lat, 50)), "p99_chunk_ms": float(np.percentile(lat, 99)),
           "rtf_p99": chunk_s / (float(np.percentile(lat, 99)) * 1e-3),
           "retunes_timed": r["retunes_timed"],
           "roofline": roofline_for(r["stats"]), "kernels": kernel_table(r["stats"]),
           "kernel_timing": "HIP events recorded by the dispatch of one launch in %d of each kernel inside "
                            "the timed steps (launches = timed launches)" % max(1, a.time_every),
           "latency_timing": "p50/p99 from HIP events around each of %d further chunks after the timed ones "
                             "and one untimed chunk (kept out of the timed steps: each event holds the "
                             "stream)" % steps}
    log("headline: %.3e tone-samples/s, %.4f ms/chunk, RTF %.1f, p99 chunk %.4f ms"
        % (value, ms, res["rtf"], res["p99_chunk_ms"]))
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = array_cpu_baseline(r, a.cpu_seconds)
    legs = set() if a.no_stream else set(x for x in a.legs.split(",") if x)
    if "static" in legs:
        log("static period leg ...")
        res["static_period"] = static_period_leg(torch, awg, W, a.static_tones, 40, a.time_every,
                                                 0 if a.no_cpu_baseline else 3.0)
    if "chunk" in legs:
        res["static_chunk"] = static_chunk_leg(torch, awg, W)
    if "playback" in legs:
        log("playback leg ...")
        res["playback"] = playback_leg(torch, awg, W, a.stream_shape)
    if "stream" in legs:
        log("streaming legs ...")
        res["streaming"] = [streaming_leg(torch, awg, W, a.stream_shape, free) for free in (False, True)]
    if "arrays" in legs:
        log("large-array legs ...")
        res["large_arrays"] = [array_leg(torch, awg, W, 5000, "mfma-bf16"), array_leg(torch, awg, W, 10000, "direct")]
    if "short" in legs:
        log("short-request leg ...")
        res["short_requests"] = short_requests_leg(torch, awg, W)
    if "serve" in legs:
        log("serving leg ...")
        res["serving"] = serving_leg(W, a.serve_seconds, a.serve_rate)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
