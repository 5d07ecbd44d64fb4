"""Benchmark of the synthesis hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--method auto|direct|mfma-f16|mfma-bf16]

Workload (the configuration the headline metric is quoted on): one period of a
static 1000-tone buffer, L = 2^24 samples at fs = 280 MS/s, bins in 60-140 MHz,
amplitudes U[0.5, 1], Schroeder phases, default gain (seeded, synthetic). A step
is one awg_synth_static call over the whole buffer into a resident int16 buffer
(exact phase words, sinusoids, weighted sum, int16 epilogue). The timed region
is K steps between device synchronisations; value = tones * samples / time.

Also reported:
  roofline      the dominant kernel's algorithmic rate against the MI355X peak
  cpu_baseline  the CPU oracle (FP64 direct sum) on a bounded contiguous sample of
                the same buffer, on this host's cores; its outputs also give the
                int16 error of the GPU result on that sample
  streaming     a chirped stream (1000 tones, 35 ms linear/cosine ramps, 2^20-sample
                chunks): per-chunk latency p50/p99 and real-time factor
  short_requests  static calls of 2^16 .. 2^22 samples on each method (wall clock)
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tone-samples/s + real-time factor at 280 MS/s (int16, <=1 LSB); p99 chunk latency"
PEAK_FP32_TFLOPS = 157.3
PEAK_MFMA16_TFLOPS = 2500.0         # dense FP16 and BF16 matrix peak of MI355X


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="auto", choices=["auto", "direct", "mfma-f16", "mfma-bf16"])
    ap.add_argument("--time-every", type=int, default=8,
                    help="time one launch in N of each kernel with HIP events inside the timed steps "
                         "(a timed launch costs the stream a few microseconds)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming, serving and large-array legs")
    ap.add_argument("--legs", default="stream,arrays,serve,short",
                    help="comma list of extra legs to run: stream, arrays, serve, short")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="seconds of Poisson arrivals of the serving leg")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="job arrivals per second of the serving leg")
    ap.add_argument("--static-tones", type=int, default=1000, help="tones of the static 2^24-sample period")
    ap.add_argument("--stream-shape", default="mixed", choices=["mixed", "linear", "cosine", "minjerk"],
                    help="ramp shape of the chirped stream")
    ap.add_argument("--arrays-tones", default="5000,10000", help="tone counts of the large-array leg")
    ap.add_argument("--arrays-methods", default="direct,mfma-f16,mfma-bf16", help="methods of the large-array leg")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


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


def cpu_baseline(w, q_gpu, seconds):
    """Oracle FP64 direct sum on a contiguous sample of the buffer (CPU, all cores)."""
    from oracle import words, csynth
    op = words.Plan(w.fs_hz, w.gain_lsb, w.period_log2, w.tones)
    pk = csynth.Packed(op)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    probe = 4096
    t0 = time.perf_counter()
    csynth.synth(op, 0, probe, threads=threads, packed=pk)
    dt = time.perf_counter() - t0
    count = int(min(w.count, max(probe, probe * seconds / max(dt, 1e-6))))
    start = int(np.random.default_rng(99).integers(0, w.count - count + 1))
    t0 = time.perf_counter()
    qo, yo = csynth.synth(op, start, count, threads=threads, packed=pk)
    dt = time.perf_counter() - t0
    ts = len(w.tones) * count
    dq = int(np.max(np.abs(q_gpu[start:start + count].astype(np.int32) - qo.astype(np.int32))))
    # the same oracle on one core, over a shorter stretch of the same sample (about 2 s)
    one = int(min(count, max(256, count * 2.0 / max(dt * threads, 1e-6))))
    t0 = time.perf_counter()
    csynth.synth(op, start, one, threads=1, packed=pk)
    dt1 = time.perf_counter() - t0
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": ts / dt, "unit": "tone-samples/s", "cores": threads, "kind": "oracle",
            "sample": "samples [%d, %d) of the %d-sample buffer, all %d tones (%.1f s)"
                      % (start, start + count, w.count, len(w.tones), dt),
            "max_dq_lsb_vs_gpu": dq,
            "value_one_core": len(w.tones) * one / dt1, "one_core_sample": "samples [%d, %d) (%.1f s)"
                                                                         % (start, start + one, dt1),
            "host_cpu": cpu}


def streaming_leg(torch, awg, W, shape="mixed"):
    """1000 tones chirped over 35 ms (mixed linear and cosine), streamed in 2^20-sample
    chunks: per-chunk latency and real-time factor."""
    w = W.chirp_35ms(shape=shape)
    plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2)
    s = torch.cuda.current_stream()
    n_chunks = w.count // w.chunk
    buf = [torch.empty(w.chunk, dtype=torch.int16, device="cuda") for _ in range(2)]
    for c in range(2):                       # warm-up
        plan.stream_next(w.chunk, out=buf[c % 2])
    plan.seek(0)
    lat = []
    for rep in range(3):
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
    return {"workload": w.name, "tones": len(w.tones), "chunk": w.chunk, "chunks": int(len(lat)),
            "p50_chunk_ms": p50, "p99_chunk_ms": p99,
            "tone_samples_per_s": len(w.tones) * w.chunk / (float(np.mean(lat)) * 1e-3),
            "rtf_p99": chunk_s / (p99 * 1e-3), "rtf_mean": chunk_s / (float(np.mean(lat)) * 1e-3),
            "latency_note": "device time per 2^20-sample chunk (hipEvents on the launch stream)"}


def serving_leg(W, seconds, rate_hz=2000.0):
    """Serving trace in real time: Poisson arrivals of chirp jobs, batched
    by the library's server; latency, throughput and deadline misses."""
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
            "deadline_misses": st["deadline_misses"], "p99_lateness_ms": st["lateness_p99_ms"], "chunks": st["chunks_done"],
            "mean_batch": st["mean_batch"], "max_batch": st["max_batch"], "steps": st["steps"],
            "wall_s": wall,
            "latency_note": "chunk latency = chunk ready - job arrival (host clock); deadline = "
                            "arrival + 5 ms + chunk start / fs"}


def large_array_leg(torch, awg, W, K, method="direct"):
    """Large-array stream: K tones, groups of 100 retuned (1 ms linear chirps)
    in turn, 2^20-sample chunks over 1 s of output; per-chunk device time. With a
    matrix-core method the chunks take the hybrid path (line tones on the matrix
    cores, ramping tones on the direct kernel); the last 11 chunks run again with
    kernel timing on for the per-kernel split."""
    w = W.array_group_chirps(K=K)
    plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, method_codes(awg)[method])
    # set up workspaces and staging before the stream starts (awg_plan_reserve)
    plan.reserve(w.chunk)
    events = sorted(w.retunes, key=lambda e: e[1])
    n_chunks = w.count // w.chunk
    buf = [torch.empty(w.chunk, dtype=torch.int16, device="cuda") for _ in range(2)]
    s = torch.cuda.current_stream()
    # the retune schedule as ready-made C arrays, one per chunk (the controller's
    # side of the stream; building them is not part of the synthesis)
    batches = []
    i = 0
    for c in range(n_chunks):
        end = (c + 1) * w.chunk
        batch = []
        while i < len(events) and events[i][1] < end:
            k, a, n, shape, f = events[i]
            batch.append((k, shape, a, n, f))
            i += 1
        batches.append(awg.retune_array(batch) if batch else None)
    ticks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_chunks)]
    evs = []
    t0 = time.perf_counter()
    for c in range(n_chunks):
        e0, e1 = ticks[c]
        e0.record(s)
        if batches[c] is not None:
            plan.retune(batches[c])
        plan.stream_next(w.chunk, out=buf[c % 2])
        e1.record(s)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    chunk_s = w.chunk / w.fs_hz
    # per-kernel split: the last 12 chunks again (within one retune cycle, so the
    # tones still hold the windows those chunks were streamed with); the first of
    # them runs untimed, since it rebuilds the B operand for lines that changed
    # since the stream's last chunk
    ctx = awg.context(0)
    first = max(0, n_chunks - 12)
    plan.synth_chirp(first * w.chunk, w.chunk, out=buf[first % 2])
    torch.cuda.synchronize()
    awg.awg_profile_read(ctx, reset=True)
    awg.awg_profile_enable(ctx, True)
    for c in range(first + 1, n_chunks):
        plan.synth_chirp(c * w.chunk, w.chunk, out=buf[c % 2])
    torch.cuda.synchronize()
    awg.awg_profile_enable(ctx, False)
    stats = awg.awg_profile_read(ctx, reset=True)
    plan.close()
    return {"workload": w.name, "method": method, "tones": K, "chunks": n_chunks, "retunes": len(events),
            "kernels_avg_ms": {k: v[1] / max(1, v[0]) for k, v in stats.items()},
            "p50_chunk_ms": float(np.percentile(lat, 50)), "p99_chunk_ms": float(np.percentile(lat, 99)),
            "first_chunk_ms": float(lat[0]), "max_chunk_ms": float(np.max(lat)),
            "tone_samples_per_s": K * w.chunk / (float(np.mean(lat)) * 1e-3),
            "rtf_mean": chunk_s / (float(np.mean(lat)) * 1e-3), "rtf_p99": chunk_s / (float(np.percentile(lat, 99)) * 1e-3),
            "wall_s": wall}


def method_codes(awg):
    return {"direct": awg.AWG_F_METHOD_DIRECT, "mfma-f16": awg.AWG_F_METHOD_MFMA_F16X3,
            "mfma-bf16": awg.AWG_F_METHOD_MFMA_BF16X3}


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


def roofline_for(method, stats, K, L):
    """Dominant kernel of the step and its algorithmic rate against the MI355X peak."""
    name, (launches, total_ms, _) = max(stats.items(), key=lambda kv: kv[1][1])
    avg_ms = total_ms / launches
    if method == "direct":
        flop = 2.0 * K * L                        # one weighting FMA per tone-sample
        ach = flop / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": name, "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS, "traffic": traffic_for(name),
                "avg_kernel_ms": avg_ms,
                "note": "2 algorithmic flop per tone-sample over the FP32 vector peak; the kernel "
                        "is bound by VALU issue including one v_sin_f32 per tone-sample"}
    kpad = 8 * ((K + 7) // 8)
    flop = 4.0 * K * L                            # two MACs per tone-sample (angle addition)
    issued = 3 * 2.0 * (2 * kpad) * L             # three hi/lo passes over the padded tones
    ach = flop / (avg_ms * 1e-3) / 1e12
    peak = PEAK_MFMA16_TFLOPS
    return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": traffic_for(name), "avg_kernel_ms": avg_ms,
            "issued_tflops": issued / (avg_ms * 1e-3) / 1e12,
            "issued_frac": issued / (avg_ms * 1e-3) / 1e12 / peak,
            "note": "achieved counts 4 algorithmic flop per tone-sample; the hi/lo split "
                    "issues 3x that on the matrix cores (issued_*)"}


def short_requests_leg(torch, awg, w, codes, reps=20):
    """Static requests shorter than the 2^24-sample period (2^16 .. 2^22 samples from
    a moving n0) on each method: wall clock per call, streams of back-to-back calls."""
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
        log("short %8d samples: direct %.3f  bf16 %.3f  f16 %.3f ms" % (
            count, row["direct"]["ms_per_call"], row["mfma-bf16"]["ms_per_call"], row["mfma-f16"]["ms_per_call"]))
        rows.append(row)
    return {"tones": K, "timing": "host wall clock over %d back-to-back calls per size" % reps, "rows": rows}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the synthesis runs on a single MI355X; "
              "--gpus %d is not supported" % a.gpus,
              file=sys.stderr)
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
    w = W.static_period(K=a.static_tones)
    K, L = len(w.tones), w.count
    codes = method_codes(awg)
    # auto: BF16 hi/lo x3, the fastest method that keeps the int16 bar (it issues the
    # same matrix instructions as FP16 but holds a higher clock under load); the
    # other two are timed on the same buffer and reported under "methods"
    primary = "mfma-bf16" if a.method == "auto" else a.method
    order = [primary] + [m for m in ("direct", "mfma-f16", "mfma-bf16") if m != primary]
    ctx = awg.context(0)
    out = torch.empty(L, dtype=torch.int16, device="cuda")
    per_method = {}
    res = None
    for m in order:
        plan = awg.Plan(w.tones, w.fs_hz, w.gain_lsb, w.period_log2, codes[m])

        def step():
            plan.synth_static(0, L, out=out)

        is_primary = m == primary
        if is_primary:
            # bring the clocks up: at least ~0.3 s of the step before timing
            t0 = time.perf_counter()
            n = 0
            while n < a.warmup or time.perf_counter() - t0 < 0.3:
                step()
                n += 1
                if n % 8 == 0:
                    torch.cuda.synchronize()
            torch.cuda.synchronize()
            awg.awg_profile_read(ctx, reset=True)
            awg.awg_profile_enable(ctx, max(1, a.time_every))
            ms, wall = timed_steps(torch, step, a.steps, 0)
            awg.awg_profile_enable(ctx, False)
            stats = awg.awg_profile_read(ctx, reset=True)
        else:
            ms, wall = timed_steps(torch, step, max(3, a.steps // 2), 1)
        per_method[m] = {"ms_per_step": ms, "tone_samples_per_s": K * L / (ms * 1e-3)}
        log("%-9s ms/step %.3f  tone-samples/s %.3e" % (m, ms, K * L / (ms * 1e-3)))
        if is_primary:
            q_gpu = out.cpu().numpy()
            value = K * L / (ms * 1e-3)
            res = {"metric": METRIC, "value": value, "unit": "tone-samples/s", "n_gpus": 1,
                   "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True,
                   "scaling": "weak", "vs_baseline": None,
                   "dtype": "f32" if m == "direct" else ("f16x3" if m == "mfma-f16" else "bf16x3"),
                   "data": "synthetic",
                   "config": {"workload": w.name, "tones": K, "samples": L, "fs_hz": w.fs_hz,
                              "method": m, "output": "int16"},
                   "rtf": (L / w.fs_hz) / (ms * 1e-3),
                   "roofline": roofline_for(m, stats, K, L),
                   "kernels": {k: {"launches": v[0], "avg_ms": v[1] / max(1, v[0])}
                               for k, v in stats.items()},
                   "kernel_timing": "HIP events recorded by the dispatch of one launch in %d of each "
                                    "kernel inside the timed steps (launches = timed launches)"
                                    % max(1, a.time_every)}
        plan.close()
    res["methods"] = per_method
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(w, q_gpu, a.cpu_seconds)
    legs = set() if a.no_stream else set(x for x in a.legs.split(",") if x)
    if "stream" in legs:
        log("streaming leg ...")
        res["streaming"] = streaming_leg(torch, awg, W, a.stream_shape)
    if "arrays" in legs:
        log("large-array legs ...")
        res["large_arrays"] = [large_array_leg(torch, awg, W, int(K), m) for K in a.arrays_tones.split(",")
                               for m in a.arrays_methods.split(",")]
    if "short" in legs:
        log("short-request leg ...")
        res["short_requests"] = short_requests_leg(torch, awg, w, codes)
    if "serve" in legs:
        log("serving leg ...")
        res["serving"] = serving_leg(W, a.serve_seconds, a.serve_rate)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
