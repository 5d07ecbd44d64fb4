"""MI355X-native multi-tone additive synthesis (arXiv 2403.15582 hot path).

Python binding of ``libawg.so`` (declared in ``include/awg.h``). The functions
named ``awg_*`` mirror the C entry points one to one and only marshal
arguments: every step of the synthesis runs in the library's HIP kernels.
Device buffers are passed as integer device pointers (e.g. a torch tensor's
``data_ptr()``) and streams as ``hipStream_t`` integers (``torch.cuda.Stream
.cuda_stream``); ``Plan`` adds a little convenience on top for callers that use
torch for device memory.

The library must have been built (``python -m paper_2403_15582_amd.build``);
importing a function when it is missing raises ``ImportError`` -- there is no
fallback implementation.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

from .abi_types import (AWG_OK, AWG_E_INVALID, AWG_E_NOMEM, AWG_E_HIP, AWG_E_RANGE,  # noqa: F401
                        AWG_E_UNSUPPORTED, AWG_E_BUSY, RAMP_NONE, RAMP_LINEAR, RAMP_COSINE,
                        RAMP_MINJERK, AWG_F_METHOD_DIRECT, AWG_F_METHOD_MFMA_F16X3,
                        AWG_F_METHOD_MFMA_BF16X3, TONE_DTYPE, make_tones)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libawg.so")

EXPORTED = [
    "awg_ctx_create", "awg_ctx_destroy", "awg_plan_tones", "awg_plan_destroy",
    "awg_plan_info_get", "awg_plan_words", "awg_ramp_table", "awg_plan_retune", "awg_plan_amplitude",
    "awg_plan_reserve",
    "awg_synth_static", "awg_synth_chirp", "awg_stream_next", "awg_stream_seek",
    "awg_stream_tell", "awg_synth_f32", "awg_synth_multiplex", "awg_stream_next_multiplex",
    "awg_phase_dump", "awg_phase_plan", "awg_phase_search", "awg_peak", "awg_peak_noalloc", "awg_strerror",
    "awg_version",
    "awg_profile_enable", "awg_profile_read",
    "awg_server_create", "awg_server_destroy", "awg_server_submit", "awg_server_poll",
    "awg_server_slot", "awg_server_read", "awg_server_release", "awg_server_stats_get",
]


class AwgError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, awg_strerror(status), status))


class awg_plan_params(ctypes.Structure):
    _fields_ = [("fs_hz", ctypes.c_double), ("gain_lsb", ctypes.c_double),
                ("period_log2", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class awg_plan_info(ctypes.Structure):
    _fields_ = [("n_tones", ctypes.c_int32), ("n_ramped", ctypes.c_int32),
                ("gain_lsb", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("period_log2", ctypes.c_uint32), ("cursor", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64)]


class awg_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("work", ctypes.c_double)]


class awg_server_params(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_jobs", ctypes.c_int32),
                ("ring_slots", ctypes.c_int32), ("chunk_len", ctypes.c_uint32),
                ("max_pending", ctypes.c_int32), ("playout_delay_ms", ctypes.c_double)]


class awg_job(ctypes.Structure):
    _fields_ = [("fs_hz", ctypes.c_double), ("gain_lsb", ctypes.c_double),
                ("period_log2", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("tones", ctypes.c_void_p), ("n_tones", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("n_samples", ctypes.c_uint64), ("user_tag", ctypes.c_uint64)]


class awg_chunk_event(ctypes.Structure):
    _fields_ = [("job_id", ctypes.c_uint64), ("user_tag", ctypes.c_uint64),
                ("chunk_index", ctypes.c_uint64), ("n0", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("slot", ctypes.c_int32), ("last", ctypes.c_int32),
                ("t_submit_ms", ctypes.c_double), ("t_ready_ms", ctypes.c_double)]


class awg_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("jobs_submitted", "jobs_admitted", "jobs_done",
                                               "jobs_pending", "jobs_active", "chunks_done", "steps",
                                               "max_batch")] + \
               [(n, ctypes.c_double) for n in ("mean_batch", "tone_samples", "audio_seconds",
                                               "device_busy_ms", "wall_ms", "chunk_latency_p50_ms",
                                               "chunk_latency_p99_ms", "first_chunk_latency_p50_ms",
                                               "first_chunk_latency_p99_ms")] + \
               [("deadline_misses", ctypes.c_uint64), ("pool_free_bytes", ctypes.c_uint64),
                ("lateness_p50_ms", ctypes.c_double), ("lateness_p99_ms", ctypes.c_double)]


class awg_retune(ctypes.Structure):
    _fields_ = [("tone", ctypes.c_int32), ("ramp", ctypes.c_int32),
                ("ramp_start", ctypes.c_uint64), ("ramp_len", ctypes.c_uint64),
                ("f_end_hz", ctypes.c_double)]


class awg_amp_ramp(ctypes.Structure):
    _fields_ = [("tone", ctypes.c_int32), ("ramp", ctypes.c_int32),
                ("ramp_start", ctypes.c_uint64), ("ramp_len", ctypes.c_uint64),
                ("amplitude_end", ctypes.c_double)]


_lib = None
_exiting = False
_VP = ctypes.c_void_p
# objects that own library handles, closed in a fixed order at interpreter exit
_live_servers = weakref.WeakSet()
_live_plans = weakref.WeakSet()


@atexit.register
def _teardown():
    """Release every library object still alive at interpreter exit while the
    HIP runtime is still fully up (Python's exit handlers all run before the
    process's C-level exit, where the runtime tears down): servers first (their
    scheduler threads launch work), then plans, then the cached contexts
    (which synchronise their device before freeing). Finalizers that run
    later see _exiting and do nothing."""
    global _exiting
    if _exiting:
        return
    try:
        for s in list(_live_servers):
            s.close()
        for p in list(_live_plans):
            p.close()
        for dev in list(_ctx_cache):
            awg_ctx_destroy(_ctx_cache.pop(dev))
    finally:
        _exiting = True

_U64 = ctypes.c_uint64
_I32 = ctypes.c_int32


def lib():
    """The loaded libawg (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libawg.so is not built; run python -m paper_2403_15582_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "awg_ctx_create": ([ctypes.c_int, ctypes.POINTER(_VP)], _I32),
        "awg_ctx_destroy": ([_VP], None),
        "awg_plan_tones": ([_VP, ctypes.POINTER(awg_plan_params), _VP, _I32, ctypes.POINTER(_VP), _VP], _I32),
        "awg_plan_destroy": ([_VP], None),
        "awg_plan_info_get": ([_VP, ctypes.POINTER(awg_plan_info)], _I32),
        "awg_plan_words": ([_VP, _VP, _VP, _VP, _VP], _I32),
        "awg_ramp_table": ([_I32, _U64, _VP], _I32),
        "awg_plan_retune": ([_VP, ctypes.POINTER(awg_retune), _I32, _VP], _I32),
        "awg_plan_amplitude": ([_VP, ctypes.POINTER(awg_amp_ramp), _I32, _VP], _I32),
        "awg_plan_reserve": ([_VP, ctypes.c_uint32, _U64], _I32),
        "awg_synth_static": ([_VP, _U64, _U64, _VP, _VP], _I32),
        "awg_synth_chirp": ([_VP, _U64, _U64, _VP, _VP], _I32),
        "awg_stream_next": ([_VP, _U64, _VP, _VP, ctypes.POINTER(_U64)], _I32),
        "awg_stream_seek": ([_VP, _U64], _I32),
        "awg_stream_tell": ([_VP, ctypes.POINTER(_U64)], _I32),
        "awg_synth_f32": ([_VP, ctypes.c_uint32, _U64, _U64, _VP, _VP], _I32),
        "awg_synth_multiplex": ([ctypes.POINTER(_VP), _I32, _U64, _U64, _VP, _VP], _I32),
        "awg_stream_next_multiplex": ([ctypes.POINTER(_VP), _I32, _U64, _VP, _VP, ctypes.POINTER(_U64)], _I32),
        "awg_phase_dump": ([_VP, _I32, _U64, _U64, _VP, _VP], _I32),
        "awg_phase_plan": ([_I32, _VP, _VP, _I32, _VP], _I32),
        "awg_phase_search": ([_VP, ctypes.c_double, ctypes.c_uint32, _VP, _VP, _I32, _I32, _VP,
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32)], _I32),
        "awg_peak": ([_VP, _U64, _U64, _VP, _VP, _VP], _I32),
        "awg_peak_noalloc": ([_VP, _U64, _U64, _VP, _VP], _I32),
        "awg_profile_enable": ([_VP, _I32], _I32),
        "awg_profile_read": ([_VP, ctypes.POINTER(awg_kernel_stat), _I32, ctypes.POINTER(_I32), _I32], _I32),
        "awg_server_create": ([_VP, ctypes.POINTER(awg_server_params), ctypes.POINTER(_VP)], _I32),
        "awg_server_destroy": ([_VP], _I32),
        "awg_server_submit": ([_VP, ctypes.POINTER(awg_job), ctypes.POINTER(_U64)], _I32),
        "awg_server_poll": ([_VP, ctypes.POINTER(awg_chunk_event), _I32, ctypes.POINTER(_I32)], _I32),
        "awg_server_slot": ([_VP, _I32, ctypes.POINTER(_VP)], _I32),
        "awg_server_read": ([_VP, _I32, _U64, _VP], _I32),
        "awg_server_release": ([_VP, _I32], _I32),
        "awg_server_stats_get": ([_VP, ctypes.POINTER(awg_server_stats)], _I32),
        "awg_strerror": ([_I32], ctypes.c_char_p),
        "awg_version": ([], _I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(status, what):
    if status != AWG_OK:
        raise AwgError(status, what)


def awg_strerror(status):
    return lib().awg_strerror(int(status)).decode()


def awg_version():
    return int(lib().awg_version())


def awg_ctx_create(device=0):
    h = _VP()
    _check(lib().awg_ctx_create(int(device), ctypes.byref(h)), "awg_ctx_create")
    return h.value


def awg_ctx_destroy(ctx):
    if ctx:
        lib().awg_ctx_destroy(ctx)


def awg_plan_tones(ctx, fs_hz, gain_lsb, period_log2, flags, tones):
    """Plan ``tones`` (TONE_DTYPE array). Returns (plan handle, quantised Hz)."""
    t = np.ascontiguousarray(tones, dtype=TONE_DTYPE)
    p = awg_plan_params(float(fs_hz), float(gain_lsb), int(period_log2), int(flags))
    fq = np.empty(len(t), dtype=np.float64)
    h = _VP()
    _check(lib().awg_plan_tones(ctx, ctypes.byref(p), t.ctypes.data, len(t), ctypes.byref(h),
                                fq.ctypes.data), "awg_plan_tones")
    return h.value, fq


def awg_plan_destroy(plan):
    if plan:
        lib().awg_plan_destroy(plan)


def awg_plan_info_get(plan):
    info = awg_plan_info()
    _check(lib().awg_plan_info_get(plan, ctypes.byref(info)), "awg_plan_info_get")
    return {f: getattr(info, f) for f, _ in awg_plan_info._fields_}


def awg_plan_words(plan, n_tones):
    out = {k: np.empty(n_tones, dtype=np.uint64) for k in ("p0", "f0", "f1")}
    out["coef"] = np.empty(n_tones, dtype=np.int64)
    _check(lib().awg_plan_words(plan, out["p0"].ctypes.data, out["f0"].ctypes.data,
                                out["f1"].ctypes.data, out["coef"].ctypes.data), "awg_plan_words")
    return out


def awg_ramp_table(shape, n):
    out = np.empty(int(n) + 1, dtype=np.uint64)
    _check(lib().awg_ramp_table(int(shape), int(n), out.ctypes.data), "awg_ramp_table")
    return out


def retune_array(events):
    """ctypes array of awg_retune from (tone, ramp, ramp_start, ramp_len, f_end_hz)
    tuples; awg_plan_retune takes it as is (callers on a hot loop build it once)."""
    ev = list(events)
    arr = (awg_retune * max(1, len(ev)))()
    for i, (k, shape, a, n, f) in enumerate(ev):
        arr[i] = awg_retune(int(k), int(shape), int(a), int(n), float(f))
    arr.n_events = len(ev)
    return arr


def awg_plan_retune(plan, events, stream=0):
    """events: iterable of (tone, ramp, ramp_start, ramp_len, f_end_hz), or an
    array from retune_array."""
    arr = events if hasattr(events, "n_events") else retune_array(events)
    _check(lib().awg_plan_retune(plan, arr, arr.n_events, stream or None), "awg_plan_retune")


def amp_ramp_array(events):
    """ctypes array of awg_amp_ramp from (tone, ramp, ramp_start, ramp_len,
    amplitude_end) tuples."""
    ev = list(events)
    arr = (awg_amp_ramp * max(1, len(ev)))()
    for i, (k, shape, a, n, amp) in enumerate(ev):
        arr[i] = awg_amp_ramp(int(k), int(shape), int(a), int(n), float(amp))
    arr.n_events = len(ev)
    return arr


def awg_plan_amplitude(plan, events, stream=0):
    """events: iterable of (tone, ramp, ramp_start, ramp_len, amplitude_end), or
    an array from amp_ramp_array."""
    arr = events if hasattr(events, "n_events") else amp_ramp_array(events)
    _check(lib().awg_plan_amplitude(plan, arr, arr.n_events, stream or None), "awg_plan_amplitude")


def awg_synth_static(plan, n0, count, d_out, stream=0):
    _check(lib().awg_synth_static(plan, int(n0), int(count), d_out, stream or None), "awg_synth_static")


def awg_plan_reserve(plan, method, max_count):
    _check(lib().awg_plan_reserve(plan, int(method), int(max_count)), "awg_plan_reserve")


def awg_synth_chirp(plan, n0, count, d_out, stream=0):
    _check(lib().awg_synth_chirp(plan, int(n0), int(count), d_out, stream or None), "awg_synth_chirp")


def awg_stream_next(plan, count, d_out, stream=0):
    n0 = _U64()
    _check(lib().awg_stream_next(plan, int(count), d_out, stream or None, ctypes.byref(n0)),
           "awg_stream_next")
    return n0.value


def awg_stream_seek(plan, n0):
    _check(lib().awg_stream_seek(plan, int(n0)), "awg_stream_seek")


def awg_stream_tell(plan):
    n0 = _U64()
    _check(lib().awg_stream_tell(plan, ctypes.byref(n0)), "awg_stream_tell")
    return n0.value


def awg_synth_f32(plan, method, n0, count, d_y, stream=0):
    _check(lib().awg_synth_f32(plan, int(method), int(n0), int(count), d_y, stream or None),
           "awg_synth_f32")


def _plan_array(plans):
    arr = (_VP * max(1, len(plans)))()
    for i, p in enumerate(plans):
        arr[i] = p
    return arr


def awg_synth_multiplex(plans, n0, count, d_out, stream=0):
    """plans: list of plan handles (1..4 channels); d_out holds len(plans)*count int16."""
    _check(lib().awg_synth_multiplex(_plan_array(plans), len(plans), int(n0), int(count), d_out, stream or None),
           "awg_synth_multiplex")


def awg_stream_next_multiplex(plans, count, d_out, stream=0):
    n0 = _U64()
    _check(lib().awg_stream_next_multiplex(_plan_array(plans), len(plans), int(count), d_out, stream or None,
                                           ctypes.byref(n0)), "awg_stream_next_multiplex")
    return n0.value


def current_stream_handle(device, stream=None):
    """The HIP stream handle for a call on `device`: `stream`'s, else that of
    torch's current stream on the device (torch's own raw query, about ten
    times cheaper per call than building a Stream object)."""
    if stream is not None:
        return stream.cuda_stream
    import torch
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return raw(device)
    return torch.cuda.current_stream(device).cuda_stream


def multiplex(plans, n0, count, out=None, stream=None):
    """Channels of `plans` (Plan objects) interleaved into an int16 tensor of
    shape (count, len(plans)): out[i, c] is channel c's sample n0 + i."""
    import torch
    if out is None:
        out = torch.empty((int(count), len(plans)), dtype=torch.int16, device="cuda:%d" % plans[0].device)
    if out.dtype != torch.int16 or not out.is_contiguous() or out.numel() < count * len(plans):
        raise ValueError("out must be a contiguous int16 tensor of at least %d elements" % (count * len(plans)))
    awg_synth_multiplex([p.handle for p in plans], n0, count, out.data_ptr(),
                        current_stream_handle(plans[0].device, stream))
    return out


AWG_PHASES_SCHROEDER, AWG_PHASES_NEWMAN, AWG_PHASES_SEARCH = 1, 2, 3


def awg_phase_plan(method, f_hz, amplitude=None):
    """Closed-form low-crest-factor phases (turns, [0, 1)) for tones at f_hz."""
    f = np.ascontiguousarray(f_hz, dtype=np.float64)
    a = None if amplitude is None else np.ascontiguousarray(amplitude, dtype=np.float64)
    out = np.empty(len(f), dtype=np.float64)
    _check(lib().awg_phase_plan(int(method), f.ctypes.data, None if a is None else a.ctypes.data, len(f),
                                out.ctypes.data), "awg_phase_plan")
    return out


def awg_peak(plan, n0, count, d_scratch, d_peak, stream=0):
    _check(lib().awg_peak(plan, int(n0), int(count), d_scratch, d_peak, stream or None), "awg_peak")


AWG_PEAK_NOALLOC_MAX = 1 << 22


def awg_peak_noalloc(plan, n0, count, d_peak, stream=0):
    _check(lib().awg_peak_noalloc(plan, int(n0), int(count), d_peak, stream or None), "awg_peak_noalloc")



def awg_phase_search(ctx, fs_hz, period_log2, f_hz, amplitude, max_evals=300):
    """Device crest-factor search: (phases in turns, crest factor, method)."""
    f = np.ascontiguousarray(f_hz, dtype=np.float64)
    a = np.ascontiguousarray(amplitude, dtype=np.float64)
    out = np.empty(len(f), dtype=np.float64)
    cf = ctypes.c_double()
    m = _I32()
    _check(lib().awg_phase_search(ctx, float(fs_hz), int(period_log2), f.ctypes.data, a.ctypes.data, len(f),
                                  int(max_evals), out.ctypes.data, ctypes.byref(cf), ctypes.byref(m)),
           "awg_phase_search")
    return out, cf.value, m.value


def plan_phases(tones, fs_hz, period_log2, max_evals=300, device=0):
    """Crest-factor-aware phase planning (awg_phase_search): the closed forms and
    the device search, the lowest measured crest factor wins. Returns
    (phases in turns, crest factor, AWG_PHASES_* of the winner)."""
    return awg_phase_search(context(device), fs_hz, period_log2, tones["f_start_hz"], tones["amplitude"], max_evals)


def awg_phase_dump(plan, tone, n0, count, d_words, stream=0):
    _check(lib().awg_phase_dump(plan, int(tone), int(n0), int(count), d_words, stream or None),
           "awg_phase_dump")


def awg_profile_enable(ctx, enable=True):
    """enable: False / 0 = off, True / 1 = every launch, n = one launch in n per kernel."""
    _check(lib().awg_profile_enable(ctx, int(enable)), "awg_profile_enable")


def awg_profile_read(ctx, reset=False):
    """{kernel name: (launches, total_ms, max_ms, work)} since the last reset;
    work = algorithmic tone-samples of the timed launches."""
    arr = (awg_kernel_stat * 64)()
    n = _I32()
    _check(lib().awg_profile_read(ctx, arr, 64, ctypes.byref(n), 1 if reset else 0), "awg_profile_read")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms, arr[i].max_ms, arr[i].work)
            for i in range(min(n.value, 64))}


def awg_server_create(ctx, mem_budget_bytes, max_jobs, ring_slots, chunk_len=1 << 20, max_pending=4096,
                      playout_delay_ms=5.0):
    p = awg_server_params(int(mem_budget_bytes), int(max_jobs), int(ring_slots), int(chunk_len),
                          int(max_pending), float(playout_delay_ms))
    h = _VP()
    _check(lib().awg_server_create(ctx, ctypes.byref(p), ctypes.byref(h)), "awg_server_create")
    return h.value


def awg_server_destroy(srv):
    if srv:
        _check(lib().awg_server_destroy(srv), "awg_server_destroy")


def awg_server_submit(srv, fs_hz, tones, n_samples, gain_lsb=0.0, period_log2=0, user_tag=0):
    t = np.ascontiguousarray(tones, dtype=TONE_DTYPE)
    j = awg_job(float(fs_hz), float(gain_lsb), int(period_log2), 0, t.ctypes.data, len(t), 0,
                int(n_samples), int(user_tag))
    jid = _U64()
    _check(lib().awg_server_submit(srv, ctypes.byref(j), ctypes.byref(jid)), "awg_server_submit")
    return jid.value


def awg_server_poll(srv, max_events=256):
    arr = (awg_chunk_event * max_events)()
    n = _I32()
    _check(lib().awg_server_poll(srv, arr, max_events, ctypes.byref(n)), "awg_server_poll")
    return [{f: getattr(arr[i], f) for f, _ in awg_chunk_event._fields_} for i in range(n.value)]


def awg_server_slot(srv, slot):
    p = _VP()
    _check(lib().awg_server_slot(srv, int(slot), ctypes.byref(p)), "awg_server_slot")
    return p.value


def awg_server_read(srv, slot, count, dst):
    _check(lib().awg_server_read(srv, int(slot), int(count), dst), "awg_server_read")


def awg_server_release(srv, slot):
    _check(lib().awg_server_release(srv, int(slot)), "awg_server_release")


def awg_server_stats_get(srv):
    st = awg_server_stats()
    _check(lib().awg_server_stats_get(srv, ctypes.byref(st)), "awg_server_stats_get")
    return {f: getattr(st, f) for f, _ in awg_server_stats._fields_}


# ------------------------------------------------------------ convenience

_ctx_cache = {}


def context(device=0):
    """A process-wide context per device (created on first use)."""
    if device not in _ctx_cache:
        _ctx_cache[device] = awg_ctx_create(device)
    return _ctx_cache[device]


class Plan:
    """Owns a plan handle; outputs are torch tensors on the plan's device."""

    def __init__(self, tones, fs_hz, gain_lsb=0.0, period_log2=0, method=AWG_F_METHOD_DIRECT,
                 device=0, host_only=False):
        self.device = device
        ctx = None if host_only else context(device)
        self.tones = np.ascontiguousarray(tones, dtype=TONE_DTYPE)
        self.method = method
        self.handle, self.f_quantised_hz = awg_plan_tones(ctx, fs_hz, gain_lsb, period_log2, method,
                                                          self.tones)
        self.n_tones = len(self.tones)
        _live_plans.add(self)

    def close(self):
        if self.handle:
            awg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return awg_plan_info_get(self.handle)

    def words(self):
        return awg_plan_words(self.handle, self.n_tones)

    def _out(self, count, dtype, out):
        import torch
        if out is None:
            return torch.empty(int(count), dtype=dtype, device="cuda:%d" % self.device)
        # the kernels write through out.data_ptr(): it must be device memory of
        # this plan's device, of the right type, contiguous and large enough
        if out.device.type != "cuda" or (out.device.index or 0) != self.device:
            raise ValueError("out must be a tensor on cuda:%d, not %s" % (self.device, out.device))
        if out.dtype != dtype or not out.is_contiguous() or out.numel() < count:
            raise ValueError("out must be a contiguous %s tensor of at least %d elements" % (dtype, count))
        return out

    def _stream(self, stream):
        return current_stream_handle(self.device, stream)

    def synth_static(self, n0, count, out=None, stream=None):
        import torch
        out = self._out(count, torch.int16, out)
        awg_synth_static(self.handle, n0, count, out.data_ptr(), self._stream(stream))
        return out

    def synth_chirp(self, n0, count, out=None, stream=None):
        import torch
        out = self._out(count, torch.int16, out)
        awg_synth_chirp(self.handle, n0, count, out.data_ptr(), self._stream(stream))
        return out

    def stream_next(self, count, out=None, stream=None):
        import torch
        out = self._out(count, torch.int16, out)
        n0 = awg_stream_next(self.handle, count, out.data_ptr(), self._stream(stream))
        return n0, out

    def synth_f32(self, n0, count, method=AWG_F_METHOD_DIRECT, out=None, stream=None):
        import torch
        out = self._out(count, torch.float32, out)
        awg_synth_f32(self.handle, method, n0, count, out.data_ptr(), self._stream(stream))
        return out

    def phase_dump(self, tone, n0, count, stream=None):
        import torch
        out = self._out(count, torch.int64, None)
        awg_phase_dump(self.handle, tone, n0, count, out.data_ptr(), self._stream(stream))
        return out

    def retune(self, events, stream=None):
        awg_plan_retune(self.handle, events, self._stream(stream))

    def amplitude(self, events, stream=None):
        """Amplitude ramps: (tone, ramp, ramp_start, ramp_len, amplitude_end) each."""
        awg_plan_amplitude(self.handle, events, self._stream(stream))

    def reserve(self, max_count, method=None):
        """Set up workspaces and staging for calls of up to max_count samples
        (method: the plan's own by default)."""
        m = (self.method if method is None else method)
        awg_plan_reserve(self.handle, m, max_count)

    def seek(self, n0):
        awg_stream_seek(self.handle, n0)

    def tell(self):
        return awg_stream_tell(self.handle)
