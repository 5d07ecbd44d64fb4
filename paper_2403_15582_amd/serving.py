"""Client side of the batched server: replay an arrival trace against it.

The server (``awg_server_*`` in the library) does admission, batching and the
synthesis; this module only submits jobs when their arrival time comes, drains
completed chunks from the ring (optionally copying chosen jobs' samples to the
host for checking) and hands the slots back, playing the part of the DAC.
"""
import time

import numpy as np

from . import (awg_server_create, awg_server_destroy, awg_server_submit, awg_server_poll,
               awg_server_read, awg_server_release, awg_server_stats_get, AwgError, AWG_E_BUSY,
               context, _live_servers)


class Server:
    def __init__(self, mem_budget_bytes=512 << 20, max_jobs=256, ring_slots=64, chunk_len=1 << 20,
                 max_pending=8192, playout_delay_ms=5.0, device=0):
        self.chunk_len = chunk_len
        self.handle = awg_server_create(context(device), mem_budget_bytes, max_jobs, ring_slots,
                                        chunk_len, max_pending, playout_delay_ms)
        _live_servers.add(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self.handle:
            awg_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def stats(self):
        return awg_server_stats_get(self.handle)

    def run_trace(self, jobs, collect=(), time_scale=1.0, timeout_s=120.0, poll_sleep_s=50e-6):
        """Submit `jobs` (objects with arrival_s, fs_hz, tones, n_samples and
        optionally gain_lsb) at arrival_s * time_scale after the start, drain
        every chunk, and return {job index: int16 samples} for the indices in
        `collect`."""
        collect = set(collect)
        out = {k: np.zeros(jobs[k].n_samples, dtype=np.int16) for k in collect}
        start = time.perf_counter()
        nxt, finished = 0, 0
        while finished < len(jobs):
            now = time.perf_counter() - start
            if now > timeout_s:
                raise TimeoutError("trace did not finish in %.0f s (%d of %d jobs)"
                                   % (timeout_s, finished, len(jobs)))
            while nxt < len(jobs) and jobs[nxt].arrival_s * time_scale <= now:
                j = jobs[nxt]
                try:
                    awg_server_submit(self.handle, j.fs_hz, j.tones, j.n_samples,
                                      gain_lsb=getattr(j, "gain_lsb", 0.0), user_tag=nxt)
                except AwgError as e:
                    if e.status == AWG_E_BUSY:
                        break                      # queue full: retry on the next pass
                    raise
                nxt += 1
            evs = awg_server_poll(self.handle)
            for ev in evs:
                k = ev["user_tag"]
                if k in collect:
                    dst = out[k][ev["n0"]:ev["n0"] + ev["count"]]
                    awg_server_read(self.handle, ev["slot"], ev["count"], dst.ctypes.data)
                awg_server_release(self.handle, ev["slot"])
                finished += ev["last"]
            if not evs:
                time.sleep(poll_sleep_s)
        return out
