"""ctypes front end of the C oracle (``synth.c``).

TEST INFRASTRUCTURE (see the package docstring). ``build()`` compiles synth.c
with gcc into ``oracle/_synth.so``; ``synth()`` packs a ``words.Plan`` into the
C records and runs the FP64 direct sum with OpenMP.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import words

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "_synth.so")


class _Ramp(ctypes.Structure):
    _fields_ = [("a", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("p_line", ctypes.c_uint64), ("f_line", ctypes.c_uint64),
                ("p_after", ctypes.c_uint64), ("f_after", ctypes.c_uint64),
                ("coef", ctypes.c_int64), ("table", ctypes.c_void_p),
                ("shape", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Amp(ctypes.Structure):
    _fields_ = [("b", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("a_from", ctypes.c_double), ("a_to", ctypes.c_double),
                ("shape", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Tone(ctypes.Structure):
    _fields_ = [("p0", ctypes.c_uint64), ("f0", ctypes.c_uint64), ("amp", ctypes.c_double),
                ("first_ramp", ctypes.c_int32), ("n_ramps", ctypes.c_int32),
                ("first_amp", ctypes.c_int32), ("n_amps", ctypes.c_int32)]


def build(force=True):
    """Compile synth.c (gcc, C99, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", "-Wall", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_synth.argtypes = [ctypes.POINTER(_Tone), ctypes.c_int32, ctypes.POINTER(_Ramp),
                                     ctypes.POINTER(_Amp), ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int32]
        lib.oracle_synth.restype = None
        lib.oracle_phases.argtypes = [ctypes.POINTER(_Tone), ctypes.POINTER(_Ramp), ctypes.c_uint64,
                                      ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_phases.restype = None
        lib.oracle_synth_at.argtypes = [ctypes.POINTER(_Tone), ctypes.c_int32, ctypes.POINTER(_Ramp),
                                        ctypes.POINTER(_Amp), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32]
        lib.oracle_amp_at.argtypes = [ctypes.POINTER(_Tone), ctypes.POINTER(_Amp), ctypes.c_uint64]
        lib.oracle_amp_at.restype = ctypes.c_double
        lib.oracle_synth_at.restype = None
        _lib = lib
    return _lib


class Packed:
    """A Plan flattened into C records; keeps the tables alive."""

    def __init__(self, plan):
        n_ramps = sum(len(t.ramps) for t in plan.tones)
        n_amps = sum(len(t.amp_ramps) for t in plan.tones)
        self.tones = (_Tone * max(1, len(plan.tones)))()
        self.ramps = (_Ramp * max(1, n_ramps))()
        self.amps = (_Amp * max(1, n_amps))()
        self.keep = []
        j = 0
        i = 0
        for k, t in enumerate(plan.tones):
            ct = self.tones[k]
            ct.p0, ct.f0, ct.amp = t.p0, t.f0, t.amp
            ct.first_amp, ct.n_amps = i, len(t.amp_ramps)
            for r in t.amp_ramps:
                ca = self.amps[i]
                ca.b, ca.m, ca.a_from, ca.a_to, ca.shape = r.b, r.M, r.a_from, r.a_to, r.shape
                i += 1
            ct.first_ramp, ct.n_ramps = j, len(t.ramps)
            for r in t.ramps:
                cr = self.ramps[j]
                cr.a, cr.n = r.a, r.N
                cr.p_line, cr.f_line = r.p_line, r.f_line
                cr.p_after, cr.f_after = r.p_after, r.f_after
                cr.coef, cr.shape = r.coef, r.shape
                if r.shape in words.SMOOTH_SHAPES:
                    tab = r.table if r.table is not None else words.ramp_table(r.shape, r.N)
                    tab = np.ascontiguousarray(tab, dtype=np.uint64)
                    self.keep.append(tab)
                    cr.table = tab.ctypes.data
                j += 1
        self.n_tones = len(plan.tones)


def synth(plan, n0, count, threads=0, packed=None):
    """(q int16[count], y float64[count]) for samples n0 .. n0+count-1."""
    lib = _load()
    pk = packed if packed is not None else Packed(plan)
    q = np.empty(int(count), dtype=np.int16)
    y = np.empty(int(count), dtype=np.float64)
    lib.oracle_synth(pk.tones, pk.n_tones, pk.ramps, pk.amps, int(n0), int(count),
                     q.ctypes.data, y.ctypes.data, int(threads))
    return q, y


def synth_at(plan, ns, threads=0, packed=None):
    """(q, y) at the absolute sample indices ``ns``."""
    lib = _load()
    pk = packed if packed is not None else Packed(plan)
    ns = np.ascontiguousarray(ns, dtype=np.uint64)
    q = np.empty(len(ns), dtype=np.int16)
    y = np.empty(len(ns), dtype=np.float64)
    lib.oracle_synth_at(pk.tones, pk.n_tones, pk.ramps, pk.amps, ns.ctypes.data, len(ns),
                        q.ctypes.data, y.ctypes.data, int(threads))
    return q, y


def sparse_tables(plan, ns):
    """Give every smooth ramp without a table one that holds only the entries
    the samples ``ns`` read (computed exactly by words.ramp_table_entries);
    lets the C sum run at sampled points of very long ramps."""
    ns = np.asarray(ns, dtype=np.int64)
    for tw in plan.tones:
        for r in tw.ramps:
            if r.shape not in words.SMOOTH_SHAPES:
                continue
            if r.table is not None and not getattr(r, "sparse", False):
                continue
            ds = ns - r.a
            ds = np.unique(ds[(ds >= 0) & (ds <= r.N)])
            key = (r.shape, r.N)
            cache = plan.__dict__.setdefault("_sparse", {})
            if key not in cache:
                cache[key] = (np.zeros(r.N + 1, dtype=np.uint64), set())
            tab, have = cache[key]
            need = [int(d) for d in ds if int(d) not in have]
            if need:
                tab[need] = words.ramp_table_entries(r.shape, r.N, need)
                have.update(need)
            r.table = tab
            r.sparse = True


def amps_at(plan, k, ns, packed=None):
    """Amplitude of tone k at the absolute samples ``ns`` from the C evaluator."""
    lib = _load()
    pk = packed if packed is not None else Packed(plan)
    tone = ctypes.pointer(pk.tones[k])
    return np.array([lib.oracle_amp_at(tone, pk.amps, int(n)) for n in ns], dtype=np.float64)


def phases(plan, k, n0, count, packed=None):
    """Exact phase words of tone k for samples n0 .. n0+count-1 (uint64)."""
    lib = _load()
    pk = packed if packed is not None else Packed(plan)
    out = np.empty(int(count), dtype=np.uint64)
    tone = ctypes.pointer(pk.tones[k])
    lib.oracle_phases(tone, pk.ramps, int(n0), int(count), out.ctypes.data)
    return out
