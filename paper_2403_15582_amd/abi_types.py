"""Plain declarations mirrored from ``include/awg.h``: status codes, ramp shapes,
flags and the ``awg_tone`` record layout.

Nothing here computes anything; it only names the constants and the packed
record that crosses the C boundary, so that input generators, the binding and
tests agree on one layout.
"""
import numpy as np

# awg_status
AWG_OK = 0
AWG_E_INVALID = -1
AWG_E_NOMEM = -2
AWG_E_HIP = -3
AWG_E_RANGE = -4
AWG_E_UNSUPPORTED = -5
AWG_E_BUSY = -6

# awg_ramp: frequency trajectory of a tone inside its ramp window
RAMP_NONE = 0      # static tone, f_end ignored
RAMP_LINEAR = 1    # f(tau) = f0 + df * tau
RAMP_COSINE = 2    # f(tau) = f0 + df * (1 - cos(pi tau)) / 2
RAMP_MINJERK = 3   # f(tau) = f0 + df * (10 tau^3 - 15 tau^4 + 6 tau^5)

RAMP_NAMES = {RAMP_NONE: "none", RAMP_LINEAR: "linear", RAMP_COSINE: "cosine",
              RAMP_MINJERK: "minjerk"}

# awg_plan_params.flags: static-synthesis method (bits 0-1)
AWG_F_METHOD_DIRECT = 0
AWG_F_METHOD_MFMA_F16X3 = 1
AWG_F_METHOD_MFMA_BF16X3 = 2
AWG_F_METHOD_MASK = 3

# One tone, 56 bytes, same field order and alignment as ``awg_tone``.
TONE_DTYPE = np.dtype([
    ("f_start_hz", "<f8"),
    ("f_end_hz", "<f8"),
    ("amplitude", "<f8"),
    ("phase_turns", "<f8"),
    ("ramp_start", "<u8"),
    ("ramp_len", "<u8"),
    ("ramp", "<i4"),
    ("reserved", "<i4"),
])
assert TONE_DTYPE.itemsize == 56


def make_tones(n):
    """Zero-initialised tone array of length ``n`` (all static)."""
    return np.zeros(int(n), dtype=TONE_DTYPE)
