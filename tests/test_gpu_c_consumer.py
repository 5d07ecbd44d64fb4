"""The C ABI from plain C: tests/c/abi_consumer (C99, only include/awg.h and the
HIP runtime's C API) synthesises 64 static tones one-shot, streamed and on the
matrix cores, checks its own invariants, and writes its tones and direct codes;
here the codes are compared with the oracle for every sample."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import words, csynth
from paper_2403_15582_amd.abi_types import TONE_DTYPE

from gpu_common import need_gpu, say, compare

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "c", "abi_consumer")

TONE = TONE_DTYPE          # the awg_tone record the C program wrote


def test_plain_c_consumer(tmp_path):
    need_gpu()
    assert os.path.exists(BIN), "tests/c/abi_consumer is not built (python -c 'import __graft_entry__ as g; g.build()')"
    out = tmp_path / "codes.bin"
    say("abi_consumer (plain C) -> %s" % out)
    r = subprocess.run([BIN, str(out)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout
    raw = out.read_bytes()
    k, n0, count = np.frombuffer(raw[:12], dtype="<u4")
    tones = np.frombuffer(raw[12:12 + k * TONE.itemsize], dtype=TONE)
    q = np.frombuffer(raw[12 + k * TONE.itemsize:], dtype="<i2")
    assert q.size == count
    op = words.Plan(280e6, 0.0, 16, tones)
    qo, _ = csynth.synth(op, int(n0), int(count))
    compare(q, None, qo, None, "plain C consumer, %d tones x %d samples" % (k, count))
