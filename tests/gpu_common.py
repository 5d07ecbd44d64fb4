"""Shared helpers of the GPU parity tests (device buffers via torch, the oracle
on the CPU). Every comparison prints what it checks before touching the GPU."""
import sys

import numpy as np
import pytest

TOL_Q = 1            # int16 codes: |q_gpu - q_oracle| <= 1 LSB
TOL_Y = 0.25         # unquantised sum: |y_gpu - y_oracle| <= 0.25 LSB (FP32 path)


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def compare(q_gpu, y_gpu, q_ora, y_ora, what, tol_y=TOL_Y):
    dq = np.abs(q_gpu.astype(np.int32) - q_ora.astype(np.int32))
    msg = "%s: max|dq|=%d (n>0: %d of %d)" % (what, int(dq.max()) if dq.size else 0,
                                               int((dq > 0).sum()), dq.size)
    if y_gpu is not None:
        dy = np.abs(y_gpu.astype(np.float64) - y_ora)
        msg += " max|dy|=%.4f LSB" % (float(dy.max()) if dy.size else 0.0)
        assert float(dy.max()) <= tol_y, msg
    say(msg)
    assert int(dq.max()) <= TOL_Q, msg
    return msg
