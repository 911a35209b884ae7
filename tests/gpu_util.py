"""Shared helpers of the GPU parity tests: seeded inputs rounded to the run's
precision and handed identically to the HIP path (through the C ABI) and to
the CPU oracle, plus the comparison metrics."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

# per-V-cycle tolerances: FP32 runs against the FP64 oracle fed the same
# rounded inputs, and FP64 runs
TOL = {"f32": 1e-5, "f64": 1e-11, "bf16": 1e-5}


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def np_dtype(prec):
    return np.float64 if prec == "f64" else np.float32


def rounded(a, prec):
    """Round an FP64 input to the run's array precision (returned as FP64)."""
    return np.asarray(a, dtype=np_dtype(prec)).astype(np.float64)


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np_dtype(prec))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = float(np.linalg.norm(b))
    na = float(np.linalg.norm(a - b))
    if nb == 0.0:
        return na
    return na / nb


def say(msg):
    print(msg, flush=True)
