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


def assert_close(a, b, tol, what=""):
    """Agreement both norm-wise and element by element:
    ||a - b||_2 <= tol ||b||_2 and max |a - b| <= tol max |b|.  The second
    bound keeps a few wrong cells from hiding inside a large field's norm."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    e2 = rel(a, b)
    mb = float(np.abs(b).max()) if b.size else 0.0
    einf = float(np.abs(a - b).max()) / mb if mb > 0 else float(np.abs(a - b).max(initial=0.0))
    assert e2 <= tol and einf <= tol, f"{what} rel2 {e2:.3e} relinf {einf:.3e} tol {tol:.1e}"
    return max(e2, einf)


def say(msg):
    print(msg, flush=True)
