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
# unit roundoff of the iterate's precision
EPS = {"f32": 2.0 ** -24, "f64": 2.0 ** -53, "bf16": 2.0 ** -24}


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


def assert_close(a, b, tol, what="", scale=None, eps=0.0):
    """Agreement both norm-wise and element by element:
    ||a - b||_2 <= tol ||b||_2 and max |a - b| <= tol max |b|.  The second
    bound keeps a few wrong cells from hiding inside a large field's norm.
    When a and b are increments of a field `scale` held in a precision of
    unit roundoff `eps`, the rounding of that field, 8 eps ||scale|| (and
    8 eps max |scale|), is allowed on top."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a - b
    nb = float(np.linalg.norm(b))
    mb = float(np.abs(b).max()) if b.size else 0.0
    f2 = finf = 0.0
    if scale is not None:
        f2 = 8.0 * eps * float(np.linalg.norm(scale))
        finf = 8.0 * eps * float(np.abs(scale).max())
    e2n = float(np.linalg.norm(d))
    einfn = float(np.abs(d).max(initial=0.0))
    e2 = e2n / nb if nb > 0 else e2n
    einf = einfn / mb if mb > 0 else einfn
    ok = e2n <= tol * nb + f2 and einfn <= tol * mb + finf
    assert ok, (f"{what} rel2 {e2:.3e} relinf {einf:.3e} tol {tol:.1e} "
                f"(rounding allowance {f2 / max(nb, 1e-300):.1e} / {finf / max(mb, 1e-300):.1e})")
    return max(e2, einf)


def say(msg):
    print(msg, flush=True)
