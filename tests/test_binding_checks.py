"""The Python binding checks every array argument (dtype, element count,
contiguity, device) against the handle before it calls into libgmg.so: the
kernels cannot see the size of a buffer, so a short or mistyped one would be
read and written past its end.  CPU-only: a stub library stands in after the
parameters are made, and fails the test if any call gets through."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2607_07687_amd import gmg as G  # noqa: E402


class _NoCalls:
    """Library stand-in: any attribute access means a call got through."""

    def __getattr__(self, name):
        raise AssertionError(f"{name} was called despite a bad argument")


@pytest.fixture
def stub(monkeypatch):
    G.load()  # the real library: builds the parameter structs
    yield lambda: monkeypatch.setattr(G, "load", lambda: _NoCalls())


class _FakeHandle(G.Handle):
    """A handle that owns nothing: its pointer never reaches the library."""

    def close(self):
        self._ptr = None


class _FakeBatch(G.Batch):
    def close(self):
        self._ptr = None


def _handle(n, dtype, cycle_dtype=None, l_storage=None, shapes=None):
    p = G.gmg_default_params(n, (False, False, False), dtype,
                             **({} if cycle_dtype is None else {"cycle_dtype": cycle_dtype}),
                             **({} if l_storage is None else {"l_storage": l_storage}))
    return _FakeHandle(ctypes.c_void_p(1), p, None, torch.device("cuda", 0),
                       shapes or [tuple(n)])


def _raises(match, f, *a, **kw):
    with pytest.raises(ValueError, match=match):
        f(*a, **kw)


def test_solve_rejects_wrong_size_and_dtype(stub):
    h = _handle((8, 8, 8), G.GMG_F32)
    stub()
    good = torch.zeros(512, dtype=torch.float32)
    _raises("512 elements", G.gmg_solve, h, torch.zeros(511), good, 1e-6, 5)
    _raises("512 elements", G.gmg_solve, h, good, torch.zeros(600), 1e-6, 5)
    _raises("torch.float32", G.gmg_solve, h, torch.zeros(512, dtype=torch.float64), good, 1e-6, 5)
    _raises("GPU tensor", G.gmg_solve, h, good, good, 1e-6, 5)
    _raises("GPU tensor", G.gmg_vcycle, h, good, good)
    _raises("512 elements", G.gmg_pcg, h, torch.zeros(8), good, 1e-6, 5)
    _raises("512 elements", G.gmg_autotune, h, good, torch.zeros(1))


def test_refinement_needs_float64_of_the_level0_size(stub):
    h = _handle((8, 8, 4), G.GMG_F64, cycle_dtype=G.GMG_F32)
    stub()
    x32 = torch.zeros(256, dtype=torch.float32)
    x64 = torch.zeros(256, dtype=torch.float64)
    _raises("torch.float64", G.gmg_solve_ir, h, x32, x64)
    _raises("256 elements", G.gmg_solve_ir, h, x64, torch.zeros(255, dtype=torch.float64))
    # whole-solve calls take the caller's dtype (F64 here; the library then
    # refuses F64 arrays with F32 cycles), the level calls the cycle dtype
    _raises("torch.float64", G.gmg_residual, h, x32, x64)
    _raises("torch.float64", G.gmg_solve, h, x32, x32, 1e-6, 5)
    _raises("torch.float32", G.gmg_smooth, h, 0, x64, x64, 2)


def test_level_calls_check_each_level_shape(stub):
    h = _handle((16, 8, 8), G.GMG_F32, shapes=[(16, 8, 8), (8, 4, 4), (4, 4, 4)])
    stub()
    f0 = torch.zeros(16 * 8 * 8)
    f1 = torch.zeros(8 * 4 * 4)
    _raises("128 elements", G.gmg_smooth, h, 1, f0, f1, 2)
    _raises("1024 elements", G.gmg_restrict_residual, h, 0, f1, f0, f1)
    _raises("64 elements", G.gmg_restrict_residual, h, 1, f1, f1, f1, f0)
    _raises("128 elements", G.gmg_prolong_correct, h, 0, f0, f0)
    _raises("out of range", G.gmg_smooth, h, 3, f0, f0, 1)
    _raises("out of range", G.gmg_restrict_residual, h, 2, torch.zeros(64), torch.zeros(64),
            torch.zeros(64))
    _raises("GPU tensor", G.gmg_smooth, h, 1, f1, f1.clone(), 2)


def test_level_faces_checks_storage_width(stub):
    h = _handle((8, 8, 8), G.GMG_F32, l_storage=G.GMG_BF16)
    stub()
    _raises("2-byte", G.gmg_level_faces, h, 0, torch.zeros(3 * 512, dtype=torch.float32))
    _raises("1536 elements", G.gmg_level_faces, h, 0, torch.zeros(512, dtype=torch.int16))
    _raises("GPU tensor", G.gmg_level_faces, h, 0, torch.zeros(3 * 512, dtype=torch.int16))


def test_setup_checks_faces(stub):
    p = G.gmg_default_params((8, 8, 8), (False, False, False), G.GMG_F64)
    stub()
    _raises("1536 elements", G.gmg_setup, p, torch.zeros(512, dtype=torch.float64))
    with pytest.raises(TypeError):
        G.gmg_setup(p, torch.zeros(1536, dtype=torch.float32))


def test_batch_checks_every_problem(stub):
    ps = [G.gmg_default_params(n, (False, False, False), G.GMG_F64, cycle_dtype=G.GMG_F32)
          for n in ((8, 8, 8), (16, 8, 8))]
    stub()
    L = [torch.zeros(3 * 512, dtype=torch.float64), torch.zeros(3 * 512, dtype=torch.float64)]
    _raises(r"L\[1\] must have 3072 elements", G.gmg_batch_setup, ps, L)
    b = _FakeBatch(ctypes.c_void_p(1), 2, None, [512, 1024], torch.device("cuda", 0))
    xs = [torch.zeros(512, dtype=torch.float64), torch.zeros(1024, dtype=torch.float64)]
    bad = [torch.zeros(512, dtype=torch.float64), torch.zeros(512, dtype=torch.float64)]
    _raises(r"x\[1\] must have 1024", G.gmg_batch_solve_ir, b, bad, xs)
    _raises(r"sigma\[0\] must be torch.float64", G.gmg_batch_solve_ir, b, xs,
            [torch.zeros(512, dtype=torch.float32), xs[1]])
    _raises("GPU tensor", G.gmg_batch_solve_ir, b, xs, xs)


def test_contiguity_is_checked(stub):
    h = _handle((8, 8, 8), G.GMG_F32)
    stub()
    t = torch.zeros(1024)[::2]
    assert t.numel() == 512 and not t.is_contiguous()
    _raises("contiguous", G.gmg_solve, h, t, torch.zeros(512), 1e-6, 5)
    assert np.prod(h.shapes[0]) == 512
