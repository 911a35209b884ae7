"""ctypes binding of libgmg.so (C ABI in include/gmg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Functions carry the C names.  Arrays are torch tensors on the GPU (device
memory and streams come from PyTorch); the work is enqueued on torch's
current stream of the tensor's device unless a stream is given.

The library is loaded from this package directory on first use; if it is
missing this raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

LIB_NAME = "libgmg.so"
_HERE = os.path.dirname(os.path.abspath(__file__))

GMG_OK, GMG_EINVAL, GMG_ESHAPE, GMG_ENOMEM, GMG_EHIP, GMG_ENOCONV = range(6)
GMG_F32, GMG_F64, GMG_BF16 = 0, 1, 2
GMG_SMOOTH_RBGS, GMG_SMOOTH_PCG = 0, 1
GMG_MAX_HISTORY = 512
STATUS_NAMES = {0: "GMG_OK", 1: "GMG_EINVAL", 2: "GMG_ESHAPE", 3: "GMG_ENOMEM",
                4: "GMG_EHIP", 5: "GMG_ENOCONV"}


class gmg_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("periodic", ctypes.c_int32 * 3),
                ("dtype", ctypes.c_int32), ("cycle_dtype", ctypes.c_int32),
                ("l_storage", ctypes.c_int32), ("anisotropic", ctypes.c_int32),
                ("min_coarse", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("nu_coarse", ctypes.c_int32), ("rollback", ctypes.c_int32),
                ("graphs", ctypes.c_int32), ("tail_cells", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("deferred_norm", ctypes.c_int32),
                ("pair_sweeps", ctypes.c_int32), ("omega0", ctypes.c_double), ("omega_min", ctypes.c_double),
                ("omega_max", ctypes.c_double), ("theta_dec", ctypes.c_double),
                ("theta_inc", ctypes.c_double), ("coarse_rtol", ctypes.c_double),
                ("coarse_max", ctypes.c_int32), ("ir_target", ctypes.c_double),
                ("uniform_bricks", ctypes.c_int32)]


class gmg_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("accepted_cycles", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("rnorm0", ctypes.c_double), ("rnorm", ctypes.c_double),
                ("snorm", ctypes.c_double), ("omega", ctypes.c_double),
                ("history", ctypes.c_double * GMG_MAX_HISTORY),
                ("omegas", ctypes.c_double * GMG_MAX_HISTORY),
                ("accepted", ctypes.c_int32 * GMG_MAX_HISTORY)]


class gmg_pcg_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("snorm", ctypes.c_double), ("rnorm0", ctypes.c_double),
                ("rnorm", ctypes.c_double), ("history", ctypes.c_double * GMG_MAX_HISTORY)]


class gmg_ir_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("inner_total", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("snorm", ctypes.c_double), ("rnorm", ctypes.c_double),
                ("history", ctypes.c_double * GMG_MAX_HISTORY),
                ("inner_cycles", ctypes.c_int32 * GMG_MAX_HISTORY)]


class gmg_tune_report(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("ty", ctypes.c_int32 * 32),
                ("kchunk", ctypes.c_int32 * 32), ("ty_default", ctypes.c_int32 * 32),
                ("kchunk_default", ctypes.c_int32 * 32), ("us", ctypes.c_double * 32),
                ("us_default", ctypes.c_double * 32), ("pair_kchunk", ctypes.c_int32 * 32),
                ("us_pair", ctypes.c_double * 32), ("pair_ty", ctypes.c_int32 * 32)]


class GMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("gmg_default_params", ctypes.c_int, [ctypes.POINTER(gmg_params)]),
    ("gmg_setup", ctypes.c_int, [ctypes.POINTER(gmg_params), ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("gmg_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("gmg_update_faces", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("gmg_num_levels", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    ("gmg_level_shape", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    ("gmg_level_faces", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    ("gmg_level_uniform", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]),
    ("gmg_residual", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    ("gmg_residual_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("gmg_smooth", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int32]),
    ("gmg_restrict_residual", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    ("gmg_prolong_correct", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    ("gmg_get_omega", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    ("gmg_set_omega", ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    ("gmg_coarse_sweeps", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    ("gmg_vcycle", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_double)]),
    ("gmg_solve", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(gmg_solve_info)]),
    ("gmg_pcg", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_double, ctypes.c_int32, ctypes.POINTER(gmg_pcg_info)]),
    ("gmg_solve_ir", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.POINTER(gmg_ir_info)]),
    ("gmg_batch_setup", ctypes.c_int, [ctypes.POINTER(gmg_params),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("gmg_batch_solve_ir", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                          ctypes.POINTER(gmg_ir_info)]),
    ("gmg_batch_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("gmg_batch_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("gmg_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.POINTER(gmg_tune_report)]),
    ("gmg_set_tiles", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32]),
    ("gmg_set_pair_sweeps", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32]),
    ("gmg_last_error", ctypes.c_char_p, []),
]


def lib_path():
    return os.path.join(_HERE, LIB_NAME)


def load():
    """Load libgmg.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_2607_07687_amd.build` (HIP, gfx950)")
        lib = ctypes.CDLL(path)
        for name, res, args in _SIGS:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return [s[0] for s in _SIGS]


def _check(status):
    if status != GMG_OK:
        raise GMGError(status, load().gmg_last_error().decode())
    return status


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return GMG_F32
    if t.dtype == torch.float64:
        return GMG_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t, what):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _torch_dtype(code):
    """torch dtype of caller arrays in gmg_dtype `code` (BF16: 2-byte raw bits)."""
    import torch
    return {GMG_F32: torch.float32, GMG_F64: torch.float64}.get(code)


def _meta(t, what, numel, dtype, optional=False):
    """dtype (a torch dtype, or an element size in bytes for raw BF16 bits)
    and element count of one tensor argument."""
    import torch
    if t is None:
        if optional:
            return
        raise ValueError(f"{what} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if isinstance(dtype, int):
        if t.element_size() != dtype:
            raise ValueError(f"{what} must have {dtype}-byte elements, got {t.dtype}")
    elif t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")


def _place(t, what, device=None):
    """Contiguity and device of one tensor argument; returns its pointer."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous GPU tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{what} is on {t.device}, the handle on {device}")
    return ctypes.c_void_p(t.data_ptr())


def _args(*specs, device=None):
    """Check tensor arguments before any library call and return their
    pointers.  specs: (tensor, name, numel, dtype[, optional]).  First the
    dtype and element count of every argument, then contiguity and device.
    The library cannot check sizes itself: a short or mistyped buffer would
    be read and written past its end by the kernels."""
    for sp in specs:
        _meta(sp[0], sp[1], sp[2], sp[3], sp[4] if len(sp) > 4 else False)
    return [_place(sp[0], sp[1], device) for sp in specs]


def _arr(t, what, numel, dtype, device=None, optional=False):
    """One checked tensor argument (see _args)."""
    return _args((t, what, numel, dtype, optional), device=device)[0]


def _cells(n):
    return int(n[0]) * int(n[1]) * int(n[2])


def _stream(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def gmg_default_params(n, periodic=(False, False, False), dtype=GMG_F32, **kw):
    """gmg_params with the library defaults, then n, periodic, dtype and any
    field given by keyword.  cycle_dtype and l_storage follow dtype unless
    given."""
    p = gmg_params()
    _check(load().gmg_default_params(ctypes.byref(p)))
    for d in range(3):
        p.n[d] = int(n[d])
        p.periodic[d] = int(bool(periodic[d]))
    p.dtype = dtype
    p.cycle_dtype = kw.pop("cycle_dtype", dtype)
    p.l_storage = kw.pop("l_storage", p.cycle_dtype)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class Handle:
    """Owns a gmg_handle*; destroyed by close() or garbage collection.
    Keeps what the bindings check arrays against: the parameters, the device
    and the cell shape (nx, ny, nz) of every level."""

    def __init__(self, ptr, params, stream, device=None, shapes=None):
        self._ptr = ptr
        self.params = params
        self.stream = stream
        self.device = device
        self.shapes = shapes if shapes is not None else [tuple(params.n)]

    def cells(self, level=0):
        if not 0 <= level < len(self.shapes):
            raise ValueError(f"level {level} out of range (0..{len(self.shapes) - 1})")
        return _cells(self.shapes[level])

    def spec(self, t, what, level=0, cycle=True, optional=False):
        """Check spec (see _args) of a cell array of `level` in the cycle
        precision, or in the caller precision `dtype` if not cycle."""
        code = self.params.cycle_dtype if cycle else self.params.dtype
        return (t, what, self.cells(level), _torch_dtype(code), optional)

    def arrs(self, *specs):
        return _args(*specs, device=self.device)

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("handle is closed")
        return self._ptr

    def close(self):
        if self._ptr is not None:
            load().gmg_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gmg_setup(params, L, stream=None):
    """Build the hierarchy from face coefficients L ([3][nz][ny][nx] tensor in
    params.dtype).  Returns a Handle."""
    if _dtype_code(L) != params.dtype:
        raise TypeError("L dtype does not match params.dtype")
    Lp = _arr(L, "L", 3 * _cells(params.n), _torch_dtype(params.dtype))
    s = _stream(stream, L.device)
    out = ctypes.c_void_p()
    _check(load().gmg_setup(ctypes.byref(params), Lp, s, ctypes.byref(out)))
    h = Handle(out, params, s, L.device)
    h.shapes = [gmg_level_shape(h, l)[0] for l in range(gmg_num_levels(h))]
    return h


def gmg_update_faces(h, L):
    """New face coefficients L ([3][nz][ny][nx] tensor in params.dtype) for
    the handle's hierarchy (same grid)."""
    if _dtype_code(L) != h.params.dtype:
        raise TypeError("L dtype does not match params.dtype")
    Lp = _arr(L, "L", 3 * h.cells(0), _torch_dtype(h.params.dtype), h.device)
    _check(load().gmg_update_faces(h.ptr, Lp))


def gmg_num_levels(h):
    n = ctypes.c_int32()
    _check(load().gmg_num_levels(h.ptr, ctypes.byref(n)))
    return n.value


def gmg_level_shape(h, level):
    n = (ctypes.c_int32 * 3)()
    c = (ctypes.c_int32 * 3)()
    _check(load().gmg_level_shape(h.ptr, level, n, c))
    return tuple(n), tuple(c)


def gmg_level_faces(h, level, out):
    ls = h.params.l_storage
    dt = 2 if ls == GMG_BF16 else _torch_dtype(ls)
    p = _arr(out, "out", 3 * h.cells(level), dt, h.device)
    _check(load().gmg_level_faces(h.ptr, level, p))
    return out


def gmg_level_uniform(h, level, active=False):
    """(uniform bricks, bricks) of a level's uniform-brick map; with active,
    (uniform bricks, uniform bricks whose cells are all active, bricks)."""
    u, a, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().gmg_level_uniform(h.ptr, level, ctypes.byref(u), ctypes.byref(a),
                                    ctypes.byref(t)))
    return (u.value, a.value, t.value) if active else (u.value, t.value)


def gmg_residual(h, x, sigma, r=None, norms=True):
    """Returns (rnorm, snorm) if norms else None; fills r if given."""
    xp, sp, rp = h.arrs(h.spec(x, "x", cycle=False), h.spec(sigma, "sigma", cycle=False),
                        h.spec(r, "r", cycle=False, optional=True))
    rn, sn = ctypes.c_double(), ctypes.c_double()
    _check(load().gmg_residual(h.ptr, xp, sp, rp,
                               ctypes.byref(rn) if norms else None,
                               ctypes.byref(sn) if norms else None))
    return (rn.value, sn.value) if norms else None


def gmg_residual_noalloc(h, x, sigma, r=None, norms=None):
    """gmg_residual without allocation and without synchronising: fills r if
    given and, if `norms` (a float64 GPU tensor of 2 elements) is given,
    writes ||r|| to norms[0] and ||sigma|| to norms[1] on the device."""
    import torch
    xp, sp, rp = h.arrs(h.spec(x, "x", cycle=False), h.spec(sigma, "sigma", cycle=False),
                        h.spec(r, "r", cycle=False, optional=True))
    np_ = _arr(norms, "norms", 2, torch.float64, h.device, optional=True)
    rnp = snp = None
    if np_ is not None:
        rnp = ctypes.c_void_p(norms.data_ptr())
        snp = ctypes.c_void_p(norms.data_ptr() + norms.element_size())
    _check(load().gmg_residual_noalloc(h.ptr, xp, sp, rp, rnp, snp))


def gmg_smooth(h, level, x, sigma, sweeps):
    xp, sp = h.arrs(h.spec(x, "x", level), h.spec(sigma, "sigma", level))
    _check(load().gmg_smooth(h.ptr, level, xp, sp, sweeps))


def gmg_restrict_residual(h, level, x, sigma, sigma_c, x_c=None):
    xp, sp, scp, xcp = h.arrs(h.spec(x, "x", level), h.spec(sigma, "sigma", level),
                              h.spec(sigma_c, "sigma_c", level + 1),
                              h.spec(x_c, "x_c", level + 1, optional=True))
    _check(load().gmg_restrict_residual(h.ptr, level, xp, sp, scp, xcp))


def gmg_prolong_correct(h, level, x_c, x):
    xcp, xp = h.arrs(h.spec(x_c, "x_c", level + 1), h.spec(x, "x", level))
    _check(load().gmg_prolong_correct(h.ptr, level, xcp, xp))


def gmg_get_omega(h):
    w = ctypes.c_double()
    _check(load().gmg_get_omega(h.ptr, ctypes.byref(w)))
    return w.value


def gmg_coarse_sweeps(h):
    n = ctypes.c_int32()
    _check(load().gmg_coarse_sweeps(h.ptr, ctypes.byref(n)))
    return n.value


def gmg_set_omega(h, omega):
    _check(load().gmg_set_omega(h.ptr, float(omega)))


def gmg_vcycle(h, x, sigma, want_norm=False):
    rn = ctypes.c_double()
    xp, sp = h.arrs(h.spec(x, "x", cycle=False), h.spec(sigma, "sigma", cycle=False))
    _check(load().gmg_vcycle(h.ptr, xp, sp, ctypes.byref(rn) if want_norm else None))
    return rn.value if want_norm else None


def info_dict(info):
    n = min(info.cycles, GMG_MAX_HISTORY)
    return dict(status=STATUS_NAMES[info.status], cycles=info.cycles,
                accepted_cycles=info.accepted_cycles, launches=info.launches,
                rnorm0=info.rnorm0, rnorm=info.rnorm, snorm=info.snorm,
                omega=info.omega, history=list(info.history[:n]),
                omegas=list(info.omegas[:n]), accepted=list(info.accepted[:n]))


def gmg_solve(h, x, sigma, rtol, max_cycles, raise_noconv=False):
    """Adaptive solve in place on x.  Returns the info dict (status
    'GMG_ENOCONV' is returned, not raised, unless raise_noconv)."""
    info = gmg_solve_info()
    xp, sp = h.arrs(h.spec(x, "x", cycle=False), h.spec(sigma, "sigma", cycle=False))
    st = load().gmg_solve(h.ptr, xp, sp, float(rtol), int(max_cycles), ctypes.byref(info))
    if st != GMG_OK and not (st == GMG_ENOCONV and not raise_noconv):
        _check(st)
    return info_dict(info)


def gmg_pcg(h, x, sigma, rtol, max_iter, raise_noconv=False):
    """Jacobi-preconditioned conjugate gradient on level 0 of the handle, in
    place on x.  Returns dict(status, iterations, snorm, rnorm0, rnorm,
    history)."""
    info = gmg_pcg_info()
    xp, sp = h.arrs(h.spec(x, "x", cycle=False), h.spec(sigma, "sigma", cycle=False))
    st = load().gmg_pcg(h.ptr, xp, sp, float(rtol), int(max_iter), ctypes.byref(info))
    if st != GMG_OK and not (st == GMG_ENOCONV and not raise_noconv):
        _check(st)
    n = min(info.iterations, GMG_MAX_HISTORY)
    return dict(status=STATUS_NAMES[info.status], iterations=info.iterations, snorm=info.snorm,
                rnorm0=info.rnorm0, rnorm=info.rnorm, history=list(info.history[:n]))


def gmg_solve_ir(h, x, sigma, rtol=1e-10, max_outer=50, max_inner=8, inner_rtol=1e-4,
                 raise_noconv=False):
    """FP64 iterative refinement around FP32 V-cycles, in place on the FP64
    tensor x.  Returns the info dict."""
    import torch
    info = gmg_ir_info()
    xp, sp = h.arrs((x, "x", h.cells(0), torch.float64), (sigma, "sigma", h.cells(0), torch.float64))
    st = load().gmg_solve_ir(h.ptr, xp, sp, float(rtol), int(max_outer), int(max_inner),
                             float(inner_rtol), ctypes.byref(info))
    if st != GMG_OK and not (st == GMG_ENOCONV and not raise_noconv):
        _check(st)
    n = min(info.outer + 1, GMG_MAX_HISTORY)
    return dict(status=STATUS_NAMES[info.status], outer=info.outer,
                inner_total=info.inner_total, snorm=info.snorm, rnorm=info.rnorm,
                history=list(info.history[:n]),
                inner_cycles=list(info.inner_cycles[:min(info.outer, GMG_MAX_HISTORY)]))


def _ir_dict(info):
    n = min(info.outer + 1, GMG_MAX_HISTORY)
    return dict(status=STATUS_NAMES[info.status], outer=info.outer,
                inner_total=info.inner_total, snorm=info.snorm, rnorm=info.rnorm,
                history=list(info.history[:n]),
                inner_cycles=list(info.inner_cycles[:min(info.outer, GMG_MAX_HISTORY)]))


class Batch:
    """Owns a gmg_batch*; keeps the cell count of every problem and the
    device for the argument checks."""

    def __init__(self, ptr, n, stream, cells=None, device=None):
        self._ptr = ptr
        self.n = n
        self.stream = stream
        self.cells = cells
        self.device = device

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("batch is closed")
        return self._ptr

    def close(self):
        if self._ptr is not None:
            load().gmg_batch_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gmg_batch_setup(params_list, L_list, stream=None):
    n = len(params_list)
    if len(L_list) != n or n == 0:
        raise ValueError("need one L per parameter set")
    dev = L_list[0].device
    for p, L in zip(params_list, L_list):
        if _dtype_code(L) != p.dtype:
            raise TypeError("L dtype does not match params.dtype")
    ptrs = [t.value for t in _args(*[(L, f"L[{q}]", 3 * _cells(p.n), _torch_dtype(p.dtype))
                                     for q, (p, L) in enumerate(zip(params_list, L_list))],
                                   device=dev)]
    parr = (gmg_params * n)(*params_list)
    larr = (ctypes.c_void_p * n)(*ptrs)
    s = _stream(stream, dev)
    out = ctypes.c_void_p()
    _check(load().gmg_batch_setup(parr, larr, n, s, ctypes.byref(out)))
    return Batch(out, n, s, [_cells(p.n) for p in params_list], dev)


def gmg_batch_solve_ir(b, xs, sigmas, rtol=1e-10, max_outer=6, max_inner=8, inner_rtol=1e-4,
                       raise_noconv=False):
    """Refinement of every problem together (with graphs: one replay per
    refinement step, until all have finished); x tensors updated in place.
    Returns the list of per-problem info dicts."""
    import torch
    if len(xs) != b.n or len(sigmas) != b.n:
        raise ValueError("need one x and one sigma per problem")
    specs = ([(t, f"x[{q}]", b.cells[q], torch.float64) for q, t in enumerate(xs)] +
             [(t, f"sigma[{q}]", b.cells[q], torch.float64) for q, t in enumerate(sigmas)])
    ptrs = [t.value for t in _args(*specs, device=b.device)]
    xarr = (ctypes.c_void_p * b.n)(*ptrs[:b.n])
    sarr = (ctypes.c_void_p * b.n)(*ptrs[b.n:])
    infos = (gmg_ir_info * b.n)()
    st = load().gmg_batch_solve_ir(b.ptr, xarr, sarr, float(rtol), int(max_outer),
                                   int(max_inner), float(inner_rtol), infos)
    if st != GMG_OK and not (st == GMG_ENOCONV and not raise_noconv):
        _check(st)
    return [_ir_dict(infos[p]) for p in range(b.n)]


def gmg_autotune(h, x, sigma, reps=5):
    """Time the sweep tile candidates of every level and keep the fastest;
    also the two-sweep pass where allowed.  Returns per-level dicts (shape,
    ty, kchunk, us, defaults, pair_kchunk (0: separate sweeps), pair_ty, us_pair)."""
    rep = gmg_tune_report()
    xp, sp = h.arrs(h.spec(x, "x", cycle=False), h.spec(sigma, "sigma", cycle=False))
    _check(load().gmg_autotune(h.ptr, xp, sp, int(reps), ctypes.byref(rep)))
    out = []
    for l in range(rep.nlevels):
        n, _ = gmg_level_shape(h, l)
        out.append(dict(level=l, n=n, ty=rep.ty[l], kchunk=rep.kchunk[l], us=rep.us[l],
                        ty_default=rep.ty_default[l], kchunk_default=rep.kchunk_default[l],
                        us_default=rep.us_default[l], pair_kchunk=rep.pair_kchunk[l],
                        pair_ty=rep.pair_ty[l], us_pair=rep.us_pair[l]))
    return out


def gmg_set_tiles(h, level, ty, kchunk):
    _check(load().gmg_set_tiles(h.ptr, int(level), int(ty), int(kchunk)))


def gmg_set_pair_sweeps(h, level, kchunk, ty=16):
    """Two-sweep passes on 64 x ty tiles (ty 8 or 16) of kchunk z-planes per
    workgroup on one level (kchunk 0: separate sweeps)."""
    _check(load().gmg_set_pair_sweeps(h.ptr, int(level), int(ty), int(kchunk)))


def gmg_batch_autotune(b, reps=5):
    _check(load().gmg_batch_autotune(b.ptr, int(reps)))


def gmg_last_error():
    return load().gmg_last_error().decode()
