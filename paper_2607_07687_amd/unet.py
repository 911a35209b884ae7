"""ctypes binding of libunet.so (C ABI in include/unet.h).

Argument marshalling only: every operation runs in the HIP library; the
functions carry the C names.  Activation tensors are torch tensors holding
BF16 bits (torch.int16 or torch.bfloat16), channels-last; a view is
(tensor, ld, off, c) mapped to unet_act.  The library is loaded from this
package directory and missing it raises.
"""
from __future__ import annotations

import ctypes
import os

LIB_NAME = "libunet.so"
_HERE = os.path.dirname(os.path.abspath(__file__))
UNET_OK, UNET_EINVAL, UNET_ENOMEM, UNET_EHIP = 0, 1, 3, 4


class unet_act(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("ld", ctypes.c_int32), ("off", ctypes.c_int32),
                ("c", ctypes.c_int32)]


class unet_shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int32), ("h", ctypes.c_int32),
                ("w", ctypes.c_int32)]


class UNetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"unet status {status}: {msg}")
        self.status = status


_V = ctypes.c_void_p
_I = ctypes.c_int32
_F = ctypes.c_float
_SIGS = [
    ("unet_conv_fwd", ctypes.c_int, [unet_shape, unet_act, _V, _V, _I, unet_act, _V, _I, _V]),
    ("unet_conv_dgrad", ctypes.c_int, [unet_shape, unet_act, _V, _I, unet_act, _V, _V]),
    ("unet_wgrad_workspace", ctypes.c_size_t, [unet_shape, _I, _I, _I]),
    ("unet_conv_wgrad", ctypes.c_int, [unet_shape, unet_act, unet_act, _I, _V, _V, _V, _V]),
    ("unet_wgrad_kernel", ctypes.c_int, [unet_shape, _I, _I, _I, _V]),
    ("unet_conv_kernel", ctypes.c_int, [unet_shape, _I, _I, _I, _V]),
    ("unet_relu_bwd", ctypes.c_int, [unet_shape, unet_act, unet_act, unet_act, _V]),
    ("unet_pool_fwd", ctypes.c_int, [unet_shape, unet_act, unet_act, _V]),
    ("unet_pool_bwd", ctypes.c_int, [unet_shape, unet_act, unet_act, _I, _V]),
    ("unet_up_fwd", ctypes.c_int, [unet_shape, unet_act, unet_act, _V]),
    ("unet_up_bwd", ctypes.c_int, [unet_shape, unet_act, unet_act, _V]),
    ("unet_head_fwd", ctypes.c_int, [unet_shape, unet_act, _V, _V, _V, _V]),
    ("unet_head_workspace", ctypes.c_size_t, [unet_shape, _I]),
    ("unet_head_bwd", ctypes.c_int, [unet_shape, unet_act, _V, _V, unet_act, _V, _V, _V, _V]),
    ("unet_mse", ctypes.c_int, [unet_shape, _V, _V, _V, _V, _V,
                                ctypes.POINTER(ctypes.c_double), _V]),
    ("unet_adam", ctypes.c_int, [ctypes.c_int64, _V, _V, _V, _V, _V, _F, _F, _F, _F, _I, _V]),
    ("unet_scale", ctypes.c_int, [ctypes.c_int64, _V, _F, _V, _V]),
    ("unet_scale_f64", ctypes.c_int, [ctypes.c_int64, _V, ctypes.c_double, _V, _V]),
    ("unet_to_bf16", ctypes.c_int, [ctypes.c_int64, _V, _V, _V]),
    ("unet_from_bf16", ctypes.c_int, [ctypes.c_int64, _V, _V, _V]),
    ("unet_pack_input", ctypes.c_int, [unet_shape, _V, _V, ctypes.POINTER(ctypes.c_float), _V, _V]),
    ("unet_mfma_selfcheck", ctypes.c_int, [_V, _V, _V, _V]),
    ("unet_last_error", ctypes.c_char_p, []),
]

_lib = None


def load():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, LIB_NAME)
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


def _check(st):
    if st != UNET_OK:
        raise UNetError(st, load().unet_last_error().decode())


def _p(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("tensor must be a contiguous GPU tensor")
    return t.data_ptr()


def _stream(stream=None):
    import torch
    return (stream or torch.cuda.current_stream()).cuda_stream


def shape(n, d, h, w):
    return unet_shape(int(n), int(d), int(h), int(w))


def act(t, ld, off, c):
    """View of channels [off, off + c) of a channels-last BF16 tensor whose
    rows hold ld channels (t may be None for an absent view)."""
    return unet_act(_p(t) if t is not None else None, int(ld), int(off), int(c))


def unet_conv_fwd(s, x, w, bias, taps, y, out_f32=None, relu=0):
    _check(load().unet_conv_fwd(s, x, _p(w), _p(bias), taps, y, _p(out_f32), int(relu), _stream()))


def unet_conv_dgrad(s, dy, w, taps, dx, wflip):
    _check(load().unet_conv_dgrad(s, dy, _p(w), taps, dx, _p(wflip), _stream()))


def unet_wgrad_workspace(s, cin, cout, taps):
    return load().unet_wgrad_workspace(s, cin, cout, taps)


def unet_conv_wgrad(s, x, dy, taps, dw, db, ws):
    _check(load().unet_conv_wgrad(s, x, dy, taps, _p(dw), _p(db), _p(ws), _stream()))


CONV_KINDS = {0: "gather", 1: "tile"}


def unet_conv_kernel(s, cin, cout, taps):
    """Kernel choice of unet_conv_fwd (host only): dict with kind ("tile" or
    "gather"), tw (tile width) or mb (voxel blocks of 16 per wave), nb (output
    blocks per wave) and groups (output-channel groups)."""
    info = (ctypes.c_int32 * 4)()
    _check(load().unet_conv_kernel(s, cin, cout, taps, ctypes.cast(info, ctypes.c_void_p)))
    kind = CONV_KINDS[info[0]]
    out = {"kind": kind, "nb": info[2], "groups": info[3]}
    out["mb" if kind == "gather" else "tw"] = info[1]
    return out


def unet_wgrad_kernel(s, cin, cout, taps):
    """Kernel choice of unet_conv_wgrad (host only): dict with rows (row-tiled
    kernel or voxel chunks), ct / ot / ws (channels and w extent of a row
    workgroup), chunks (partial rows) and dper (d planes per chunk)."""
    info = (ctypes.c_int32 * 6)()
    _check(load().unet_wgrad_kernel(s, cin, cout, taps, ctypes.cast(info, ctypes.c_void_p)))
    return {"rows": bool(info[0]), "ct": info[1], "ot": info[2], "ws": info[3],
            "chunks": info[4], "dper": info[5]}


def unet_relu_bwd(s, y, dy, out):
    _check(load().unet_relu_bwd(s, y, dy, out, _stream()))


def unet_pool_fwd(fine, x, y):
    _check(load().unet_pool_fwd(fine, x, y, _stream()))


def unet_pool_bwd(fine, dy, dx, accumulate=0):
    _check(load().unet_pool_bwd(fine, dy, dx, int(accumulate), _stream()))


def unet_up_fwd(coarse, x, y):
    _check(load().unet_up_fwd(coarse, x, y, _stream()))


def unet_up_bwd(coarse, dy, dx):
    _check(load().unet_up_bwd(coarse, dy, dx, _stream()))


def unet_head_fwd(s, x, w, b, y):
    _check(load().unet_head_fwd(s, x, _p(w), _p(b), _p(y), _stream()))


def unet_head_workspace(s, cin):
    return load().unet_head_workspace(s, cin)


def unet_head_bwd(s, x, w, dy, dx, dw, db, ws):
    _check(load().unet_head_bwd(s, x, _p(w), _p(dy), dx, _p(dw), _p(db), _p(ws), _stream()))


def unet_mse(s, pred, target, mask, dpred, stats, want_loss=True):
    loss = ctypes.c_double()
    _check(load().unet_mse(s, _p(pred), _p(target), _p(mask), _p(dpred), _p(stats),
                           ctypes.byref(loss) if want_loss else None, _stream()))
    return loss.value if want_loss else None


def unet_adam(master, m, v, g, bf16_out, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().unet_adam(master.numel(), _p(master), _p(m), _p(v), _p(g), _p(bf16_out),
                            float(lr), float(beta1), float(beta2), float(eps), int(t), _stream()))


def unet_scale(x, a, out):
    _check(load().unet_scale(x.numel(), _p(x), float(a), _p(out), _stream()))


def unet_scale_f64(x, a, out):
    _check(load().unet_scale_f64(x.numel(), _p(x), float(a), _p(out), _stream()))


def unet_to_bf16(x, out):
    _check(load().unet_to_bf16(x.numel(), _p(x), _p(out), _stream()))


def unet_from_bf16(x, out):
    _check(load().unet_from_bf16(x.numel(), _p(x), _p(out), _stream()))


def unet_pack_input(s, sigma, L, scales, x):
    arr = (ctypes.c_float * len(scales))(*[float(v) for v in scales])
    _check(load().unet_pack_input(s, _p(sigma), _p(L), arr, _p(x), _stream()))


def unet_mfma_selfcheck(a, b, out):
    _check(load().unet_mfma_selfcheck(_p(a), _p(b), _p(out), _stream()))


def unet_last_error():
    return load().unet_last_error().decode()
