"""The U-Net warm start assembled from libunet.so operations.

This module owns the network's buffers (allocated as torch tensors: device
memory only) and issues the C-ABI calls of include/unet.h in U-Net order:
every arithmetic step - convolutions, pooling, upsampling, ReLU gradients,
the head, the loss, Adam - runs in the HIP kernels.

Parameters live in one flat FP32 vector (master weights), with flat FP32
gradient and Adam-moment vectors of the same layout and a flat BF16 copy that
the convolutions read.  Per layer, in the order of ``layers()``: the weights
[C_out][taps][C_in] then the biases [C_out]; the input layer's C_in is padded
from 4 to 8 with zero channels.

Activations are BF16, channels-last.  The skip connection is free: encoder
level i writes its output into channels [c_i, 2 c_i) of the concatenation
buffer whose channels [0, c_i) the decoder's up-convolution fills.
"""
from __future__ import annotations

import math

import numpy as np

from . import unet as UN

IN_CH = 8  # 4 input fields padded to 8 channels


def layers(chans=(16, 32, 64, 128), in_ch=IN_CH):
    """(name, C_in, C_out, taps) of every layer, in parameter order."""
    out = []
    c_prev = in_ch
    for i, c in enumerate(chans):
        out.append((f"enc{i}a", c_prev, c, 27))
        out.append((f"enc{i}b", c, c, 27))
        c_prev = c
    for i in range(len(chans) - 2, -1, -1):
        out.append((f"up{i}", chans[i + 1], chans[i], 27))
        out.append((f"dec{i}a", 2 * chans[i], chans[i], 27))
        out.append((f"dec{i}b", chans[i], chans[i], 27))
    out.append(("head", chans[0], 1, 1))
    return out


class UNet:
    def __init__(self, chans=(16, 32, 64, 128), device="cuda"):
        import torch
        self.torch = torch
        self.chans = tuple(chans)
        self.nl = len(chans)
        self.dev = device
        self.layers = layers(self.chans)
        self.offs = {}
        off = 0
        for name, ci, co, taps in self.layers:
            self.offs[name] = (off, off + co * taps * ci, ci, co, taps)
            off += co * taps * ci + co
        self.nparams = off
        z = lambda: torch.zeros(off, dtype=torch.float32, device=device)
        self.master, self.grad, self.m, self.v = z(), z(), z(), z()
        self.wbf = torch.zeros(off, dtype=torch.int16, device=device)
        self.step = 0
        self._bufs = None
        self._shape = None

    # -- parameters ---------------------------------------------------------
    def init_he(self, seed):
        """He-normal weights (zero for the padded input channels), zero biases."""
        rng = np.random.default_rng(seed)
        flat = np.zeros(self.nparams, dtype=np.float32)
        for name, ci, co, taps in self.layers:
            w0, b0, _, _, _ = self.offs[name]
            cin_true = 4 if name == "enc0a" else ci
            std = math.sqrt(2.0 / (cin_true * taps))
            w = rng.standard_normal((co, taps, ci)) * std
            if name == "enc0a":
                w[:, :, 4:] = 0.0
            flat[w0:b0] = w.reshape(-1)
        self.set_flat(flat)

    def set_flat(self, flat):
        self.master.copy_(self.torch.from_numpy(np.asarray(flat, dtype=np.float32)))
        self.m.zero_()
        self.v.zero_()
        self.step = 0
        UN.unet_to_bf16(self.master, self.wbf)

    def get_flat(self):
        return self.master.cpu().numpy()

    def _w(self, name):
        w0, b0, ci, co, taps = self.offs[name]
        return self.wbf[w0:b0], self.master[b0:b0 + co]

    # -- buffers ------------------------------------------------------------
    def _alloc(self, n, d, h, w):
        torch = self.torch
        if self._shape == (n, d, h, w):
            return self._bufs
        div = 2 ** (self.nl - 1)
        if d % div or h % div or w % div:
            raise ValueError(f"grid must be divisible by {div}")
        B = {}
        i16 = dict(dtype=torch.int16, device=self.dev)
        sh = [(n, d >> i, h >> i, w >> i) for i in range(self.nl)]
        B["shape"] = sh
        for i, c in enumerate(self.chans):
            for k in ("Ea", "gEa", "Db", "gDb", "Da", "gDa"):
                B[f"{k}{i}"] = torch.zeros(sh[i] + (c,), **i16)
            if i < self.nl - 1:
                B[f"CAT{i}"] = torch.zeros(sh[i] + (2 * c,), **i16)
                B[f"gCAT{i}"] = torch.zeros(sh[i] + (2 * c,), **i16)
                B[f"U{i}"] = torch.zeros(sh[i] + (self.chans[i + 1],), **i16)
                B[f"gU{i}"] = torch.zeros(sh[i] + (self.chans[i + 1],), **i16)
            if i > 0:
                B[f"P{i}"] = torch.zeros(sh[i] + (self.chans[i - 1],), **i16)
                B[f"gP{i}"] = torch.zeros(sh[i] + (self.chans[i - 1],), **i16)
        B["Eb"] = torch.zeros(sh[-1] + (self.chans[-1],), **i16)
        B["gEb"] = torch.zeros(sh[-1] + (self.chans[-1],), **i16)
        B["out"] = torch.zeros(sh[0], dtype=torch.float32, device=self.dev)
        B["dout"] = torch.zeros(sh[0], dtype=torch.float32, device=self.dev)
        B["stats"] = torch.zeros(2 + 512, dtype=torch.float64, device=self.dev)
        wsz, fl = 0, 0
        for name, ci, co, taps in self.layers:
            lvl = int("".join(ch for ch in name if ch.isdigit())) if name != "head" else 0
            s = UN.shape(*sh[lvl])
            if name == "head":
                wsz = max(wsz, UN.unet_head_workspace(s, ci))
            else:
                wsz = max(wsz, UN.unet_wgrad_workspace(s, ci, co, taps))
            fl = max(fl, ci * co * taps)
        B["ws"] = torch.empty(wsz // 4 + 16, dtype=torch.float32, device=self.dev)
        B["wflip"] = torch.empty(fl, dtype=torch.int16, device=self.dev)
        self._bufs, self._shape = B, (n, d, h, w)
        return B

    # -- forward ------------------------------------------------------------
    def forward(self, x_in, n, d, h, w):
        """x_in: BF16 channels-last [n][d][h][w][8].  Returns the FP32 output
        [n][d][h][w] (a view of an internal buffer)."""
        B = self._alloc(n, d, h, w)
        sh, ch = B["shape"], self.chans
        A = UN.act
        hv, hs = A(x_in, IN_CH, 0, IN_CH), sh[0]
        for i, c in enumerate(ch):
            s = UN.shape(*sh[i])
            wa, ba = self._w(f"enc{i}a")
            UN.unet_conv_fwd(s, hv, wa, ba, 27, A(B[f"Ea{i}"], c, 0, c), None, 1)
            wb, bb = self._w(f"enc{i}b")
            if i < self.nl - 1:
                skip = A(B[f"CAT{i}"], 2 * c, c, c)
                UN.unet_conv_fwd(s, A(B[f"Ea{i}"], c, 0, c), wb, bb, 27, skip, None, 1)
                UN.unet_pool_fwd(s, skip, A(B[f"P{i + 1}"], c, 0, c))
                hv = A(B[f"P{i + 1}"], c, 0, c)
            else:
                UN.unet_conv_fwd(s, A(B[f"Ea{i}"], c, 0, c), wb, bb, 27, A(B["Eb"], c, 0, c),
                                 None, 1)
                hv = A(B["Eb"], c, 0, c)
        for i in range(self.nl - 2, -1, -1):
            c, cu = ch[i], ch[i + 1]
            s = UN.shape(*sh[i])
            UN.unet_up_fwd(UN.shape(*sh[i + 1]), hv, A(B[f"U{i}"], cu, 0, cu))
            wu, bu = self._w(f"up{i}")
            UN.unet_conv_fwd(s, A(B[f"U{i}"], cu, 0, cu), wu, bu, 27, A(B[f"CAT{i}"], 2 * c, 0, c),
                             None, 1)
            wa, ba = self._w(f"dec{i}a")
            UN.unet_conv_fwd(s, A(B[f"CAT{i}"], 2 * c, 0, 2 * c), wa, ba, 27,
                             A(B[f"Da{i}"], c, 0, c), None, 1)
            wb, bb = self._w(f"dec{i}b")
            UN.unet_conv_fwd(s, A(B[f"Da{i}"], c, 0, c), wb, bb, 27, A(B[f"Db{i}"], c, 0, c),
                             None, 1)
            hv = A(B[f"Db{i}"], c, 0, c)
        w0, b0, _, _, _ = self.offs["head"]
        UN.unet_head_fwd(UN.shape(*sh[0]), hv, self.master[w0:b0], self.master[b0:b0 + 1],
                         B["out"])
        return B["out"]

    # -- backward -----------------------------------------------------------
    def backward(self, x_in, target, mask, want_loss=True):
        """Gradients of the masked MSE of the last forward's output against
        target (FP32 [n][d][h][w]) into self.grad; returns the loss."""
        B = self._bufs
        sh, ch = B["shape"], self.chans
        A = UN.act
        G = self.grad
        s0 = UN.shape(*sh[0])
        loss = UN.unet_mse(s0, B["out"], target, mask, B["dout"], B["stats"], want_loss)

        def gw(name):
            w0, b0, ci, co, taps = self.offs[name]
            return G[w0:b0], G[b0:b0 + co]

        c0 = ch[0]
        hw0, hb0 = gw("head")
        w0, b0, _, _, _ = self.offs["head"]
        UN.unet_head_bwd(s0, A(B["Db0"], c0, 0, c0), self.master[w0:b0], B["dout"],
                         A(B["gDb0"], c0, 0, c0), hw0, hb0, B["ws"])
        for i in range(self.nl - 1):
            c, cu = ch[i], ch[i + 1]
            s = UN.shape(*sh[i])
            gDb = A(B[f"gDb{i}"], c, 0, c)
            UN.unet_relu_bwd(s, A(B[f"Db{i}"], c, 0, c), gDb, gDb)
            dw, db = gw(f"dec{i}b")
            UN.unet_conv_wgrad(s, A(B[f"Da{i}"], c, 0, c), gDb, 27, dw, db, B["ws"])
            UN.unet_conv_dgrad(s, gDb, self._w(f"dec{i}b")[0], 27, A(B[f"gDa{i}"], c, 0, c),
                               B["wflip"])
            gDa = A(B[f"gDa{i}"], c, 0, c)
            UN.unet_relu_bwd(s, A(B[f"Da{i}"], c, 0, c), gDa, gDa)
            dw, db = gw(f"dec{i}a")
            UN.unet_conv_wgrad(s, A(B[f"CAT{i}"], 2 * c, 0, 2 * c), gDa, 27, dw, db, B["ws"])
            UN.unet_conv_dgrad(s, gDa, self._w(f"dec{i}a")[0], 27,
                               A(B[f"gCAT{i}"], 2 * c, 0, 2 * c), B["wflip"])
            gup = A(B[f"gCAT{i}"], 2 * c, 0, c)
            UN.unet_relu_bwd(s, A(B[f"CAT{i}"], 2 * c, 0, c), gup, gup)
            dw, db = gw(f"up{i}")
            UN.unet_conv_wgrad(s, A(B[f"U{i}"], cu, 0, cu), gup, 27, dw, db, B["ws"])
            UN.unet_conv_dgrad(s, gup, self._w(f"up{i}")[0], 27, A(B[f"gU{i}"], cu, 0, cu),
                               B["wflip"])
            dst = B["gEb"] if i + 1 == self.nl - 1 else B[f"gDb{i + 1}"]
            UN.unet_up_bwd(UN.shape(*sh[i + 1]), A(B[f"gU{i}"], cu, 0, cu), A(dst, cu, 0, cu))
        for i in range(self.nl - 1, -1, -1):
            c = ch[i]
            s = UN.shape(*sh[i])
            if i == self.nl - 1:
                yb, gyb = A(B["Eb"], c, 0, c), A(B["gEb"], c, 0, c)
            else:
                yb, gyb = A(B[f"CAT{i}"], 2 * c, c, c), A(B[f"gCAT{i}"], 2 * c, c, c)
                UN.unet_pool_bwd(s, A(B[f"gP{i + 1}"], c, 0, c), gyb, 1)
            UN.unet_relu_bwd(s, yb, gyb, gyb)
            dw, db = gw(f"enc{i}b")
            UN.unet_conv_wgrad(s, A(B[f"Ea{i}"], c, 0, c), gyb, 27, dw, db, B["ws"])
            UN.unet_conv_dgrad(s, gyb, self._w(f"enc{i}b")[0], 27, A(B[f"gEa{i}"], c, 0, c),
                               B["wflip"])
            gEa = A(B[f"gEa{i}"], c, 0, c)
            UN.unet_relu_bwd(s, A(B[f"Ea{i}"], c, 0, c), gEa, gEa)
            dw, db = gw(f"enc{i}a")
            if i == 0:
                UN.unet_conv_wgrad(s, A(x_in, IN_CH, 0, IN_CH), gEa, 27, dw, db, B["ws"])
            else:
                cp = ch[i - 1]
                UN.unet_conv_wgrad(s, A(B[f"P{i}"], cp, 0, cp), gEa, 27, dw, db, B["ws"])
                UN.unet_conv_dgrad(s, gEa, self._w(f"enc{i}a")[0], 27, A(B[f"gP{i}"], cp, 0, cp),
                                   B["wflip"])
        return loss

    def adam(self, lr):
        self.step += 1
        UN.unet_adam(self.master, self.m, self.v, self.grad, self.wbf, lr, self.step)
