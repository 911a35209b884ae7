"""Plain CPU FP64 oracle of the 3-D U-Net warm start for the GMG solver.

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path; it
shares no code with the HIP kernels.

The network predicts the pressure of the Poisson problem from (sigma / s, L_x,
L_y, L_z), s = RMS of sigma over the active cells, so that GMG can start from
its prediction instead of zero.  The paper has no network; its architecture
is the reading taken here (4 levels, 16 -> 128 channels, 3x3x3 convolutions with
zero padding 1, ReLU, 2x2x2 average pooling, nearest x2 upsampling, skip
concatenation, 1x1x1 head, MSE loss, Adam).

Everything is whole-array NumPy FP64.  Arrays are [C, D, H, W] per sample (D
= z, H = y, W = x); weights are [C_out, C_in, kd, kh, kw]; convolution is the
cross-correlation y[o, v] = b[o] + sum_{c, t} w[o, c, t] x[c, v + t - 1].
Every backward function is the exact gradient of its forward, written from
the definition.
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------------------
# Layers
# ----------------------------------------------------------------------------

def conv3d(x, w, b):
    """Cross-correlation with zero padding (k - 1) / 2, stride 1."""
    co, ci, kd, kh, kw = w.shape
    pd, ph, pw = kd // 2, kh // 2, kw // 2
    C, D, H, W = x.shape
    assert C == ci
    xp = np.pad(x, ((0, 0), (pd, pd), (ph, ph), (pw, pw)))
    y = np.zeros((co, D, H, W))
    for a in range(kd):
        for bb in range(kh):
            for c in range(kw):
                y += np.einsum("oc,cdhw->odhw", w[:, :, a, bb, c],
                               xp[:, a:a + D, bb:bb + H, c:c + W])
    return y + b[:, None, None, None]


def conv3d_backward(x, w, dy):
    """Gradients of conv3d: (dx, dw, db)."""
    co, ci, kd, kh, kw = w.shape
    pd, ph, pw = kd // 2, kh // 2, kw // 2
    C, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (pd, pd), (ph, ph), (pw, pw)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(kd):
        for bb in range(kh):
            for c in range(kw):
                win = (slice(None), slice(a, a + D), slice(bb, bb + H), slice(c, c + W))
                dw[:, :, a, bb, c] = np.einsum("odhw,cdhw->oc", dy, xp[win])
                dxp[win] += np.einsum("oc,odhw->cdhw", w[:, :, a, bb, c], dy)
    dx = dxp[:, pd:pd + D, ph:ph + H, pw:pw + W]
    db = dy.sum(axis=(1, 2, 3))
    return dx, dw, db


def conv3d_points(x, w, b, pts):
    """conv3d at selected voxels, from the definition: for each (d, h, w)
    in pts, y[o] = b[o] + sum over c and taps t of w[o, c, t] x[c, v + t -
    (k - 1) / 2] (zero outside the grid).  Returns y [len(pts), C_out]."""
    k = w.shape[2]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (p, p)))
    out = np.zeros((len(pts), w.shape[0]))
    for i, (d, h, ww) in enumerate(pts):
        patch = xp[:, d:d + k, h:h + k, ww:ww + k]
        out[i] = b + np.tensordot(w, patch, axes=([1, 2, 3, 4], [0, 1, 2, 3]))
    return out


def conv3d_wgrad_pairs(x, dy, pairs, k=3):
    """Selected weight-gradient entries of conv3d, from the definition:
    for each (o, c) in pairs, g[o, c][a, b, e] = sum over voxels v of
    dy[o, v] x[c, v + (a, b, e) - (k - 1) / 2] (zero outside the grid), one
    dot product per tap.  Returns (g [len(pairs), k, k, k], db[C_out] = sum
    over voxels of dy[o])."""
    p = k // 2
    C, D, H, W = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (p, p)))
    out = np.zeros((len(pairs), k, k, k))
    for i, (o, c) in enumerate(pairs):
        for a in range(k):
            for b in range(k):
                for e in range(k):
                    out[i, a, b, e] = np.sum(dy[o] * xp[c, a:a + D, b:b + H, e:e + W])
    return out, dy.sum(axis=(1, 2, 3))


def bf16(a):
    """Round to BF16 (round to nearest even on the FP32 bit pattern, after
    rounding to FP32) and return the value in FP64: the storage rounding of
    a BF16 activation or gradient whose value was accumulated in FP32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(y, dy):
    """Gradient through ReLU given its output y."""
    return dy * (y > 0.0)


def avgpool2(x):
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def upsample2(x):
    """Nearest-neighbour x2 upsampling."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def upsample2_backward(dy):
    C, D, H, W = dy.shape
    return dy.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))


def mse(pred, target, mask):
    """Mean squared error over the masked cells and its gradient."""
    n = max(int(mask.sum()), 1)
    d = (pred - target) * mask
    return float(np.sum(d * d)) / n, 2.0 * d / n


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------

def layer_list(in_ch=4, chans=(16, 32, 64, 128)):
    """Ordered (name, C_in, C_out, k) of every convolution."""
    layers = []
    c_prev = in_ch
    for i, c in enumerate(chans):
        layers.append((f"enc{i}a", c_prev, c, 3))
        layers.append((f"enc{i}b", c, c, 3))
        c_prev = c
    for i in range(len(chans) - 2, -1, -1):
        layers.append((f"up{i}", chans[i + 1], chans[i], 3))
        layers.append((f"dec{i}a", 2 * chans[i], chans[i], 3))
        layers.append((f"dec{i}b", chans[i], chans[i], 3))
    layers.append(("head", chans[0], 1, 1))
    return layers


def init_params(seed, in_ch=4, chans=(16, 32, 64, 128)):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, ci, co, k in layer_list(in_ch, chans):
        std = math.sqrt(2.0 / (ci * k ** 3))
        params[name + ".w"] = rng.standard_normal((co, ci, k, k, k)) * std
        params[name + ".b"] = np.zeros(co)
    return params


def forward(params, x, chans=(16, 32, 64, 128), store_bf16=False):
    """U-Net forward for one sample x[C_in, D, H, W]; returns (y[1, D, H, W],
    cache of every intermediate for backward).  store_bf16: every stored
    activation (each convolution + ReLU output and each pooling output) is
    rounded to BF16, as a network that keeps its activations in BF16 stores
    them; the head's output is not."""
    nl = len(chans)
    rnd = bf16 if store_bf16 else (lambda v: v)
    cache = {"x": x}
    h = x
    for i in range(nl):
        a = rnd(relu(conv3d(h, params[f"enc{i}a.w"], params[f"enc{i}a.b"])))
        bb = rnd(relu(conv3d(a, params[f"enc{i}b.w"], params[f"enc{i}b.b"])))
        cache[f"enc{i}in"], cache[f"enc{i}a"], cache[f"enc{i}b"] = h, a, bb
        h = rnd(avgpool2(bb)) if i < nl - 1 else bb
    for i in range(nl - 2, -1, -1):
        u = upsample2(h)
        c = rnd(relu(conv3d(u, params[f"up{i}.w"], params[f"up{i}.b"])))
        cat = np.concatenate([c, cache[f"enc{i}b"]], axis=0)
        a = rnd(relu(conv3d(cat, params[f"dec{i}a.w"], params[f"dec{i}a.b"])))
        bb = rnd(relu(conv3d(a, params[f"dec{i}b.w"], params[f"dec{i}b.b"])))
        cache[f"up{i}in"], cache[f"up{i}"], cache[f"cat{i}"] = u, c, cat
        cache[f"dec{i}a"], cache[f"dec{i}b"] = a, bb
        h = bb
    y = conv3d(h, params["head.w"], params["head.b"])
    cache["headin"] = h
    return y, cache


def backward(params, cache, dy, chans=(16, 32, 64, 128), store_bf16=False):
    """Gradients of every parameter (and of the input) given dL/dy.
    store_bf16: every stored activation gradient (each convolution's input
    gradient, each upsampling and pooling backward, and the encoder's sum of
    pooled and skip gradients) is rounded to BF16; parameter gradients are
    not."""
    nl = len(chans)
    rnd = bf16 if store_bf16 else (lambda v: v)
    g = {}
    dh, g["head.w"], g["head.b"] = conv3d_backward(cache["headin"], params["head.w"], dy)
    dh = rnd(dh)
    dskip = {}
    for i in range(nl - 1):
        d = relu_backward(cache[f"dec{i}b"], dh)
        d, g[f"dec{i}b.w"], g[f"dec{i}b.b"] = conv3d_backward(cache[f"dec{i}a"],
                                                              params[f"dec{i}b.w"], d)
        d = relu_backward(cache[f"dec{i}a"], rnd(d))
        dcat, g[f"dec{i}a.w"], g[f"dec{i}a.b"] = conv3d_backward(cache[f"cat{i}"],
                                                                 params[f"dec{i}a.w"], d)
        dcat = rnd(dcat)
        c = chans[i]
        dc, dskip[i] = dcat[:c], dcat[c:]
        d = relu_backward(cache[f"up{i}"], dc)
        du, g[f"up{i}.w"], g[f"up{i}.b"] = conv3d_backward(cache[f"up{i}in"],
                                                           params[f"up{i}.w"], d)
        dh = rnd(upsample2_backward(rnd(du)))
    for i in range(nl - 1, -1, -1):
        # the bottom level feeds the decoder directly; the others feed the
        # pooling to the next level and the skip concatenation
        d = dh if i == nl - 1 else rnd(avgpool2_backward(dh) + dskip[i])
        d = relu_backward(cache[f"enc{i}b"], d)
        d, g[f"enc{i}b.w"], g[f"enc{i}b.b"] = conv3d_backward(cache[f"enc{i}a"],
                                                              params[f"enc{i}b.w"], d)
        d = relu_backward(cache[f"enc{i}a"], rnd(d))
        dh, g[f"enc{i}a.w"], g[f"enc{i}a.b"] = conv3d_backward(cache[f"enc{i}in"],
                                                               params[f"enc{i}a.w"], d)
        dh = rnd(dh)
    return g, dh


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, gk in grads.items():
        m = state.setdefault("m." + k, np.zeros_like(gk))
        v = state.setdefault("v." + k, np.zeros_like(gk))
        m *= beta1
        m += (1 - beta1) * gk
        v *= beta2
        v += (1 - beta2) * gk * gk
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)
