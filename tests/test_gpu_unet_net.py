"""GPU parity of the whole U-Net (forward output, every parameter gradient)
against the FP64 oracle on a small grid, with the same BF16-rounded weights
and inputs, the oracle storing every activation and every activation
gradient in BF16 at the points libunet.so does (store_bf16).

What then separates the two is the order and precision of the sums inside
each convolution: FP32 accumulation of K = 27 C_in products on the GPU, FP64
in the oracle.  Before a BF16 store the two values differ by at most about
K u32 of the sum's magnitude (u32 = 2^-24, K <= 27 * 64 = 1728 here: 1e-4),
so they round to different BF16 neighbours only when they straddle a
rounding boundary, for a fraction of at most 2 K u32 / u16 (u16 = 2^-8: 0.05)
of the elements, each then off by one BF16 spacing (2 u16).  A stored tensor
so differs by at most sqrt(0.05) * 2 u16 = 1.7e-3 norm-wise, and through the
ten stores of the forward pass, or the twenty of the deepest gradient
(random walk), by at most 6e-3 and 8e-3.  The bounds are 1e-2 for the output
and the loss, and 2e-2 with a cosine above 0.9995 for every parameter
gradient.  (Typical sums are far from the worst case, and the errors seen
are some ten times smaller.)  A wrong index or operand gives errors of order
one."""
import numpy as np
import pytest

from oracle import unet_oracle as UO
from paper_2607_07687_amd import unet as UN
from paper_2607_07687_amd import unet_net as NET
from tests.gpu_util import require_gpu, say
from tests.test_gpu_unet_ops import bf16_round, bf16_to_f64, cl, to_dev_bf16

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def oracle_params(net, flat, chans):
    """Flat GPU layout (BF16-rounded conv weights, FP32 biases and head) ->
    oracle dict with 4 input channels."""
    P = {}
    for name, ci, co, taps in net.layers:
        w0, b0, _, _, _ = net.offs[name]
        w = flat[w0:b0].astype(np.float64)
        if name != "head":
            w = bf16_to_f64(bf16_round(flat[w0:b0]))
        w = w.reshape(co, taps, ci)
        if name == "enc0a":
            w = w[:, :, :4]
        k = 3 if taps == 27 else 1
        P[name + ".w"] = np.ascontiguousarray(w.transpose(0, 2, 1)).reshape(co, -1, k, k, k)
        P[name + ".b"] = flat[b0:b0 + co].astype(np.float64)
    return P


def test_unet_forward_backward_matches_oracle():
    require_gpu()
    chans = (16, 32)
    net = NET.UNet(chans)
    net.init_he(3)
    rng = np.random.default_rng(9)
    flat = net.get_flat().copy()
    for name, ci, co, taps in net.layers:  # nonzero biases exercise db
        w0, b0, _, _, _ = net.offs[name]
        flat[b0:b0 + co] = rng.standard_normal(co) * 0.05
    net.set_flat(flat)
    n, d, h, w = 2, 8, 8, 12
    x4 = rng.standard_normal((n, 4, d, h, w))
    x8 = np.concatenate([x4, np.zeros_like(x4)], axis=1)
    xd, x64 = to_dev_bf16(cl(x8))
    tgt = rng.standard_normal((n, d, h, w)).astype(np.float32)
    mask = (rng.uniform(size=(n, d, h, w)) > 0.2).astype(np.uint8)
    out = net.forward(xd, n, d, h, w)
    loss = net.backward(xd, torch.from_numpy(tgt).cuda(), torch.from_numpy(mask).cuda())
    P = oracle_params(net, flat, chans)
    gsum, ltot = None, 0.0
    outs = []
    cnt = int(mask.sum())
    for i in range(n):
        xo = np.moveaxis(x64[i], -1, 0)[:4]
        y, cache = UO.forward(P, xo, chans, store_bf16=True)
        outs.append(y[0])
        dlt = (y[0] - tgt[i]) * mask[i]
        ltot += float(np.sum(dlt * dlt))
        g, _ = UO.backward(P, cache, (2.0 * dlt / cnt)[None], chans, store_bf16=True)
        gsum = g if gsum is None else {k: gsum[k] + g[k] for k in g}
    want = np.stack(outs)
    got = out.cpu().numpy().astype(np.float64)
    e_out = np.linalg.norm(got - want) / np.linalg.norm(want)
    say(f"unet out rel err {e_out:.2e}, loss {loss:.4f} vs {ltot / cnt:.4f}")
    assert e_out <= 1e-2
    assert abs(loss - ltot / cnt) <= 1e-2 * ltot / cnt
    G = net.grad.cpu().numpy().astype(np.float64)
    bad = []
    for name, ci, co, taps in net.layers:
        w0, b0, _, _, _ = net.offs[name]
        gw = G[w0:b0].reshape(co, taps, ci)
        if name == "enc0a":
            gw = gw[:, :, :4]
        k = 3 if taps == 27 else 1
        gw = np.ascontiguousarray(gw.transpose(0, 2, 1)).reshape(co, -1, k, k, k)
        for got_g, want_g, tag in ((gw, gsum[name + ".w"], "w"), (G[b0:b0 + co], gsum[name + ".b"], "b")):
            e = np.linalg.norm(got_g - want_g) / max(np.linalg.norm(want_g), 1e-30)
            cos = float(np.sum(got_g * want_g) / (np.linalg.norm(got_g) * np.linalg.norm(want_g) + 1e-300))
            say(f"  {name}.{tag}: rel {e:.2e} cos {cos:.5f}")
            bad.append((name, tag, e, cos)) if (e > 2e-2 or cos < 0.9995) else None
    assert not bad, bad


def test_pack_input_and_adam_step_moves_loss_down():
    require_gpu()
    chans = (16, 32)
    net = NET.UNet(chans)
    net.init_he(1)
    rng = np.random.default_rng(2)
    n, d, h, w = 1, 8, 8, 8
    sig = rng.standard_normal((n, d, h, w)).astype(np.float32)
    L = rng.uniform(0.5, 1.0, (n, 3, d, h, w)).astype(np.float32)
    x = torch.zeros((n, d, h, w, 8), dtype=torch.int16, device="cuda")
    UN.unet_pack_input(UN.shape(n, d, h, w), torch.from_numpy(sig).cuda(),
                       torch.from_numpy(L).cuda(), [2.0], x)
    got = bf16_to_f64(x.cpu().numpy().view(np.uint16))
    want = np.stack([sig / 2.0, L[:, 0], L[:, 1], L[:, 2]], axis=-1)
    assert np.array_equal(got[..., :4], bf16_to_f64(bf16_round(want)))
    assert np.all(got[..., 4:] == 0)
    tgt = torch.from_numpy(rng.standard_normal((n, d, h, w)).astype(np.float32)).cuda()
    mask = torch.ones((n, d, h, w), dtype=torch.uint8, device="cuda")
    losses = []
    for _ in range(30):
        net.forward(x, n, d, h, w)
        losses.append(net.backward(x, tgt, mask))
        net.adam(3e-3)
    say(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]
