"""Pins of the U-Net oracle: convolution and selected weight-gradient entries
against torch's CPU float64 conv3d and its autograd (library routines) and
the closed form of a delta input, pooling /
upsampling adjointness, exact gradients of every layer and of a whole small
U-Net against central finite differences, and the closed form of the first
Adam step."""
import numpy as np
import pytest

from oracle import unet_oracle as U

torch = pytest.importorskip("torch")


def test_conv3d_matches_torch_cpu_float64():
    rng = np.random.default_rng(0)
    for ci, co, k, shp in [(3, 5, 3, (4, 6, 5)), (8, 2, 1, (3, 3, 4)), (2, 4, 3, (1, 2, 3))]:
        x = rng.standard_normal((ci,) + shp)
        w = rng.standard_normal((co, ci, k, k, k))
        b = rng.standard_normal(co)
        want = torch.nn.functional.conv3d(torch.from_numpy(x)[None], torch.from_numpy(w),
                                          torch.from_numpy(b), padding=k // 2)[0].numpy()
        assert np.allclose(U.conv3d(x, w, b), want, rtol=0, atol=1e-12)


def test_conv3d_points_match_torch_cpu_float64():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((4, 5, 6, 7))
    w = rng.standard_normal((3, 4, 3, 3, 3))
    b = rng.standard_normal(3)
    want = torch.nn.functional.conv3d(torch.from_numpy(x)[None], torch.from_numpy(w),
                                      torch.from_numpy(b), padding=1)[0].numpy()
    pts = [(0, 0, 0), (4, 5, 6), (2, 3, 0), (1, 0, 6), (3, 2, 4)]
    got = U.conv3d_points(x, w, b, pts)
    for i, (d, h, ww) in enumerate(pts):
        assert np.allclose(got[i], want[:, d, h, ww], rtol=0, atol=1e-12)


def test_conv3d_of_delta_is_flipped_kernel():
    # cross-correlation: a unit impulse at the centre returns w reversed in
    # every spatial direction
    rng = np.random.default_rng(1)
    w = rng.standard_normal((2, 1, 3, 3, 3))
    x = np.zeros((1, 5, 5, 5))
    x[0, 2, 2, 2] = 1.0
    y = U.conv3d(x, w, np.zeros(2))
    assert np.allclose(y[:, 1:4, 1:4, 1:4], w[:, 0, ::-1, ::-1, ::-1], atol=0)
    assert np.count_nonzero(y[:, [0, 4]]) == 0


def test_pool_upsample_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 6, 8))
    y = rng.standard_normal((3, 2, 3, 4))
    assert abs(np.sum(U.avgpool2(x) * y) - np.sum(x * U.upsample2(y)) / 8.0) <= 1e-12
    assert np.allclose(U.avgpool2(np.ones((2, 4, 4, 4))), 1.0)
    assert np.allclose(U.avgpool2_backward(y), U.upsample2(y) / 8.0)
    assert np.allclose(U.upsample2_backward(x), 8.0 * U.avgpool2(x))


def _fd_check(f, x, g, idxs, h=1e-6, tol=1e-7):
    for idx in idxs:
        old = x[idx]
        x[idx] = old + h
        fp = f()
        x[idx] = old - h
        fm = f()
        x[idx] = old
        num = (fp - fm) / (2 * h)
        assert abs(num - g[idx]) <= tol * max(1.0, abs(num)), (idx, num, g[idx])


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 3, 4, 3))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    r = rng.standard_normal((2, 3, 4, 3))
    loss = lambda: float(np.sum(U.conv3d(x, w, b) * r))
    dx, dw, db = U.conv3d_backward(x, w, r)
    _fd_check(loss, x, dx, [(0, 0, 0, 0), (2, 1, 3, 2), (1, 2, 1, 1)])
    _fd_check(loss, w, dw, [(0, 0, 0, 0, 0), (1, 2, 2, 1, 0), (0, 1, 1, 1, 1)])
    _fd_check(loss, b, db, [(0,), (1,)])


def test_wgrad_pairs_match_torch_weight_gradient():
    # the selected-entry weight gradient against torch's CPU float64 autograd
    # of conv3d (a library routine), on a grid with walls on every side
    rng = np.random.default_rng(11)
    x = rng.standard_normal((5, 4, 6, 7))
    dy = rng.standard_normal((3, 4, 6, 7))
    xt = torch.from_numpy(x)[None]
    wt = torch.zeros((3, 5, 3, 3, 3), dtype=torch.float64, requires_grad=True)
    bt = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    y = torch.nn.functional.conv3d(xt, wt, bt, padding=1)
    (y * torch.from_numpy(dy)[None]).sum().backward()
    want = wt.grad.numpy()
    pairs = [(0, 0), (2, 4), (1, 3), (2, 0)]
    got, db = U.conv3d_wgrad_pairs(x, dy, pairs)
    for i, (o, c) in enumerate(pairs):
        assert np.allclose(got[i], want[o, c], rtol=0, atol=1e-12)
    assert np.allclose(db, bt.grad.numpy(), rtol=0, atol=1e-12)


def test_unet_backward_finite_differences():
    chans = (2, 4)
    params = U.init_params(5, in_ch=3, chans=chans)
    rng = np.random.default_rng(6)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.standard_normal(params[k].shape) * 0.1
    x = rng.standard_normal((3, 4, 4, 4))
    tgt = rng.standard_normal((1, 4, 4, 4))
    mask = rng.uniform(size=(1, 4, 4, 4)) > 0.2

    def loss():
        y, _ = U.forward(params, x, chans)
        return U.mse(y, tgt, mask)[0]

    y, cache = U.forward(params, x, chans)
    _, dy = U.mse(y, tgt, mask)
    g, dx = U.backward(params, cache, dy, chans)
    assert set(g) == set(params)
    for name in ["enc0a.w", "enc1b.w", "up0.w", "dec0a.w", "dec0b.b", "head.w", "enc1a.b"]:
        arr = params[name]
        idxs = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(3)]
        _fd_check(loss, arr, g[name], idxs, tol=1e-6)
    _fd_check(loss, x, dx, [(0, 1, 2, 3), (2, 0, 0, 0)], tol=1e-6)


def test_first_adam_step_closed_form():
    # with zero moments the bias-corrected first step is lr * g / (|g| + eps)
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    st = {}
    U.adam_step(p, g, st, lr=0.1)
    want = np.array([1.0, -2.0, 3.0]) - 0.1 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, atol=1e-12)


def test_parameter_count():
    params = U.init_params(0)
    n = sum(v.size for v in params.values())
    assert 1.5e6 < n < 1.7e6


def test_bf16_storage_rounding_is_round_to_nearest_even():
    # BF16 keeps 8 significant bits: between 1 and 2 the spacing is 2^-7.
    # Halfway cases go to the even neighbour; others to the nearest; values
    # already in BF16 are kept; FP64 inputs are rounded to FP32 first
    u = 2.0 ** -7
    x = np.array([1.0, 1.0 + u / 2, 1.0 + 3 * u / 2, 1.0 + 0.49 * u, 1.0 + 0.51 * u, -1.5,
                  3.0 * 2.0 ** -130, 65504.0])
    want = np.array([1.0, 1.0, 1.0 + 2 * u, 1.0, 1.0 + u, -1.5, 3.0 * 2.0 ** -130, 65536.0])
    assert np.array_equal(U.bf16(x), want)
    # idempotent, and within half a BF16 spacing (unit roundoff 2^-8) of the input
    r = np.random.default_rng(0).standard_normal(1000)
    b = U.bf16(r)
    assert np.array_equal(U.bf16(b), b)
    assert np.all(np.abs(b - r) <= 2.0 ** -8 * np.abs(r))


def test_bf16_storage_changes_the_forward_only_by_its_rounding():
    # with BF16 storage each stored activation is within 2^-8 of the value it
    # rounds; over the network the output then moves by a few 2^-8 relative
    chans = (8, 16)
    P = U.init_params(4, 4, chans)
    x = np.random.default_rng(1).standard_normal((4, 8, 8, 8))
    y, _ = U.forward(P, x, chans)
    yb, cb = U.forward(P, x, chans, store_bf16=True)
    for k in ("enc0a", "enc0b", "enc1a", "enc1b", "up0", "dec0a", "dec0b"):
        assert np.array_equal(U.bf16(cb[k]), cb[k]), k
    e = np.linalg.norm(yb - y) / np.linalg.norm(y)
    assert 0 < e < 10 * 2.0 ** -8
