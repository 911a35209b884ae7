"""GPU parity of the U-Net operations (libunet.so) against the FP64 U-Net
oracle fed the same BF16-rounded inputs: the MFMA lane layout, convolution
forward (FP32 and BF16 outputs), data and weight gradients, pooling,
upsampling, ReLU backward, the 1x1x1 head, the masked MSE and Adam.

Tolerances: FP32-output results differ from the oracle only by FP32
accumulation order (1e-5 relative); BF16-output results also by the final
rounding to BF16 (2^-8 relative per element)."""
import numpy as np
import pytest

from oracle import unet_oracle as UO
from paper_2607_07687_amd import unet as UN
from tests.gpu_util import require_gpu, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def bf16_round(a):
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return u


def bf16_to_f64(u):
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def to_dev_bf16(a):
    """FP64 array -> (device int16 tensor of BF16 bits, FP64 of the rounded values)."""
    u = bf16_round(a)
    return torch.from_numpy(u.view(np.int16).copy()).cuda(), bf16_to_f64(u)


def from_dev_bf16(t):
    return bf16_to_f64(t.cpu().numpy().view(np.uint16))


def cl(x):
    """[n][C][D][H][W] -> channels-last [n][D][H][W][C]."""
    return np.ascontiguousarray(np.moveaxis(x, 1, -1))


def cf(x):
    return np.ascontiguousarray(np.moveaxis(x, -1, 1))


def w_gpu(w):
    """oracle [co][ci][3][3][3] -> [co][27][ci]"""
    co, ci = w.shape[:2]
    return np.ascontiguousarray(w.reshape(co, ci, -1).transpose(0, 2, 1))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_mfma_lane_layout():
    require_gpu()
    rng = np.random.default_rng(0)
    A = rng.integers(-4, 5, (16, 32)).astype(np.float64)
    B = rng.integers(-4, 5, (32, 16)).astype(np.float64)
    Ad, _ = to_dev_bf16(A)
    Bd, _ = to_dev_bf16(B)
    out = torch.zeros(256, dtype=torch.float32, device="cuda")
    UN.unet_mfma_selfcheck(Ad, Bd, out)
    assert np.array_equal(out.cpu().numpy().reshape(16, 16), (A @ B).astype(np.float32))


CONV_CASES = [(2, 8, 16, (5, 6, 7)), (1, 16, 32, (4, 4, 9)), (2, 32, 64, (3, 5, 4)),
              (1, 64, 128, (4, 3, 3)), (1, 128, 16, (2, 3, 4)),
              # w a multiple of 64 and h of 4, 16 or 32 channels in and out: the
              # LDS-tiled kernel (walls of the tile's neighbourhood on every side)
              (1, 16, 16, (3, 8, 64)), (2, 32, 32, (2, 4, 64)), (1, 16, 32, (2, 4, 128)),
              (1, 32, 16, (3, 4, 64)), (2, 8, 16, (2, 4, 64)), (1, 8, 32, (3, 8, 64)),
              (1, 64, 64, (2, 4, 64)), (1, 32, 64, (3, 4, 64)), (1, 64, 16, (2, 8, 64)),
              # w = 32, h a multiple of 8: 32 x 8 tiles
              (2, 32, 64, (2, 8, 32)), (1, 64, 64, (3, 16, 32)), (1, 16, 32, (2, 8, 32)),
              (2, 8, 16, (3, 8, 32))]


@pytest.mark.parametrize("n,cin,cout,dhw", CONV_CASES)
def test_conv_forward(n, cin, cout, dhw):
    require_gpu()
    say(f"conv fwd {n} {cin}->{cout} {dhw}")
    rng = np.random.default_rng(cin + cout)
    x = rng.standard_normal((n, cin) + dhw)
    w = rng.standard_normal((cout, cin, 3, 3, 3)) / np.sqrt(27 * cin)
    b = rng.standard_normal(cout) * 0.1
    xd, x64 = to_dev_bf16(cl(x))
    wd, w64 = to_dev_bf16(w_gpu(w))
    bd = torch.from_numpy(b.astype(np.float32)).cuda()
    w64o = w64.reshape(cout, 27, cin).transpose(0, 2, 1).reshape(cout, cin, 3, 3, 3)
    want = np.stack([UO.conv3d(cf(x64)[i], w64o, b.astype(np.float32)) for i in range(n)])
    s = UN.shape(n, *dhw)
    yf = torch.zeros((n,) + dhw + (cout,), dtype=torch.float32, device="cuda")
    UN.unet_conv_fwd(s, UN.act(xd, cin, 0, cin), wd, bd, 27, UN.act(None, cout, 0, cout), yf, 0)
    assert rel(cf(yf.cpu().numpy().astype(np.float64)), want) <= 1e-5
    # BF16 output with ReLU, written into channel slice [cout, 2 cout) of a wider row
    yb = torch.zeros((n,) + dhw + (2 * cout,), dtype=torch.int16, device="cuda")
    UN.unet_conv_fwd(s, UN.act(xd, cin, 0, cin), wd, bd, 27, UN.act(yb, 2 * cout, cout, cout),
                     None, 1)
    got = cf(from_dev_bf16(yb)[..., cout:])
    wr = np.maximum(want, 0.0)
    assert np.all(np.abs(got - wr) <= 2.0 ** -8 * np.abs(wr) + 1e-5 * np.abs(wr).max())
    assert np.all(from_dev_bf16(yb)[..., :cout] == 0.0)


@pytest.mark.parametrize("n,cin,cout,dhw", [c for c in CONV_CASES if c[1] >= 16])
def test_conv_dgrad_and_wgrad(n, cin, cout, dhw):
    require_gpu()
    say(f"conv bwd {n} {cin}->{cout} {dhw}")
    rng = np.random.default_rng(7 + cin)
    x = rng.standard_normal((n, cin) + dhw)
    w = rng.standard_normal((cout, cin, 3, 3, 3)) / np.sqrt(27 * cin)
    dy = rng.standard_normal((n, cout) + dhw)
    xd, x64 = to_dev_bf16(cl(x))
    wd, w64 = to_dev_bf16(w_gpu(w))
    dyd, dy64 = to_dev_bf16(cl(dy))
    w64o = w64.reshape(cout, 27, cin).transpose(0, 2, 1).reshape(cout, cin, 3, 3, 3)
    dxs, dws, dbs = [], 0.0, 0.0
    for i in range(n):
        dx_i, dw_i, db_i = UO.conv3d_backward(cf(x64)[i], w64o, cf(dy64)[i])
        dxs.append(dx_i)
        dws = dws + dw_i
        dbs = dbs + db_i
    s = UN.shape(n, *dhw)
    dx = torch.zeros((n,) + dhw + (cin,), dtype=torch.int16, device="cuda")
    wflip = torch.empty(cout * 27 * cin, dtype=torch.int16, device="cuda")
    UN.unet_conv_dgrad(s, UN.act(dyd, cout, 0, cout), wd, 27, UN.act(dx, cin, 0, cin), wflip)
    want = np.stack(dxs)
    got = cf(from_dev_bf16(dx))
    assert np.all(np.abs(got - want) <= 2.0 ** -8 * np.abs(want) + 1e-5 * np.abs(want).max())
    ws = torch.empty(UN.unet_wgrad_workspace(s, cin, cout, 27) // 4 + 1, dtype=torch.float32,
                     device="cuda")
    dw = torch.zeros(cout * 27 * cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    UN.unet_conv_wgrad(s, UN.act(xd, cin, 0, cin), UN.act(dyd, cout, 0, cout), 27, dw, db, ws)
    got_w = dw.cpu().numpy().astype(np.float64).reshape(cout, 27, cin).transpose(0, 2, 1)
    assert rel(got_w.reshape(cout, cin, 3, 3, 3), dws) <= 1e-5
    assert rel(db.cpu().numpy().astype(np.float64), dbs) <= 1e-5


# Forward cases on larger grids, compared at sampled voxels (every output
# channel), chosen so that with CONV_CASES every kernel instance the launch
# plan can pick runs at least once (tests/test_unet_plan.py checks this on
# the host).  LDS tiles with 2 and 4 output blocks per wave for 8, 16, 32 and
# 64 input channels on 64 x 4 and 32 x 8 tiles (grids with enough tiles that
# the output channels are not split); gathered operands with 64 voxels per
# wave and 8, 4 (of 8), 2 (of 4) and 1 output blocks, or 16 voxels and 2 (of
# 8).  Small grids, as in CONV_CASES, take one output block per wave.
CONV_LARGE_CASES = ([(1, cin, 16 * nb, (64, 64, 64) if tw == 64 else (128, 64, 32))
                     for cin in (8, 16, 32, 64) for nb in (2, 4) for tw in (64, 32)]
                    + [(1, 24, 128, (16, 64, 64)), (1, 64, 128, (32, 32, 32)),
                       (1, 128, 64, (32, 32, 32)), (1, 24, 16, (16, 64, 64)),
                       (1, 128, 128, (16, 16, 16))])


@pytest.mark.parametrize("n,cin,cout,dhw", CONV_LARGE_CASES)
def test_conv_forward_large(n, cin, cout, dhw):
    require_gpu()
    say(f"conv fwd large {n} {cin}->{cout} {dhw}")
    rng = np.random.default_rng(200 + cin + cout)
    x = rng.standard_normal((n, cin) + dhw).astype(np.float32)
    w = rng.standard_normal((cout, cin, 3, 3, 3)) / np.sqrt(27 * cin)
    b = rng.standard_normal(cout) * 0.1
    xd, x64 = to_dev_bf16(cl(x))
    wd, w64 = to_dev_bf16(w_gpu(w))
    bd = torch.from_numpy(b.astype(np.float32)).cuda()
    w64o = w64.reshape(cout, 27, cin).transpose(0, 2, 1).reshape(cout, cin, 3, 3, 3)
    d, h, ww = dhw
    pts = [(0, 0, 0), (d - 1, h - 1, ww - 1), (0, h - 1, 0), (d - 1, 0, ww - 1)]
    pts += [tuple(int(rng.integers(0, m)) for m in dhw) for _ in range(60)]
    want = UO.conv3d_points(cf(x64)[0], w64o, b.astype(np.float32).astype(np.float64), pts)
    s = UN.shape(n, *dhw)
    yf = torch.full((n,) + dhw + (cout,), np.nan, dtype=torch.float32, device="cuda")
    UN.unet_conv_fwd(s, UN.act(xd, cin, 0, cin), wd, bd, 27, UN.act(None, cout, 0, cout), yf, 0)
    y = yf.cpu().numpy()
    assert np.all(np.isfinite(y))
    got = np.stack([y[0][p] for p in pts]).astype(np.float64)
    assert rel(got, want) <= 1e-5


# Weight-gradient cases of the row-tiled kernel, one or more per channel tiling
# (input channels, output channels, w extent of a workgroup): 4-row blocks of
# w = 32k or w = 16 grids, several d ranges per sample, XCD-grouped chunk
# order (chunk count a multiple of 8) and two-level partial sums (more than 64
# chunks).  Entries are compared on sampled (o, c) pairs (all 27 taps) and the
# whole bias gradient.
WGRAD_ROW_CASES = [
    (1, 8, 16, (16, 8, 64)), (1, 8, 32, (128, 64, 32)), (1, 16, 16, (12, 8, 96)),
    (1, 16, 32, (128, 64, 32)), (1, 32, 16, (128, 64, 32)), (1, 64, 64, (64, 32, 32)),
    (1, 8, 32, (8, 8, 16)), (2, 16, 32, (4, 8, 16)), (1, 32, 16, (6, 4, 16)),
    (1, 128, 128, (32, 16, 16))]


@pytest.mark.parametrize("n,cin,cout,dhw", WGRAD_ROW_CASES)
def test_conv_wgrad_rows(n, cin, cout, dhw):
    require_gpu()
    plan = UN.unet_wgrad_kernel(UN.shape(n, *dhw), cin, cout, 27)
    say(f"conv wgrad rows {n} {cin}->{cout} {dhw} {plan}")
    assert plan["rows"]
    rng = np.random.default_rng(100 + cin + cout)
    x = rng.standard_normal((n, cin) + dhw)
    dy = rng.standard_normal((n, cout) + dhw)
    # x as a channel slice [8, 8 + cin) of a wider row, dy plain
    xw = np.zeros((n,) + dhw + (cin + 16,))
    xw[..., 8:8 + cin] = cl(x)
    xd, xw64 = to_dev_bf16(xw)
    x64 = cf(xw64[..., 8:8 + cin])
    dyd, dy64 = to_dev_bf16(cl(dy))
    dy64 = cf(dy64)
    pairs = sorted({(int(o), int(c)) for o, c in zip(rng.integers(0, cout, 24),
                                                    rng.integers(0, cin, 24))}
                   | {(0, 0), (cout - 1, cin - 1)})
    want = 0.0
    want_b = 0.0
    for i in range(n):
        g, b = UO.conv3d_wgrad_pairs(x64[i], dy64[i], pairs)
        want = want + g
        want_b = want_b + b
    s = UN.shape(n, *dhw)
    ws = torch.empty(UN.unet_wgrad_workspace(s, cin, cout, 27) // 4 + 1, dtype=torch.float32,
                     device="cuda")
    dw = torch.full((cout * 27 * cin,), np.nan, dtype=torch.float32, device="cuda")
    db = torch.full((cout,), np.nan, dtype=torch.float32, device="cuda")
    UN.unet_conv_wgrad(s, UN.act(xd, cin + 16, 8, cin), UN.act(dyd, cout, 0, cout), 27, dw, db, ws)
    got = dw.cpu().numpy().astype(np.float64).reshape(cout, 3, 3, 3, cin)
    assert np.all(np.isfinite(got))
    got_p = np.stack([got[o, :, :, :, c] for o, c in pairs])
    assert rel(got_p, want) <= 1e-5
    assert rel(db.cpu().numpy().astype(np.float64), want_b) <= 1e-5
    # a second call gives bitwise the same result (fixed summation order)
    dw2 = torch.empty_like(dw)
    db2 = torch.empty_like(db)
    UN.unet_conv_wgrad(s, UN.act(xd, cin + 16, 8, cin), UN.act(dyd, cout, 0, cout), 27, dw2, db2,
                       ws)
    assert torch.equal(dw, dw2) and torch.equal(db, db2)


def put(a_cl, ld):
    """channels-last FP64 array -> (device BF16 rows of ld channels holding a
    in the first C, FP64 of the rounded values)."""
    c = a_cl.shape[-1]
    full = np.zeros(a_cl.shape[:-1] + (ld,))
    full[..., :c] = a_cl
    d, r = to_dev_bf16(full)
    return d, r[..., :c]


def zeros_ld(shape, ld):
    return torch.zeros(tuple(shape) + (ld,), dtype=torch.int16, device="cuda")


def got_c(t, c):
    """device BF16 rows -> FP64 [n][C][...] of the first c channels; the
    channels beyond c must be untouched (zero)."""
    a = from_dev_bf16(t)
    assert np.all(a[..., c:] == 0.0)
    return cf(a[..., :c])


# (channels, row length): 8-channel vector kernels, and one-channel kernels
# for a count that is not a multiple of 8
@pytest.mark.parametrize("c,ld", [(16, 16), (16, 24), (4, 8), (12, 16)])
def test_pool_upsample_relu_bwd(c, ld):
    require_gpu()
    say(f"pool/upsample/relu c={c} ld={ld}")
    rng = np.random.default_rng(3)
    n, dhw = 2, (4, 6, 8)
    x = rng.standard_normal((n, c) + dhw)
    xd, x64 = put(cl(x), ld)
    x64 = cf(x64)
    fine = UN.shape(n, *dhw)
    coarse = UN.shape(n, 2, 3, 4)
    yp = zeros_ld((n, 2, 3, 4), ld)
    UN.unet_pool_fwd(fine, UN.act(xd, ld, 0, c), UN.act(yp, ld, 0, c))
    want = np.stack([UO.avgpool2(x64[i]) for i in range(n)])
    got = got_c(yp, c)
    assert np.all(np.abs(got - want) <= 2.0 ** -8 * np.abs(want) + 1e-7)
    # upsample of the pooled values, and the adjoint sums
    yu = zeros_ld((n,) + dhw, ld)
    UN.unet_up_fwd(coarse, UN.act(yp, ld, 0, c), UN.act(yu, ld, 0, c))
    assert np.array_equal(got_c(yu, c), np.stack([UO.upsample2(g) for g in got]))
    dyd, dy64 = put(cl(rng.standard_normal((n, c) + dhw)), ld)
    dy64 = cf(dy64)
    du = zeros_ld((n, 2, 3, 4), ld)
    UN.unet_up_bwd(coarse, UN.act(dyd, ld, 0, c), UN.act(du, ld, 0, c))
    want = np.stack([UO.upsample2_backward(dy64[i]) for i in range(n)])
    gu = got_c(du, c)
    assert np.all(np.abs(gu - want) <= 2.0 ** -8 * np.abs(want) + 1e-6)
    dp = zeros_ld((n,) + dhw, ld)
    UN.unet_pool_bwd(fine, UN.act(du, ld, 0, c), UN.act(dp, ld, 0, c), 0)
    want = np.stack([UO.avgpool2_backward(gu[i]) for i in range(n)])
    assert np.array_equal(got_c(dp, c), want)
    # accumulate = 1 adds the pooled gradient to what dx holds (BF16 sum)
    UN.unet_pool_bwd(fine, UN.act(du, ld, 0, c), UN.act(dp, ld, 0, c), 1)
    assert np.all(np.abs(got_c(dp, c) - 2 * want) <= 2.0 ** -8 * np.abs(2 * want))
    # ReLU backward keeps dy where y > 0
    ro = zeros_ld((n,) + dhw, ld)
    UN.unet_relu_bwd(fine, UN.act(xd, ld, 0, c), UN.act(dyd, ld, 0, c), UN.act(ro, ld, 0, c))
    want = np.stack([UO.relu_backward(x64[i], dy64[i]) for i in range(n)])
    assert np.array_equal(got_c(ro, c), want)


@pytest.mark.parametrize("c,ld", [(16, 16), (12, 16)])
def test_head_mse_adam(c, ld):
    require_gpu()
    say(f"head/mse/adam c={c} ld={ld}")
    rng = np.random.default_rng(4)
    n, dhw = 2, (3, 4, 5)
    x = rng.standard_normal((n, c) + dhw)
    xd, x64 = put(cl(x), ld)
    w = rng.standard_normal(c).astype(np.float32)
    b = np.float32(0.3)
    s = UN.shape(n, *dhw)
    wd = torch.from_numpy(w).cuda()
    bd = torch.tensor([b], dtype=torch.float32, device="cuda")
    y = torch.zeros((n,) + dhw, dtype=torch.float32, device="cuda")
    UN.unet_head_fwd(s, UN.act(xd, ld, 0, c), wd, bd, y)
    w5 = w.astype(np.float64).reshape(1, c, 1, 1, 1)
    want = np.stack([UO.conv3d(cf(x64)[i], w5, np.array([float(b)]))[0] for i in range(n)])
    assert rel(y.cpu().numpy().astype(np.float64), want) <= 1e-6
    tgt = rng.standard_normal((n,) + dhw).astype(np.float32)
    mask = (rng.uniform(size=(n,) + dhw) > 0.3).astype(np.uint8)
    dpred = torch.zeros_like(y)
    stats = torch.zeros(2 + 512, dtype=torch.float64, device="cuda")
    loss = UN.unet_mse(s, y, torch.from_numpy(tgt).cuda(), torch.from_numpy(mask).cuda(), dpred,
                       stats)
    yl = y.cpu().numpy().astype(np.float64)
    lo, dlo = UO.mse(yl, tgt.astype(np.float64), mask.astype(bool))
    assert abs(loss - lo) <= 1e-9 * lo
    assert rel(dpred.cpu().numpy().astype(np.float64), dlo) <= 1e-6
    ws = torch.empty(UN.unet_head_workspace(s, c) // 4 + 1, dtype=torch.float32, device="cuda")
    dw = torch.zeros(c, dtype=torch.float32, device="cuda")
    db = torch.zeros(1, dtype=torch.float32, device="cuda")
    dx = torch.zeros_like(xd)
    UN.unet_head_bwd(s, UN.act(xd, ld, 0, c), wd, dpred, UN.act(dx, ld, 0, c), dw, db, ws)
    dp64 = dpred.cpu().numpy().astype(np.float64)
    gx, gw, gb = 0.0, 0.0, 0.0
    dxs = []
    for i in range(n):
        dx_i, dw_i, db_i = UO.conv3d_backward(cf(x64)[i], w5, dp64[i][None])
        dxs.append(dx_i)
        gw, gb = gw + dw_i, gb + db_i
    assert rel(dw.cpu().numpy().astype(np.float64), gw.reshape(c)) <= 1e-5
    assert abs(float(db.item()) - float(gb[0])) <= 1e-5 * abs(float(gb[0])) + 1e-7
    want = np.stack(dxs)
    assert np.all(np.abs(got_c(dx, c) - want) <= 2.0 ** -8 * np.abs(want) + 1e-7)
    # Adam: two steps against the oracle's
    p0 = rng.standard_normal(1000)
    g1, g2 = rng.standard_normal(1000), rng.standard_normal(1000)
    master = torch.from_numpy(p0.astype(np.float32)).cuda()
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    out16 = torch.zeros(1000, dtype=torch.int16, device="cuda")
    po = {"p": p0.astype(np.float32).astype(np.float64)}
    st = {}
    for t, g in ((1, g1), (2, g2)):
        gd = torch.from_numpy(g.astype(np.float32)).cuda()
        UN.unet_adam(master, m, v, gd, out16, 1e-3, t)
        UO.adam_step(po, {"p": g.astype(np.float32).astype(np.float64)}, st, 1e-3)
    assert rel(master.cpu().numpy().astype(np.float64) - p0, po["p"] - p0) <= 1e-4
    assert np.array_equal(out16.cpu().numpy().view(np.uint16), bf16_round(master.cpu().numpy()))


def test_head_backward_many_chunks():
    # 131072 voxels: 128 voxel chunks, summed in two levels
    require_gpu()
    rng = np.random.default_rng(5)
    n, c, dhw = 2, 16, (16, 64, 64)
    x = rng.standard_normal((n, c) + dhw)
    xd, x64 = to_dev_bf16(cl(x))
    w = rng.standard_normal(c).astype(np.float32)
    dy = rng.standard_normal((n,) + dhw).astype(np.float32)
    s = UN.shape(n, *dhw)
    ws = torch.empty(UN.unet_head_workspace(s, c) // 4 + 1, dtype=torch.float32, device="cuda")
    dw = torch.zeros(c, dtype=torch.float32, device="cuda")
    db = torch.zeros(1, dtype=torch.float32, device="cuda")
    UN.unet_head_bwd(s, UN.act(xd, c, 0, c), torch.from_numpy(w).cuda(),
                     torch.from_numpy(dy).cuda(), UN.act(None, c, 0, c), dw, db, ws)
    w5 = w.astype(np.float64).reshape(1, c, 1, 1, 1)
    gw, gb = 0.0, 0.0
    for i in range(n):
        _, dw_i, db_i = UO.conv3d_backward(cf(x64)[i], w5, dy[i].astype(np.float64)[None])
        gw, gb = gw + dw_i, gb + db_i
    assert rel(dw.cpu().numpy().astype(np.float64), gw.reshape(c)) <= 1e-5
    assert abs(float(db.item()) - float(gb[0])) <= 1e-5 * np.abs(dy).sum()


def test_scale_to_fp32_and_fp64():
    require_gpu()
    v = np.random.default_rng(8).standard_normal(1000).astype(np.float32)
    vd = torch.from_numpy(v).cuda()
    o32 = torch.zeros_like(vd)
    o64 = torch.zeros(1000, dtype=torch.float64, device="cuda")
    UN.unet_scale(vd, 2.5, o32)
    UN.unet_scale_f64(vd, 0.1, o64)
    assert np.array_equal(o32.cpu().numpy(), (np.float32(2.5) * v).astype(np.float32))
    assert np.array_equal(o64.cpu().numpy(), 0.1 * v.astype(np.float64))
