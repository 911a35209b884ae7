"""Host-side choice of the weight-gradient kernel (no GPU call): the parity
cases of the row-tiled kernel cover every channel tiling it is built for,
and shapes outside its conditions take the voxel-chunk kernel."""
from paper_2607_07687_amd import unet as UN
from tests.test_gpu_unet_ops import CONV_CASES, WGRAD_ROW_CASES

ROW_TILINGS = {(8, 16, 32), (8, 32, 32), (16, 16, 32), (16, 32, 32), (32, 16, 32),
               (32, 32, 32), (8, 32, 16), (16, 32, 16), (32, 16, 16), (32, 32, 16)}


def plan(n, cin, cout, dhw):
    return UN.unet_wgrad_kernel(UN.shape(n, *dhw), cin, cout, 27)


def test_row_cases_cover_every_tiling():
    seen = set()
    for n, cin, cout, dhw in WGRAD_ROW_CASES:
        p = plan(n, cin, cout, dhw)
        assert p["rows"], (n, cin, cout, dhw)
        seen.add((p["ct"], p["ot"], p["ws"]))
    assert seen == ROW_TILINGS
    # several d ranges, a chunk count that is a multiple of 8 and one above 64
    chunks = [plan(*c)["chunks"] for c in WGRAD_ROW_CASES]
    assert any(c % 8 == 0 for c in chunks) and any(c > 64 for c in chunks)
    assert any(plan(*c)["dper"] < c[3][0] for c in WGRAD_ROW_CASES)


def test_voxel_chunk_kernel_outside_row_conditions():
    for n, cin, cout, dhw in CONV_CASES:
        p = plan(n, cin, cout, dhw)
        ok = dhw[2] % 32 == 0 or dhw[2] == 16
        if not ok or dhw[1] % 4:
            assert not p["rows"]
    assert not UN.unet_wgrad_kernel(UN.shape(1, 8, 8, 64), 16, 16, 1)["rows"]   # 1x1x1 taps
    assert not UN.unet_wgrad_kernel(UN.shape(1, 8, 8, 64), 24, 16, 27)["rows"]  # 24 channels
    assert not UN.unet_wgrad_kernel(UN.shape(1, 8, 6, 64), 16, 16, 27)["rows"]  # h = 6


def test_unet_level_shapes_take_the_row_kernel():
    # the per-level shapes of a 128^3 sample: every layer on the row kernel,
    # with partial rows within 8 Mi floats
    for cin, cout, m in [(8, 16, 128), (16, 16, 128), (32, 16, 128), (16, 32, 64), (32, 32, 64),
                         (64, 32, 64), (32, 64, 32), (64, 64, 32), (128, 64, 32), (64, 128, 16),
                         (128, 128, 16)]:
        p = plan(1, cin, cout, (m, m, m))
        assert p["rows"], (cin, cout, m)
        assert p["chunks"] * (cout * 27 * cin + cout) <= 8 << 20


def conv_instance(n, cin, cout, dhw):
    p = UN.unet_conv_kernel(UN.shape(n, *dhw), cin, cout, 27)
    return (p["kind"], cin if p["kind"] == "tile" else 0, p.get("tw", p.get("mb")), p["nb"])


def test_conv_cases_cover_every_forward_instance():
    # every (kind, input channels, tile width or voxel blocks, output blocks)
    # the plan can choose is run by a forward parity case, or by the data
    # gradient of one (a forward convolution from C_out to C_in channels)
    from tests.test_gpu_unet_ops import CONV_LARGE_CASES
    seen = {conv_instance(*c) for c in CONV_CASES + CONV_LARGE_CASES}
    seen |= {conv_instance(n, co, ci, dhw) for n, ci, co, dhw in CONV_CASES if ci >= 16}
    want = {("tile", c, tw, nb) for c in (8, 16, 32, 64) for tw in (64, 32) for nb in (1, 2, 4)}
    want |= {("gather", 0, 4, nb) for nb in (1, 2, 4, 8)} | {("gather", 0, 1, 1), ("gather", 0, 1, 2)}
    assert want <= seen, sorted(want - seen)


def test_conv_plan_fills_the_chip_on_unet_levels():
    # the U-Net's levels for a 128^3 sample: every launch of a forward or
    # data-gradient convolution has at least 256 workgroups (one per CU),
    # counting the output-channel groups, except where the output channels
    # are already split as far as they go
    for cin, cout, m in [(8, 16, 128), (16, 16, 128), (32, 16, 128), (16, 32, 64), (32, 32, 64),
                         (64, 32, 64), (32, 64, 32), (64, 64, 32), (128, 64, 32), (64, 128, 16),
                         (128, 128, 16)]:
        for ci, co in [(cin, cout), (cout, cin)]:
            if co % 16 or co > 128:
                continue
            p = UN.unet_conv_kernel(UN.shape(1, m, m, m), ci, co, 27)
            if p["kind"] == "tile":
                wgs = m ** 3 // 256 * p["groups"]
            else:
                wgs = -(-m ** 3 // (64 * p["mb"])) * p["groups"]
            assert wgs >= 256 or p["nb"] == 1, (ci, co, m, p)
