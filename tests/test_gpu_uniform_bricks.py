"""GPU checks of the uniform-brick map (blocks of 128 x 2 x 2 cells whose
faces are one constant per direction, low walls at zero, and whether all
their cells are active): the map of every level agrees with the rule
evaluated on the host from the level's faces, and every entry point whose
kernels read it (residual and its norms, the allocation-free residual, the
fused residual + restriction, the two-sweep pass through its table of tile
modes, V-cycles, solves, the deferred decision) gives bitwise the results of
a handle without the map, on walls, periodic directions, holes, ragged
tails, FP32/FP64 iterates and FP32/BF16/FP64 faces, after gmg_update_faces
and after a change of tiling.  The kernels without the map are themselves
checked against the oracle in test_gpu_parity.py."""
import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P
from tests.gpu_util import dev, require_gpu, rounded, say, torch
from tests.test_gpu_parity import STORE

pytestmark = pytest.mark.gpu

UBX, UBY, UBZ = 128, 2, 2


def layered(n, per, split=8):
    """L = 1 below plane `split` and (x, y faces) 2 above, z faces 1: bricks
    on both sides are uniform with different constants, so a z-range that
    spans both must take the stored faces."""
    L = np.ones((3, n[2], n[1], n[0]))
    L[0, split:] = 2.0
    L[1, split:] = 2.0
    L = P.zero_wall_faces(L, per)
    u = np.random.default_rng(5).uniform(-1.0, 1.0, L.shape)
    return L, P.rhs_from_velocity(L, u, per), per


def solid_slab(n, per, lo=10, hi=20):
    """L = 1 except a slab of planes [lo, hi) whose faces (and the z faces
    into it from above) are 0: inactive cells in bricks of uniform zero
    faces, next to uniform active bricks."""
    L = np.ones((3, n[2], n[1], n[0]))
    L[:, lo:hi] = 0.0
    L[2, hi] = 0.0
    L = P.zero_wall_faces(L, per)
    u = np.random.default_rng(8).uniform(-1.0, 1.0, L.shape)
    return L, P.rhs_from_velocity(L, u, per), per


# (name, builder) -> (L, sigma, periodic); level 0 at least 128 cells in x
CASES = {
    "sphere_walls": lambda: P.sphere_box((256, 40, 36), (128.0, 20.0, 18.0), 7.0, "uniform", 1),
    "tgv_periodic": lambda: P.tgv_periodic(128, seed=0),
    "holes_mixed": lambda: P.random_problem((256, 18, 22), (True, False, False), seed=4,
                                            contrast=0.0, holes=0.002),
    "ragged_walls": lambda: P.sphere_box((300, 21, 19), (60.0, 10.0, 9.0), 4.0, "uniform", 2),
    "layered_z": lambda: layered((256, 16, 40), (False, True, True)),
    "solid_slab": lambda: solid_slab((256, 16, 40), (True, True, False)),
    # 2^23 cells: the default mode's two-sweep pass takes the map on level 0
    "sphere_2p23": lambda: P.sphere_box((256, 256, 128), (128.0, 128.0, 64.0), 32.0,
                                        "uniform", 3),
}
SMALL = [c for c in CASES if c != "sphere_2p23"]


def level_faces(h, l, storage, prec):
    (nx, ny, nz), _ = G.gmg_level_shape(h, l)
    shape = (3, nz, ny, nx)
    if storage == "bf16":
        raw = torch.empty(shape, dtype=torch.int16, device="cuda")
        G.gmg_level_faces(h, l, raw)
        bits = raw.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
        return bits.view(np.float32).astype(np.float64)
    dt = torch.float64 if storage == "f64" else torch.float32
    out = torch.empty(shape, dtype=dt, device="cuda")
    G.gmg_level_faces(h, l, out)
    return out.cpu().numpy().astype(np.float64)


def host_uniform(L, per, active=False):
    """(uniform bricks, bricks) by the rule, from a level's faces as FP64;
    with active, (uniform bricks, those whose cells are all active by the
    oracle's active set, bricks)."""
    _, nz, ny, nx = L.shape
    bits = L.view(np.int64)
    act = O.active_set(L, per)
    nact = 0
    nbx, nby, nbz = -(-nx // UBX), -(-ny // UBY), -(-nz // UBZ)
    count = 0
    for bz in range(nbz):
        k0 = bz * UBZ
        for by in range(nby):
            j0 = by * UBY
            for bx in range(nbx):
                i0 = bx * UBX
                if i0 + UBX > nx or j0 + UBY > ny or k0 + UBZ > nz:
                    continue
                u = L[:, k0 + 1, j0 + 1, i0 + 1]
                ok = True
                for d in range(3):
                    want = np.full((UBZ, UBY, UBX), u[d])
                    lo = (i0, j0, k0)[d]
                    if lo == 0 and not per[d]:
                        sl = [slice(None)] * 3
                        sl[2 - d] = 0
                        want[tuple(sl)] = 0.0
                    got = bits[d, k0:k0 + UBZ, j0:j0 + UBY, i0:i0 + UBX]
                    ok &= bool(np.array_equal(got, want.view(np.int64)))
                    # the faces beyond the brick's high side, unless a wall
                    hi = (i0 + UBX, j0 + UBY, k0 + UBZ)[d]
                    nd = (nx, ny, nz)[d]
                    if hi < nd or per[d]:
                        h0 = hi % nd
                        if d == 0:
                            got = bits[0, k0:k0 + UBZ, j0:j0 + UBY, h0]
                        elif d == 1:
                            got = bits[1, k0:k0 + UBZ, h0, i0:i0 + UBX]
                        else:
                            got = bits[2, h0, j0:j0 + UBY, i0:i0 + UBX]
                        ok &= bool(np.all(got == np.float64(u[d]).view(np.int64)))
                count += ok
                nact += ok and bool(act[k0:k0 + UBZ, j0:j0 + UBY, i0:i0 + UBX].all())
    return (count, nact, nbx * nby * nbz) if active else (count, nbx * nby * nbz)


def pair(name, prec, storage, mode=2):
    """Handles with the map (mode 2: on every level, so that these small
    grids exercise it; 1: the default, on levels of at least 2^21 cells)
    and without it, on the same inputs."""
    require_gpu()
    L, s, per = CASES[name]()
    n = (L.shape[3], L.shape[2], L.shape[1])
    dt = G.GMG_F64 if prec == "f64" else G.GMG_F32
    Ld, sd = dev(rounded(L, prec), prec), dev(rounded(s, prec), prec)
    hu = G.gmg_setup(G.gmg_default_params(n, per, dt, l_storage=STORE[storage],
                                          uniform_bricks=mode), Ld)
    ho = G.gmg_setup(G.gmg_default_params(n, per, dt, l_storage=STORE[storage],
                                          uniform_bricks=0), Ld)
    return hu, ho, sd, per


PRECS = [("f32", "f32"), ("f32", "bf16"), ("f64", "f64")]


@pytest.mark.parametrize("prec,storage", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_map_matches_host_rule(name, prec, storage):
    say(f"uniform map {name} {prec}/{storage}")
    hu, ho, _, per = pair(name, prec, storage)
    for l in range(G.gmg_num_levels(hu)):
        got = G.gmg_level_uniform(hu, l, active=True)
        want = host_uniform(level_faces(hu, l, storage, prec), per, active=True)
        assert got == want, f"level {l}: {got} vs {want}"
        assert G.gmg_level_uniform(ho, l) == (0, 0)
    if name in ("sphere_walls", "tgv_periodic", "layered_z", "solid_slab"):
        u, a, t = G.gmg_level_uniform(hu, 0, active=True)
        assert u >= t // 2 > 0, (u, t)  # the constant-face path is exercised
        if name == "solid_slab":
            assert 0 < a < u  # uniform bricks of inactive cells too
    hu.close()
    ho.close()


def check_same(hu, ho, sd, prec, seed=3):
    x = dev(rounded(np.random.default_rng(seed).standard_normal(tuple(sd.shape)), prec), prec)
    # residual and its norms
    ra, rb = torch.empty_like(sd), torch.empty_like(sd)
    na = G.gmg_residual(hu, x, sd, ra)
    nb = G.gmg_residual(ho, x, sd, rb)
    assert torch.equal(ra, rb)
    assert na == nb
    # the allocation-free residual
    ra.zero_()
    rb.zero_()
    za = torch.zeros(2, dtype=torch.float64, device="cuda")
    zb = torch.zeros(2, dtype=torch.float64, device="cuda")
    G.gmg_residual_noalloc(hu, x, sd, ra, za)
    G.gmg_residual_noalloc(ho, x, sd, rb, zb)
    torch.cuda.synchronize()
    assert torch.equal(ra, rb) and torch.equal(za, zb)
    # fused residual + restriction on every level that has a coarser one
    for l in range(G.gmg_num_levels(hu) - 1):
        (nx, ny, nz), _ = G.gmg_level_shape(hu, l)
        (cx, cy, cz), _ = G.gmg_level_shape(hu, l + 1)
        g = np.random.default_rng(seed + l)
        xl = dev(g.standard_normal((nz, ny, nx)), prec)
        sl = dev(g.standard_normal((nz, ny, nx)), prec)
        outs = []
        for h in (hu, ho):
            sc = torch.full((cz, cy, cx), 7.0, dtype=sd.dtype, device="cuda")
            xc = torch.full((cz, cy, cx), 7.0, dtype=sd.dtype, device="cuda")
            G.gmg_restrict_residual(h, l, xl, sl, sc, xc)
            outs.append((sc, xc))
        assert torch.equal(outs[0][0], outs[1][0]), f"level {l}"
        assert torch.equal(outs[0][1], outs[1][1]), f"level {l}"
    # V-cycles from a random and from a zero guess, then a whole solve
    xa, xb = x.clone(), x.clone()
    assert G.gmg_vcycle(hu, xa, sd, True) == G.gmg_vcycle(ho, xb, sd, True)
    assert torch.equal(xa, xb)
    xa.zero_()
    xb.zero_()
    ia = G.gmg_solve(hu, xa, sd, 1e-5, 40)
    ib = G.gmg_solve(ho, xb, sd, 1e-5, 40)
    assert torch.equal(xa, xb)
    assert ia["history"] == ib["history"] and ia["status"] == ib["status"]


@pytest.mark.parametrize("prec,storage", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_bitwise_with_and_without_map(name, prec, storage):
    say(f"uniform bitwise {name} {prec}/{storage}")
    hu, ho, sd, _ = pair(name, prec, storage)
    check_same(hu, ho, sd, prec)
    hu.close()
    ho.close()


@pytest.mark.parametrize("prec,storage", [("f32", "f32"), ("f32", "bf16")])
def test_update_faces_rebuilds_map(prec, storage):
    """A body that moves: the map follows gmg_update_faces (the same as a
    fresh handle's), and results stay bitwise those without the map."""
    say(f"uniform update {prec}/{storage}")
    hu, ho, sd, per = pair("sphere_walls", prec, storage)
    L2, s2, _ = P.sphere_box((256, 40, 36), (200.0, 26.0, 15.0), 9.0, "uniform", 4)
    L2d, s2d = dev(rounded(L2, prec), prec), dev(rounded(s2, prec), prec)
    before = G.gmg_level_uniform(hu, 0)
    G.gmg_update_faces(hu, L2d)
    G.gmg_update_faces(ho, L2d)
    fresh = G.gmg_setup(G.gmg_default_params((256, 40, 36), per, G.GMG_F32,
                                             l_storage=STORE[storage], uniform_bricks=2), L2d)
    for l in range(G.gmg_num_levels(hu)):
        assert G.gmg_level_uniform(hu, l) == G.gmg_level_uniform(fresh, l)
        assert G.gmg_level_uniform(hu, l) == host_uniform(level_faces(hu, l, storage, prec), per)
    assert G.gmg_level_uniform(hu, 0) != before
    check_same(hu, ho, s2d, prec, seed=9)
    for h in (hu, ho, fresh):
        h.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_default_mode_at_2p23_cells(storage):
    """The default mode on a level of 2^23 cells (its kernels take the map
    there, tiles near the sphere not): bitwise the results without the
    map."""
    say(f"uniform default mode 256x256x128 f32/{storage}")
    hu, ho, sd, per = pair("sphere_2p23", "f32", storage, mode=1)
    u, t = G.gmg_level_uniform(hu, 0)
    assert t == 2 * 128 * 64 and 0 < u < t
    check_same(hu, ho, sd, "f32")
    hu.close()
    ho.close()


def set_pairs_everywhere(h, ty, kc):
    """Two-sweep passes on every level with an even nx (z-chunk min(kc, nz))."""
    for l in range(G.gmg_num_levels(h)):
        (nx, _, nz), _ = G.gmg_level_shape(h, l)
        G.gmg_set_pair_sweeps(h, l, min(kc, nz) if nx % 2 == 0 else 0, ty)


@pytest.mark.parametrize("tiling", [(16, 3), (8, 2), (16, 8)], ids=lambda t: f"{t[0]}x{t[1]}")
@pytest.mark.parametrize("name", ["sphere_walls", "tgv_periodic", "solid_slab", "layered_z"])
def test_pass_tile_modes_on_every_level(name, tiling):
    """Passes on every level read the table of their tiles' face modes (found
    when the tiling is set): bitwise the passes without the map, through
    V-cycles and a solve, then again after the tiling changes."""
    say(f"uniform tile modes {name} {tiling}")
    hu, ho, sd, _ = pair(name, "f32", "f32")
    for ty, kc in (tiling, (16 if tiling[0] == 8 else 8, tiling[1] + 1)):
        for h in (hu, ho):
            set_pairs_everywhere(h, ty, kc)
        check_same(hu, ho, sd, "f32", seed=11)
    hu.close()
    ho.close()


@pytest.mark.parametrize("name", ["sphere_walls", "tgv_periodic", "solid_slab"])
def test_deferred_norm_pass_with_map(name):
    """The deferred decision's first pass (which also sums its input's
    residual, one partial per workgroup) in the uniform-face variants: solves
    bitwise those without the map, histories and decisions included, at the
    same pass tiling (the default z-chunk differs with the map, and with it
    the partials' grouping)."""
    say(f"uniform deferred norm {name}")
    require_gpu()
    L, s, per = CASES[name]()
    n = (L.shape[3], L.shape[2], L.shape[1])
    Ld, sd = dev(rounded(L, "f32"), "f32"), dev(rounded(s, "f32"), "f32")
    hs = [G.gmg_setup(G.gmg_default_params(n, per, G.GMG_F32, uniform_bricks=m, deferred_norm=1),
                      Ld) for m in (2, 0)]
    for h in hs:
        G.gmg_set_pair_sweeps(h, 0, min(6, n[2]), 16)
    xs = [torch.zeros_like(sd) for _ in hs]
    infos = [G.gmg_solve(h, x, sd, 1e-5, 40) for h, x in zip(hs, xs)]
    assert torch.equal(xs[0], xs[1])
    assert infos[0]["history"] == infos[1]["history"]
    assert infos[0]["accepted"] == infos[1]["accepted"]
    for h in hs:
        h.close()
