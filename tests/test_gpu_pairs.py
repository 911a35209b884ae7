"""GPU checks of the two-sweep pass (two consecutive red-black sweeps of one
smoothing step in one launch, temporal blocking): bitwise equal to separate
sweeps on every level, in V-cycles (with the coarse correction folded into the
first post-smoothing pass) and over whole solves; walls, periodic directions,
ragged tiles and z-chunks, FP32 and BF16 faces, odd sweep counts; and the
parameter checks.  Separate sweeps are themselves checked against the oracle
in test_gpu_parity.py."""
import zlib

import numpy as np
import pytest

from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P
from tests.gpu_util import dev, require_gpu, rounded, say, torch
from tests.test_gpu_parity import SMALL, STORE

pytestmark = pytest.mark.gpu

EVEN = [c for c in SMALL if c[1][0] % 2 == 0]

# (name, n, periodic): several 64 x 8 tiles, ragged tails, many z-chunks
LARGER = [
    ("walls_192", (192, 40, 37), (False, False, False)),
    ("periodic_128", (128, 32, 48), (True, True, True)),
    ("mixed_136", (136, 18, 22), (False, True, False)),
]


def handles(L, s, per, prec, storage, **kw):
    require_gpu()
    n = (L.shape[3], L.shape[2], L.shape[1])
    dt = G.GMG_F64 if prec == "f64" else G.GMG_F32
    Ld, sd = dev(rounded(L, prec), prec), dev(rounded(s, prec), prec)
    hp = G.gmg_setup(G.gmg_default_params(n, per, dt, l_storage=STORE[storage], **kw), Ld)
    hs = G.gmg_setup(G.gmg_default_params(n, per, dt, l_storage=STORE[storage], pair_sweeps=0,
                                          **kw), Ld)
    return hp, hs, sd


def set_pairs(h, kc, ty=16):
    """Two-sweep passes on every level that allows them, z-chunk kc(l, nz),
    tiles of 64 x ty cells."""
    on = []
    for l in range(G.gmg_num_levels(h)):
        (nx, ny, nz), _ = G.gmg_level_shape(h, l)
        if nx % 2 == 0:
            G.gmg_set_pair_sweeps(h, l, kc(l, nz), ty)
            on.append(l)
        else:
            G.gmg_set_pair_sweeps(h, l, 0)
    return on


def same_cycles_and_solve(hp, hs, sd, prec, seed=2):
    x0 = dev(rounded(np.random.default_rng(seed).standard_normal(tuple(sd.shape)), prec), prec)
    xa, xb = x0.clone(), x0.clone()
    G.gmg_vcycle(hp, xa, sd)
    G.gmg_vcycle(hs, xb, sd)
    assert torch.equal(xa, xb)
    xa.zero_()
    xb.zero_()
    G.gmg_vcycle(hp, xa, sd)
    G.gmg_vcycle(hs, xb, sd)
    assert torch.equal(xa, xb)
    xa.zero_()
    xb.zero_()
    ra = G.gmg_solve(hp, xa, sd, 1e-5, 60)
    rb = G.gmg_solve(hs, xb, sd, 1e-5, 60)
    assert torch.equal(xa, xb)
    assert ra["history"] == rb["history"] and ra["accepted"] == rb["accepted"]
    return ra


KCS = {"one": lambda l, nz: 1, "three": lambda l, nz: min(3, nz), "whole": lambda l, nz: nz}


@pytest.mark.parametrize("ty", [16, 8])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("kc", list(KCS), ids=list(KCS))
@pytest.mark.parametrize("case", EVEN, ids=lambda c: c[0])
def test_pairs_match_separate_sweeps(case, kc, storage, ty):
    name, n, per, contrast, holes = case
    L, s, _ = P.random_problem(n, per, seed=zlib.crc32(name.encode()) % 1000, contrast=contrast,
                               holes=holes)
    hp, hs, sd = handles(L, s, per, "f32", storage)
    on = set_pairs(hp, KCS[kc], ty)
    assert 0 in on
    r = same_cycles_and_solve(hp, hs, sd, "f32")
    say(f"{name} {storage} kc={kc} ty={ty}: passes on levels {on}, {r['cycles']} cycles, "
        "bitwise equal")
    hp.close()
    hs.close()


@pytest.mark.parametrize("case", LARGER, ids=lambda c: c[0])
def test_pairs_match_on_larger_grids(case):
    name, n, per = case
    L, s, _ = P.random_problem(n, per, seed=zlib.crc32(name.encode()) % 1000, contrast=2.0,
                               holes=0.05)
    hp, hs, sd = handles(L, s, per, "f32", "f32")
    for kc, ty in ((lambda l, nz: 0 if l else 5, 8), (lambda l, nz: 16 if l == 0 else min(4, nz), 8),
                   (lambda l, nz: 0 if l else 7, 16), (lambda l, nz: 12 if l == 0 else min(3, nz), 16)):
        on = set_pairs(hp, kc, ty)
        same_cycles_and_solve(hp, hs, sd, "f32", seed=len(on) + ty)
    hp.close()
    hs.close()


@pytest.mark.parametrize("nu", [(3, 1, 5), (1, 2, 2), (4, 4, 4)])
def test_pairs_with_other_sweep_counts(nu):
    # odd counts mix passes and single sweeps within one smoothing step
    L, s, per = P.sphere_box((64, 24, 20), (30.0, 12.0, 10.0), 6.0, "uniform", 3)
    hp, hs, sd = handles(L, s, per, "f32", "f32", nu_pre=nu[0], nu_post=nu[1], nu_coarse=nu[2],
                         tail_cells=0)
    set_pairs(hp, lambda l, nz: min(7, nz))
    same_cycles_and_solve(hp, hs, sd, "f32")
    hp.close()
    hs.close()


def test_pairs_default_and_autotune():
    L, s, per = P.sphere_box((96, 48, 40), (40.0, 24.0, 20.0), 8.0, "uniform", 5)
    hp, hs, sd = handles(L, s, per, "f32", "f32")
    x = torch.zeros_like(sd)
    rep = G.gmg_autotune(hp, x, sd, 2)
    assert rep[0]["us_pair"] > 0 and rep[0]["pair_ty"] in (8, 16)
    say("autotune: " + ", ".join(f"L{r['level']} pair {r['pair_ty']}x{r['pair_kchunk']} "
                                 f"({r['us_pair']:.1f} us) vs sweep {r['us']:.1f} us" for r in rep))
    same_cycles_and_solve(hp, hs, sd, "f32")
    hp.close()
    hs.close()


def test_pair_parameter_checks():
    require_gpu()
    L = torch.ones((3, 8, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(G.GMGError) as e:
        G.gmg_setup(G.gmg_default_params((8, 8, 8), (False,) * 3, pair_sweeps=2), L)
    assert e.value.status == G.GMG_EINVAL
    h = G.gmg_setup(G.gmg_default_params((8, 8, 8), (False,) * 3), L)
    for level, kc, ty in ((0, 9, 16), (0, -1, 16), (7, 1, 16), (0, 2, 4), (0, 2, 12)):
        with pytest.raises(G.GMGError) as e:
            G.gmg_set_pair_sweeps(h, level, kc, ty)
        assert e.value.status == G.GMG_EINVAL
    G.gmg_set_pair_sweeps(h, 0, 0)
    G.gmg_set_pair_sweeps(h, 0, 8, 8)
    G.gmg_set_pair_sweeps(h, 0, 8, 16)
    h.close()
    # FP64 cycles, the PCG smoother, pair_sweeps 0 and an odd nx do not allow passes
    for kw, Lt, n in ((dict(dtype=G.GMG_F64), L.double(), (8, 8, 8)),
                      (dict(smoother=G.GMG_SMOOTH_PCG), L, (8, 8, 8)),
                      (dict(pair_sweeps=0), L, (8, 8, 8)),
                      ({}, torch.ones((3, 8, 8, 7), dtype=torch.float32, device="cuda"),
                       (7, 8, 8))):
        h = G.gmg_setup(G.gmg_default_params(n, (False,) * 3, **kw), Lt)
        with pytest.raises(G.GMGError) as e:
            G.gmg_set_pair_sweeps(h, 0, 2)
        assert e.value.status == G.GMG_EINVAL
        G.gmg_set_pair_sweeps(h, 0, 0)
        h.close()


def test_pair_refused_above_buffer_limit():
    # the pass addresses each field with 32-bit buffer offsets: a level of
    # more than 2^28 cells must run separate sweeps (3.2 GB of faces here)
    require_gpu()
    n = (2048, 512, 257)
    assert n[0] * n[1] * n[2] > 1 << 28
    L = torch.ones((3, n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    h = G.gmg_setup(G.gmg_default_params(n, (False,) * 3), L)
    del L
    with pytest.raises(G.GMGError) as e:
        G.gmg_set_pair_sweeps(h, 0, 8)
    assert e.value.status == G.GMG_EINVAL
    # level 1 is below the limit and keeps its passes
    G.gmg_set_pair_sweeps(h, 1, 8)
    h.close()
