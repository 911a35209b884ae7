"""GPU parity of every step of the V-cycle against the CPU oracle, through the
C ABI: hierarchy and face restriction, residual, red-black smoothing,
fused residual + restriction, prolongation + correction, one V-cycle, and the
adaptive solve (history, relaxation decisions, result).  Sizes span several
128 x 2 cell-kernel tiles and 64 x TY sweep tiles with ragged tails, both
boundary kinds, inactive cells, FP32, FP64 and BF16 face storage."""
import zlib

import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P
from tests.gpu_util import assert_close, EPS, TOL, dev, host, rel, require_gpu, rounded, say, torch

pytestmark = pytest.mark.gpu

STORE = {"f32": G.GMG_F32, "f64": G.GMG_F64, "bf16": G.GMG_BF16}

# (name, n, periodic, contrast, holes)
SMALL = [
    ("walls_ragged", (70, 9, 5), (False, False, False), 2.0, 0.1),
    ("periodic_tiles", (132, 6, 8), (True, True, True), 1.0, 0.0),
    ("mixed", (20, 20, 8), (True, False, False), 3.0, 0.15),
    ("odd_walls", (37, 11, 13), (False, False, False), 1.0, 0.05),
    ("flat_2d", (40, 24, 1), (False, False, False), 1.0, 0.0),
]


def setup_case(case, prec, storage=None, **kw):
    name, n, per, contrast, holes = case
    L, s, _ = P.random_problem(n, per, seed=zlib.crc32(name.encode()) % 1000, contrast=contrast, holes=holes)
    return build(L, s, per, prec, storage, **kw)


def build(L, s, per, prec, storage=None, **kw):
    """Round inputs, build the GPU handle and the oracle hierarchy on the same
    rounded values.  Returns (handle, Ld, sd, levels, L64, s64)."""
    require_gpu()
    storage = storage or prec
    L64, s64 = rounded(L, prec), rounded(s, prec)
    dt = G.GMG_F64 if prec == "f64" else G.GMG_F32
    n = (L.shape[3], L.shape[2], L.shape[1])
    params = G.gmg_default_params(n, per, dt, l_storage=STORE[storage], **kw)
    Ld, sd = dev(L64, prec), dev(s64, prec)
    h = G.gmg_setup(params, Ld)
    levels = O.build_hierarchy(L64, per, anisotropic=bool(params.anisotropic),
                               min_coarse=params.min_coarse, max_levels=params.max_levels,
                               storage=storage)
    return h, Ld, sd, levels, L64, s64


@pytest.mark.parametrize("prec,storage", [("f32", "f32"), ("f64", "f64"), ("f32", "bf16")])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: c[0])
def test_hierarchy_faces(case, prec, storage):
    say(f"hierarchy {case[0]} {prec}/{storage}")
    h, Ld, sd, levels, _, _ = setup_case(case, prec, storage)
    assert G.gmg_num_levels(h) == len(levels)
    for l, lv in enumerate(levels):
        n, c = G.gmg_level_shape(h, l)
        assert (n[2], n[1], n[0]) == lv["L"].shape[1:]
        assert (c if any(c) else None) == lv["c"]
        shape = (3,) + lv["L"].shape[1:]
        if storage == "bf16":
            raw = torch.empty(shape, dtype=torch.int16, device="cuda")
            G.gmg_level_faces(h, l, raw)
            bits = raw.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
            got = bits.view(np.float32).astype(np.float64)
            tol = 2.0 ** -8  # one BF16 ulp of relative difference
        else:
            out = torch.empty(shape, dtype=torch.float64 if prec == "f64" else torch.float32,
                              device="cuda")
            G.gmg_level_faces(h, l, out)
            got = host(out)
            tol = 1e-15 if prec == "f64" else 2.0 ** -23
        want = lv["L"]
        assert np.all(np.abs(got - want) <= tol * np.abs(want)), f"level {l}"
    h.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: c[0])
def test_residual(case, prec):
    say(f"residual {case[0]} {prec}")
    h, Ld, sd, levels, L64, s64 = setup_case(case, prec)
    x = rounded(np.random.default_rng(1).standard_normal(s64.shape), prec)
    r = torch.empty_like(sd)
    rn, sn = G.gmg_residual(h, dev(x, prec), sd, r)
    ro = O.residual(x, s64, levels[0]["L"], case[2])
    assert_close(host(r), ro, TOL[prec])
    act = levels[0]["active"]
    assert np.all(host(r)[~act] == 0.0)
    assert abs(rn - O.norm2(ro)) <= TOL[prec] * O.norm2(ro)
    assert abs(sn - O.norm2(s64, act)) <= 1e-12 * O.norm2(s64, act)
    h.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: c[0])
def test_smoother_sweeps(case, prec):
    say(f"smooth {case[0]} {prec}")
    h, Ld, sd, levels, L64, s64 = setup_case(case, prec)
    per = case[2]
    x0 = rounded(np.random.default_rng(2).standard_normal(s64.shape), prec)
    G.gmg_set_omega(h, 0.8)
    for sweeps in (1, 2):
        xd = dev(x0, prec)
        G.gmg_smooth(h, 0, xd, sd, sweeps)
        xo = x0.copy()
        for _ in range(sweeps):
            xo = O.rb_sweep(xo, s64, levels[0]["L"], per, 0.8)
        assert_close(host(xd) - x0, xo - x0, TOL[prec], f"{sweeps} sweeps")
    # a coarse level with its own faces
    if len(levels) > 1:
        shp = levels[1]["L"].shape[1:]
        rng = np.random.default_rng(3)
        xc = rounded(rng.standard_normal(shp), prec)
        sc = rounded(rng.standard_normal(shp), prec)
        xd = dev(xc, prec)
        G.gmg_smooth(h, 1, xd, dev(sc, prec), 2)
        xo = O.rb_sweep(O.rb_sweep(xc, sc, levels[1]["L"], per, 0.8), sc, levels[1]["L"], per, 0.8)
        assert_close(host(xd) - xc, xo - xc, TOL[prec])
    h.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: c[0])
def test_restrict_and_prolong(case, prec):
    say(f"transfers {case[0]} {prec}")
    h, Ld, sd, levels, L64, s64 = setup_case(case, prec)
    if len(levels) < 2:
        h.close()
        pytest.skip("single level")
    per, c = case[2], levels[0]["c"]
    rng = np.random.default_rng(4)
    x = rounded(rng.standard_normal(s64.shape), prec)
    shp = levels[1]["L"].shape[1:]
    sc = torch.empty(shp, dtype=sd.dtype, device="cuda")
    xc = torch.full(shp, 7.0, dtype=sd.dtype, device="cuda")
    G.gmg_restrict_residual(h, 0, dev(x, prec), sd, sc, xc)
    want = O.restrict(O.residual(x, s64, levels[0]["L"], per), c)
    assert_close(host(sc), want, TOL[prec])
    assert torch.count_nonzero(xc).item() == 0
    y = rounded(rng.standard_normal(shp), prec)
    xd = dev(x, prec)
    G.gmg_prolong_correct(h, 0, dev(y, prec), xd)
    act = levels[0]["active"]
    want = x.copy()
    want[act] += O.prolong(y, c)[act]
    assert_close(host(xd), want, (1e-7 if prec == "f32" else 1e-15))
    assert np.array_equal(host(xd)[~act], x[~act])
    h.close()


@pytest.mark.parametrize("prec,storage", [("f32", "f32"), ("f64", "f64"), ("f32", "bf16")])
@pytest.mark.parametrize("case", SMALL, ids=lambda c: c[0])
def test_vcycle(case, prec, storage):
    say(f"vcycle {case[0]} {prec}/{storage}")
    h, Ld, sd, levels, L64, s64 = setup_case(case, prec, storage)
    G.gmg_set_omega(h, 0.9)
    # (i) first cycle from x = 0
    xd = torch.zeros_like(sd)
    G.gmg_vcycle(h, xd, sd)
    xo = O.vcycle(levels, np.zeros_like(s64), s64, 0.9)
    assert_close(host(xd), xo, TOL[prec])
    # (ii) a later cycle fed the oracle's iterate rounded to the run precision
    xin = rounded(xo, prec)
    xd = dev(xin, prec)
    G.gmg_vcycle(h, xd, sd)
    xo2 = O.vcycle(levels, xin, s64, 0.9)
    assert_close(host(xd), xo2, TOL[prec])
    # the cycle's increment, allowing for the rounding of the iterate itself
    assert_close(host(xd) - xin, xo2 - xin, TOL[prec], "increment", scale=xo2, eps=EPS[prec])
    h.close()


def test_vcycle_tgv32_fp64():
    L, s, per = P.tgv_periodic(32, seed=0)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f64")
    assert len(levels) == 4
    xd = torch.zeros_like(sd)
    xo = np.zeros_like(s64)
    for _ in range(3):
        G.gmg_vcycle(h, xd, sd)
        xo = O.vcycle(levels, xo, s64, 1.0)
        assert_close(host(xd), xo, 1e-11)
    h.close()


def test_vcycle_sphere64_fp32():
    L, s, per = P.sphere_box((64, 64, 64), (32.0, 32.0, 32.0), 8.0, "uniform", 1)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f32")
    xd = torch.zeros_like(sd)
    G.gmg_vcycle(h, xd, sd)
    xo = O.vcycle(levels, np.zeros_like(s64), s64, 1.0)
    assert_close(host(xd), xo, 1e-5)
    h.close()


def rounding_floor(levels, res_orc, prec):
    """Relative-residual noise of evaluating sigma - A x once x is rounded to
    the run precision: ||A dx|| <= ||A|| eps ||x|| with ||A|| <= 2 max|D|,
    relative to ||sigma||; computed from the oracle's values only."""
    eps = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    maxD = float(np.abs(O.diagonal(levels[0]["L"], levels[0]["periodic"])).max())
    return 8.0 * eps * 2.0 * maxD * float(np.linalg.norm(res_orc["x"])) / res_orc["snorm"]


def _compare_solve(res_gpu, res_orc, prec, floor):
    """Same cycle count, status, relaxation decisions and omega trajectory;
    residual histories within the per-cycle tolerance plus the rounding
    floor (below the floor a history value is rounding noise)."""
    assert res_gpu["cycles"] == res_orc["cycles"]
    assert res_gpu["status"] == ("GMG_OK" if res_orc["status"] == "ok" else "GMG_ENOCONV")
    for hg, ho in zip(res_gpu["history"], res_orc["history"]):
        assert abs(hg - ho) <= TOL[prec] * ho + floor
    assert res_gpu["accepted"] == [1 if f else 0 for f in res_orc["accepted_flags"]]
    assert np.allclose(res_gpu["omegas"], res_orc["omegas"])


@pytest.mark.parametrize("deferred", [0, 1])
def test_solve_tgv32_fp64_to_1e10(deferred):
    L, s, per = P.tgv_periodic(32, seed=0)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f64", deferred_norm=deferred)
    xd = torch.zeros_like(sd)
    rg = G.gmg_solve(h, xd, sd, 1e-10, 100)
    ro = O.solve(levels, np.zeros_like(s64), s64, 1e-10, 100)
    say(f"tgv32 fp64 cycles gpu {rg['cycles']} oracle {ro['cycles']}")
    assert rg["status"] == "GMG_OK"
    _compare_solve(rg, ro, "f64", rounding_floor(levels, ro, "f64"))
    assert_close(host(xd), ro["x"], 1e-9)
    rn, sn = G.gmg_residual(h, xd, sd)
    assert rn <= 1e-10 * sn
    h.close()


@pytest.mark.parametrize("deferred", [0, 1])
def test_solve_sphere64_fp32_to_1e6(deferred):
    L, s, per = P.sphere_box((64, 64, 64), (32.0, 32.0, 32.0), 8.0, "uniform", 1)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f32", deferred_norm=deferred)
    xd = torch.zeros_like(sd)
    rg = G.gmg_solve(h, xd, sd, 1e-6, 60)
    ro = O.solve(levels, np.zeros_like(s64), s64, 1e-6, 60)
    say(f"sphere64 fp32 cycles gpu {rg['cycles']} oracle {ro['cycles']}")
    assert rg["status"] == "GMG_OK"
    _compare_solve(rg, ro, "f32", rounding_floor(levels, ro, "f32"))
    act = levels[0]["active"]
    e = host(xd)[act] - ro["x"][act]
    assert np.linalg.norm(e - e.mean()) <= 1e-4 * np.linalg.norm(ro["x"][act])
    h.close()


@pytest.mark.parametrize("deferred", [0, 1])
def test_solve_rollback_decisions_match(deferred):
    case = ("rollback", (16, 16, 16), (False, False, False), 4.0, 0.0)
    kw = dict(omega0=3.0, omega_max=3.0, theta_inc=1.0)
    h, Ld, sd, levels, L64, s64 = setup_case(case, "f64", deferred_norm=deferred, **kw)
    xd = torch.zeros_like(sd)
    rg = G.gmg_solve(h, xd, sd, 1e-9, 80)
    ro = O.solve(levels, np.zeros_like(s64), s64, 1e-9, 80, **kw)
    assert ro["accepted_flags"][0] is False
    _compare_solve(rg, ro, "f64", rounding_floor(levels, ro, "f64"))
    assert_close(host(xd), ro["x"], 1e-9)
    h.close()


@pytest.mark.parametrize("deferred", [0, 1])
def test_solve_edge_cases(deferred):
    require_gpu()
    # sigma = 0: nothing to do
    L, s, per = P.tgv_periodic(8, seed=0)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f64", deferred_norm=deferred)
    xd = torch.zeros_like(sd)
    rg = G.gmg_solve(h, xd, torch.zeros_like(sd), 1e-6, 5)
    assert rg["status"] == "GMG_OK" and rg["cycles"] == 0
    # ... and x is left as it was (the first round of cycles is launched
    # before the host reads the start's decision, and must do nothing)
    x1 = torch.ones_like(sd)
    rg = G.gmg_solve(h, x1, torch.zeros_like(sd), 1e-6, 5)
    assert rg["cycles"] == 0 and torch.all(x1 == 1.0)
    # max_cycles = 0 -> not converged, x untouched
    x0 = torch.ones_like(sd)
    rg = G.gmg_solve(h, x0, sd, 1e-6, 0)
    assert rg["status"] == "GMG_ENOCONV" and rg["cycles"] == 0
    assert torch.all(x0 == 1.0)
    # ENOCONV with history
    rg = G.gmg_solve(h, xd, sd, 1e-15, 3)
    assert rg["status"] == "GMG_ENOCONV" and rg["cycles"] == 3
    with pytest.raises(G.GMGError):
        G.gmg_solve(h, xd, sd, 1e-15, 2, raise_noconv=True)
    h.close()
    # single-level grid (nothing coarsens): the cycle is nu_coarse sweeps
    case = ("single", (6, 6, 6), (False, False, False), 1.0, 0.0)
    h, Ld, sd, levels, L64, s64 = setup_case(case, "f64")
    assert len(levels) == 1 and G.gmg_num_levels(h) == 1
    xd = torch.zeros_like(sd)
    G.gmg_vcycle(h, xd, sd)
    assert_close(host(xd), O.vcycle(levels, np.zeros_like(s64), s64, 1.0), 1e-11)
    h.close()


@pytest.mark.parametrize("kw", [dict(anisotropic=0), dict(max_levels=2),
                                dict(nu_pre=0, nu_post=3, nu_coarse=1),
                                dict(nu_pre=1, nu_post=0), dict(min_coarse=2)])
def test_vcycle_parameter_variants(kw):
    L, s, per = P.sphere_box((48, 24, 16), (20.0, 12.0, 8.0), 5.0, "uniform", 9)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f64", **kw)
    p = h.params
    xd = torch.zeros_like(sd)
    G.gmg_vcycle(h, xd, sd)
    xo = O.vcycle(levels, np.zeros_like(s64), s64, 1.0, p.nu_pre, p.nu_post, p.nu_coarse)
    assert_close(host(xd), xo, 1e-11)
    h.close()


def test_abi_errors():
    require_gpu()
    L = torch.ones((3, 4, 4, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(TypeError):
        G.gmg_setup(G.gmg_default_params((6, 4, 4), (True, False, False)), L.double())
    p = G.gmg_default_params((5, 4, 4), (True, False, False))
    with pytest.raises(G.GMGError) as e:
        G.gmg_setup(p, torch.ones((3, 4, 4, 5), device="cuda"))
    assert e.value.status == G.GMG_ESHAPE
    p = G.gmg_default_params((6, 4, 4), (False, False, False), l_storage=G.GMG_F64)
    with pytest.raises(G.GMGError) as e:
        G.gmg_setup(p, L)
    assert e.value.status == G.GMG_EINVAL
    p = G.gmg_default_params((6, 4, 4), (False, False, False))
    h = G.gmg_setup(p, L)
    with pytest.raises(G.GMGError):
        G.gmg_set_omega(h, -1.0)
    with pytest.raises(ValueError):  # single level: the binding finds no coarser level
        G.gmg_restrict_residual(h, 0, L[0], L[0], L[0])
    h.close()


@pytest.mark.parametrize("deferred", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_graph_replays_match_direct_launches(prec, deferred):
    # the captured V-cycle is replayed many times per solve and reused across
    # solves; every replay must give exactly what direct launches give
    L, s, per = P.sphere_box((64, 32, 32), (30.0, 16.0, 16.0), 6.0, "uniform", 4)
    hg, Ld, sd, levels, L64, s64 = build(L, s, per, prec, graphs=1, deferred_norm=deferred)
    he = G.gmg_setup(G.gmg_default_params((64, 32, 32), per, hg.params.dtype, graphs=0,
                                          deferred_norm=deferred), Ld)
    outs = []
    for h in (hg, he, hg):
        x = torch.zeros_like(sd)
        res = G.gmg_solve(h, x, sd, 1e-8 if prec == "f64" else 1e-6, 60)
        torch.cuda.synchronize()
        outs.append((x.clone(), res))
    for x, res in outs[1:]:
        assert torch.equal(x, outs[0][0])
        assert res["history"] == outs[0][1]["history"]
        assert res["cycles"] == outs[0][1]["cycles"]
    # a different right-hand side buffer forces a new capture
    s2 = sd * 0.5
    x = torch.zeros_like(sd)
    r2 = G.gmg_solve(hg, x, s2, 1e-6, 60)
    x2 = torch.zeros_like(sd)
    r3 = G.gmg_solve(he, x2, s2, 1e-6, 60)
    assert torch.equal(x, x2) and r2["history"] == r3["history"]
    hg.close()
    he.close()


def test_autotune_keeps_results_bitwise(tmp_path):
    from paper_2607_07687_amd import autotune as AT
    L, s, per = P.sphere_box((96, 64, 48), (40.0, 32.0, 24.0), 8.0, "uniform", 6)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f32")
    x0 = torch.zeros_like(sd)
    r0 = G.gmg_solve(h, x0, sd, 1e-6, 60)
    scratch = torch.zeros_like(sd)
    rep = AT.tune(h, scratch, sd, cache=str(tmp_path / "tiles.json"), reps=3)
    say("tiles " + ", ".join(f"L{r['level']}:{r['ty']}x{r['kchunk']}" for r in rep))
    assert len(rep) == len(levels)
    for r in rep:
        assert r["ty"] in (1, 4, 8) and r["kchunk"] >= 1
        assert r["us"] <= r["us_default"] * 1.05 + 1.0
    x1 = torch.zeros_like(sd)
    r1 = G.gmg_solve(h, x1, sd, 1e-6, 60)
    assert torch.equal(x0, x1) and r0["history"] == r1["history"]
    # cached choices are applied on a fresh handle
    h2 = G.gmg_setup(h.params, Ld)
    rep2 = AT.tune(h2, scratch, sd, cache=str(tmp_path / "tiles.json"))
    assert all(r["cached"] for r in rep2)
    with pytest.raises(G.GMGError):
        G.gmg_set_tiles(h2, 0, 6, 4)
    with pytest.raises(G.GMGError):
        G.gmg_set_tiles(h2, 0, 8, 1000)
    h.close()
    h2.close()


# (name, n, periodic, anisotropic) for the single-workgroup tail
TAIL_CASES = [
    ("sphere_walls", (48, 24, 16), None, 1),
    ("periodic_iso", (32, 32, 32), (True, True, True), 0),
    ("channel_aniso", (64, 16, 12), (True, False, False), 1),
    ("odd_coarsest", (60, 24, 24), (False, False, False), 1),
]


@pytest.mark.parametrize("crule", [0.1, 0.0], ids=["coarse_rule", "fixed_coarse"])
@pytest.mark.parametrize("prec,storage", [("f32", "f32"), ("f64", "f64"), ("f32", "bf16")])
@pytest.mark.parametrize("case", TAIL_CASES, ids=lambda c: c[0])
def test_tail_matches_grid_kernels(case, prec, storage, crule):
    # the coarse levels cycled by one workgroup in LDS give bitwise what the
    # grid-wide kernels give (the coarsest level then runs alone through the
    # tail from global memory), and the V-cycle still matches the oracle
    name, n, per, aniso = case
    if per is None:
        L, s, per = P.sphere_box(n, tuple(0.4 * v for v in n), n[2] / 4, "uniform", 3)
    else:
        L, s, _ = P.random_problem(n, per, seed=zlib.crc32(name.encode()) % 1000,
                                   contrast=2.0, holes=0.05)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, prec, storage, anisotropic=aniso,
                                        tail_cells=32768, coarse_rtol=crule)
    p0 = G.gmg_default_params(h.params.n, per, h.params.dtype, l_storage=h.params.l_storage,
                              anisotropic=aniso, tail_cells=0, coarse_rtol=crule)
    h0 = G.gmg_setup(p0, Ld)
    say(f"{name} {prec}/{storage} coarse_rtol {crule}: {len(levels)} levels")
    xt, x0 = torch.zeros_like(sd), torch.zeros_like(sd)
    G.gmg_vcycle(h, xt, sd)
    G.gmg_vcycle(h0, x0, sd)
    assert torch.equal(xt, x0)
    assert G.gmg_coarse_sweeps(h) == G.gmg_coarse_sweeps(h0)
    xo = O.vcycle(levels, np.zeros_like(s64), s64, 1.0, coarse_rtol=crule)
    assert_close(host(xt), xo, TOL[prec if storage != "bf16" else "bf16"])
    tol = 1e-8 if prec == "f64" else 1e-5
    xt.zero_()
    x0.zero_()
    rt = G.gmg_solve(h, xt, sd, tol, 120)
    r0 = G.gmg_solve(h0, x0, sd, tol, 120)
    assert torch.equal(xt, x0)
    assert rt["history"] == r0["history"] and rt["omegas"] == r0["omegas"]
    h.close()
    h0.close()


def test_tail_cells_bounds():
    require_gpu()
    L = torch.ones((3, 8, 8, 8), dtype=torch.float32, device="cuda")
    p = G.gmg_default_params((8, 8, 8), (False, False, False), tail_cells=32769)
    with pytest.raises(G.GMGError) as e:
        G.gmg_setup(p, L)
    assert e.value.status == G.GMG_EINVAL
    assert G.gmg_default_params((8, 8, 8), (False,) * 3).tail_cells == 4096


@pytest.mark.parametrize("rollback", [1, 0])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nu_pre", [2, 3, 1])
def test_deferred_norm_gives_the_same_solve(prec, rollback, nu_pre):
    # the norm taken by the next cycle's first smoothing step (a two-sweep
    # pass in FP32 with nu_pre >= 2, else a fused sweep) leads to the same
    # decisions and the same iterates as the separate norm kernel; only the
    # summation order of the norm differs
    case = ("rollback", (48, 32, 24), (False, True, False), 3.0, 0.05)
    kw = dict(omega0=2.5, omega_max=2.5, theta_inc=1.0, rollback=rollback, nu_pre=nu_pre)
    out = []
    for deferred in (0, 1):
        h, Ld, sd, levels, L64, s64 = setup_case(case, prec, deferred_norm=deferred, **kw)
        x = torch.zeros_like(sd)
        out.append((G.gmg_solve(h, x, sd, 1e-6 if prec == "f32" else 1e-10, 60), x.clone()))
        h.close()
    (r0, x0), (r1, x1) = out
    say(f"deferred vs separate: {r1['cycles']} / {r0['cycles']} cycles, accepted {r1['accepted']}")
    assert r0["cycles"] == r1["cycles"] and r0["accepted"] == r1["accepted"]
    assert r0["omegas"] == r1["omegas"] and 0 in r0["accepted"] + [0] * (1 - rollback)
    assert torch.equal(x0, x1)
    assert np.allclose(r0["history"], r1["history"], rtol=1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec,storage", [("f32", "f32"), ("f64", "f64"), ("f32", "bf16")])
@pytest.mark.parametrize("case", SMALL[:4], ids=lambda c: c[0])
def test_split_sweeps_match_fused(case, prec, storage):
    # the sweep as red and black half-sweep launches gives bitwise what the
    # fused sweep gives: level by level, in a V-cycle (with the correction
    # folded into the first post-sweep) and over a whole solve (single sweeps
    # only: no two-sweep passes)
    h, Ld, sd, levels, L64, s64 = setup_case(case, prec, storage, pair_sweeps=0)
    hs = G.gmg_setup(h.params, Ld)
    for l in range(len(levels)):
        G.gmg_set_tiles(hs, l, 1, 1)
    n0 = levels[0]["L"].shape[1:]
    x0 = dev(rounded(np.random.default_rng(2).standard_normal(n0), prec), prec)
    xa, xb = x0.clone(), x0.clone()
    G.gmg_smooth(h, 0, xa, sd, 3)
    G.gmg_smooth(hs, 0, xb, sd, 3)
    assert torch.equal(xa, xb)
    xa.zero_()
    xb.zero_()
    G.gmg_vcycle(h, xa, sd)
    G.gmg_vcycle(hs, xb, sd)
    assert torch.equal(xa, xb)
    xa.zero_()
    xb.zero_()
    ra = G.gmg_solve(h, xa, sd, 1e-5 if prec == "f32" else 1e-9, 60)
    rb = G.gmg_solve(hs, xb, sd, 1e-5 if prec == "f32" else 1e-9, 60)
    assert torch.equal(xa, xb) and ra["history"] == rb["history"]
    h.close()
    hs.close()
