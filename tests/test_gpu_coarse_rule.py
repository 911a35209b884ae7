"""The coarsest-level rule (Sec. 3.2: the coarsest grid is where the
smoother removes the lowest wavenumbers): sweeps until the coarsest
residual has fallen by coarse_rtol, at least one and at most coarse_max.
GPU V-cycles against the oracle's, including the sweep count the rule chose
(an integer: compared exactly), the cap, the LDS and global-memory tails,
and the solves the rule is for."""
import zlib

import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P
from tests.gpu_util import TOL, assert_close, dev, host, require_gpu, say, torch
from tests.test_gpu_parity import _compare_solve, build, rounding_floor

pytestmark = pytest.mark.gpu

CASES = [
    # name, n, periodic, storage, extra params
    ("sphere_walls_f64", (48, 24, 16), None, "f64", {}),
    ("mixed_periodic_f64", (40, 16, 24), (True, False, True), "f64", {}),
    ("odd_coarsest_f32", (72, 32, 32), None, "f32", {}),
    ("aniso_channel_bf16", (96, 16, 16), (False, True, False), "bf16", {}),
    ("global_tail_f64", (60, 24, 24), None, "f64", {"tail_cells": 0}),
    ("tight_cap_f64", (48, 24, 16), None, "f64", {"coarse_rtol": 1e-4, "coarse_max": 3}),
    ("loose_rule_f32", (64, 64, 32), None, "f32", {"coarse_rtol": 0.5, "coarse_max": 200}),
]


def _problem(name, n, per):
    if per is None:
        return P.sphere_box(n, tuple(0.45 * v for v in n), min(n) / 5, "uniform",
                            zlib.crc32(name.encode()) % 1000)
    L, s, _ = P.random_problem(n, per, seed=zlib.crc32(name.encode()) % 1000, contrast=2.0,
                               holes=0.05)
    return L, s, per


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_vcycle_and_sweep_count_match_oracle(case):
    name, n, per, storage, kw = case
    L, s, per = _problem(name, n, per)
    prec = "f64" if storage == "f64" else "f32"
    h, Ld, sd, levels, L64, s64 = build(L, s, per, prec, storage, **kw)
    crtol, cmax = h.params.coarse_rtol, h.params.coarse_max
    rng = np.random.default_rng(5)
    act = levels[0]["active"]
    for start in ("zero", "random"):
        x0 = np.zeros_like(s64) if start == "zero" else \
            np.where(act, rng.standard_normal(s64.shape), 0.0)
        x0 = np.asarray(x0, dtype=np.float32 if prec == "f32" else np.float64).astype(np.float64)
        xd = dev(x0, prec)
        for omega in (1.0, 0.6):
            G.gmg_set_omega(h, omega)
            xd.copy_(dev(x0, prec))
            G.gmg_vcycle(h, xd, sd)
            ng = G.gmg_coarse_sweeps(h)
            st = []
            xo = O.vcycle(levels, x0, s64, omega, coarse_rtol=crtol, coarse_max=cmax, stats=st)
            say(f"{name} {start} omega {omega}: {len(levels)} levels, coarsest "
                f"{levels[-1]['L'].shape[1:][::-1]}, sweeps gpu {ng} oracle {st}")
            assert [ng] == st
            assert 1 <= ng <= cmax
            assert_close(host(xd), xo, TOL[storage])
    if "tight_cap" in name:
        assert ng == 3
    h.close()


def test_rule_off_gives_fixed_sweeps():
    L, s, per = _problem("fixed", (48, 24, 16), None)
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f64", coarse_rtol=0.0, nu_coarse=7)
    xd = torch.zeros_like(sd)
    G.gmg_vcycle(h, xd, sd)
    assert G.gmg_coarse_sweeps(h) == 7
    xo = O.vcycle(levels, np.zeros_like(s64), s64, 1.0, nu_coarse=7, coarse_rtol=0.0)
    assert_close(host(xd), xo, TOL["f64"])
    h.close()


def test_batch_problem_with_odd_coarsest_converges_fast():
    # a 72 x 32 x 32 batch problem stops coarsening at 9 x 4 x 4; four fixed
    # sweeps there left it converging at about 0.77 per cycle.  With the rule
    # the FP64 solve to 1e-10 takes a handful of cycles, as in the oracle
    sp = P.batch_specs(64, 3)[57]
    L, s, per = P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
    h, Ld, sd, levels, L64, s64 = build(L, s, per, "f64")
    xd = torch.zeros_like(sd)
    rg = G.gmg_solve(h, xd, sd, 1e-10, 100)
    ro = O.solve(levels, np.zeros_like(s64), s64, 1e-10, 100)
    say(f"batch problem 57 {sp['n']}: gpu {rg['cycles']} cycles, oracle {ro['cycles']}")
    _compare_solve(rg, ro, "f64", rounding_floor(levels, ro, "f64"))
    assert rg["status"] == "GMG_OK" and rg["cycles"] <= 12
    h.close()


def test_rule_parameter_errors():
    require_gpu()
    L = torch.ones((3, 8, 8, 8), dtype=torch.float64, device="cuda")
    for kw in ({"coarse_rtol": 1.0}, {"coarse_rtol": -0.1}, {"coarse_rtol": float("nan")},
               {"coarse_rtol": 0.1, "coarse_max": 0}, {"coarse_rtol": 0.1, "coarse_max": 5000}):
        with pytest.raises(G.GMGError) as e:
            G.gmg_setup(G.gmg_default_params((8, 8, 8), (False,) * 3, G.GMG_F64, **kw), L)
        assert e.value.status == G.GMG_EINVAL, kw
    # a coarsest level above 2^20 cells cannot run the rule: refused, and
    # accepted with fixed sweeps
    n = (4098, 1026, 1)
    Lb = torch.ones((3, 1, 1026, 4098), dtype=torch.float32, device="cuda")
    with pytest.raises(G.GMGError) as e:
        G.gmg_setup(G.gmg_default_params(n, (False,) * 3, G.GMG_F32), Lb)
    assert e.value.status == G.GMG_ESHAPE
    h = G.gmg_setup(G.gmg_default_params(n, (False,) * 3, G.GMG_F32, coarse_rtol=0.0), Lb)
    assert G.gmg_num_levels(h) == 2
    h.close()
