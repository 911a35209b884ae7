"""Pins of the oracle's hierarchy and grid transfers: the level tables that the
coarsening rule gives for the workloads (hand-derived, stored under
tests/golden), adjointness and conservation of restriction and prolongation,
the finite-volume rediscretisation closed form of the coarse coefficients for
L = 1, and the half-Galerkin identity of isotropic coarsening."""
import json
import math
import os

import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden", "level_plans.json")


def _plans():
    with open(GOLD) as f:
        return json.load(f)["plans"]


@pytest.mark.parametrize("case", _plans(), ids=lambda c: c["name"])
def test_level_plan_golden(case):
    plan = O.level_plan(case["n"], case["periodic"], case["anisotropic"],
                        case["min_coarse"])
    got = [list(n) for n, _ in plan]
    assert got == case["levels"]
    facs = [list(c) for _, c in plan if c is not None]
    assert facs == case["factors"]


FACTORS = [(2, 2, 2), (2, 1, 1), (1, 2, 2), (2, 2, 1), (1, 1, 2)]


@pytest.mark.parametrize("c", FACTORS)
def test_restriction_is_adjoint_of_prolongation(c):
    rng = np.random.default_rng(0)
    nf = (4, 6, 8)  # (nz, ny, nx)
    r = rng.standard_normal(nf)
    y = rng.standard_normal((nf[0] // c[2], nf[1] // c[1], nf[2] // c[0]))
    lhs = float(np.sum(O.restrict(r, c) * y))
    rhs = float(np.sum(r * O.prolong(y, c)))
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(r).sum() * np.abs(y).max())
    assert abs(O.restrict(r, c).sum() - r.sum()) <= 1e-13 * np.abs(r).sum()
    # prolongation of a coarse constant is the fine constant
    assert np.array_equal(O.prolong(np.ones_like(y), c), np.ones_like(r))


@pytest.mark.parametrize("c", FACTORS)
@pytest.mark.parametrize("per", [(True, True, True), (False, False, False)])
def test_coarse_faces_rediscretise_unit_coefficient(c, per):
    # finite-volume rediscretisation on the coarse mesh (cell size c) gives a
    # face coefficient of face area / spacing = prod_{e != d} c_e / c_d
    n = (8, 8, 8)
    L = O.normalize_faces(np.ones((3, 8, 8, 8)), per)
    Lc = O.restrict_faces(L, c)
    for d in range(3):
        want = math.prod(c[e] for e in range(3) if e != d) / c[d]
        inner = Lc[d][tuple(slice(1, None) if (not per[d] and O.AX[d] == a)
                            else slice(None) for a in range(3))]
        assert np.allclose(inner, want)
        if not per[d]:
            assert np.all(Lc[d][O._index(d, 0)] == 0.0)  # walls stay walls


def test_isotropic_coarse_operator_is_half_galerkin():
    # with piecewise-constant P and R = P^T, the coarse face coefficients
    # (1/2) * (sum of the four fine faces) make A_c = (1/2) P^T A P exactly,
    # for any coefficients and boundary conditions
    rng = np.random.default_rng(3)
    for per in [(True, True, True), (False, True, False)]:
        n = (8, 4, 6)
        L, _, _ = P.random_problem(n, per, seed=8, contrast=2.0, holes=0.1)
        L = O.normalize_faces(L, per)
        c = (2, 2, 2)
        Lc = O.restrict_faces(L, c)
        y = rng.standard_normal((n[2] // 2, n[1] // 2, n[0] // 2))
        lhs = O.apply_A(y, Lc, per)
        rhs = 0.5 * O.restrict(O.apply_A(O.prolong(y, c), L, per), c)
        assert np.allclose(lhs, rhs, atol=1e-13 * np.abs(rhs).max())


def test_hierarchy_propagates_inactive_and_walls():
    n, per = (16, 8, 8), (False, False, False)
    L, _, _ = P.sphere_box(n, (8.0, 4.0, 4.0), 3.0, "uniform", 0)
    levels = O.build_hierarchy(L, per)
    assert [lv["L"].shape[1:] for lv in levels] == [(8, 8, 16), (4, 4, 8), (4, 4, 4)]
    for lv in levels:
        Lc = lv["L"]
        for d in range(3):
            assert np.all(Lc[d][O._index(d, 0)] == 0.0)
        assert np.all(Lc >= 0.0)
