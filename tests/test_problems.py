"""Pins of the seeded input generators: the Taylor-Green field is discretely
divergence-free on the staggered grid, right-hand sides sum to zero over the
active cells (compatibility of the singular periodic/Neumann problem), the
smoothed step takes its closed-form values, and the 256^3 sphere's inactive
cell count agrees with a brute-force count of cells whose six face centres
all lie at least one cell inside the sphere."""
import math

import numpy as np
import pytest

from paper_2607_07687_amd import problems as P


def test_tgv_is_discretely_divergence_free():
    n = (32, 32, 32)
    L = np.ones((3, 32, 32, 32))
    u = P.tgv_velocity(n, period=32)
    s = P.flux_divergence(L, u, (True, True, True))
    assert np.abs(s).max() <= 1e-14
    u = P.tgv_velocity((24, 16, 16), period=16)
    s = P.flux_divergence(np.ones((3, 16, 16, 24)), u, (False, True, True))
    # walls in x break the wrap: only the x = 0 and x = n-1 layers may differ
    assert np.abs(s[:, :, 1:-1]).max() <= 1e-14


def test_rhs_compatible_and_zero_off_active():
    for L, s, per in [P.tgv_periodic(16, seed=0),
                      P.sphere_box((24, 16, 16), (12.0, 8.0, 8.0), 5.0, "uniform", 1),
                      P.random_problem((10, 8, 6), (True, False, False), 2,
                                       contrast=2.0, holes=0.2)]:
        t = P.touched_cells(L, per)
        assert abs(s[t].sum()) <= 1e-12 * np.abs(s).sum()
        assert np.all(s[~t] == 0.0)


def test_mu0_closed_form():
    d = np.array([-2.0, -1.0, 0.0, 1.0, 2.0, 0.5, -0.5])
    m = P.mu0(d)
    assert m[0] == 0.0 and m[1] == 0.0 and m[3] == 1.0 and m[4] == 1.0
    assert abs(m[2] - 0.5) <= 1e-16
    assert abs(m[5] - (0.75 + 1 / (2 * math.pi))) <= 1e-15
    assert abs(m[5] + m[6] - 1.0) <= 1e-15  # odd symmetry about (0, 1/2)
    # C1 at the band edges: the derivative (1 + cos(pi d)) / 2 vanishes there
    h = 1e-6
    assert P.mu0(np.array([1 - h]))[0] > 1 - 1e-12
    assert P.mu0(np.array([-1 + h]))[0] < 1e-12


def test_sphere256_inactive_cells_brute_force():
    L = P.sphere_faces((256, 256, 256), (False,) * 3, (128.0, 128.0, 128.0), 32.0)
    t = P.touched_cells(L, (False,) * 3)
    n_inactive = int((~t).sum())
    # brute force: a cell is inactive iff its six face centres are all at
    # distance <= R - 1 = 31 from the centre; scan the bounding cube only
    cnt = 0
    offs = [(0, .5, .5), (1, .5, .5), (.5, 0, .5), (.5, 1, .5), (.5, .5, 0), (.5, .5, 1)]
    for k in range(96, 160):
        for j in range(96, 160):
            i = np.arange(96, 160, dtype=np.float64)
            ok = np.ones(64, dtype=bool)
            for (a, b, c) in offs:
                r2 = (i + a - 128) ** 2 + (j + b - 128) ** 2 + (k + c - 128) ** 2
                ok &= r2 <= 31.0 ** 2
            cnt += int(ok.sum())
    assert n_inactive == cnt == 119808


def test_batch_specs_fit():
    specs = P.batch_specs()
    assert len(specs) == 64
    for sp in specs:
        n = sp["n"]
        assert 32 <= n[0] <= 128 and 32 <= n[1] <= 64 and 32 <= n[2] <= 64
        assert all(v % 8 == 0 for v in n)
        assert 4.0 <= sp["radius"] <= 12.0
        for d in range(3):
            assert sp["radius"] + 3 <= sp["centre"][d] <= n[d] - sp["radius"] - 3


@pytest.mark.parametrize("kind", P.IMPULSIVE_KINDS)
def test_impulsive_rhs_inlet_outlet_and_mirror_symmetry(kind):
    m = 16
    L, s, per = P.impulsive_problem(kind, 4, m)
    nz, ny, nx = s.shape
    assert abs(s.sum()) <= 1e-12 * np.abs(s).sum()
    # far from the body the unit inflow enters through the closed inlet wall
    # and leaves through the outlet: +1 and -1 on those planes, 0 between
    far = slice(2 * m, nx - 1)
    assert np.allclose(s[..., 0], 1.0, atol=1e-12)
    assert np.allclose(s[..., -1], -1.0, atol=1e-12)
    assert np.allclose(s[..., far], 0.0, atol=1e-12)
    # the body's band term L(x + 1/2) - L(x - 1/2) is odd under the x-mirror
    # through the body centre (x = m/2) and even under the y and z mirrors
    near = s[..., 1:m - 1]
    assert np.allclose(near, -near[..., ::-1], atol=1e-12)
    assert np.allclose(s, s[:, ::-1, :], atol=1e-12)
    assert np.allclose(s, s[::-1, :, :], atol=1e-12)
    assert np.abs(near).max() > 0.1  # the body is resolved
