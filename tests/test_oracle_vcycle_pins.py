"""Pins of the oracle's V-cycle composition and of one refinement step,
against a brute-force reconstruction built from the method's definitions
(GMG = smoothing plus coarse-grid correction, Sec. 3; red-black Gauss-Seidel
with one relaxation factor, Sec. 3.1; coarsening per direction, Sec. 3.2)
with none of the oracle's array code:

* every level's operator is ASSEMBLED as a dense matrix, face by face, from
  its face coefficients (the coarse faces are summed by explicit loops over
  the fine faces that tile each coarse face), not by applying the oracle's
  operator to unit vectors;
* smoothing is textbook sequential Gauss-Seidel on that matrix, one cell at
  a time in colour order (red cells, then black), each update seeing the
  latest values;
* the transfers are explicit matrices: P (piecewise-constant prolongation)
  and R = P^T, the correction applied on the active cells only;
* the cycle is the recursion written out: pre-sweeps, restrict the
  residual, recurse from zero, correct, post-sweeps; the coarsest level gets
  its own sweep count, fixed, or (the coarsest-level rule) sweeps until its
  residual norm has dropped by a given factor, within a cap.

Sweep counts (1, 3, 5) and omega = 0.7 are chosen so that a swapped pre/post
count, a wrong coarsest count, a correction applied after the post-sweeps, a
transfer that averages instead of sums, an inactive cell touched by the
correction or a level smoothed with another factor all change the result.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import problems as P


def _cells(shape_zyx):
    nz, ny, nx = shape_zyx
    return [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]


def _lin(i, j, k, n):
    nx, ny, _ = n
    return (k * ny + j) * nx + i


def assemble(L, periodic):
    """Dense operator from face coefficients.  Face L[d][I] joins cell I to
    its low neighbour I - e_d: across the domain boundary that is the last
    cell if d is periodic, and nothing (a wall) otherwise.  Each face adds
    its flux coefficient to the two off-diagonal entries and subtracts it
    from the two diagonal ones."""
    nz, ny, nx = L.shape[1:]
    n = (nx, ny, nz)
    N = nx * ny * nz
    A = np.zeros((N, N))
    for (i, j, k) in _cells((nz, ny, nx)):
        a = _lin(i, j, k, n)
        for d in range(3):
            c = [i, j, k]
            if c[d] == 0:
                if not periodic[d]:
                    continue
                c[d] = n[d] - 1
            else:
                c[d] -= 1
            b = _lin(c[0], c[1], c[2], n)
            w = L[d][k, j, i]
            A[a, b] += w
            A[b, a] += w
            A[a, a] -= w
            A[b, b] -= w
    return A


def zero_wall_low_faces(L, periodic):
    L = np.array(L, dtype=np.float64, copy=True)
    nz, ny, nx = L.shape[1:]
    for (i, j, k) in _cells((nz, ny, nx)):
        for d in range(3):
            if not periodic[d] and (i, j, k)[d] == 0:
                L[d][k, j, i] = 0.0
    return L


def coarse_faces_by_loops(L, c):
    """L_c,d[J] = (1/c_d) * sum of the fine d-faces on coarse cell J's low
    d-face: fine cells c*J + s with s_d = 0 and 0 <= s_e < c_e otherwise."""
    nz, ny, nx = L.shape[1:]
    n = (nx // c[0], ny // c[1], nz // c[2])
    out = np.zeros((3, n[2], n[1], n[0]))
    for (I, J, K) in _cells((n[2], n[1], n[0])):
        for d in range(3):
            ext = [1 if e == d else c[e] for e in range(3)]
            s = 0.0
            for sx, sy, sz in itertools.product(range(ext[0]), range(ext[1]), range(ext[2])):
                s += L[d][K * c[2] + sz, J * c[1] + sy, I * c[0] + sx]
            out[d][K, J, I] = s / c[d]
    return out


def prolongation(fine_zyx, c):
    """P[a, J] = 1 iff fine cell a lies in coarse cell J (a_d // c_d = J_d)."""
    nz, ny, nx = fine_zyx
    nf = (nx, ny, nz)
    nc = (nx // c[0], ny // c[1], nz // c[2])
    Pm = np.zeros((nx * ny * nz, nc[0] * nc[1] * nc[2]))
    for (i, j, k) in _cells(fine_zyx):
        Pm[_lin(i, j, k, nf), _lin(i // c[0], j // c[1], k // c[2], nc)] = 1.0
    return Pm


def gauss_seidel(A, colour, x, b, omega, sweeps):
    """Sequential relaxed Gauss-Seidel: per sweep, visit the red cells one at
    a time, then the black ones; a row with zero diagonal is skipped."""
    x = x.copy()
    for _ in range(sweeps):
        for c in (0, 1):
            for I in range(x.size):
                if colour[I] == c and A[I, I] != 0.0:
                    x[I] += omega * (b[I] - A[I] @ x) / A[I, I]
    return x


def build_reference(L, periodic, storage, anisotropic=True, max_levels=0):
    """Per level: assembled matrix, colours, active set, factor and P."""
    nz, ny, nx = L.shape[1:]
    plan = O.level_plan((nx, ny, nz), periodic, anisotropic, 4, max_levels)
    Lc = O.round_to(zero_wall_low_faces(L, periodic), storage)
    refs = []
    for (n, c) in plan:
        shape = (n[2], n[1], n[0])
        A = assemble(Lc, periodic)
        k, j, i = np.meshgrid(*(np.arange(v) for v in shape), indexing="ij")
        refs.append(dict(A=A, colour=((i + j + k) % 2).ravel(), active=np.diag(A) != 0.0,
                         c=c, P=None if c is None else prolongation(shape, c)))
        if c is not None:
            Lc = O.round_to(coarse_faces_by_loops(Lc, c), storage)
    return refs


def coarsest_reference(r, x, b, omega, nuc, crtol, counts=None, group=1):
    """crtol = 0: nuc sweeps.  crtol > 0: remove the mean of b over the
    active cells, then sweep in groups of `group`, checking the residual
    norm on the active cells after each group, until it is at most crtol
    times its value on entry or nuc (the cap) sweeps are done."""
    if crtol <= 0.0:
        return gauss_seidel(r["A"], r["colour"], x, b, omega, nuc)
    act = r["active"]
    b = b.copy()
    b[act] -= sum(b[act]) / int(act.sum())

    def rnorm(v):
        res = np.where(act, b - r["A"] @ v, 0.0)
        return math.sqrt(float(res @ res))

    r0 = rnorm(x)
    n = 0
    while n < nuc:
        k = min(group, nuc - n)
        x = gauss_seidel(r["A"], r["colour"], x, b, omega, k)
        n += k
        if n < nuc and rnorm(x) <= crtol * r0:
            break
    if counts is not None:
        counts.append(n)
    return x


def vcycle_reference(refs, x, b, omega, nu1, nu2, nuc, l=0, crtol=0.0, counts=None, group=1):
    r = refs[l]
    if r["c"] is None:
        return coarsest_reference(r, x, b, omega, nuc, crtol, counts, group)
    x = gauss_seidel(r["A"], r["colour"], x, b, omega, nu1)
    res = np.where(r["active"], b - r["A"] @ x, 0.0)
    bc = r["P"].T @ res  # R = P^T
    xc = vcycle_reference(refs, np.zeros(bc.size), bc, omega, nu1, nu2, nuc, l + 1, crtol, counts,
                          group)
    x = x + np.where(r["active"], r["P"] @ xc, 0.0)
    return gauss_seidel(r["A"], r["colour"], x, b, omega, nu2)


CASES = [
    # name, n, periodic, storage, anisotropic, max_levels
    ("walls_two_levels", (8, 8, 8), (False, False, False), "f64", True, 2),
    ("walls_three_levels", (8, 8, 8), (False, False, False), "f64", True, 0),
    ("periodic_x_bf16", (12, 8, 8), (True, False, False), "bf16", True, 0),
    ("aniso_periodic_yz", (8, 16, 8), (False, True, True), "f32", True, 0),
    ("iso_stops_early", (8, 16, 8), (False, False, False), "f64", False, 0),
]


@pytest.mark.parametrize("name,n,per,storage,aniso,maxl", CASES, ids=[c[0] for c in CASES])
def test_vcycle_equals_assembled_reconstruction(name, n, per, storage, aniso, maxl):
    L, s, _ = P.random_problem(n, per, seed=sum(map(ord, name)) % 97, contrast=2.0, holes=0.08)
    levels = O.build_hierarchy(L, per, anisotropic=aniso, max_levels=maxl, storage=storage)
    refs = build_reference(L, per, storage, anisotropic=aniso, max_levels=maxl)
    assert len(refs) == len(levels) >= 2
    for lv, r in zip(levels, refs):  # operators agree level by level
        M = assemble(lv["L"], per)
        assert np.allclose(M, r["A"], rtol=0, atol=1e-14 * np.abs(r["A"]).max())
        assert np.array_equal(lv["active"].ravel(), r["active"])
    rng = np.random.default_rng(3)
    x0 = np.where(levels[0]["active"], rng.standard_normal(s.shape), 0.0)
    for (nu1, nu2, nuc, omega, crtol, grp) in ((1, 3, 5, 0.7, 0.0, 1), (2, 2, 4, 1.0, 0.0, 1),
                                              (2, 2, 64, 1.0, 0.1, 4), (1, 2, 40, 0.8, 0.01, 3),
                                              (2, 1, 30, 0.9, 0.05, 1)):
        st, counts = [], []
        got = O.vcycle(levels, x0, s, omega, nu1, nu2, nuc if crtol == 0 else grp,
                       coarse_rtol=crtol, coarse_max=nuc, stats=st)
        want = vcycle_reference(refs, x0.ravel(), s.ravel(), omega, nu1, nu2, nuc, crtol=crtol,
                                counts=counts, group=grp)
        scale = np.abs(want).max()
        assert np.abs(got.ravel() - want).max() <= 1e-12 * scale, (nu1, nu2, nuc, omega, crtol)
        if crtol > 0:
            assert st == counts and 1 <= st[0] <= nuc
            assert st[0] == nuc or st[0] % grp == 0


def test_reconstruction_detects_plausible_mistakes():
    # the brute force separates the cycle from each of its plausible
    # misreadings: they all differ from it by far more than the tolerance
    per = (False, True, False)
    L, s, _ = P.random_problem((8, 8, 8), per, seed=5, contrast=2.0, holes=0.08)
    refs = build_reference(L, per, "f64")
    x0 = np.zeros(s.size)
    want = vcycle_reference(refs, x0, s.ravel(), 0.7, 1, 3, 5)
    scale = np.abs(want).max()

    def far(v):
        return np.abs(v - want).max() > 1e-6 * scale

    assert far(vcycle_reference(refs, x0, s.ravel(), 0.7, 3, 1, 5))  # pre/post swapped
    assert far(vcycle_reference(refs, x0, s.ravel(), 0.7, 1, 3, 4))  # coarsest count
    # the adaptive coarsest rule: its stopping factor decides the sweep count
    c1, c2 = [], []
    a1 = vcycle_reference(refs, x0, s.ravel(), 0.7, 1, 3, 64, crtol=0.1, counts=c1, group=2)
    a2 = vcycle_reference(refs, x0, s.ravel(), 0.7, 1, 3, 64, crtol=0.01, counts=c2, group=2)
    assert c1[0] < c2[0] and np.abs(a1 - a2).max() > 1e-6 * np.abs(a2).max()
    r0 = refs[0]
    # correction after the post-sweeps
    x = gauss_seidel(r0["A"], r0["colour"], x0, s.ravel(), 0.7, 1)
    bc = r0["P"].T @ np.where(r0["active"], s.ravel() - r0["A"] @ x, 0.0)
    xc = vcycle_reference(refs, np.zeros(bc.size), bc, 0.7, 1, 3, 5, 1)
    late = gauss_seidel(r0["A"], r0["colour"], x, s.ravel(), 0.7, 3)
    assert far(late + np.where(r0["active"], r0["P"] @ xc, 0.0))
    # averaging restriction (R = P^T / 8)
    xc8 = vcycle_reference(refs, np.zeros(bc.size), bc / 8.0, 0.7, 1, 3, 5, 1)
    avg = gauss_seidel(r0["A"], r0["colour"], x + np.where(r0["active"], r0["P"] @ xc8, 0.0),
                       s.ravel(), 0.7, 3)
    assert far(avg)


# ----------------------------------------------------------------------------
# One step of the FP64 iterative refinement
# ----------------------------------------------------------------------------

def _round32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_refinement_step_by_hand(storage):
    # outer step: r = sigma - A x with the EXACT faces (assembled here in FP64),
    # beta = ||r|| / sqrt(#active), b = fp32(r / beta), an adaptive inner solve
    # of A_s e = b from zero on the storage-rounded hierarchy (omega reset),
    # then x + beta e; the history holds ||r|| / ||sigma|| before and after
    per = (False, False, True)
    L, s, _ = P.random_problem((16, 8, 8), per, seed=21, contrast=1.5, holes=0.05)
    A = assemble(zero_wall_low_faces(L, per), per)
    act = np.diag(A) != 0.0
    rng = np.random.default_rng(8)
    x0 = np.where(act.reshape(s.shape), rng.standard_normal(s.shape), 0.0)
    got = O.solve_ir(L, per, x0, s, rtol=1e-14, max_outer=1, max_inner=3,
                     inner_rtol=1e-3, inner_storage=storage)
    r = np.where(act, s.ravel() - A @ x0.ravel(), 0.0)
    rn = math.sqrt(float(r @ r))
    beta = rn / math.sqrt(int(act.sum()))
    b = _round32(r / beta).reshape(s.shape)
    levels = O.build_hierarchy(L, per, storage=storage)
    e = O.solve(levels, np.zeros_like(b), b, 1e-3, 3)
    x1 = x0 + beta * e["x"]
    sn = math.sqrt(float(np.sum(s.ravel()[act] ** 2)))
    assert got["outer"] == 1 and got["inner_total"] == e["cycles"]
    assert np.abs(got["x"] - x1).max() <= 1e-14 * np.abs(x1).max()
    assert abs(got["history"][0] - rn / sn) <= 1e-13 * rn / sn
    r1 = np.where(act, s.ravel() - A @ x1.ravel(), 0.0)
    assert abs(got["history"][1] - math.sqrt(float(r1 @ r1)) / sn) <= 1e-12 * got["history"][1]


def test_refinement_step_detects_plausible_mistakes():
    # a misread scale, a missing FP32 rounding or the rounded faces in the
    # outer residual each move the step's result by far more than the 1e-14
    # the test above allows
    per = (False, False, False)
    L, s, _ = P.random_problem((16, 8, 8), per, seed=4, contrast=1.5, holes=0.05)
    A = assemble(zero_wall_low_faces(L, per), per)
    act = np.diag(A) != 0.0
    x0 = np.where(act, np.random.default_rng(2).standard_normal(s.size), 0.0)
    levels = O.build_hierarchy(L, per, storage="bf16")
    r = np.where(act, s.ravel() - A @ x0, 0.0)
    rn = math.sqrt(float(r @ r))

    def step(beta, rounding=True):
        b = (r / beta).reshape(s.shape)
        if rounding:
            b = _round32(b)
        return x0 + beta * O.solve(levels, np.zeros_like(b), b, 1e-3, 3)["x"].ravel()

    want = step(rn / math.sqrt(int(act.sum())))
    scale = np.abs(want).max()
    assert np.abs(step(rn) - want).max() > 1e-12 * scale
    assert np.abs(step(rn / math.sqrt(int(act.sum())), rounding=False) - want).max() > 1e-12 * scale
    Ab = assemble(levels[0]["L"], per)
    rb = np.where(act, s.ravel() - Ab @ x0, 0.0)
    assert np.abs(rb - r).max() > 1e-6 * np.abs(r).max()


def test_single_level_cycle_is_fixed_sweeps_whatever_the_rule():
    # a grid that cannot coarsen has no coarse-grid correction: its cycle is
    # nu_coarse plain sweeps, with or without the coarsest-level rule
    per = (False, False, False)
    L, s, _ = P.random_problem((7, 5, 6), per, seed=9, contrast=1.0, holes=0.05)
    levels = O.build_hierarchy(L, per)
    refs = build_reference(L, per, "f64")
    assert len(levels) == len(refs) == 1
    x0 = np.zeros(s.size)
    want = gauss_seidel(refs[0]["A"], refs[0]["colour"], x0, s.ravel(), 0.9, 5)
    for crtol in (0.0, 0.1, 0.5):
        got = O.vcycle(levels, x0.reshape(s.shape), s, 0.9, 2, 2, 5, coarse_rtol=crtol)
        assert np.abs(got.ravel() - want).max() <= 1e-13 * np.abs(want).max()


def test_coarse_rule_projects_out_the_mean():
    # on a singular level a right-hand side with a nonzero mean (in the
    # cycle: its rounding) cannot be solved; without the projection its
    # residual norm stalls above the stopping factor and the rule runs to its
    # cap, drifting x along the constants.  With it the rule stops early,
    # and the result is that of the mean-free right-hand side
    per = (False, False, False)
    L, s, _ = P.random_problem((8, 8, 8), per, seed=13, contrast=1.0, holes=0.0)
    levels = O.build_hierarchy(L, per, max_levels=1)
    refs = build_reference(L, per, "f64", max_levels=1)
    act = refs[0]["active"]
    b = s.ravel().copy()
    b[act] += 0.3 * math.sqrt(float(b[act] @ b[act]) / act.sum())  # a constant, 0.3 ||b||
    c_ref = []
    want = coarsest_reference(refs[0], np.zeros(b.size), b, 1.0, 64, 0.1, c_ref, group=4)
    x, n = O.coarsest_sweeps(np.zeros_like(s), b.reshape(s.shape), levels[0]["L"], per, 1.0, 4,
                             0.1, 64, levels[0]["active"])
    assert n == c_ref[0] < 64
    assert np.abs(x.ravel() - want).max() <= 1e-12 * np.abs(want).max()
    bz = s.ravel().copy()
    bz[act] -= bz[act].mean()
    xz, nz = O.coarsest_sweeps(np.zeros_like(s), bz.reshape(s.shape), levels[0]["L"], per, 1.0,
                               4, 0.1, 64, levels[0]["active"])
    assert nz == n and np.abs(xz - x).max() <= 1e-12 * np.abs(x).max()
    # without the projection the plain residual norm stays above 0.1 ||b||
    xs = gauss_seidel(refs[0]["A"], refs[0]["colour"], np.zeros(b.size), b, 1.0, 64)
    res = np.where(act, b - refs[0]["A"] @ xs, 0.0)
    assert math.sqrt(float(res @ res)) > 0.1 * math.sqrt(float(b[act] @ b[act]))
