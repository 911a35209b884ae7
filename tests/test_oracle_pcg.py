"""Pins of the PCG and GMG-PCG oracles (CPU): iterate-by-iterate agreement
with scipy's conjugate-gradient routine on the assembled matrix, the finite
termination of CG fixed by the spectrum of a periodic Laplacian, the PCG
smoother inside a V-cycle, and agreement of the solvers' solutions."""
import numpy as np
import pytest
import scipy.sparse.linalg as sl

from oracle import gmg_oracle as O
from oracle import pcg_oracle as PO
from paper_2607_07687_amd import problems as P


def assembled(L, per):
    """Dense -A on the active cells (columns from unit vectors) and the
    active index list, plus diag(-A) there."""
    Ln = O.normalize_faces(L, per)
    act = O.active_set(Ln, per)
    idx = np.flatnonzero(act.ravel())
    cols = []
    for j in idx:
        e = np.zeros(act.size)
        e[j] = 1.0
        cols.append(-O.apply_A(e.reshape(act.shape), Ln, per).ravel()[idx])
    return np.array(cols).T, idx, act, -O.diagonal(Ln, per).ravel()[idx]


def scipy_pcg(B, b, x0, dg, k):
    x, _ = sl.cg(B, b, x0=x0, rtol=0.0, atol=0.0, maxiter=k, M=np.diag(1.0 / dg))
    return x


@pytest.mark.parametrize("per", [(False, False, False), (True, False, True)])
def test_pcg_iterates_equal_scipy_cg(per):
    L, s, _ = P.random_problem((6, 5, 4), per, seed=3, contrast=2.0, holes=0.1)
    B, idx, act, dg = assembled(L, per)
    assert np.allclose(B, B.T)
    x0 = np.random.default_rng(1).standard_normal(act.shape)
    for k in range(1, 8):
        got = PO.pcg(x0, s, L, per, k)["x"]
        want = scipy_pcg(B, -s.ravel()[idx], x0.ravel()[idx], dg, k)
        assert np.allclose(got.ravel()[idx], want, rtol=1e-9, atol=1e-11 * np.abs(want).max())
        # inactive cells keep the initial guess
        assert np.array_equal(got[~act], x0[~act])


def test_cg_terminates_after_distinct_eigenvalue_count():
    # The 4^3 periodic Laplacian (L = 1) has eigenvalues sum_d (2 - 2 cos(pi k_d / 2)):
    # 0, 2, ..., 12, i.e. six distinct nonzero ones; its Jacobi preconditioner is
    # 6 I.  CG on a mean-free right-hand side with components in every
    # eigenspace therefore needs exactly six iterations.
    per = (True, True, True)
    L = np.ones((3, 4, 4, 4))
    s = np.random.default_rng(5).standard_normal((4, 4, 4))
    s -= s.mean()
    sn = np.linalg.norm(s)
    five = PO.pcg(np.zeros_like(s), s, L, per, 5)
    six = PO.pcg(np.zeros_like(s), s, L, per, 6)
    assert five["history"][-1] > 1e-6
    assert six["history"][-1] <= 1e-12
    assert np.linalg.norm(O.residual(six["x"], s, L, per)) <= 1e-12 * sn


def test_pcg_smoother_in_vcycle_matches_scipy_smoothing():
    per = (False, True, False)
    L, s, _ = P.random_problem((16, 8, 8), per, seed=7, contrast=1.0, holes=0.05)
    levels = O.build_hierarchy(L, per, max_levels=2)
    x0 = np.zeros_like(s)
    got = PO.vcycle_pcg(levels, x0, s, 2, 3, 5)

    def smooth(lev, x, sigma, k):
        B, idx, act, dg = assembled(lev["L"], lev["periodic"])
        out = np.array(x, dtype=np.float64, copy=True)
        out.ravel()[idx] = scipy_pcg(B, -sigma.ravel()[idx], x.ravel()[idx], dg, k)
        return out

    l0, l1 = levels
    x = smooth(l0, x0, s, 2)
    sc = O.restrict(O.residual(x, s, l0["L"], per), l0["c"])
    xc = smooth(l1, np.zeros_like(sc), sc, 5)
    x[l0["active"]] += O.prolong(xc, l0["c"])[l0["active"]]
    want = smooth(l0, x, s, 3)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-11 * np.abs(want).max())


def test_pcg_and_gmg_pcg_solve_the_same_problem():
    L, s, per = P.sphere_box((32, 16, 16), (12.0, 8.0, 8.0), 4.0, "uniform", 2)
    levels = O.build_hierarchy(L, per)
    g = PO.solve_gmg_pcg(levels, np.zeros_like(s), s, 1e-9, 80)
    c = PO.pcg_solve(L, per, np.zeros_like(s), s, 1e-9, 2000)
    assert g["status"] == "ok" and c["status"] == "ok"
    # GMG-PCG needs far fewer cycles than PCG needs iterations
    assert g["cycles"] * 10 < c["iterations"]
    act = levels[0]["active"]
    # wall-bounded (Neumann) problem: solutions agree up to a constant
    d = g["x"] - c["x"]
    d = d[act] - d[act].mean()
    assert np.linalg.norm(d) <= 1e-6 * np.linalg.norm(c["x"][act])
    # the recursive PCG residual tracks the true one
    true = O.norm2(O.residual(c["x"], s, L, per)) / c["snorm"]
    assert true <= 2e-9
