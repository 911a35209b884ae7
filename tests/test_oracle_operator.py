"""Pins of the oracle's operator, residual and smoother against what the
mathematics fixes: symmetry and semi-definiteness of the flux-form operator,
the constant null vector, closed-form eigenmodes (periodic Fourier and
Neumann cosine modes), textbook Gauss-Seidel on the assembled matrix, and the
exactness property of a Gauss-Seidel half-sweep."""
import math

import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import problems as P

CASES = [
    ((6, 5, 4), (False, False, False), 1.0, 0.0),
    ((6, 4, 8), (True, True, True), 2.0, 0.0),
    ((4, 6, 6), (True, False, True), 3.0, 0.15),
    ((5, 7, 3), (False, False, False), 2.0, 0.2),
]


def _ip(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("n,per,contrast,holes", CASES)
def test_symmetric_negative_semidefinite(n, per, contrast, holes):
    L, _, _ = P.random_problem(n, per, seed=11, contrast=contrast, holes=holes)
    L = O.normalize_faces(L, per)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n[2], n[1], n[0]))
    y = rng.standard_normal((n[2], n[1], n[0]))
    Ax, Ay = O.apply_A(x, L, per), O.apply_A(y, L, per)
    scale = np.abs(Ax).sum() * np.abs(y).max()
    assert abs(_ip(Ax, y) - _ip(x, Ay)) <= 1e-13 * scale
    assert _ip(x, Ax) <= 1e-13 * scale
    # constants are in the null space, and the flux form conserves: sum(Ax) = 0
    assert np.abs(O.apply_A(np.ones_like(x), L, per)).max() <= 1e-14
    assert abs(Ax.sum()) <= 1e-12 * np.abs(Ax).sum()


def test_periodic_fourier_eigenmodes():
    # L = 1 on a periodic grid: exp(2 pi i m.I / n) is an eigenvector with
    # eigenvalue -sum_d 4 sin^2(pi m_d / n_d) (second difference, unit spacing)
    n = (8, 6, 4)
    per = (True, True, True)
    L = np.ones((3, n[2], n[1], n[0]))
    k, j, i = np.meshgrid(*(np.arange(v) for v in n[::-1]), indexing="ij")
    for m in [(1, 0, 0), (2, 1, 1), (3, 2, 1), (4, 3, 2)]:
        phase = 2 * math.pi * (m[0] * i / n[0] + m[1] * j / n[1] + m[2] * k / n[2])
        lam = -sum(4 * math.sin(math.pi * m[d] / n[d]) ** 2 for d in range(3))
        for v in (np.cos(phase), np.sin(phase)):
            assert np.allclose(O.apply_A(v, L, per), lam * v, atol=1e-13)


def test_neumann_cosine_eigenmodes():
    # L = 1 with walls: cos(pi m (i + 1/2) / n) per direction (DCT-II modes)
    # with eigenvalue -sum_d 4 sin^2(pi m_d / (2 n_d))
    n = (7, 5, 6)
    per = (False, False, False)
    L = O.normalize_faces(np.ones((3, n[2], n[1], n[0])), per)
    k, j, i = np.meshgrid(*(np.arange(v) for v in n[::-1]), indexing="ij")
    for m in [(1, 0, 0), (0, 2, 1), (3, 1, 5), (6, 4, 2)]:
        v = (np.cos(math.pi * m[0] * (i + 0.5) / n[0]) *
             np.cos(math.pi * m[1] * (j + 0.5) / n[1]) *
             np.cos(math.pi * m[2] * (k + 0.5) / n[2]))
        lam = -sum(4 * math.sin(math.pi * m[d] / (2 * n[d])) ** 2 for d in range(3))
        assert np.allclose(O.apply_A(v, L, per), lam * v, atol=1e-13)


def test_residual_zero_off_active_set():
    n, per = (6, 6, 6), (False, True, False)
    L, s, _ = P.random_problem(n, per, seed=3, contrast=1.0, holes=0.2)
    L = O.normalize_faces(L, per)
    act = O.active_set(L, per)
    assert (~act).sum() > 0
    x = np.random.default_rng(1).standard_normal(s.shape)
    r = O.residual(x, s, L, per)
    assert np.all(r[~act] == 0.0)
    assert np.allclose(r[act], (s - O.apply_A(x, L, per))[act])


def _dense(L, per, shape):
    N = int(np.prod(shape))
    M = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        M[:, c] = O.apply_A(e.reshape(shape), L, per).ravel()
    return M


@pytest.mark.parametrize("n,per", [((4, 4, 4), (True, True, True)),
                                   ((5, 4, 3), (False, False, False)),
                                   ((6, 4, 4), (True, False, False))])
def test_half_sweeps_equal_sequential_gauss_seidel(n, per):
    # textbook Gauss-Seidel on the assembled matrix, visiting the red cells
    # one at a time (each update seeing the latest values) and then the black
    # ones, must equal the simultaneous colour updates: same-colour cells are
    # never coupled, the periodic wrap included (even periodic sizes)
    shape = (n[2], n[1], n[0])
    L, s, _ = P.random_problem(n, per, seed=7, contrast=2.0, holes=0.1)
    L = O.normalize_faces(L, per)
    M = _dense(L, per, shape)
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(shape)
    omega = 0.7
    col = O.colour(shape).ravel()
    xs = x0.ravel().copy()
    b = s.ravel()
    for c in (0, 1):
        for I in range(xs.size):
            if col[I] == c and M[I, I] != 0.0:
                xs[I] += omega * (b[I] - M[I] @ xs) / M[I, I]
    xv = O.rb_sweep(x0, s, L, per, omega)
    assert np.allclose(xv.ravel(), xs, rtol=0, atol=1e-13 * np.abs(xs).max())


def test_gauss_seidel_half_sweep_exactness():
    # after a half-sweep of colour c, the residual of every updated cell is
    # (1 - omega) times its value before (0 for omega = 1)
    n, per = (8, 6, 4), (False, True, False)
    shape = (n[2], n[1], n[0])
    L, s, _ = P.random_problem(n, per, seed=9, contrast=2.0, holes=0.1)
    L = O.normalize_faces(L, per)
    act = O.active_set(L, per)
    x = np.random.default_rng(4).standard_normal(shape)
    for c in (0, 1):
        for omega in (1.0, 0.6):
            m = (O.colour(shape) == c) & act
            r0 = O.residual(x, s, L, per)
            x1 = O.rb_half_sweep(x, s, L, per, c, omega)
            r1 = O.residual(x1, s, L, per)
            assert np.allclose(r1[m], (1 - omega) * r0[m], atol=1e-12)
            # inactive cells and the other colour are untouched
            assert np.array_equal(x1[~m], x[~m])
