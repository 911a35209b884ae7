"""The moving-body sequence generator: pinned properties of its inputs."""
import numpy as np

from paper_2607_07687_amd import problems as P


def test_moving_body_moves_and_accelerates():
    n = (64, 16, 16)
    dt, u0, a = 0.5, 1.0, 0.05
    cx = []
    for step in range(4):
        L, s, per = P.moving_body_problem("sphere", n, step, dt=dt, u0=u0, accel=a, wave=0.0)
        # the body's centre: the x-weighted centroid of the blocked part of L_x
        w = 1.0 - L[0][:, :, 1:]
        X = np.arange(1, n[0])[None, None, :]
        cx.append(float((w * X).sum() / w.sum()))
        assert abs(s.sum()) < 1e-9 * np.abs(s).sum()  # compatible right-hand side
        assert per == (False, False, False)
    t = np.arange(4) * dt
    want = n[1] + u0 * t + 0.5 * a * t * t
    assert np.allclose(np.diff(cx), np.diff(want), atol=0.02)


def test_cylinder_is_uniform_along_its_axis():
    L, s, _ = P.moving_body_problem("cylinder", (48, 16, 8), 2, wave=0.0)
    assert np.allclose(L[0], L[0][:1]) and np.allclose(s, s[:1])
