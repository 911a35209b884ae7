"""Seeded synthetic inputs for the GMG Poisson solver.

This module only builds inputs: face-coefficient fields L and right-hand sides
sigma.  It holds none of the solver's arithmetic and imports neither the HIP
library nor the CPU oracle, so both can be fed the very same arrays.

Conventions (shared with the C ABI): cell-centred fields are C-order
``[nz][ny][nx]``; ``L[d]`` (d = 0, 1, 2 for x, y, z) holds the coefficient of
the LOW d-face of each cell; ``periodic`` is a 3-tuple in (x, y, z) order.
Positions are in cell units: cell (i, j, k) spans [i, i+1] x [j, j+1] x [k, k+1],
so its low x-face centre is (i, j+1/2, k+1/2), and likewise for y and z.

Every generator returns FP64 arrays; a run rounds them to its own precision
before either the GPU path or the oracle sees them.

Workloads (the paper's test cases are a Taylor-Green vortex in a
triple-periodic box and flow past a sphere in a (16 x 6 x 6) D box, Sec. 2;
immersed bodies make the coefficients heterogeneous, Sec. 3.1):

* ``tgv_periodic``: 32^3 triple-periodic box, L = 1 on every face; sigma is
  the divergence of a Taylor-Green velocity plus N(0, 0.01^2) face noise.
* ``sphere_box``: wall-bounded box with an immersed sphere smoothed over a
  2-cell band by a cosine kernel; sigma from a uniform-random face velocity
  (256^3, sphere diameter 64 at the centre) or from the Taylor-Green field
  (512 x 192 x 192 box, sphere of diameter 32 at x = 128).
* ``batch_problems``: 64 independent wall-bounded sphere problems of uneven
  sizes.
* ``moving_body_problem``: one time step of a sequence of pressure problems
  past an accelerating sphere or cylinder that moves through the box, the
  time-correlated problems a flow solver hands its pressure solver.
"""
from __future__ import annotations

import math

import numpy as np

AX = (2, 1, 0)  # numpy axis of direction d


def _sel(d, i):
    idx = [slice(None)] * 3
    idx[AX[d]] = i
    return tuple(idx)


def face_centres(n, d):
    """Cell-unit coordinates (X, Y, Z) of the low d-face centres, as arrays
    that broadcast to shape (nz, ny, nx)."""
    nx, ny, nz = n
    X = np.arange(nx, dtype=np.float64)[None, None, :] + (0.0 if d == 0 else 0.5)
    Y = np.arange(ny, dtype=np.float64)[None, :, None] + (0.0 if d == 1 else 0.5)
    Z = np.arange(nz, dtype=np.float64)[:, None, None] + (0.0 if d == 2 else 0.5)
    return X, Y, Z


def mu0(dist):
    """Cosine-kernel smoothed step over a 2-cell band: 0 for dist <= -1,
    1 for dist >= 1, and (1 + dist)/2 + sin(pi dist)/(2 pi) in between (the
    integral of the kernel (1 + cos(pi s))/2 over s <= dist)."""
    d = np.asarray(dist, dtype=np.float64)
    out = (d >= 1.0).astype(np.float64)
    band = (d > -1.0) & (d < 1.0)
    db = d[band]
    out[band] = 0.5 * (1.0 + db) + np.sin(math.pi * db) / (2.0 * math.pi)
    return out


def zero_wall_faces(L, periodic):
    """Faces on a wall carry no flux: zero L_d at index 0 of each wall
    direction (the high wall face is outside the stored array)."""
    L = np.array(L, dtype=np.float64, copy=True)
    for d in range(3):
        if not periodic[d]:
            L[d][_sel(d, 0)] = 0.0
    return L


def sphere_faces(n, periodic, centre, radius):
    """L_d = mu0(|f - C| - R) at every face centre f; wall faces zeroed."""
    L = np.empty((3, n[2], n[1], n[0]), dtype=np.float64)
    for d in range(3):
        X, Y, Z = face_centres(n, d)
        r = np.sqrt(((X - centre[0]) ** 2 + (Y - centre[1]) ** 2) +
                    (Z - centre[2]) ** 2)
        L[d] = mu0(r - radius)
    return zero_wall_faces(L, periodic)


def body_faces(n, periodic, centre, radius, axis=None):
    """L_d = mu0(dist - R) at every face centre, dist being the distance to
    the point `centre` (sphere, axis None) or to the line through `centre`
    along direction `axis` (cylinder); wall faces zeroed."""
    L = np.empty((3, n[2], n[1], n[0]), dtype=np.float64)
    for d in range(3):
        P = face_centres(n, d)
        r2 = 0.0
        for e in range(3):
            if e != axis:
                r2 = r2 + (P[e] - centre[e]) ** 2
        L[d] = mu0(np.sqrt(r2) - radius)
    return zero_wall_faces(L, periodic)


IMPULSIVE_KINDS = ("cylinder2d", "cylinder3d", "sphere")


def impulsive_problem(kind, aspect, m):
    """Impulsive start of the flow past a body (the three cases of the
    anisotropic-coarsening study, Sec. 3.2): unit velocity along x on every
    face, sigma its flux divergence through L with the mean removed; it is
    nonzero on the body's band and on the walled inlet and outlet planes,
    whose pressure difference is the low axial mode.
      cylinder2d: aspect*m x m x 1, walls, cylinder along z;
      cylinder3d: aspect*m x m x m/2, periodic in z (spanwise), cylinder along z;
      sphere:     aspect*m x m x m, walls.
    Body diameter m/4, centred at x = m/2 and mid-height.  Returns
    (L, sigma, periodic)."""
    if kind == "cylinder2d":
        n, per, axis = (aspect * m, m, 1), (False, False, False), 2
    elif kind == "cylinder3d":
        n, per, axis = (aspect * m, m, m // 2), (False, False, True), 2
    elif kind == "sphere":
        n, per, axis = (aspect * m, m, m), (False, False, False), None
    else:
        raise ValueError(kind)
    centre = (m / 2, n[1] / 2, n[2] / 2)
    L = body_faces(n, per, centre, m / 8, axis)
    u = np.zeros_like(L)
    u[0] = 1.0
    return L, rhs_from_velocity(L, u, per), per


def touched_cells(L, periodic):
    """Cells with at least one nonzero face among their six (low faces L_d[I]
    and high faces L_d[I + e_d], the latter wrapping when periodic)."""
    t = np.zeros(L.shape[1:], dtype=bool)
    for d in range(3):
        hi = np.roll(L[d], -1, axis=AX[d])
        if not periodic[d]:
            hi[_sel(d, -1)] = 0.0
        t |= (L[d] != 0.0) | (hi != 0.0)
    return t


def flux_divergence(L, u, periodic):
    """sigma(I) = sum_d F_d(I + e_d) - F_d(I) with face fluxes F_d = L_d u_d;
    the high flux at a wall is 0 and wraps when periodic."""
    s = np.zeros(L.shape[1:], dtype=np.float64)
    for d in range(3):
        F = L[d] * u[d]
        Fh = np.roll(F, -1, axis=AX[d])
        if not periodic[d]:
            Fh[_sel(d, -1)] = 0.0
        s += Fh - F
    return s


def rhs_from_velocity(L, u, periodic):
    """Flux divergence, then the mean over the touched cells removed and sigma
    set to 0 on untouched cells."""
    s = flux_divergence(L, u, periodic)
    t = touched_cells(L, periodic)
    if t.any():
        s[t] -= s[t].mean()
    s[~t] = 0.0
    return s


def tgv_velocity(n, period, kx=1, ky=1, kz=1, phase=(0.0, 0.0, 0.0)):
    """Taylor-Green face velocity u = sin X cos Y cos Z, v = -cos X sin Y cos Z,
    w = 0, sampled at the face centres with X = 2 pi k_x (x + phase_x) / period
    (and likewise Y, Z)."""
    u = np.zeros((3, n[2], n[1], n[0]), dtype=np.float64)
    for d in range(2):
        X, Y, Z = face_centres(n, d)
        X = 2 * math.pi * kx * (X + phase[0]) / period
        Y = 2 * math.pi * ky * (Y + phase[1]) / period
        Z = 2 * math.pi * kz * (Z + phase[2]) / period
        if d == 0:
            u[0] = (np.sin(X) * np.cos(Y)) * np.cos(Z)
        else:
            u[1] = -(np.cos(X) * np.sin(Y)) * np.cos(Z)
    return u


def normal_face_noise(n, seed, std=1e-2):
    """i.i.d. N(0, std^2) on every face component, drawn u, v, w in turn,
    each in C order."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.standard_normal((n[2], n[1], n[0])) * std
                     for _ in range(3)])


def uniform_face_velocity(n, seed):
    """i.i.d. U[-1, 1] on every face component, drawn u, v, w in turn."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-1.0, 1.0, (n[2], n[1], n[0]))
                     for _ in range(3)])


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def tgv_periodic(n=32, seed=0):
    """32^3 triple-periodic box, L = 1 everywhere (wrap faces included),
    sigma = div(TGV + noise).  Returns (L, sigma, periodic)."""
    shape = (n, n, n)
    periodic = (True, True, True)
    L = np.ones((3, n, n, n), dtype=np.float64)
    u = tgv_velocity(shape, period=n) + normal_face_noise(shape, seed)
    return L, rhs_from_velocity(L, u, periodic), periodic


def sphere_box(n=(256, 256, 256), centre=(128.0, 128.0, 128.0), radius=32.0,
               velocity="uniform", seed=1, period=None):
    """Wall-bounded box with an immersed sphere.  velocity = 'uniform'
    (U[-1, 1] per face) or 'tgv' (Taylor-Green with the given period plus
    N(0, 0.01^2) noise).  Returns (L, sigma, periodic)."""
    periodic = (False, False, False)
    L = sphere_faces(n, periodic, centre, radius)
    if velocity == "uniform":
        u = uniform_face_velocity(n, seed)
    elif velocity == "tgv":
        u = tgv_velocity(n, period=period) + normal_face_noise(n, seed)
    else:
        raise ValueError(velocity)
    return L, rhs_from_velocity(L, u, periodic), periodic


def sphere_256(seed=1):
    """256^3 walls, sphere diameter 64 at the centre, uniform velocity."""
    return sphere_box((256, 256, 256), (128.0, 128.0, 128.0), 32.0,
                      "uniform", seed)


def sphere_channel(seed=2):
    """512 x 192 x 192 walls ((16 x 6 x 6) D with D = 32), sphere at x = 4 D,
    Taylor-Green velocity with period 192 plus noise."""
    return sphere_box((512, 192, 192), (128.0, 96.0, 96.0), 16.0, "tgv",
                      seed, period=192.0)


def batch_specs(count=64, seed=3):
    """Sizes and spheres of the uneven batch: n_x in {32, 40, ..., 128},
    n_y, n_z in {32, ..., 64}, sphere diameter U[8, 24], centre uniform such
    that the sphere, its 2-cell band and one more cell fit inside."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = (8 * int(rng.integers(4, 17)), 8 * int(rng.integers(4, 9)),
             8 * int(rng.integers(4, 9)))
        radius = 0.5 * float(rng.uniform(8.0, 24.0))
        centre = tuple(float(rng.uniform(radius + 3.0, n[d] - radius - 3.0))
                       for d in range(3))
        specs.append(dict(n=n, centre=centre, radius=radius, seed=seed + i))
    return specs


def batch_problems(count=64, seed=3):
    """List of (L, sigma, periodic) for the uneven batch."""
    return [sphere_box(s["n"], s["centre"], s["radius"], "uniform", s["seed"])
            for s in batch_specs(count, seed)]


def random_problem(n, periodic, seed, contrast=1.0, holes=0.0):
    """Small generic test problem: L_d = 10^(-contrast * U[0, 1]) on every
    face (L = 1 when contrast = 0), a fraction ``holes`` of cells made fully
    inactive by zeroing their six faces, wall faces zeroed, and sigma the
    flux divergence of a U[-1, 1] face velocity with the mean removed."""
    rng = np.random.default_rng(seed)
    shape = (3, n[2], n[1], n[0])
    L = 10.0 ** (-contrast * rng.uniform(0.0, 1.0, shape))
    if holes > 0:
        dead = rng.uniform(0.0, 1.0, shape[1:]) < holes
        for d in range(3):
            L[d][dead] = 0.0
            L[d][np.roll(dead, 1, axis=AX[d])] = 0.0
    L = zero_wall_faces(L, periodic)
    u = rng.uniform(-1.0, 1.0, shape)
    return L, rhs_from_velocity(L, u, periodic), periodic


def tgv_modes_velocity(n, rng, modes=3, kmax=4):
    """Sum of `modes` Taylor-Green modes with random amplitude a ~ U[-1, 1],
    wavenumber k in {1..kmax}, phase in [0, 2 pi)^3 and a random assignment of
    the mode's (u, v, w = 0) components to the three axes; the period is the
    box length along each axis."""
    u = np.zeros((3, n[2], n[1], n[0]), dtype=np.float64)
    for _ in range(modes):
        a = rng.uniform(-1.0, 1.0)
        k = int(rng.integers(1, kmax + 1))
        ph = rng.uniform(0.0, 2 * math.pi, 3)
        perm = rng.permutation(3)  # mode component c acts along axis perm[c]
        for c in range(2):
            d = int(perm[c])
            pos = face_centres(n, d)
            ang = [k * 2 * math.pi * pos[int(perm[e])] / n[int(perm[e])] + ph[e] for e in range(3)]
            if c == 0:
                f = (np.sin(ang[0]) * np.cos(ang[1])) * np.cos(ang[2])
            else:
                f = -(np.cos(ang[0]) * np.sin(ang[1])) * np.cos(ang[2])
            u[d] += a * np.broadcast_to(f, u[d].shape)
    return u


def tgv_modes_sphere(n, seed, dmin=8.0, dmax=24.0):
    """Warm-start training/evaluation problem: walls, a sphere of diameter
    U[dmin, dmax] at a random centre (sphere, band and one cell inside), and
    sigma from a sum of random Taylor-Green modes.  Returns (L, sigma,
    periodic)."""
    rng = np.random.default_rng(seed)
    radius = 0.5 * float(rng.uniform(dmin, dmax))
    centre = tuple(float(rng.uniform(radius + 3.0, n[d] - radius - 3.0)) for d in range(3))
    periodic = (False, False, False)
    L = sphere_faces(n, periodic, centre, radius)
    u = tgv_modes_velocity(n, rng)
    return L, rhs_from_velocity(L, u, periodic), periodic


def moving_body_problem(kind, n, step, dt=0.5, u0=1.0, accel=0.05, x0=None, wave=0.1):
    """Pressure problem of time step `step` of a body moving through a
    walled box (time-correlated problems: consecutive steps differ by a
    fraction of a cell of body motion and a small change of velocity).

    The body (kind 'sphere', diameter n_y / 4, or 'cylinder' along z, same
    diameter) is centred at x = x0 + u0 t + accel t^2 / 2 (x0 default n_y),
    mid-height, at t = step * dt.  The face velocity is the body's speed
    U(t) = u0 + accel t along x plus a Taylor-Green wave of relative
    amplitude `wave` that travels with the flow (phase U t along x), and
    sigma is its flux divergence through L with the mean removed
    (``rhs_from_velocity``), as for the impulsive start.  Returns
    (L, sigma, periodic)."""
    periodic = (False, False, False)
    t = step * dt
    U = u0 + accel * t
    xc = (n[1] if x0 is None else x0) + u0 * t + 0.5 * accel * t * t
    centre = (xc, n[1] / 2, n[2] / 2)
    axis = None if kind == "sphere" else 2
    if kind not in ("sphere", "cylinder"):
        raise ValueError(kind)
    L = body_faces(n, periodic, centre, n[1] / 8, axis)
    u = np.zeros_like(L)
    u[0] = U
    if wave:
        u += wave * U * tgv_velocity(n, period=n[1], phase=(-U * t, 0.0, 0.0))
    return L, rhs_from_velocity(L, u, periodic), periodic
