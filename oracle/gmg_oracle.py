"""Plain CPU FP64 oracle of the geometric-multigrid (GMG) Poisson V-cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library and imports
nothing from the package.

What it computes (the paper: "Scaling WaterLily.jl with MPI and an improved
geometric multigrid solver", Sec. 3 and 3.1-3.2):

* the variable-coefficient pressure Poisson problem  div(L grad p) = sigma  on
  a Cartesian grid, written as a 7-point face-coefficient operator in
  finite-volume form with unit cell size (Sec. 3.1 names the variable
  coefficients of immersed-boundary flows; the operator form is the reading
  stated in the design notes);
* GMG = smoothing plus coarse-grid correction (Sec. 3, first paragraph);
* red-black Gauss-Seidel smoothing, under-relaxed by a factor omega that
  adapts to residual growth or decay after every V-cycle (Sec. 3.1);
* anisotropic coarsening that halves every direction independently until it
  reaches the coarsening limit, or isotropic coarsening that stops as soon as
  one direction cannot be halved (Sec. 3.2);
* an FP64 iterative-refinement driver around reduced-precision V-cycles.

Everything is written as whole-array NumPy FP64 operations in the order the
method states them; there is no blocking, fusion or reordering.

Array conventions: cell-centred fields are C-order ``[nz][ny][nx]`` (x
fastest).  Face coefficients are ``L[3][nz][ny][nx]`` with ``L[d][I]`` the
coefficient of the LOW d-face of cell I (between I - e_d and I), d = 0, 1, 2
for x, y, z.  ``periodic`` is a 3-tuple of booleans in (x, y, z) order.

Parity status of each function against the paper:
* operator, smoother, transfers, hierarchy, V-cycle: pinned by invariants,
  closed forms, brute force and direct/FFT solves in the tests;
* the adaptive-omega constants (decrease factor, increase factor, bounds,
  rollback): the paper fixes only that omega reacts to growth or decay after
  each V-cycle, so the constants are PARITY UNPINNED against the paper; the
  accepted-residual monotonicity they are meant to ensure is pinned;
* the coarsest-level stopping factor and sweep cap (coarse_rtol, coarse_max):
  the paper says only that the coarsest level is where the smoother removes
  the low wavenumbers, so their values are PARITY UNPINNED against the paper;
  the rule itself is pinned by a brute-force reconstruction.
"""
from __future__ import annotations

import math

import numpy as np

# numpy axis of direction d (x -> axis 2, y -> axis 1, z -> axis 0)
AX = (2, 1, 0)


def _index(d, i):
    """Index tuple selecting position i along direction d of a 3-D array."""
    idx = [slice(None)] * 3
    idx[AX[d]] = i
    return tuple(idx)


# ----------------------------------------------------------------------------
# Operator (Sec. 3.1: variable-coefficient Poisson problem)
# ----------------------------------------------------------------------------

def normalize_faces(L, periodic):
    """Boundary normalisation: a wall direction has no flux through the
    domain's low boundary face, so L_d is zeroed at index 0 there.  The high
    boundary face is handled by ``high_face``.  Returns a new FP64 array."""
    L = np.array(L, dtype=np.float64, copy=True)
    for d in range(3):
        if not periodic[d]:
            L[d][_index(d, 0)] = 0.0
    return L


def high_face(Ld, d, periodic):
    """Coefficient of the HIGH d-face of every cell: L_d[I + e_d], which wraps
    to index 0 in a periodic direction and is 0 at a wall."""
    H = np.roll(Ld, -1, axis=AX[d])
    if not periodic[d]:
        H[_index(d, -1)] = 0.0
    return H


def diagonal(L, periodic):
    """D(I) = -(sum of the six face coefficients of cell I)."""
    D = np.zeros(L.shape[1:], dtype=np.float64)
    for d in range(3):
        D -= L[d] + high_face(L[d], d, periodic)
    return D


def active_set(L, periodic):
    """Cells with D != 0.  Inactive cells (all six faces zero) are decoupled
    from the rest of the grid."""
    return diagonal(L, periodic) != 0.0


def apply_A(x, L, periodic):
    """(A x)(I) = sum_d  L_d^+(I) (x(I+e_d) - x(I)) + L_d(I) (x(I-e_d) - x(I)).

    Flux form of div(L grad x) with unit spacing.  Neighbours across a wall
    are multiplied by a zero coefficient, so the wrapped value from np.roll
    never contributes there."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for d in range(3):
        up = np.roll(x, -1, axis=AX[d])
        dn = np.roll(x, 1, axis=AX[d])
        out += high_face(L[d], d, periodic) * (up - x)
        out += L[d] * (dn - x)
    return out


def residual(x, sigma, L, periodic):
    """r = sigma - A x on the active set, 0 elsewhere."""
    r = np.asarray(sigma, dtype=np.float64) - apply_A(x, L, periodic)
    r[~active_set(L, periodic)] = 0.0
    return r


def norm2(v, mask=None):
    """Euclidean norm over the masked cells, accumulated in FP64."""
    v = np.asarray(v, dtype=np.float64)
    if mask is not None:
        v = v[mask]
    return math.sqrt(float(np.sum(v * v)))


# ----------------------------------------------------------------------------
# Red-black Gauss-Seidel smoother (Sec. 3.1)
# ----------------------------------------------------------------------------

def colour(shape):
    """(i + j + k) mod 2 for every cell of a level (0 = red, 1 = black)."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    return (i + j + k) % 2


def rb_half_sweep(x, sigma, L, periodic, c, omega):
    """Update every active cell of colour c at once, from the residual of x as
    it was before this half-sweep:  x(I) += omega * r(I) / D(I).

    With omega = 1 this is exact Gauss-Seidel on the cell's row; omega < 1
    under-relaxes it.  Returns a new array."""
    D = diagonal(L, periodic)
    r = residual(x, sigma, L, periodic)
    upd = (colour(x.shape) == c) & (D != 0.0)
    x = np.array(x, dtype=np.float64, copy=True)
    x[upd] += omega * r[upd] / D[upd]
    return x


def rb_sweep(x, sigma, L, periodic, omega):
    """One full sweep: red half-sweep, then black."""
    x = rb_half_sweep(x, sigma, L, periodic, 0, omega)
    return rb_half_sweep(x, sigma, L, periodic, 1, omega)


# ----------------------------------------------------------------------------
# Hierarchy and transfers (Sec. 3.2: anisotropic coarsening)
# ----------------------------------------------------------------------------

def can_coarsen(n, periodic, min_coarse):
    """Direction coarsens iff n is even, n/2 >= min_coarse, and (periodic
    directions) n/2 stays even so the red-black colouring survives the wrap."""
    if n % 2 != 0 or n // 2 < min_coarse:
        return False
    if periodic and (n // 2) % 2 != 0:
        return False
    return True


def level_plan(n, periodic, anisotropic=True, min_coarse=4, max_levels=0):
    """List of (shape (nx, ny, nz), factor c (cx, cy, cz) to the next level or
    None on the coarsest) for every level."""
    plan = []
    n = tuple(int(v) for v in n)
    # the problem's dimensions: a direction of extent 1 (a 2-D problem) is
    # not one, and isotropic coarsening leaves it alone
    dims = [d for d in range(3) if n[d] > 1]
    while True:
        ok = [can_coarsen(n[d], periodic[d], min_coarse) for d in range(3)]
        if anisotropic:
            c = tuple(2 if ok[d] else 1 for d in range(3))
            stop = not any(ok)
        else:
            c = tuple(2 if d in dims else 1 for d in range(3))
            stop = not dims or not all(ok[d] for d in dims)
        if max_levels and len(plan) + 1 >= max_levels:
            stop = True
        if stop:
            plan.append((n, None))
            return plan
        plan.append((n, c))
        n = tuple(n[d] // c[d] for d in range(3))


def restrict_faces(L, c):
    """Coarse face coefficients: L_d^c[J] = (1/c_d) * sum of the fine d-faces
    that tile the coarse cell's low d-face (offset 0 along d, every offset
    0..c_e-1 along the other directions e)."""
    nz, ny, nx = L.shape[1:]
    cx, cy, cz = c
    out = np.zeros((3, nz // cz, ny // cy, nx // cx), dtype=np.float64)
    for d in range(3):
        # pick offset 0 along d, then sum over the remaining block offsets
        sub = L[d]
        sl = [slice(None)] * 3
        sl[AX[d]] = slice(0, None, c[d])
        sub = sub[tuple(sl)]
        shp = list(sub.shape)
        cc = [1, 1, 1]  # block size per numpy axis after the pick
        for e in range(3):
            if e != d:
                cc[AX[e]] = c[e]
        blk = sub.reshape(shp[0] // cc[0], cc[0], shp[1] // cc[1], cc[1],
                          shp[2] // cc[2], cc[2])
        out[d] = blk.sum(axis=(1, 3, 5)) / c[d]
    return out


def restrict(r, c):
    """sigma_c[J] = sum of r over the fine cells c*J + s, 0 <= s < c."""
    cx, cy, cz = c
    nz, ny, nx = r.shape
    return r.reshape(nz // cz, cz, ny // cy, cy, nx // cx, cx).sum(axis=(1, 3, 5))


def prolong(y, c):
    """Piecewise-constant prolongation: (P y)[a] = y[a // c]."""
    cx, cy, cz = c
    return np.repeat(np.repeat(np.repeat(y, cz, axis=0), cy, axis=1), cx, axis=2)


def build_hierarchy(L, periodic, anisotropic=True, min_coarse=4, max_levels=0,
                    storage="f64"):
    """Level list: dicts with 'L' (normalised faces, promoted to FP64), 'c'
    (factor to the next level or None), 'periodic', 'active'.

    ``storage`` ('f64', 'f32', 'bf16') is the format the faces of every level
    are kept in: level 0 is rounded to it, and each coarser level is
    restricted from the stored finer one and rounded to it again."""
    L0 = round_to(normalize_faces(L, periodic), storage)
    nz, ny, nx = L0.shape[1:]
    plan = level_plan((nx, ny, nz), periodic, anisotropic, min_coarse, max_levels)
    levels = []
    Lc = L0
    for (n, c) in plan:
        assert Lc.shape[1:] == (n[2], n[1], n[0])
        levels.append({"L": Lc, "c": c, "periodic": tuple(periodic),
                       "active": active_set(Lc, periodic)})
        if c is not None:
            Lc = round_to(restrict_faces(Lc, c), storage)
    return levels


# ----------------------------------------------------------------------------
# V-cycle and adaptive solve (Sec. 3 and 3.1)
# ----------------------------------------------------------------------------

def coarsest_sweeps(x, sigma, L, per, omega, nu_coarse, coarse_rtol, coarse_max, act=None):
    """Smoothing on the coarsest level, where the smoother itself has to
    remove the lowest wavenumbers (Sec. 3.2).  coarse_rtol = 0: exactly
    nu_coarse sweeps.  coarse_rtol > 0: first sigma loses its mean over the
    active cells ``act`` (with walls and periodic directions only the level
    is singular, constants being in the null space, and only a zero-mean
    right-hand side is solvable; the restricted residual has zero mean in
    exact arithmetic), then sweeps in groups of g = max(1, nu_coarse), the
    residual norm over the active cells checked after each group, until it
    is at most coarse_rtol times its value on entry or coarse_max sweeps are
    done (the last group cut to fit).  No direct solve either way.  Returns
    (x, sweeps)."""
    if coarse_rtol <= 0.0:
        for _ in range(nu_coarse):
            x = rb_sweep(x, sigma, L, per, omega)
        return x, nu_coarse
    if act is None:
        act = active_set(L, per)
    sigma = np.array(sigma, dtype=np.float64, copy=True)
    if act.any():
        sigma[act] -= sigma[act].mean()
    r0 = norm2(residual(x, sigma, L, per))
    group = max(1, nu_coarse)
    n = 0
    while n < coarse_max:
        for _ in range(min(group, coarse_max - n)):
            x = rb_sweep(x, sigma, L, per, omega)
            n += 1
        if n < coarse_max and norm2(residual(x, sigma, L, per)) <= coarse_rtol * r0:
            break
    return x, n


def vcycle(levels, x, sigma, omega, nu_pre=2, nu_post=2, nu_coarse=4, l=0, coarse_rtol=0.1,
           coarse_max=64, stats=None):
    """One V(nu_pre, nu_post) cycle from level l with the same omega
    everywhere.  The coarsest level of a hierarchy of two or more levels is
    smoothed by ``coarsest_sweeps`` (no direct solve); a single-level
    hierarchy has no coarse-grid correction, and its cycle is nu_coarse plain
    sweeps.  Returns the new x (a new array); the sweep count of the coarsest
    level is appended to ``stats`` if given."""
    lev = levels[l]
    L, per = lev["L"], lev["periodic"]
    x = np.array(x, dtype=np.float64, copy=True)
    if lev["c"] is None:
        x, n = coarsest_sweeps(x, sigma, L, per, omega, nu_coarse,
                               coarse_rtol if l > 0 else 0.0, coarse_max, lev["active"])
        if stats is not None:
            stats.append(n)
        return x
    for _ in range(nu_pre):
        x = rb_sweep(x, sigma, L, per, omega)
    r = residual(x, sigma, L, per)
    sigma_c = restrict(r, lev["c"])
    x_c = np.zeros_like(sigma_c)
    x_c = vcycle(levels, x_c, sigma_c, omega, nu_pre, nu_post, nu_coarse, l + 1, coarse_rtol,
                 coarse_max, stats)
    corr = prolong(x_c, lev["c"])
    x[lev["active"]] += corr[lev["active"]]
    for _ in range(nu_post):
        x = rb_sweep(x, sigma, L, per, omega)
    return x


DEFAULTS = dict(nu_pre=2, nu_post=2, nu_coarse=4, coarse_rtol=0.1, coarse_max=64, omega0=1.0,
                omega_min=0.1, omega_max=1.0, theta_dec=0.5, theta_inc=1.2, rollback=True)


def solve(levels, x0, sigma, rtol, max_cycles, **kw):
    """Adaptive under-relaxed GMG solve.

    After every V-cycle the new residual norm rho' is compared with the last
    accepted one rho: growth (rho' > rho) lowers omega by theta_dec (not
    below omega_min) and, with rollback, discards the cycle; decay (or a tie)
    accepts it and raises omega by theta_inc (not above omega_max).  Stops when
    rho / ||sigma|| <= rtol or after max_cycles cycles.

    Returns dict(x, status ('ok' | 'noconv'), cycles, accepted, rho0, rho,
    snorm, omega, history (relative residual after every cycle), omegas (omega
    used by every cycle), accepted_flags)."""
    p = dict(DEFAULTS)
    p.update(kw)
    L, per = levels[0]["L"], levels[0]["periodic"]
    act = levels[0]["active"]
    x = np.array(x0, dtype=np.float64, copy=True)
    snorm = norm2(sigma, act)
    rho = norm2(residual(x, sigma, L, per))
    rho0 = rho
    omega = p["omega0"]
    hist, omegas, flags = [], [], []
    k = acc = 0
    if snorm == 0.0:
        return dict(x=x, status="ok", cycles=0, accepted=0, rho0=rho0, rho=rho,
                    snorm=snorm, omega=omega, history=hist, omegas=omegas,
                    accepted_flags=flags)
    status = "noconv"
    while True:
        if rho / snorm <= rtol:
            status = "ok"
            break
        if k >= max_cycles:
            break
        xn = vcycle(levels, x, sigma, omega, p["nu_pre"], p["nu_post"],
                    p["nu_coarse"], coarse_rtol=p["coarse_rtol"], coarse_max=p["coarse_max"])
        rn = norm2(residual(xn, sigma, L, per))
        omegas.append(omega)
        if rn > rho:
            omega = max(p["omega_min"], p["theta_dec"] * omega)
            if not p["rollback"]:
                x, rho = xn, rn
            flags.append(False)
        else:
            x, rho = xn, rn
            omega = min(p["omega_max"], p["theta_inc"] * omega)
            acc += 1
            flags.append(True)
        hist.append(rn / snorm)
        k += 1
    return dict(x=x, status=status, cycles=k, accepted=acc, rho0=rho0, rho=rho,
                snorm=snorm, omega=omega, history=hist, omegas=omegas,
                accepted_flags=flags)


# ----------------------------------------------------------------------------
# FP64 iterative refinement around reduced-precision V-cycles
# ----------------------------------------------------------------------------

def round_to(a, storage):
    """Round an FP64 array to the storage format ('f64', 'f32', 'bf16', the
    latter round-to-nearest-even on the FP32 bit pattern) and return it
    promoted back to FP64."""
    a = np.asarray(a, dtype=np.float64)
    if storage == "f64":
        return a.copy()
    f = a.astype(np.float32)
    if storage == "f32":
        return f.astype(np.float64)
    if storage == "bf16":
        u = f.view(np.uint32).astype(np.uint64)
        lsb = (u >> 16) & 1
        u = ((u + 0x7FFF + lsb) >> 16) << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(storage)


def solve_ir(L, periodic, x0, sigma, rtol=1e-10, max_outer=50, max_inner=8,
             inner_rtol=1e-4, inner_storage="f32", anisotropic=True,
             min_coarse=4, max_levels=0, inner_target=0.5, **kw):
    """Iterative refinement: the outer residual and update are FP64 on the
    exact (normalised) L; each correction comes from an inner adaptive GMG
    solve on the hierarchy built from L rounded to ``inner_storage``, with its
    right-hand side rounded to FP32 after scaling by beta = ||r|| /
    sqrt(|active|).  The inner cycles here are evaluated in FP64 on those
    rounded inputs.  The inner solve of a step that starts from residual
    norm ||r|| stops at max(inner_rtol, inner_target * rtol * ||sigma|| /
    ||r||) relative to its own right-hand side: once the correction brings
    the outer residual within reach of rtol there is no point in reducing
    the inner residual further (the refinement is this build's addition, not
    the paper's; inner_target = 0 keeps inner_rtol).  Returns dict(x,
    status, outer, inner_total, history, inner_tols)."""
    L64 = normalize_faces(L, periodic)
    act = active_set(L64, periodic)
    levels = build_hierarchy(L64, periodic, anisotropic, min_coarse,
                             max_levels, storage=inner_storage)
    x = np.array(x0, dtype=np.float64, copy=True)
    snorm = norm2(sigma, act)
    hist = []
    tols = []
    inner_total = 0
    n_act = int(act.sum())
    status = "noconv"
    for it in range(max_outer + 1):
        r = residual(x, sigma, L64, periodic)
        rn = norm2(r)
        hist.append(rn / snorm if snorm > 0 else 0.0)
        if snorm == 0.0 or rn / snorm <= rtol:
            status = "ok"
            break
        if it == max_outer:
            break
        beta = rn / math.sqrt(n_act)
        b = round_to(r / beta, "f32")
        tol = inner_rtol
        if inner_target > 0 and rn > 0:
            tol = max(inner_rtol, inner_target * rtol * snorm / rn)
        tols.append(tol)
        res = solve(levels, np.zeros_like(b), b, tol, max_inner, **kw)
        inner_total += res["cycles"]
        x = x + beta * res["x"]
    return dict(x=x, status=status, outer=len(hist) - 1,
                inner_total=inner_total, history=hist, inner_tols=tols)
