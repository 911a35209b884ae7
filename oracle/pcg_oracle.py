"""Plain CPU FP64 oracle of the two comparison solvers of the paper's solver
table (Sec. 3 and Table 1): the general-purpose preconditioned conjugate
gradient (PCG) solver, and GMG with PCG in place of the red-black smoother
(GMG-PCG).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library; it builds on the
operator, transfer and hierarchy functions of gmg_oracle (same oracle).

Readings (the paper names the solvers, not their details):
* PCG is the textbook conjugate-gradient iteration on the symmetric positive
  (semi)definite form  (-A) x = -sigma  over the active cells, with the
  Jacobi preconditioner M = diag(-A) (the sum of a cell's six faces).
  Inactive cells keep x and carry zero residual and direction.
* The PCG smoother of GMG-PCG is that iteration, restarted from the current
  iterate at every smoothing step, with nu_pre / nu_post / nu_coarse
  iterations in place of red-black sweeps.  It has no relaxation factor, so
  the GMG-PCG solve accepts every cycle (no rollback).
* Stopping test as for GMG: ||r|| / ||sigma|| over active cells.

Parity status: PCG is pinned against scipy's conjugate-gradient routine on
the assembled matrix and against the closed-form finite termination of CG on
a periodic Laplacian; GMG-PCG's smoother is pinned the same way, its cycle
structure is gmg_oracle's (pinned there).
"""
from __future__ import annotations

import numpy as np

from . import gmg_oracle as O


def _dot(a, b, mask):
    """Inner product over the masked cells, accumulated in FP64."""
    return float(np.sum(a[mask].astype(np.float64) * b[mask].astype(np.float64)))


def pcg(x0, sigma, L, periodic, iters, rtol=0.0, snorm=None):
    """Up to `iters` Jacobi-PCG iterations on (-A) x = -sigma from x0; stops
    early when ||r|| / ||sigma|| <= rtol (rtol > 0).  Returns dict(x,
    iterations, history = ||r|| / ||sigma|| after every iteration, rnorm0)."""
    Ln = O.normalize_faces(L, periodic)
    act = O.active_set(Ln, periodic)
    s = -O.diagonal(Ln, periodic)  # the preconditioner: diag(-A) > 0 on active cells
    if snorm is None:
        snorm = O.norm2(sigma, act)
    x = np.array(x0, dtype=np.float64, copy=True)
    r = -O.residual(x, sigma, Ln, periodic)  # b - B x with B = -A, b = -sigma
    rnorm0 = O.norm2(r, act)
    hist = []
    z = np.zeros_like(r)
    z[act] = r[act] / s[act]
    p = z.copy()
    rz = _dot(r, z, act)
    k = 0
    while k < iters:
        if rtol > 0.0 and snorm > 0.0 and O.norm2(r, act) / snorm <= rtol:
            break
        q = np.zeros_like(p)
        q[act] = -O.apply_A(p, Ln, periodic)[act]  # B p
        pq = _dot(p, q, act)
        if pq == 0.0:
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        hist.append(O.norm2(r, act) / snorm if snorm > 0.0 else 0.0)
        z = np.zeros_like(r)
        z[act] = r[act] / s[act]
        rz_new = _dot(r, z, act)
        beta = rz_new / rz if rz != 0.0 else 0.0
        rz = rz_new
        p = z + beta * p
    return dict(x=x, iterations=k, history=hist, rnorm0=rnorm0)


def pcg_solve(L, periodic, x0, sigma, rtol, max_iter):
    """The PCG solver: iterate until ||r|| / ||sigma|| <= rtol or max_iter.
    status 'ok' or 'noconv'."""
    act = O.active_set(O.normalize_faces(L, periodic), periodic)
    snorm = O.norm2(sigma, act)
    res = pcg(x0, sigma, L, periodic, max_iter, rtol=rtol, snorm=snorm)
    final = res["history"][-1] if res["history"] else (res["rnorm0"] / snorm if snorm else 0.0)
    res["status"] = "ok" if final <= rtol else "noconv"
    res["snorm"] = snorm
    return res


def vcycle_pcg(levels, x, sigma, nu_pre=2, nu_post=2, nu_coarse=4, l=0):
    """One V-cycle with the PCG smoother: as gmg_oracle.vcycle, with every
    smoothing step replaced by a restarted PCG run of that many iterations."""
    lev = levels[l]
    L, per = lev["L"], lev["periodic"]
    x = np.array(x, dtype=np.float64, copy=True)
    if lev["c"] is None:
        return pcg(x, sigma, L, per, nu_coarse)["x"]
    x = pcg(x, sigma, L, per, nu_pre)["x"]
    r = O.residual(x, sigma, L, per)
    sigma_c = O.restrict(r, lev["c"])
    x_c = vcycle_pcg(levels, np.zeros_like(sigma_c), sigma_c, nu_pre, nu_post, nu_coarse, l + 1)
    corr = O.prolong(x_c, lev["c"])
    x[lev["active"]] += corr[lev["active"]]
    return pcg(x, sigma, L, per, nu_post)["x"]


def solve_gmg_pcg(levels, x0, sigma, rtol, max_cycles, nu_pre=2, nu_post=2, nu_coarse=4):
    """GMG-PCG: V-cycles with the PCG smoother until ||r|| / ||sigma|| <=
    rtol or max_cycles; every cycle is accepted.  Returns dict(x, status,
    cycles, history)."""
    L, per = levels[0]["L"], levels[0]["periodic"]
    act = levels[0]["active"]
    x = np.array(x0, dtype=np.float64, copy=True)
    snorm = O.norm2(sigma, act)
    hist = []
    rho = O.norm2(O.residual(x, sigma, L, per))
    k = 0
    status = "noconv"
    while True:
        if snorm == 0.0 or rho / snorm <= rtol:
            status = "ok"
            break
        if k >= max_cycles:
            break
        x = vcycle_pcg(levels, x, sigma, nu_pre, nu_post, nu_coarse)
        rho = O.norm2(O.residual(x, sigma, L, per))
        hist.append(rho / snorm)
        k += 1
    return dict(x=x, status=status, cycles=k, history=hist, snorm=snorm)
