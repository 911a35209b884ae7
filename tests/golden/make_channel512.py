"""Write tests/golden/channel512_oracle.json: oracle results on the
512 x 192 x 192 wall-bounded sphere channel ((16 x 6 x 6) D with D = 32,
sphere of diameter D at x = 4 D, Taylor-Green velocity of period 192 plus
N(0, 0.01^2) face noise, seed 2), FP32-rounded inputs, faces stored in FP32
on every level, default V(2,2) cycle and coarsest-level rule, omega = 1, for
anisotropic (8 levels) and isotropic (6 levels) coarsening (Sec. 3.2).

Calls only the CPU oracle and the input generators.  Takes about 15 minutes:

    python tests/golden/make_channel512.py

Stored per coarsening: the level shapes, 2048 seeded sample cells of x after
the first V-cycle from x = 0, the norms of that x and of its residual, and
the relative-residual history, omega trajectory and accepted flags of the
adaptive solve to 1e-5 (this right-hand side leaves an FP32 residual floor
near 7e-6, so 1e-6 is out of reach of FP32 cycles), plus the FP32 rounding
floor of a history value, 16 eps_32 max|D| ||x|| / ||sigma||.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gmg_oracle as O  # noqa: E402
from paper_2607_07687_amd import problems as P  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "channel512_oracle.json")
RTOL = 1e-5
MAX_CYCLES = 150


def main():
    t0 = time.time()
    L, s, per = P.sphere_channel(seed=2)
    L = L.astype(np.float32).astype(np.float64)
    s = s.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(54321)
    idx = np.sort(rng.choice(s.size, 2048, replace=False))
    out = dict(source="oracle/gmg_oracle.py via tests/golden/make_channel512.py",
               workload="512x192x192 walls, sphere d=32 at x=128, TGV period 192 + noise seed 2, "
                        "FP32 inputs", rtol=RTOL, sample_index=idx.tolist())
    for name, aniso in (("aniso", True), ("iso", False)):
        levels = O.build_hierarchy(L, per, anisotropic=aniso, storage="f32")
        x1 = O.vcycle(levels, np.zeros_like(s), s, 1.0)
        r1 = O.residual(x1, s, levels[0]["L"], per)
        snorm = O.norm2(s, levels[0]["active"])
        print(f"{name}: {len(levels)} levels, first cycle rel {O.norm2(r1) / snorm:.3e} "
              f"{time.time() - t0:.0f}s", flush=True)
        res = O.solve(levels, np.zeros_like(s), s, RTOL, MAX_CYCLES)
        maxD = float(np.abs(O.diagonal(levels[0]["L"], per)).max())
        floor = 16.0 * 2.0 ** -24 * maxD * float(np.linalg.norm(res["x"])) / snorm
        out[name] = dict(levels=[list(lv["L"].shape[1:][::-1]) for lv in levels],
                         x1_sample=x1.ravel()[idx].tolist(), x1_norm=float(np.linalg.norm(x1)),
                         r1_norm=O.norm2(r1), snorm=snorm, solve_status=res["status"],
                         solve_cycles=res["cycles"], solve_history=res["history"],
                         solve_omegas=res["omegas"],
                         solve_accepted=[bool(a) for a in res["accepted_flags"]],
                         fp32_floor=floor)
        print(f"{name}: solve {res['status']} {res['cycles']} cycles, floor {floor:.2e} "
              f"{time.time() - t0:.0f}s", flush=True)
        del levels, x1, r1, res
        with open(OUT, "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
