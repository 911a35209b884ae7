"""Write tests/golden/sphere256_oracle.json: oracle results on the 256^3
wall-bounded sphere workload (sphere of diameter 64 at the centre, cosine
band of 2 cells, uniform-random face velocity, seed 1), FP32-rounded inputs,
faces stored in FP32 on every level, V(2,2) with the default coarsest-level
rule (groups of 4 sweeps until the coarsest residual falls by 0.1, at most
64), omega = 1.

Calls only the CPU oracle and the input generators.  Takes a few minutes:

    python tests/golden/make_sphere256.py [--no-solve]

Stored: 2048 seeded sample cells of x after the first V-cycle from x = 0,
the norms of that x and of its residual, and the relative-residual history,
omega trajectory and accepted flags of the adaptive solve to 1e-6.
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere256_oracle.json")


def main():
    t0 = time.time()
    L, s, per = P.sphere_256(seed=1)
    L = L.astype(np.float32).astype(np.float64)
    s = s.astype(np.float32).astype(np.float64)
    levels = O.build_hierarchy(L, per, storage="f32")
    print(f"inputs + hierarchy {time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(s.size, 2048, replace=False))
    x1 = O.vcycle(levels, np.zeros_like(s), s, 1.0)
    r1 = O.residual(x1, s, levels[0]["L"], per)
    out = dict(
        source="oracle/gmg_oracle.py via tests/golden/make_sphere256.py",
        workload="256^3 walls, sphere d=64 at centre, uniform face velocity seed 1, FP32 inputs",
        sample_index=idx.tolist(),
        x1_sample=x1.ravel()[idx].tolist(),
        x1_norm=float(np.linalg.norm(x1)),
        r1_norm=O.norm2(r1),
        snorm=O.norm2(s, levels[0]["active"]),
    )
    print(f"vcycle done {time.time() - t0:.0f}s rel {out['r1_norm'] / out['snorm']:.3e}", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f)
    if "--no-solve" in sys.argv:
        return
    res = O.solve(levels, x1 * 0.0, s, 1e-6, 40)
    out.update(solve_status=res["status"], solve_cycles=res["cycles"],
               solve_history=res["history"], solve_omegas=res["omegas"],
               solve_accepted=[bool(a) for a in res["accepted_flags"]])
    print(f"solve {res['status']} {res['cycles']} cycles {time.time() - t0:.0f}s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
