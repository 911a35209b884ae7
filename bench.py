"""Benchmark: GMG V-cycles/s and time to 1e-6 relative residual on the 256^3
FP32 wall-bounded sphere problem, on one MI355X, through the C ABI.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one V-cycle of the adaptive solve (V(2,2) over all 7 levels, the
level-0 residual norm, and the on-device relaxation / rollback / convergence
decision).  K steps run inside one gmg_solve call with rtol = 0, bracketed by
device synchronisations.  Inputs are resident in HBM before timing starts.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GMG V-cycles/s + time to 1e-6 rel. residual at 256³ FP32; % HBM peak"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell of one fused red-black sweep launch (FP32):
# read x (4), sigma (4), the three face arrays (12); write x (4)
SWEEP_BYTES_PER_CELL = 24.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline():
    """The CPU oracle, untuned, on a bounded sample: one V-cycle plus the
    residual norm of the same workload recipe at 128^3 (sphere diameter 32 at
    the centre, uniform face velocity seed 1), scaled by the cell ratio to
    256^3."""
    from oracle import gmg_oracle as O
    from paper_2607_07687_amd import problems as P

    n = 128
    L, s, per = P.sphere_box((n, n, n), (n / 2,) * 3, n / 8, "uniform", 1)
    L = L.astype(np.float32).astype(np.float64)
    s = s.astype(np.float32).astype(np.float64)
    levels = O.build_hierarchy(L, per, storage="f32")
    t0 = time.perf_counter()
    x = O.vcycle(levels, np.zeros_like(s), s, 1.0)
    O.norm2(O.residual(x, s, levels[0]["L"], per))
    dt = time.perf_counter() - t0
    scale = (n ** 3) / (256 ** 3)
    return {"value": scale / dt, "unit": "V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"1 oracle V-cycle + residual norm at 128^3 (same recipe), "
                      f"{dt:.1f} s, scaled by 1/8 to 256^3; NumPy elementwise, one thread; "
                      f"host has {os.cpu_count()} logical CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol-runs", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_07687_amd import gmg as G
    from paper_2607_07687_amd import problems as P

    G.load()  # fail loudly without the HIP library
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    log("generating 256^3 sphere inputs")
    L, s, per = P.sphere_256(seed=1)
    Ld = torch.from_numpy(L.astype(np.float32)).to(dev)
    sd = torch.from_numpy(s.astype(np.float32)).to(dev)
    del L, s
    n = (256, 256, 256)
    params = G.gmg_default_params(n, per, G.GMG_F32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = G.gmg_setup(params, Ld)
    setup_ms = (time.perf_counter() - t0) * 1e3
    nlev = G.gmg_num_levels(h)
    x = torch.zeros_like(sd)

    # warm-up, then K timed cycles of the adaptive solve
    G.gmg_solve(h, x, sd, 0.0, max(1, args.warmup))
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = G.gmg_solve(h, x, sd, 0.0, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert info["cycles"] == args.steps, info["cycles"]
    log(f"{args.steps} cycles in {dt * 1e3:.2f} ms")

    # time to 1e-6 from x = 0 (median of runs)
    ttt, cyc = [], []
    for _ in range(args.tol_runs):
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = G.gmg_solve(h, x, sd, 1e-6, 200)
        torch.cuda.synchronize()
        ttt.append((time.perf_counter() - t1) * 1e3)
        cyc.append(res["cycles"])
        assert res["status"] == "GMG_OK", res["status"]
    rn, sn = G.gmg_residual(h, x, sd)
    log(f"time to 1e-6: {sorted(ttt)} ms, cycles {cyc}, final rel {rn / sn:.3e}")

    # dominant kernel: the level-0 fused red-black sweep (one launch per
    # sweep), timed with HIP events on the stream the library launches on
    # (torch's current stream); an even sweep count needs no copy-back
    sweeps = 20
    stream = torch.cuda.current_stream(dev)
    G.gmg_smooth(h, 0, x, sd, 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    G.gmg_smooth(h, 0, x, sd, sweeps)
    e1.record(stream)
    torch.cuda.synchronize()
    sweep_ms = e0.elapsed_time(e1) / sweeps
    cells = 256 ** 3
    alg_bytes = SWEEP_BYTES_PER_CELL * cells
    achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    h.close()

    out = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sphere256_walls_fp32", "n": list(n), "levels": nlev,
                   "cycle": "V(2,2), 4 coarsest sweeps, adaptive omega with rollback",
                   "sphere_diameter": 64, "rhs": "flux divergence of U[-1,1] face velocity"},
        "time_to_tol_ms": float(np.median(ttt)),
        "cycles_to_tol": int(np.median(cyc)),
        "final_rel_residual": rn / sn,
        "setup_ms": setup_ms,
        "roofline": {"bound": "hbm", "kernel": "k_rb_sweep<float,float,8> (level-0 fused sweep)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": sweep_ms * 1e3,
                     "alg_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
