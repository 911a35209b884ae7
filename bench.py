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
# algorithmic bytes per cell of one launch of either level-0 smoothing
# kernel (FP32): read x (4), sigma (4), the three face arrays (12); write x
# (4).  The fused sweep does one sweep per launch, the two-sweep pass two.
SWEEP_BYTES_PER_CELL = 24.0

# hardware-counter summaries of the level-0 smoothing kernels (rocprofv3
# FETCH_SIZE and WRITE_SIZE runs of `bench.py --kernel-probe`), each naming
# the hash of the sources the counted kernel was built from, and everything
# that kernel is compiled from (kernel, helpers, flags)
_CSRC = "paper_2607_07687_amd/csrc/"
KERNELS = {
    "fused": (os.path.join(ROOT, "profiles", "sweep256_fp32_counters.md"),
              [_CSRC + "gmg_sweep.h", _CSRC + "gmg_device.h", "paper_2607_07687_amd/build.py"]),
    "pair": (os.path.join(ROOT, "profiles", "sweep2_256_fp32_counters.md"),
             [_CSRC + "gmg_sweep2.h", _CSRC + "gmg_sweep.h", _CSRC + "gmg_device.h",
              "paper_2607_07687_amd/build.py"]),
}


def device_copy_gbs(stream, mib=256, reps=10):
    """Bandwidth of a plain device-to-device copy of `mib` MiB (read + write
    bytes over time, HIP events), the practical ceiling the kernels are also
    reported against."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_source_hash(kind="fused"):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNELS[kind][1]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kind="fused"):
    """HBM bytes per launch of a level-0 smoothing kernel from the committed
    counter runs: FETCH_SIZE scaled by the copy-kernel calibration factor,
    plus WRITE_SIZE.  None when the summary is missing or the kernel's
    sources have changed since the counters were taken."""
    import re
    try:
        text = open(KERNELS[kind][0]).read()
    except OSError:
        return None
    vals = dict(re.findall(r"^- (\w+): ([0-9a-f.]+)\s*$", text, re.M))
    try:
        if vals["source_hash"] != sweep_source_hash(kind):
            return None
        kib = float(vals["fetch_kib_per_launch"]) * float(vals["fetch_factor"]) + \
            float(vals["write_kib_per_launch"]) * float(vals["write_factor"])
    except (KeyError, ValueError):
        return None
    return kib * 1024.0


def cpu_baseline(cycles=2):
    """The CPU oracle, untuned, on a bounded sample of the benchmark workload
    itself: `cycles` V-cycles, each followed by the residual norm, on the
    same 256^3 sphere problem rounded to FP32 (hierarchy built untimed)."""
    from oracle import gmg_oracle as O
    from paper_2607_07687_amd import problems as P

    L, s, per = P.sphere_256(seed=1)
    L = L.astype(np.float32).astype(np.float64)
    s = s.astype(np.float32).astype(np.float64)
    levels = O.build_hierarchy(L, per, storage="f32")
    del L
    x = np.zeros_like(s)
    t0 = time.perf_counter()
    for _ in range(cycles):
        x = O.vcycle(levels, x, s, 1.0)
        O.norm2(O.residual(x, s, levels[0]["L"], per))
    dt = time.perf_counter() - t0
    return {"value": cycles / dt, "unit": "V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{cycles} oracle V-cycles, each with its residual norm, on the 256^3 "
                      f"benchmark problem: {dt:.1f} s; NumPy elementwise, one thread; "
                      f"host has {os.cpu_count()} logical CPUs"}


def timed(fn, reps=3):
    import torch
    ts, out = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts)), out


def solver_comparison(rtol=1e-6, reps=3):
    """The paper's solver table on synthetic stand-ins: generic PCG, GMG with
    the PCG smoother and GMG with the adaptive red-black smoother, FP32 from
    x = 0 to rtol, on walled boxes with a sphere at the table's grid sizes
    4 * 2^(3p) (p = 5, 6: 2:1:2 boxes) and on the 256^3 benchmark problem.
    Iterations are PCG iterations or V-cycles; cost is wall time per cell."""
    import torch
    from paper_2607_07687_amd import gmg as G
    from paper_2607_07687_amd import problems as P
    out = {}
    for name, n in (("p5_64x32x64", (64, 32, 64)), ("p6_128x64x128", (128, 64, 128)),
                    ("sphere256", (256, 256, 256))):
        if n[0] == 256:
            L, s, per = P.sphere_256(seed=1)
        else:
            L, s, per = P.sphere_box(n, tuple(v / 2 for v in n), n[1] / 4, "uniform", 1)
        Ld = torch.from_numpy(L.astype(np.float32)).cuda()
        sd = torch.from_numpy(s.astype(np.float32)).cuda()
        del L, s
        cells = n[0] * n[1] * n[2]
        row = {}
        for solver in ("PCG", "GMG-PCG", "GMG-RBGS"):
            smoother = G.GMG_SMOOTH_PCG if solver == "GMG-PCG" else G.GMG_SMOOTH_RBGS
            h = G.gmg_setup(G.gmg_default_params(n, per, G.GMG_F32, smoother=smoother), Ld)
            x = torch.zeros_like(sd)

            def run():
                x.zero_()
                if solver == "PCG":
                    i = G.gmg_pcg(h, x, sd, rtol, 20000)
                    return i["status"], i["iterations"]
                i = G.gmg_solve(h, x, sd, rtol, 500)
                return i["status"], i["cycles"]

            run()  # capture / warm-up
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                status, its = run()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            rn, sn = G.gmg_residual(h, x, sd)
            ms = 1e3 * float(np.median(ts))
            row[solver] = {"iterations": its, "status": status, "final_rel": rn / sn, "ms": ms,
                           "ns_per_cell": 1e6 * ms / cells}
            h.close()
        base = row["GMG-RBGS"]["ms"]
        row["cost_ratio_vs_gmg_rbgs"] = {k: row[k]["ms"] / base for k in ("PCG", "GMG-PCG")}
        out[name] = row
        log(f"{name}: " + ", ".join(f"{k} {row[k]['iterations']} it {row[k]['ms']:.2f} ms"
                                    for k in ("PCG", "GMG-PCG", "GMG-RBGS")))
    return out


def coarsening_sweep(m=64, aspects=(1, 2, 4, 8), rtol=1e-8, max_cycles=3000):
    """Anisotropic against isotropic coarsening on impulsive-start problems
    (unit inflow along x past a 2-D cylinder, a spanwise-periodic cylinder
    and a sphere in boxes of aspect ratio N = aspect x 1 x 1): FP64 V(2,2)
    cycles from x = 0 to rtol, and the wall time of each solve."""
    import torch
    from paper_2607_07687_amd import gmg as G
    from paper_2607_07687_amd import problems as P
    out = {}
    for kind in P.IMPULSIVE_KINDS:
        for N in aspects:
            L, s, per = P.impulsive_problem(kind, N, m)
            n = (L.shape[3], L.shape[2], L.shape[1])
            Ld = torch.from_numpy(L).cuda()
            sd = torch.from_numpy(s).cuda()
            del L, s
            row = {"n": list(n)}
            for aniso in (1, 0):
                h = G.gmg_setup(G.gmg_default_params(n, per, G.GMG_F64, anisotropic=aniso), Ld)
                x = torch.zeros_like(sd)
                G.gmg_solve(h, x, sd, rtol, 1)  # capture the cycle graph
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = G.gmg_solve(h, x, sd, rtol, max_cycles)
                torch.cuda.synchronize()
                row["aniso" if aniso else "iso"] = {
                    "levels": G.gmg_num_levels(h), "cycles": info["cycles"],
                    "status": info["status"], "ms": 1e3 * (time.perf_counter() - t0)}
                h.close()
            row["cycle_ratio_iso_over_aniso"] = row["iso"]["cycles"] / max(1, row["aniso"]["cycles"])
            out[f"{kind}_N{N}"] = row
            log(f"{kind} N={N} {tuple(n)}: aniso {row['aniso']['cycles']} cycles "
                f"({row['aniso']['levels']} levels), iso {row['iso']['cycles']} "
                f"({row['iso']['levels']} levels)")
    return out


def extra_configs():
    """The other workloads, each on one GPU: the 32^3 periodic FP64 solve to
    1e-10, anisotropic vs isotropic coarsening on the 512 x 192 x 192 sphere
    channel, and 64 uneven problems refined to 1e-10 (one graph replay per refinement step)."""
    import torch
    from paper_2607_07687_amd import gmg as G
    from paper_2607_07687_amd import problems as P
    out = {}
    # 32^3 triple-periodic TGV, FP64, to 1e-10
    L, s, per = P.tgv_periodic(32, seed=0)
    h = G.gmg_setup(G.gmg_default_params((32, 32, 32), per, G.GMG_F64),
                    torch.from_numpy(L).cuda())
    sd = torch.from_numpy(s).cuda()
    x = torch.zeros_like(sd)

    def run():
        x.zero_()
        return G.gmg_solve(h, x, sd, 1e-10, 100)
    run()
    ms, res = timed(run, 5)
    out["tgv32_fp64"] = {"time_to_1e-10_ms": ms, "cycles": res["cycles"], "status": res["status"]}
    h.close()
    log(f"tgv32: {out['tgv32_fp64']}")
    # 512 x 192 x 192 sphere channel: anisotropic vs isotropic coarsening.
    # Its smooth Taylor-Green right-hand side leaves an FP32 residual floor
    # near 7e-6, so cycles are counted to 1e-5
    L, s, per = P.sphere_channel(seed=2)
    Ld = torch.from_numpy(L.astype(np.float32)).cuda()
    sd = torch.from_numpy(s.astype(np.float32)).cuda()
    del L, s
    ch = {}
    for name, aniso in (("aniso", 1), ("iso", 0)):
        h = G.gmg_setup(G.gmg_default_params((512, 192, 192), per, G.GMG_F32,
                                             anisotropic=aniso), Ld)
        x = torch.zeros_like(sd)

        def run():
            x.zero_()
            return G.gmg_solve(h, x, sd, 1e-5, 300)
        run()
        ms, res = timed(run, 3)
        ch[name] = {"levels": G.gmg_num_levels(h), "rtol": 1e-5, "cycles": res["cycles"],
                    "status": res["status"], "time_ms": ms,
                    "final_rel": res["history"][-1] if res["history"] else None}
        h.close()
    out["channel512x192x192_fp32"] = ch
    log(f"channel: {ch}")
    del Ld, sd
    # 64 uneven problems, FP64 refinement to 1e-10, one graph replay per step
    probs = P.batch_problems(64, seed=3)
    Ls = [torch.from_numpy(L).cuda() for L, _, _ in probs]
    ss = [torch.from_numpy(s).cuda() for _, s, _ in probs]
    prms = [G.gmg_default_params((L.shape[3], L.shape[2], L.shape[1]), per, G.GMG_F64,
                                 cycle_dtype=G.GMG_F32) for L, _, per in probs]
    cells = int(sum(L[0].size for L, _, _ in probs))
    del probs
    b = G.gmg_batch_setup(prms, Ls)
    G.gmg_batch_autotune(b, reps=3)
    xs = [torch.zeros_like(s) for s in ss]

    def run():
        for t in xs:
            t.zero_()
        return G.gmg_batch_solve_ir(b, xs, ss, rtol=1e-10, max_outer=30, max_inner=8)
    run()  # records the graph
    ms, infos = timed(run, 3)
    out["batch64_ir_fp64"] = {"problems": 64, "cells": cells, "time_to_1e-10_ms": ms,
                              "all_ok": all(i["status"] == "GMG_OK" for i in infos),
                              "max_outer": max(i["outer"] for i in infos),
                              "worst_final_rel": max(i["history"][-1] for i in infos),
                              "graph_launches": 1 + max(i["outer"] for i in infos)}
    b.close()
    log(f"batch: {out['batch64_ir_fp64']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol-runs", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only run a 256 MiB device copy (counter calibration), 4 level-0 "
                         "sweeps at 256^3 as two two-sweep passes, then 4 as fused sweeps, "
                         "for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_07687_amd import autotune as AT
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
    if args.kernel_probe:
        a = torch.ones(64 * 2 ** 20, dtype=torch.float32, device=dev)  # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        G.gmg_smooth(h, 0, x, sd, 4)
        G.gmg_set_pair_sweeps(h, 0, 0)
        G.gmg_smooth(h, 0, x, sd, 4)
        torch.cuda.synchronize()
        log("kernel probe done: copy of 256 MiB, 2 two-sweep passes, 4 fused sweeps")
        h.close()
        return

    # warm-up, then K timed cycles of the adaptive solve
    tiles = AT.tune(h, x, sd, cache=None)  # timed sweep tiles per level (setup, untimed)
    log("tiles " + ", ".join(f"L{t['level']}:{t['ty']}x{t['kchunk']}" +
                             (f"+pass{t.get('pair_ty', 16)}x{t['pair_kchunk']}"
                              if t.get("pair_kchunk") else "")
                             for t in tiles))
    x.zero_()
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

    # dominant kernel: the level-0 smoothing launch the solve uses (the
    # two-sweep pass, or the fused sweep where the tuner turned passes off),
    # timed with HIP events on the stream the library launches on (torch's
    # current stream); an even sweep count needs no copy-back.  The other
    # kernel is timed the same way for comparison.
    sweeps = 20
    stream = torch.cuda.current_stream(dev)

    def launch_ms(per_launch):
        G.gmg_smooth(h, 0, x, sd, 2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        G.gmg_smooth(h, 0, x, sd, sweeps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / (sweeps // per_launch)

    pair_kc = tiles[0].get("pair_kchunk", 0)
    pass_ms = launch_ms(2) if pair_kc else None
    G.gmg_set_pair_sweeps(h, 0, 0)
    fused_ms = launch_ms(1)
    kind = "pair" if pair_kc else "fused"
    launch = pass_ms if pair_kc else fused_ms
    copy_gbs = device_copy_gbs(stream)
    cells = 256 ** 3
    alg_bytes = SWEEP_BYTES_PER_CELL * cells
    achieved = alg_bytes / (launch * 1e-3) / 1e9
    h.close()
    if pair_kc:
        kname = (f"k_rb_sweep2<float,float,{tiles[0].get('pair_ty', 16)},false> "
                 "(level-0 two-sweep pass, 2 sweeps per launch)")
    elif tiles[0]["ty"] != 1:
        kname = f"k_rb_sweep<float,float,{tiles[0]['ty']},2> (level-0 fused sweep)"
    else:
        kname = "k_half_sweep<float,float> (level-0 split sweep)"

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
        "tiles": [{"level": t["level"], "ty": t["ty"], "kchunk": t["kchunk"],
                   "pass_ty": t.get("pair_ty", 16), "pass_kchunk": t.get("pair_kchunk", 0)}
                  for t in tiles],
        "roofline": {"bound": "hbm", "kernel": kname,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kind),
                     "traffic_unit": "HBM bytes per launch (counters)",
                     "avg_launch_us": launch * 1e3,
                     "alg_bytes_per_launch": alg_bytes,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "level0_smoothing": {
            "two_sweep_pass_us": pass_ms * 1e3 if pass_ms else None,
            "fused_sweep_us": fused_ms * 1e3,
            "us_per_sweep": (pass_ms / 2 if pass_ms else fused_ms) * 1e3,
            "fused_sweep_frac": alg_bytes / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "fused_sweep_traffic": measured_traffic("fused")},
    }
    if not args.no_extras:
        out["other_configs"] = extra_configs()
        out["other_configs"]["solver_table"] = solver_comparison()
        out["other_configs"]["coarsening_sweep"] = coarsening_sweep()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
