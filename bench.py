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
# algorithmic bytes per cell and red-black sweep (FP32): read x (4), sigma
# (4), the three face arrays (12) and write x (4) once per sweep.  A launch
# moves this times the sweeps it performs (the fused sweep one, the
# two-sweep pass two).  The pass's own minimum, one read of everything and
# one write of x for both sweeps, is the same 24 B per cell per launch.
SWEEP_BYTES_PER_CELL = 24.0
# With the uniform-brick map the faces of a uniform brick (128 x 2 x 2
# cells whose faces are one constant per direction) are not data: the
# kernels take them from the map's 32-B entry.  Per sweep the method then
# moves 12 B per cell (x, sigma, x) plus the 12 B of faces per cell of the
# other bricks plus the map.
SWEEP_BYTES_NO_FACES = 12.0
FACE_BYTES_PER_CELL = 12.0
BRICK_CELLS = 128 * 2 * 2
BRICK_BYTES = 32.0

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
              _CSRC + "gmg_kernels.h", "include/gmg.h", "paper_2607_07687_amd/build.py"]),
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


def _oracle_cycles(L, s, per, cycles, **kw):
    """Seconds for `cycles` oracle V-cycles, each with its residual norm, on
    FP32-rounded inputs (hierarchy built untimed)."""
    from oracle import gmg_oracle as O
    L = L.astype(np.float32).astype(np.float64)
    s = s.astype(np.float32).astype(np.float64)
    levels = O.build_hierarchy(L, per, storage="f32", **kw)
    del L
    x = np.zeros_like(s)
    t0 = time.perf_counter()
    for _ in range(cycles):
        x = O.vcycle(levels, x, s, 1.0)
        O.norm2(O.residual(x, s, levels[0]["L"], per))
    return time.perf_counter() - t0


def _oracle_batch_problem(i):
    """One problem of the uneven batch refined to 1e-10 by the oracle."""
    from oracle import gmg_oracle as O
    from paper_2607_07687_amd import problems as P
    sp = P.batch_specs(64, 3)[i]
    L, s, per = P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
    res = O.solve_ir(L, per, np.zeros_like(s), s, rtol=1e-10, max_outer=30, max_inner=8)
    return res["outer"], res["inner_total"], res["status"]


def cpu_baseline(cycles=2, others=True):
    """The CPU oracle, untuned, on bounded samples of the workloads: `cycles`
    V-cycles (each with its residual norm) of the 256^3 benchmark problem
    (the reported value), and beside it the 32^3 periodic FP64 solve to 1e-10
    in full, 2 V-cycles of the 512 x 192 x 192 channel and the 64-problem
    batch refined to 1e-10 in a process pool over the host cores."""
    from oracle import gmg_oracle as O
    from paper_2607_07687_amd import problems as P

    L, s, per = P.sphere_256(seed=1)
    dt = _oracle_cycles(L, s, per, cycles)
    del L, s
    out = {"value": cycles / dt, "unit": "V-cycles/s", "cores": 1, "kind": "oracle",
           "sample": f"{cycles} oracle V-cycles, each with its residual norm, on the 256^3 "
                     f"benchmark problem: {dt:.1f} s; NumPy elementwise, one thread; "
                     f"host has {os.cpu_count()} logical CPUs"}
    if not others:
        return out
    legs = {}
    log("oracle: 32^3 periodic FP64 solve")
    L, s, per = P.tgv_periodic(32, seed=0)
    levels = O.build_hierarchy(L, per)
    t0 = time.perf_counter()
    res = O.solve(levels, np.zeros_like(s), s, 1e-10, 100)
    legs["tgv32_fp64_solve"] = {"value": 1e3 * (time.perf_counter() - t0), "unit": "ms to 1e-10",
                                "cycles": res["cycles"], "cores": 1,
                                "sample": "full oracle solve from x = 0, FP64"}
    log("oracle: 512 x 192 x 192 channel cycles")
    L, s, per = P.sphere_channel(seed=2)
    dt = _oracle_cycles(L, s, per, cycles)
    del L, s
    legs["channel512_fp32_aniso"] = {"value": cycles / dt, "unit": "V-cycles/s", "cores": 1,
                                     "sample": f"{cycles} oracle V-cycles with residual norms, "
                                               f"anisotropic hierarchy: {dt:.1f} s"}
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    log(f"oracle: 64-problem batch over {workers} processes")
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        rs = list(ex.map(_oracle_batch_problem, range(64)))
    dt = time.perf_counter() - t0
    legs["batch64_ir_fp64"] = {"value": 1e3 * dt, "unit": "ms to 1e-10 (all 64 problems)",
                               "cores": workers, "all_ok": all(r[2] == "ok" for r in rs),
                               "max_outer": max(r[0] for r in rs),
                               "sample": f"the 64 problems refined to 1e-10 by the oracle, "
                                         f"one per task in a pool of {workers} processes"}
    out["other_configs"] = legs
    return out


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
            # the default coarsest-level rule, and fixed nu_coarse = 4 sweeps
            for rule, crtol in (("", None), ("_fixed4", 0.0)):
                for aniso in (1, 0):
                    kw = {} if crtol is None else {"coarse_rtol": crtol, "nu_coarse": 4}
                    h = G.gmg_setup(G.gmg_default_params(n, per, G.GMG_F64, anisotropic=aniso,
                                                         **kw), Ld)
                    x = torch.zeros_like(sd)
                    G.gmg_solve(h, x, sd, rtol, 1)  # capture the cycle graph
                    x.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    info = G.gmg_solve(h, x, sd, rtol, max_cycles)
                    torch.cuda.synchronize()
                    row[("aniso" if aniso else "iso") + rule] = {
                        "levels": G.gmg_num_levels(h), "cycles": info["cycles"],
                        "status": info["status"], "ms": 1e3 * (time.perf_counter() - t0)}
                    h.close()
                row["cycle_ratio_iso_over_aniso" + rule] = \
                    row["iso" + rule]["cycles"] / max(1, row["aniso" + rule]["cycles"])
            out[f"{kind}_N{N}"] = row
            log(f"{kind} N={N} {tuple(n)}: aniso {row['aniso']['cycles']} cycles "
                f"({row['aniso']['levels']} levels), iso {row['iso']['cycles']} "
                f"({row['iso']['levels']} levels); fixed 4 coarsest sweeps: aniso "
                f"{row['aniso_fixed4']['cycles']}, iso {row['iso_fixed4']['cycles']}")
    return out


def sequence_solves(n=(256, 64, 64), steps=12, rtol=1e-6):
    """Time-correlated pressure solves (the regime of Table 1): a sphere
    accelerating through a walled 4:1:1 box, one solve per time step after
    replacing the hierarchy's faces in place (gmg_update_faces): FP64
    refinement around FP32 V-cycles to rtol (these smooth pressures sit
    below the FP32 residual floor), from zero, from the previous step's
    pressure, and from its linear extrapolation 2 p(t-1) - p(t-2).  Reports
    V-cycles per solve (mean over the steps after the second), refinement
    steps, the final relative residual and the wall time per step (face
    update + solve) per cell."""
    import torch
    from paper_2607_07687_amd import gmg as G
    from paper_2607_07687_amd import problems as P
    seq = [P.moving_body_problem("sphere", n, k) for k in range(steps)]
    per = seq[0][2]
    Ls = [torch.from_numpy(L).cuda() for L, _, _ in seq]
    ss = [torch.from_numpy(s).cuda() for _, s, _ in seq]
    del seq
    h = G.gmg_setup(G.gmg_default_params(n, per, G.GMG_F64, cycle_dtype=G.GMG_F32), Ls[0])
    cells = n[0] * n[1] * n[2]
    out = {"n": list(n), "steps": steps, "rtol": rtol,
           "solve": "FP64 refinement around FP32 V(2,2) cycles"}
    for mode in ("cold", "previous", "extrapolated"):
        x = torch.zeros_like(ss[0])
        p1 = torch.zeros_like(x)
        p2 = torch.zeros_like(x)
        cyc, outer, fin, ms = [], [], [], []
        G.gmg_solve_ir(h, x, ss[0], rtol, 30)  # graph capture
        for k in range(steps):
            if mode == "cold" or k == 0:
                x.zero_()
            elif mode == "previous" or k == 1:
                x.copy_(p1)
            else:
                torch.sub(p1 * 2.0, p2, out=x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            G.gmg_update_faces(h, Ls[k])
            info = G.gmg_solve_ir(h, x, ss[k], rtol, 30)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
            cyc.append(info["inner_total"])
            outer.append(info["outer"])
            fin.append(info["history"][-1])
            assert info["status"] == "GMG_OK", (mode, k, info["status"])
            p2.copy_(p1)
            p1.copy_(x)
        out[mode] = {"cycles_per_solve": float(np.mean(cyc[2:])), "cycles": cyc,
                     "refinement_steps": outer, "worst_final_rel": max(fin),
                     "ms_per_step": float(np.median(ms[2:])),
                     "ns_per_cell_step": 1e6 * float(np.median(ms[2:])) / cells}
        log(f"sequence {mode}: cycles {cyc}, {out[mode]['ms_per_step']:.2f} ms per step")
    h.close()
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
    out["batch64_ir_fp64"] = batch_solves()
    return out


def batch_solves(reps=3):
    """64 uneven problems, FP64 refinement to 1e-10, one graph replay per
    refinement step (the median of `reps` timed solves after one that
    records the graphs)."""
    import torch
    from paper_2607_07687_amd import gmg as G
    from paper_2607_07687_amd import problems as P
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
    ms, infos = timed(run, reps)
    outer = [i["outer"] for i in infos]
    inner = [i["inner_total"] for i in infos]
    res = {"problems": 64, "cells": cells, "time_to_1e-10_ms": ms,
                              "all_ok": all(i["status"] == "GMG_OK" for i in infos),
                              "max_outer": max(outer),
                              "outer_histogram": {str(k): outer.count(k)
                                                  for k in sorted(set(outer))},
                              "inner_cycles_min_median_max": [min(inner),
                                                              float(np.median(inner)),
                                                              max(inner)],
                              "slowest_problem": int(np.argmax(inner)),
                              "worst_final_rel": max(i["history"][-1] for i in infos),
                              "graph_launches": 1 + max(outer)}
    b.close()
    log(f"batch: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol-runs", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--batch-probe", action="store_true",
                    help="only the 64-problem batch solve (3 timed runs), for kernel traces")
    ap.add_argument("--deferred-norm", type=int, default=None, choices=(0, 1),
                    help="override the library's default deferred_norm for the 256^3 solve")
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
    if args.batch_probe:
        print(json.dumps(batch_solves()), flush=True)
        return
    dev = torch.device("cuda:0")
    log("generating 256^3 sphere inputs")
    L, s, per = P.sphere_256(seed=1)
    Ld = torch.from_numpy(L.astype(np.float32)).to(dev)
    sd = torch.from_numpy(s.astype(np.float32)).to(dev)
    del L, s
    n = (256, 256, 256)
    params = G.gmg_default_params(n, per, G.GMG_F32)
    if args.deferred_norm is not None:
        params.deferred_norm = args.deferred_norm
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
    floor_sweeps = G.gmg_coarse_sweeps(h)
    log(f"{args.steps} cycles in {dt * 1e3:.2f} ms (coarsest sweeps in the last: {floor_sweeps})")

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
    coarse_last = G.gmg_coarse_sweeps(h)
    log(f"time to 1e-6: {sorted(ttt)} ms, cycles {cyc}, final rel {rn / sn:.3e}, "
        f"coarsest sweeps in the last cycle {coarse_last}")

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
    pair_ty = tiles[0].get("pair_ty", 16)
    pass_ms = launch_ms(2) if pair_kc else None
    G.gmg_set_pair_sweeps(h, 0, 0)
    fused_ms = launch_ms(1)
    kind = "pair" if pair_kc else "fused"
    launch = pass_ms if pair_kc else fused_ms
    uni_bricks, bricks = G.gmg_level_uniform(h, 0)
    h.close()
    # the same kernel with no map (every face loaded), at the same tiling
    nomap_ms = None
    if pair_kc:
        params.uniform_bricks = 0
        h = G.gmg_setup(params, Ld)
        G.gmg_set_pair_sweeps(h, 0, pair_kc, pair_ty)
        nomap_ms = launch_ms(2)
        h.close()
    copy_gbs = device_copy_gbs(stream)
    cells = 256 ** 3
    sweeps_per_launch = 2 if pair_kc else 1
    # the pass reads the map; the fused sweep loads every face
    face_cells = (bricks - uni_bricks) * BRICK_CELLS if pair_kc else cells
    map_bytes = bricks * BRICK_BYTES if pair_kc else 0.0
    sweep_bytes = SWEEP_BYTES_NO_FACES * cells + FACE_BYTES_PER_CELL * face_cells + map_bytes
    alg_bytes = sweep_bytes * sweeps_per_launch
    achieved = alg_bytes / (launch * 1e-3) / 1e9
    one_read_gbs = sweep_bytes / (launch * 1e-3) / 1e9
    dense_bytes = SWEEP_BYTES_PER_CELL * sweeps_per_launch * cells
    traffic = measured_traffic(kind)
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
                   "cycle": f"V({params.nu_pre},{params.nu_post}), coarsest level swept until "
                            f"its residual falls by {params.coarse_rtol:g} (at most "
                            f"{params.coarse_max} sweeps), adaptive omega with rollback",
                   "deferred_norm": int(params.deferred_norm),
                   "sphere_diameter": 64, "rhs": "flux divergence of U[-1,1] face velocity"},
        "time_to_tol_ms": float(np.median(ttt)),
        "cycles_to_tol": int(np.median(cyc)),
        "final_rel_residual": rn / sn,
        "setup_ms": setup_ms,
        "coarsest_sweeps_last_cycle": {"solve_to_1e-6": coarse_last,
                                       "timed_run": floor_sweeps},
        "tiles": [{"level": t["level"], "ty": t["ty"], "kchunk": t["kchunk"],
                   "pass_ty": t.get("pair_ty", 16), "pass_kchunk": t.get("pair_kchunk", 0)}
                  for t in tiles],
        "roofline": {"bound": "hbm", "kernel": kname,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (counters)",
                     "avg_launch_us": launch * 1e3,
                     "alg_bytes_per_launch": alg_bytes,
                     "alg_bytes_rule": f"per sweep {SWEEP_BYTES_NO_FACES:g} B per cell (read x, "
                                       f"sigma; write x) x {cells} cells + "
                                       f"{FACE_BYTES_PER_CELL:g} B of faces per cell outside "
                                       f"uniform bricks x {face_cells} cells + "
                                       f"{map_bytes:g} B of brick map; x {sweeps_per_launch} "
                                       "sweep(s) per launch",
                     "uniform_bricks": [uni_bricks, bricks],
                     "dense_faces": {
                         "rule": f"{SWEEP_BYTES_PER_CELL:g} B per cell per sweep (every face "
                                 f"loaded) x {sweeps_per_launch} x {cells} cells",
                         "alg_bytes_per_launch": dense_bytes,
                         "frac_at_map_launch": dense_bytes / (launch * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "note": "frac_at_map_launch prices the map pass at bytes it does not "
                                 "move (uniform faces); above 1 it is no roofline, the map "
                                 "rule above is",
                         "no_map_launch_us": nomap_ms * 1e3 if nomap_ms else None,
                         "no_map_frac": dense_bytes / (nomap_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                         if nomap_ms else None},
                     "one_read_min_gbs": one_read_gbs,
                     "one_read_min_frac": one_read_gbs / HBM_PEAK_GBS,
                     "traffic_gbs": traffic / (launch * 1e-3) / 1e9 if traffic else None,
                     "traffic_frac": traffic / (launch * 1e-3) / 1e9 / HBM_PEAK_GBS
                     if traffic else None,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "level0_smoothing": {
            "two_sweep_pass_us": pass_ms * 1e3 if pass_ms else None,
            "fused_sweep_us": fused_ms * 1e3,
            "us_per_sweep": (pass_ms / 2 if pass_ms else fused_ms) * 1e3,
            "fused_sweep_frac": SWEEP_BYTES_PER_CELL * cells / (fused_ms * 1e-3) / 1e9
            / HBM_PEAK_GBS,
            "fused_sweep_traffic": measured_traffic("fused")},
    }
    if not args.no_extras:
        out["other_configs"] = extra_configs()
        out["other_configs"]["solver_table"] = solver_comparison()
        out["other_configs"]["coarsening_sweep"] = coarsening_sweep()
        out["other_configs"]["moving_sphere_sequence"] = sequence_solves()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
