"""Learned warm start for the GMG solve: data from the solver itself,
training with the project's kernels, and the timed comparison with plain GMG.

* Data: warm-start problems (walls, a random sphere, sigma from random
  Taylor-Green modes) generated on the host; each is solved on the GPU by
  the FP64 iterative refinement of libgmg.so to 1e-10; the target is p / s
  with its mean over the active cells removed, s = RMS of sigma there.
* Training: the U-Net of unet_net.py (BF16 activations and weights, FP32
  master weights and accumulation), masked MSE over the active cells, Adam
  with a cosine learning-rate decay.
* Use: x0 = s * U(sigma / s, L); then the adaptive GMG solve from x0.  The
  final residual judges the prediction: if the warm-started solve misses the
  tolerance in its cycle budget, plain GMG from zero runs instead.

Run on an MI355X:  python -m paper_2607_07687_amd.warmstart --help
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import gmg as G
from . import problems as P
from . import unet as UN
from . import unet_net as NET


def _gen(args):
    n, seed = args
    L, s, per = P.tgv_modes_sphere(n, seed)
    return L.astype(np.float64), s.astype(np.float64), per


def generate(n, seeds, workers=8, chunk=32):
    """Host-side generation of the warm-start problems (process pool),
    yielded in order chunk by chunk so that at most a few chunks of FP64
    problems are held on the host at a time."""
    seeds = list(seeds)
    if workers <= 1:
        for s in seeds:
            yield _gen((n, s))
        return
    with ProcessPoolExecutor(workers) as ex:
        for c0 in range(0, len(seeds), chunk):
            part = [(n, s) for s in seeds[c0:c0 + chunk]]
            yield from ex.map(_gen, part, chunksize=max(1, len(part) // workers))


class Sample:
    """Device tensors of one problem: FP32 sigma and faces (network input and
    FP32 solve), target p / s, active mask, scale s."""

    def __init__(self, L, s, per, p=None, keep64=False):
        import torch
        t = P.touched_cells(L, per)
        self.n = (L.shape[3], L.shape[2], L.shape[1])
        self.per = per
        self.scale = float(np.sqrt(np.mean(s[t] ** 2))) if t.any() else 1.0
        self.sigma = torch.from_numpy(s.astype(np.float32)).cuda()
        self.L = torch.from_numpy(L.astype(np.float32)).cuda()
        self.mask = torch.from_numpy(t.astype(np.uint8)).cuda()
        # FP64 copies for the refinement solves of the evaluation
        self.sigma64 = torch.from_numpy(s).cuda() if keep64 else None
        self.L64 = torch.from_numpy(L).cuda() if keep64 else None
        self.target = None
        if p is not None:
            q = p - p[t].mean()
            self.target = torch.from_numpy((q / self.scale).astype(np.float32)).cuda()


def solve_fp64(L, s, per):
    """FP64 iterative-refinement solve to 1e-10 on the GPU."""
    import torch
    n = (L.shape[3], L.shape[2], L.shape[1])
    prm = G.gmg_default_params(n, per, G.GMG_F64, cycle_dtype=G.GMG_F32)
    h = G.gmg_setup(prm, torch.from_numpy(L).cuda())
    sd = torch.from_numpy(s).cuda()
    x = torch.zeros_like(sd)
    info = G.gmg_solve_ir(h, x, sd, rtol=1e-10, max_outer=20)
    h.close()
    if info["status"] != "GMG_OK":
        raise RuntimeError(f"training target solve failed: {info}")
    return x.cpu().numpy()


def make_samples(n, seeds, workers=8, with_target=True, keep64=False):
    out = []
    t0 = time.perf_counter()
    for L, s, per in generate(n, seeds, workers):
        p = solve_fp64(L, s, per) if with_target else None
        out.append(Sample(L, s, per, p, keep64))
        if len(out) % 100 == 0:
            print(f"{len(out)} samples at {n} ({time.perf_counter() - t0:.1f}s)", flush=True)
    return out


def pack(samples, x_buf):
    """BF16 network input of a batch of samples into x_buf [B][d][h][w][8]."""
    import torch
    B = len(samples)
    nx, ny, nz = samples[0].n
    sig = torch.stack([sm.sigma for sm in samples]) if B > 1 else samples[0].sigma[None]
    L = torch.stack([sm.L for sm in samples]) if B > 1 else samples[0].L[None]
    UN.unet_pack_input(UN.shape(B, nz, ny, nx), sig.contiguous(), L.contiguous(),
                       [sm.scale for sm in samples], x_buf)


def train(net, samples, steps, batch=2, lr=1e-3, seed=0, log_every=50):
    import torch
    rng = np.random.default_rng(seed)
    nx, ny, nz = samples[0].n
    x = torch.zeros((batch, nz, ny, nx, NET.IN_CH), dtype=torch.int16, device="cuda")
    losses = []
    t0 = time.perf_counter()
    for it in range(steps):
        idx = rng.choice(len(samples), batch, replace=False)
        bs = [samples[i] for i in idx]
        pack(bs, x)
        tgt = torch.stack([b.target for b in bs]).contiguous()
        msk = torch.stack([b.mask for b in bs]).contiguous()
        net.forward(x, batch, nz, ny, nx)
        want = (it % log_every == 0) or it == steps - 1
        loss = net.backward(x, tgt, msk, want_loss=want)
        net.adam(lr * 0.5 * (1.0 + math.cos(math.pi * it / steps)))
        if want:
            losses.append((it, loss))
            print(f"step {it} loss {loss:.5f} ({time.perf_counter() - t0:.1f}s)", flush=True)
    return losses


def predict(net, sm, x_buf, out):
    """x0 = s * U(sigma / s, L) into out (FP32 [d][h][w])."""
    nx, ny, nz = sm.n
    pack([sm], x_buf)
    y = net.forward(x_buf, 1, nz, ny, nx)
    UN.unet_scale(y, sm.scale, out)
    return out


# a prediction whose residual exceeds this many times ||sigma|| is not used
PRED_LIMIT = 10.0


class HalfRes:
    """Half-resolution inference: the network runs on the problem restricted
    to the hierarchy's level 1 (sigma summed over 2x2x2 blocks, the level's
    faces), and its prediction is prolongated back.  For a smooth pressure
    the level-1 problem A_1 p_1 = R sigma has p_1 close to p at the coarse
    cells (the level-1 faces are twice the mean of the fine faces they
    cover, and R sums eight right-hand sides).  The network, trained on
    faces in [0, 1], is fed the level-1 faces halved and R sigma / (8 s);
    its output q then solves the problem with the halved faces, so
    p_1 = 4 s q.  Every step runs in the libraries: the restriction and
    level-1 faces from libgmg.so, scaling and packing in libunet.so, and
    the piecewise-constant prolongation on the active cells from libgmg.so.
    Needs a grid that coarsens by 2 in every direction to level 1."""

    def __init__(self, h, sm):
        import torch
        n1, c = G.gmg_level_shape(h, 1)
        if tuple(c) != (2, 2, 2):
            raise ValueError("half-resolution inference needs 2x2x2 coarsening to level 1")
        self.h, self.sm, self.n1 = h, sm, n1
        nx, ny, nz = n1
        dev = sm.sigma.device
        self.zero = torch.zeros_like(sm.sigma)
        self.x32 = torch.zeros_like(sm.sigma)
        self.s1 = torch.zeros((nz, ny, nx), dtype=torch.float32, device=dev)
        self.L1 = torch.zeros((3, nz, ny, nx), dtype=torch.float32, device=dev)
        self.Lin = torch.zeros_like(self.L1)
        self.x1 = torch.zeros_like(self.s1)
        self.xb = torch.zeros((1, nz, ny, nx, NET.IN_CH), dtype=torch.int16, device=dev)
        G.gmg_level_faces(h, 1, self.L1)
        UN.unet_scale(self.L1, 0.5, self.Lin)

    def predict(self, net, x64):
        """x64 (FP64, level 0) <- P (4 s U(R sigma / (8 s), L_1 / 2))."""
        nx, ny, nz = self.n1
        s = self.sm.scale
        G.gmg_restrict_residual(self.h, 0, self.zero, self.sm.sigma, self.s1)
        UN.unet_pack_input(UN.shape(1, nz, ny, nx), self.s1, self.Lin, [8.0 * s], self.xb)
        y = net.forward(self.xb, 1, nz, ny, nx)
        UN.unet_scale(y, 4.0 * s, self.x1)
        self.x32.zero_()
        G.gmg_prolong_correct(self.h, 0, self.x1, self.x32)
        UN.unet_scale_f64(self.x32, 1.0, x64)


def warm_solve(h, net, sm, x, x_buf, rtol=1e-6, max_outer=30, half=None):
    """Solve with the learned warm start and plain GMG as the fallback.

    x0 = s * U(sigma / s, L) is written into x (FP64); its residual judges
    it.  A useful prediction can have a residual above ||sigma||: its error
    has high-frequency content that the operator amplifies and the first
    sweeps remove at once.  So x is zeroed before the solve only when the
    prediction is clearly broken, ||sigma - A x0|| > PRED_LIMIT ||sigma|| or
    not finite.  The refinement solve then runs from x; if it misses rtol
    within max_outer steps from a prediction, x is zeroed and the solve runs
    again from zero.  Returns (info of the solve whose x is returned,
    fallback reason or None)."""
    nx, ny, nz = sm.n
    if half is not None:
        half.predict(net, x)
    else:
        pack([sm], x_buf)
        y = net.forward(x_buf, 1, nz, ny, nx)
        UN.unet_scale_f64(y, sm.scale, x)
    rn, sn = G.gmg_residual(h, x, sm.sigma64)
    reason = None
    if not (rn <= PRED_LIMIT * sn):  # also catches a non-finite prediction
        x.zero_()
        reason = "prediction residual far above the zero guess's"
    info = G.gmg_solve_ir(h, x, sm.sigma64, rtol, max_outer)
    if info["status"] != "GMG_OK" and reason is None:
        x.zero_()
        reason = "warm-started solve missed the tolerance"
        info = G.gmg_solve_ir(h, x, sm.sigma64, rtol, max_outer)
    return info, reason


def compare(net, samples, rtol=1e-6, reps=10, max_outer=30, half=False):
    """Wall time of plain GMG (x0 = 0) against U-Net inference + GMG from its
    prediction, on the same GPU; medians over reps.  Both solves are the FP64
    iterative refinement around FP32 V-cycles (each outer step one captured
    graph): the smooth low-mode right-hand sides of these problems put the
    FP32 residual floor above 1e-6.  half: the network runs on the problem
    restricted to level 1 (HalfRes)."""
    import torch
    res = []
    for sm in samples:
        nx, ny, nz = sm.n
        prm = G.gmg_default_params(sm.n, sm.per, G.GMG_F64, cycle_dtype=G.GMG_F32)
        h = G.gmg_setup(prm, sm.L64)
        x = torch.zeros_like(sm.sigma64)
        xb = None if half else torch.zeros((1, nz, ny, nx, NET.IN_CH), dtype=torch.int16,
                                           device="cuda")
        hr = HalfRes(h, sm) if half else None

        def warm():
            if hr is not None:
                hr.predict(net, x)
                return
            pack([sm], xb)
            y = net.forward(xb, 1, nz, ny, nx)
            UN.unet_scale_f64(y, sm.scale, x)

        G.gmg_solve_ir(h, x, sm.sigma64, rtol, max_outer)  # warm-up (graph capture)
        warm_solve(h, net, sm, x, xb, rtol, max_outer, hr)
        tp, tw, ti = [], [], []
        reasons = set()
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ip = G.gmg_solve_ir(h, x, sm.sigma64, rtol, max_outer)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            warm()
            torch.cuda.synchronize()
            ti.append(time.perf_counter() - t0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iw, why = warm_solve(h, net, sm, x, xb, rtol, max_outer, hr)
            torch.cuda.synchronize()
            tw.append(time.perf_counter() - t0)
            if why:
                reasons.add(why)
        # relative residual of the prediction alone (first history entry)
        rel0 = iw["history"][0] if iw["history"] and not reasons else float("nan")
        res.append(dict(plain_ms=1e3 * float(np.median(tp)), warm_ms=1e3 * float(np.median(tw)),
                        infer_ms=1e3 * float(np.median(ti)),
                        plain_outer=ip["outer"], plain_inner=ip["inner_total"],
                        warm_outer=iw["outer"], warm_inner=iw["inner_total"],
                        plain_status=ip["status"], warm_status=iw["status"], warm_rel_r0=rel0,
                        fallback=sorted(reasons)))
        h.close()
        r = res[-1]
        print(f"eval {len(res)} {sm.n[0]}^3{' (half-res inference)' if half else ''}: plain {r['plain_ms']:.2f} ms ({r['plain_inner']} "
              f"V-cycles, {r['plain_status']}), warm {r['warm_ms']:.2f} ms ({r['warm_inner']} "
              f"V-cycles, {r['warm_status']}; inference {r['infer_ms']:.2f} ms), "
              f"prediction r/s {rel0:.3e}", flush=True)
    return res


def conv_throughput(n=128, reps=5):
    """Measured TFLOP/s of the convolution kernels at the U-Net's per-level
    shapes for one n^3 sample (forward, data and weight gradient)."""
    import torch
    out = []
    chans = [(8, 16, n), (16, 16, n), (32, 16, n), (16, 32, n // 2), (32, 32, n // 2),
             (32, 64, n // 4), (64, 64, n // 4), (64, 128, n // 8), (128, 128, n // 8),
             (128, 64, n // 4)]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for cin, cout, m in chans:
        s = UN.shape(1, m, m, m)
        x = torch.zeros((m, m, m, cin), dtype=torch.int16, device="cuda")
        y = torch.zeros((m, m, m, cout), dtype=torch.int16, device="cuda")
        w = torch.zeros(cout * 27 * cin, dtype=torch.int16, device="cuda")
        b = torch.zeros(cout, dtype=torch.float32, device="cuda")
        flops = 2.0 * 27 * cin * cout * m ** 3
        res = {"cin": cin, "cout": cout, "n": m}
        ws = torch.empty(UN.unet_wgrad_workspace(s, cin, cout, 27) // 4 + 1, dtype=torch.float32,
                         device="cuda")
        dw = torch.zeros(cout * 27 * cin, dtype=torch.float32, device="cuda")
        wf = torch.empty_like(w)
        ops = {"fwd": lambda: UN.unet_conv_fwd(s, UN.act(x, cin, 0, cin), w, b, 27,
                                               UN.act(y, cout, 0, cout), None, 1),
               "wgrad": lambda: UN.unet_conv_wgrad(s, UN.act(x, cin, 0, cin),
                                                   UN.act(y, cout, 0, cout), 27, dw, b, ws)}
        if cin % 16 == 0:
            ops["dgrad"] = lambda: UN.unet_conv_dgrad(s, UN.act(y, cout, 0, cout), w, 27,
                                                      UN.act(x, cin, 0, cin), wf)
        for name, fn in ops.items():
            fn()
            ev0.record()
            for _ in range(reps):
                fn()
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / reps
            res[name + "_tflops"] = flops / (ms * 1e-3) / 1e12
            res[name + "_ms"] = ms
        out.append(res)
        print(res, flush=True)
    return out


def train_throughput(n=128, batch=2, steps=20, warmup=3):
    """Measured time of one training step (forward, backward, Adam) at batch
    x n^3 on synthetic data: random BF16 inputs, random targets, every cell
    active.  HIP-event timing of `steps` steps after `warmup`."""
    import torch
    net = NET.UNet()
    net.init_he(0)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = (torch.randn((batch, n, n, n, NET.IN_CH), device="cuda", generator=g)
         .to(torch.bfloat16).view(torch.int16).contiguous())
    tgt = torch.randn((batch, n, n, n), device="cuda", generator=g).contiguous()
    msk = torch.ones((batch, n, n, n), dtype=torch.uint8, device="cuda")

    def step():
        net.forward(x, batch, n, n, n)
        net.backward(x, tgt, msk, want_loss=False)
        net.adam(1e-4)

    for _ in range(warmup):
        step()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    res = {"n": n, "batch": batch, "steps": steps, "ms_per_step": ev0.elapsed_time(ev1) / steps}
    print(res, flush=True)
    return res


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128, help="training grid")
    ap.add_argument("--eval-n", default="128,256", help="evaluation grids, comma-separated")
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--eval-samples", type=int, default=32)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default="warmstart_out")
    ap.add_argument("--conv-throughput", action="store_true")
    ap.add_argument("--train-throughput", action="store_true",
                    help="time training steps on synthetic data at --n and --batch")
    ap.add_argument("--params", default="", help="trained weights (.npy): evaluate only")
    ap.add_argument("--half-n", default="",
                    help="evaluation grids (comma-separated) also run with half-resolution "
                         "inference")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    G.load()
    UN.load()
    assert torch.cuda.is_available()
    if args.conv_throughput:
        res = conv_throughput(args.n)
        with open(os.path.join(args.out, "conv_throughput.json"), "w") as f:
            json.dump(res, f, indent=1)
        return
    if args.train_throughput:
        res = train_throughput(args.n, args.batch)
        with open(os.path.join(args.out, "train_throughput.json"), "w") as f:
            json.dump(res, f, indent=1)
        return
    net = NET.UNet()
    summary = dict(train_n=args.n, samples=args.samples, steps=args.steps, batch=args.batch)
    if args.params:  # evaluate trained weights, no training
        net.set_flat(np.load(args.params, allow_pickle=False))
        summary["params"] = args.params
    else:
        t0 = time.perf_counter()
        train_set = make_samples((args.n,) * 3, range(10000, 10000 + args.samples), args.workers)
        t_data = time.perf_counter() - t0
        print(f"{len(train_set)} training pairs in {t_data:.1f}s", flush=True)
        net.init_he(0)
        t0 = time.perf_counter()
        losses = train(net, train_set, args.steps, args.batch, args.lr)
        torch.cuda.synchronize()
        summary.update(data_s=t_data, train_s=time.perf_counter() - t0, losses=losses)
        np.save(os.path.join(args.out, "unet_params.npy"), net.get_flat())
        del train_set
    summary["eval"] = {}
    half_n = [int(v) for v in args.half_n.split(",") if v]
    for en in [int(v) for v in args.eval_n.split(",")]:
        evals = make_samples((en,) * 3, range(20000, 20000 + args.eval_samples), args.workers,
                             with_target=False, keep64=True)
        for half in ([False, True] if en in half_n else [False]):
            res = compare(net, evals, half=half)
            med = lambda key: float(np.median([r[key] for r in res]))
            key = f"{en}_half" if half else str(en)
            summary["eval"][key] = dict(
                per_sample=res, plain_ms_median=med("plain_ms"), warm_ms_median=med("warm_ms"),
                infer_ms_median=med("infer_ms"), plain_vcycles_median=med("plain_inner"),
                warm_vcycles_median=med("warm_inner"),
                prediction_rel_residual_median=med("warm_rel_r0"),
                fallbacks=sum(1 for r in res if r["fallback"]))
            print(json.dumps({"eval": key, **{k: v for k, v in summary["eval"][key].items()
                                              if k != "per_sample"}}), flush=True)
        del evals
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(summary, f, indent=1)


if __name__ == "__main__":
    main()
