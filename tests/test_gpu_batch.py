"""GPU tests of the batched refinement solve (many uneven problems, one graph
replay per refinement step): every problem's result is bitwise identical to a separate
gmg_solve_ir of the same problem (same kernels, same reduction order), and
agrees with the oracle's refinement driver; replays of the kept graph give
the same results."""
import numpy as np
import pytest

from oracle import gmg_oracle as O
from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P
from tests.gpu_util import dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu


def _params(L, per, storage):
    n = (L.shape[3], L.shape[2], L.shape[1])
    return G.gmg_default_params(n, per, G.GMG_F64, cycle_dtype=G.GMG_F32,
                                l_storage=G.GMG_BF16 if storage == "bf16" else G.GMG_F32)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batch_equals_single_solves(storage):
    require_gpu()
    specs = P.batch_specs(count=6, seed=3)
    probs = [P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
             for sp in specs]
    # a periodic and an odd-sized wall problem in the mix
    probs.append(P.tgv_periodic(16, seed=1))
    probs.append(P.random_problem((40, 20, 12), (False, False, False), 3, contrast=1.0,
                                  holes=0.05))
    Ls = [dev(L, "f64") for L, _, _ in probs]
    ss = [dev(s, "f64") for _, s, _ in probs]
    params = [_params(L, per, storage) for L, _, per in probs]
    b = G.gmg_batch_setup(params, Ls)
    xs = [torch.zeros_like(s) for s in ss]
    say(f"batch of {len(probs)} ({storage})")
    infos = G.gmg_batch_solve_ir(b, xs, ss, rtol=1e-10, max_outer=30, max_inner=8)
    for p, ((L, s, per), prm) in enumerate(zip(probs, params)):
        h = G.gmg_setup(prm, Ls[p])
        x1 = torch.zeros_like(ss[p])
        r1 = G.gmg_solve_ir(h, x1, ss[p], rtol=1e-10, max_outer=30, max_inner=8)
        say(f"  p{p} n={prm.n[0]}x{prm.n[1]}x{prm.n[2]} outer {infos[p]['outer']} "
            f"final {infos[p]['history'][-1]:.2e}")
        assert infos[p]["status"] == "GMG_OK"
        assert infos[p]["history"] == r1["history"]
        assert infos[p]["inner_cycles"] == r1["inner_cycles"]
        assert torch.equal(xs[p], x1)
        h.close()
    # replay of the kept graph from fresh zero guesses
    for x in xs:
        x.zero_()
    infos2 = G.gmg_batch_solve_ir(b, xs, ss, rtol=1e-10, max_outer=30, max_inner=8)
    assert [i["history"] for i in infos2] == [i["history"] for i in infos]
    b.close()


@pytest.mark.parametrize("nu", [(3, 1), (1, 2)])
def test_batch_other_sweep_counts(nu):
    # odd sweep counts mix two-sweep passes with single sweeps, and leave the
    # coarse levels' iterate in either of their two buffers: the batch must
    # take the prolongation from the one the smoothing ended on
    require_gpu()
    specs = P.batch_specs(count=4, seed=5)
    probs = [P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
             for sp in specs]
    Ls = [dev(L, "f64") for L, _, _ in probs]
    ss = [dev(s, "f64") for _, s, _ in probs]
    params = []
    for L, _, per in probs:
        prm = _params(L, per, "f32")
        prm.nu_pre, prm.nu_post, prm.nu_coarse = nu[0], nu[1], nu[0] + nu[1]
        params.append(prm)
    b = G.gmg_batch_setup(params, Ls)
    xs = [torch.zeros_like(s) for s in ss]
    infos = G.gmg_batch_solve_ir(b, xs, ss, rtol=1e-10, max_outer=30, max_inner=8)
    for p, prm in enumerate(params):
        h = G.gmg_setup(prm, Ls[p])
        x1 = torch.zeros_like(ss[p])
        r1 = G.gmg_solve_ir(h, x1, ss[p], rtol=1e-10, max_outer=30, max_inner=8)
        say(f"  nu {nu} p{p} outer {infos[p]['outer']} final {infos[p]['history'][-1]:.2e}")
        assert infos[p]["history"] == r1["history"]
        assert torch.equal(xs[p], x1)
        h.close()
    b.close()


def test_batch_matches_oracle_subset():
    require_gpu()
    specs = P.batch_specs(count=3, seed=3)
    probs = [P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
             for sp in specs]
    Ls = [dev(L, "f64") for L, _, _ in probs]
    ss = [dev(s, "f64") for _, s, _ in probs]
    b = G.gmg_batch_setup([_params(L, per, "f32") for L, _, per in probs], Ls)
    xs = [torch.zeros_like(s) for s in ss]
    infos = G.gmg_batch_solve_ir(b, xs, ss, rtol=1e-10, max_outer=30, max_inner=8)
    for p, (L, s, per) in enumerate(probs):
        ro = O.solve_ir(L, per, np.zeros_like(s), s, rtol=1e-10, max_outer=30, max_inner=8,
                        inner_rtol=1e-4, inner_storage="f32")
        assert ro["status"] == "ok" and infos[p]["status"] == "GMG_OK"
        assert abs(infos[p]["outer"] - ro["outer"]) <= 1
        # the returned x meets the tolerance under the oracle's exact FP64
        # residual (ir_target 0.5 stops the last step near half of it)
        L64 = O.normalize_faces(L, per)
        act = O.active_set(L64, per)
        assert O.norm2(O.residual(host(xs[p]), s, L64, per), act) <= 1e-10 * O.norm2(s, act)
        # and the two solutions differ by what 2e-10 of the residual allows:
        # A (x - x_o) = r_o - r, whose norm is at most 2e-10 ||sigma||
        d = host(xs[p]) - ro["x"]
        assert O.norm2(O.residual(d, np.zeros_like(s), L64, per), act) <= 2e-10 * O.norm2(s, act)
    b.close()


def test_batch_argument_errors():
    require_gpu()
    L, s, per = P.tgv_periodic(8, seed=0)
    prm = G.gmg_default_params((8, 8, 8), per, G.GMG_F64)  # F64 cycles: not allowed
    with pytest.raises(G.GMGError):
        G.gmg_batch_setup([prm], [dev(L, "f64")])
    # a single-level problem (6^3 walls cannot coarsen) smooths in the
    # descent and the ascent: nu_coarse must be nu_pre + nu_post
    L1, _, per1 = P.random_problem((6, 6, 6), (False, False, False), 2)
    prm = _params(L1, per1, "f32")
    prm.nu_coarse = 3
    with pytest.raises(G.GMGError):
        G.gmg_batch_setup([prm], [dev(L1, "f64")])
    # with two levels the tail smooths the coarsest level: any nu_coarse
    prm = _params(L, per, "f32")
    prm.nu_coarse = 3
    G.gmg_batch_setup([prm], [dev(L, "f64")]).close()
    # problems must share the coarsest-level rule
    p1, p2 = _params(L, per, "f32"), _params(L, per, "f32")
    p2.coarse_rtol = 0.2
    with pytest.raises(G.GMGError):
        G.gmg_batch_setup([p1, p2], [dev(L, "f64"), dev(L, "f64")])


def test_batch_autotune_keeps_results_bitwise():
    require_gpu()
    specs = P.batch_specs(count=4, seed=5)
    probs = [P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
             for sp in specs]
    Ls = [dev(L, "f64") for L, _, _ in probs]
    ss = [dev(s, "f64") for _, s, _ in probs]
    b = G.gmg_batch_setup([_params(L, per, "f32") for L, _, per in probs], Ls)
    xs = [torch.zeros_like(s) for s in ss]
    i0 = G.gmg_batch_solve_ir(b, xs, ss, max_outer=30)
    G.gmg_batch_autotune(b, reps=2)
    ys = [torch.zeros_like(s) for s in ss]
    i1 = G.gmg_batch_solve_ir(b, ys, ss, max_outer=30)
    assert [i["history"] for i in i0] == [i["history"] for i in i1]
    assert all(torch.equal(a, c) for a, c in zip(xs, ys))
    b.close()


@pytest.mark.parametrize("max_outer", [0, 2, 30])
def test_batch_step_replays_match_eager_launches(max_outer):
    # the step graph is replayed until every problem has finished or max_outer
    # times: the results, step counts and statuses equal those of launching
    # every kernel eagerly (graphs off), also when max_outer cuts the solve
    require_gpu()
    specs = P.batch_specs(count=4, seed=7)
    probs = [P.sphere_box(sp["n"], sp["centre"], sp["radius"], "uniform", sp["seed"])
             for sp in specs]
    Ls = [dev(L, "f64") for L, _, _ in probs]
    ss = [dev(s, "f64") for _, s, _ in probs]
    out = []
    for graphs in (1, 0):
        params = []
        for L, _, per in probs:
            prm = _params(L, per, "f32")
            prm.graphs = graphs
            params.append(prm)
        b = G.gmg_batch_setup(params, Ls)
        xs = [torch.zeros_like(s) for s in ss]
        say(f"  max_outer {max_outer} graphs {graphs}")
        infos = G.gmg_batch_solve_ir(b, xs, ss, rtol=1e-10, max_outer=max_outer, max_inner=8)
        out.append((infos, xs))
        b.close()
    (ig, xg), (ie, xe) = out
    for a, c in zip(ig, ie):
        assert a["status"] == c["status"] and a["outer"] == c["outer"]
        assert a["history"] == c["history"]
        assert a["outer"] <= max_outer
    assert all(torch.equal(a, c) for a, c in zip(xg, xe))
    for i in ig:
        assert i["status"] == "GMG_OK" or i["outer"] == max_outer
    if max_outer == 0:
        assert all(i["status"] != "GMG_OK" for i in ig)
    if max_outer == 30:
        assert all(i["status"] == "GMG_OK" for i in ig)
