"""Full-size parity on the 256^3 FP32 wall-bounded sphere workload, in the
launch configuration bench.py times (default tiles, graphs on): the first
V-cycle from x = 0 at 2048 seeded sample cells and in norm, and the adaptive
solve to 1e-6 (cycle count, residual history, omega decisions), against the
oracle's results stored in tests/golden/sphere256_oracle.json (written by
tests/golden/make_sphere256.py, which calls only the oracle)."""
import json
import os

import numpy as np
import pytest

from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P
from tests.gpu_util import require_gpu, say, torch

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "sphere256_oracle.json")


@pytest.fixture(scope="module")
def sphere256():
    require_gpu()
    with open(GOLD) as f:
        gold = json.load(f)
    L, s, per = P.sphere_256(seed=1)
    Ld = torch.from_numpy(L.astype(np.float32)).cuda()
    sd = torch.from_numpy(s.astype(np.float32)).cuda()
    h = G.gmg_setup(G.gmg_default_params((256, 256, 256), per, G.GMG_F32), Ld)
    yield gold, h, sd
    h.close()


def test_first_vcycle_sampled(sphere256):
    gold, h, sd = sphere256
    x = torch.zeros_like(sd)
    rn = G.gmg_vcycle(h, x, sd, want_norm=True)
    xs = x.flatten()[torch.tensor(gold["sample_index"], device="cuda")].cpu().numpy()
    want = np.array(gold["x1_sample"])
    e = np.linalg.norm(xs - want) / np.linalg.norm(want)
    einf = np.abs(xs - want).max() / np.abs(want).max()
    xn = float(torch.linalg.vector_norm(x.double()).item())
    say(f"256^3 first cycle: sampled rel {e:.2e}, |x| {xn:.6e} vs {gold['x1_norm']:.6e}, "
        f"|r| {rn:.6e} vs {gold['r1_norm']:.6e}")
    assert e <= 1e-5 and einf <= 1e-5, (e, einf)
    assert abs(xn - gold["x1_norm"]) <= 1e-5 * gold["x1_norm"]
    assert abs(rn - gold["r1_norm"]) <= 1e-5 * gold["r1_norm"]


def test_solve_to_1e6(sphere256):
    gold, h, sd = sphere256
    if "solve_history" not in gold:
        pytest.skip("golden file holds no solve history")
    x = torch.zeros_like(sd)
    res = G.gmg_solve(h, x, sd, 1e-6, 40)
    say(f"256^3 solve: {res['cycles']} cycles, history {['%.3e' % v for v in res['history']]}")
    assert res["status"] == "GMG_OK"
    assert res["cycles"] == gold["solve_cycles"]
    assert res["accepted"] == [1 if a else 0 for a in gold["solve_accepted"]]
    for hg, ho in zip(res["history"], gold["solve_history"]):
        assert abs(hg - ho) <= 1e-5 * ho + 1e-7
    rn, sn = G.gmg_residual(h, x, sd)
    assert rn <= 1e-6 * sn and abs(sn - gold["snorm"]) <= 1e-6 * gold["snorm"]
