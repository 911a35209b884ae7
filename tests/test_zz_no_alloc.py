"""gmg_residual_noalloc (the allocation-free variant of gmg_residual) against
gmg_residual itself, through the C ABI: two calls in a row on one device,
the second on a smaller grid, each checked for the residual field and both
norms; and the size limit of its fixed scratch array."""
import numpy as np
import pytest

from paper_2607_07687_amd import gmg as G
from paper_2607_07687_amd import problems as P

from .gpu_util import dev, host, require_gpu, say, torch

pytestmark = pytest.mark.gpu


def _one(n, periodic, prec, seed, holes):
    L, s, per = P.random_problem(n, periodic, seed, contrast=1.0, holes=holes)
    code = G.GMG_F64 if prec == "f64" else G.GMG_F32
    h = G.gmg_setup(G.gmg_default_params(n, per, code), dev(L, prec))
    sd = dev(s, prec)
    x = dev(np.random.default_rng(seed + 1).uniform(-1.0, 1.0, s.shape), prec)
    r_ref = torch.empty_like(sd)
    rn_ref, sn_ref = G.gmg_residual(h, x, sd, r_ref)
    r = torch.full_like(sd, float("nan"))
    norms = torch.full((2,), float("nan"), dtype=torch.float64, device=sd.device)
    G.gmg_residual_noalloc(h, x, sd, r, norms)
    torch.cuda.synchronize()
    rn, sn = host(norms)
    say(f"noalloc {n} {prec}: rnorm {rn:.17e} vs {rn_ref:.17e}, snorm {sn:.17e} vs {sn_ref:.17e}")
    # the same kernels on the same inputs: the field bitwise, the norms to
    # the last bit or one rounding of the final square root
    assert torch.equal(r, r_ref)
    assert abs(rn - rn_ref) <= 1e-15 * rn_ref and abs(sn - sn_ref) <= 1e-15 * sn_ref
    # norms only (no r), then r only (no norms)
    norms.fill_(float("nan"))
    G.gmg_residual_noalloc(h, x, sd, None, norms)
    r.fill_(float("nan"))
    G.gmg_residual_noalloc(h, x, sd, r, None)
    torch.cuda.synchronize()
    assert np.array_equal(host(norms), np.array([rn, sn])) and torch.equal(r, r_ref)
    h.close()


def test_noalloc_residual_matches_gmg_residual_twice_second_smaller():
    require_gpu()
    _one((72, 40, 36), (False, False, False), "f32", 11, 0.05)
    _one((20, 12, 16), (True, False, True), "f64", 12, 0.1)


def test_noalloc_residual_rejects_grids_beyond_its_scratch():
    require_gpu()
    # 1 x 65538 x 128 cells: 1 * 32769 * 8 reduction blocks > 2^18
    n = (1, 65538, 128)
    L = torch.ones((3, n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    h = G.gmg_setup(G.gmg_default_params(n, (False, False, False), G.GMG_F32), L)
    x = torch.zeros((n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GMGError) as e:
        G.gmg_residual_noalloc(h, x, x, None, norms)
    assert e.value.status == G.GMG_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(norms, torch.zeros_like(norms))
    h.close()
