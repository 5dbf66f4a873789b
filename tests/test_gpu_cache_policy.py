"""The cache policy of the stream-collide kernels (non-temporal hints or
cached accesses) changes no arithmetic: both give the same stored state bit
for bit.  The small parity cases run the cached kernels (LBM_CACHE_AUTO keeps
lattices under 192 MiB cache-resident) and the full-size ones the streaming
kernels, so this equality ties the two sets of parity tests together."""
import numpy as np
import pytest
import torch

import lbm_inputs
from _helpers import case, host, lattice, random_blobs

pytestmark = pytest.mark.gpu

CASES = {
    "I-TRT-f32": dict(dtype="f32", trt=True),
    "S-SRT-f64": dict(dtype="f64"),
    "I-TRT-f16s-stochastic": dict(dtype="f16s", trt=True, rounding="stochastic"),
    "I3-MRT-bf16s": dict(dtype="bf16s", improved=2, mrt=(1.6, 1.2)),
    "Q27-TRT-f32s": dict(dtype="f32s", trt=True, stencil=27, improved=0),
}


@pytest.mark.parametrize("pattern", ["two_grid", "aa"])
@pytest.mark.parametrize("name", list(CASES))
def test_cache_policies_agree_bit_for_bit(name, pattern):
    kw_case = dict(CASES[name])
    dtype = kw_case.pop("dtype")
    extra = {}
    if "rounding" in kw_case:
        extra = dict(rounding=kw_case.pop("rounding"), seed=9)
    solid = random_blobs((14, 18, 40), seed=120)
    cfg, kw = case(40, 18, 14, periodic=(1, 0, 1), omega=1.8, accel=(1e-5, 2e-6, 0),
                   solid=solid, **kw_case)
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=121, amax=0.06)
    out = {}
    for policy in ("stream", "keep", "auto"):
        lat = lattice(cfg, kw, u0, dtype=dtype, pattern=pattern, cache_policy=policy, **extra)
        lat.step(7)
        out[policy] = lat.state_view(lat.state).clone()
        lat.close()
    torch.cuda.synchronize()
    for policy in ("keep", "auto"):
        assert torch.equal(out[policy].view(torch.uint8), out["stream"].view(torch.uint8)), policy
    assert np.isfinite(host(out["stream"].float())).all()


@pytest.mark.parametrize("name", ["I-TRT-f32", "I-TRT-f16s-stochastic", "Q27-TRT-f32s"])
def test_adjoint_cache_policies_agree_bit_for_bit(name):
    """The adjoint step under both policies: same lam_prev, same gradient."""
    kw_case = dict(CASES[name])
    dtype = kw_case.pop("dtype")
    kw_case.pop("rounding", None)
    solid = random_blobs((14, 18, 40), seed=122)
    cfg, kw = case(40, 18, 14, periodic=(1, 0, 1), omega=1.8, accel=(1e-5, 2e-6, 0),
                   solid=solid, **kw_case)
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=123, amax=0.06)
    out = {}
    for policy in ("stream", "keep"):
        lat = lattice(cfg, kw, u0, dtype=dtype, cache_policy=policy)
        lat.step(3)
        ln, lp = lat.new_adjoint(), lat.new_adjoint()
        o = torch.zeros(4, dtype=torch.float64, device="cuda")
        lat.objective(0, lat.state, o, ln)
        grad = torch.zeros(4, dtype=torch.float64, device="cuda")
        for _ in range(3):
            lat.adjoint_step(lat.state, ln, lp, grad)
            ln, lp = lp, ln
        out[policy] = (lat.state_view(ln).clone(), grad.clone())
        lat.close()
    torch.cuda.synchronize()
    assert torch.equal(out["keep"][0], out["stream"][0])
    assert torch.equal(out["keep"][1], out["stream"][1])
