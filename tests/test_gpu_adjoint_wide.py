"""GPU parity of the adjoint of the widened forward path (D3Q27, the
third-order D3Q19-I equilibrium, MRT) against the FP64 oracle, whose
transpose is pinned by dot-product tests and finite differences."""
import numpy as np
import pytest
import torch

import oracle
from _helpers import assert_adjoint_parity, case, dev, host, lattice, random_blobs, weights_for

pytestmark = pytest.mark.gpu

WIDE = {
    "Q27-SRT": dict(stencil=27, improved=0),
    "Q27-TRT": dict(stencil=27, improved=0, trt=True),
    "I3-SRT": dict(improved=2),
    "I3-TRT": dict(improved=2, trt=True),
    "MRT-S": dict(improved=0, mrt=(1.7, 0.9)),
    "MRT-I": dict(improved=1, mrt=(1.7, 0.9)),
    "MRT-I3": dict(improved=2, mrt=(0.8, 1.6)),
}


def _noisy(cfg, seed, amp=0.02, uamp=0.05):
    w = weights_for(cfg.q)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * w[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = w[:, None]
    return f


def _load(lat, buf, arr):
    lat.state_view(buf).copy_(dev(arr, buf.dtype))


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("name", list(WIDE))
def test_wide_adjoint_step_matches_oracle(name, dtype):
    solid = random_blobs((13, 17, 37), seed=110)
    cfg, kw = case(37, 17, 13, periodic=(1, 0, 1), omega=1.7, accel=(3e-4, -1e-4, 2e-4),
                   solid=solid, **WIDE[name])
    f = _noisy(cfg, 111)
    lam = np.random.default_rng(112).standard_normal(f.shape)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype)
    lat.set_pdfs(dev(f))
    f_stored = host(lat.get_pdfs())       # the state as stored (rounded below FP64)
    ln, lp = lat.new_adjoint(), lat.new_adjoint()
    assert lat.state_view(ln).shape[0] == cfg.q
    _load(lat, ln, lam)
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    lat.adjoint_step(lat.state, ln, lp, grad)
    got = host(lat.state_view(lp)).astype(np.float64)
    want, gw = oracle.adjoint_step(cfg, f_stored, lam)
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert_adjoint_parity(got, want, dtype, name)
    np.testing.assert_allclose(host(grad), gw, rtol=tol * 10, atol=tol * np.abs(gw).max())
    lat.close()


@pytest.mark.parametrize("kind", [0, 1])
def test_d3q27_objective_and_seed_match_oracle(kind):
    solid = random_blobs((11, 12, 13), seed=113)
    cfg, kw = case(13, 12, 11, periodic=(1, 0, 0), trt=True, omega=1.4, accel=(1e-4, 0, 0),
                   solid=solid, stencil=27, improved=0)
    f = _noisy(cfg, 114)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape))
    lat.set_pdfs(dev(f))
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    lam = lat.new_adjoint()
    lat.objective(kind, lat.state, out, lam)
    J, lam_o, da = oracle.objective(cfg, f, kind)
    o = host(out)
    assert abs(o[0] - J) <= 1e-12 * max(abs(J), 1e-3)
    np.testing.assert_allclose(o[1:], da, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(host(lat.state_view(lam)), lam_o, rtol=0, atol=1e-12)
    lat.close()


@pytest.mark.parametrize("name", ["Q27-SRT", "I3-SRT"])
def test_wide_init_vjp_matches_oracle(name):
    solid = random_blobs((9, 10, 11), seed=115)
    cfg, kw = case(11, 10, 9, solid=solid, **WIDE[name])
    rng = np.random.default_rng(116)
    u0 = rng.uniform(-0.08, 0.08, size=(3,) + cfg.shape)
    lam = rng.standard_normal((cfg.q,) + cfg.shape)
    lat = lattice(cfg, kw, u0)
    l0 = lat.new_adjoint()
    _load(lat, l0, lam)
    gu = torch.empty((3,) + cfg.shape, dtype=torch.float64, device="cuda")
    lat.init_vjp(dev(u0), l0, gu)
    np.testing.assert_allclose(host(gu), oracle.init_vjp(cfg, u0, lam), rtol=0, atol=1e-13)
    lat.close()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("name", ["Q27-TRT", "I3-TRT", "MRT-I"])
def test_wide_rollout_gradient_matches_oracle_fp64(name, kind):
    """Checkpointed autograd rollout (FP64, T = 11, segments of 4) against the
    oracle's full-trajectory gradient."""
    from paper_1803_04937_amd import RolloutConfig, rollout_objective
    solid = random_blobs((10, 12, 16), seed=117)
    m = WIDE[name]
    cfg, _ = case(16, 12, 10, periodic=(1, 0, 0), omega=1.5, accel=(2e-4, 1e-5, 0), solid=solid,
                  **m)
    rng = np.random.default_rng(118)
    u0 = rng.uniform(-0.04, 0.04, size=(3,) + cfg.shape)
    T = 11
    extra = {}
    if "mrt" in m:
        extra = dict(collision="mrt", mrt_omega3=m["mrt"][0], mrt_omega4=m["mrt"][1])
    else:
        extra = dict(collision="trt" if m.get("trt") else "srt")
    rc = RolloutConfig(16, 12, 10, steps=T, periodic=(1, 0, 0),
                       equilibrium={0: "standard", 1: "improved", 2: "improved3"}[m["improved"]],
                       dtype="f64", objective=kind, checkpoint_every=4,
                       solid=dev(solid, torch.uint8), stencil=m.get("stencil", 19), **extra)
    u = dev(u0).requires_grad_(True)
    a = torch.tensor([2e-4, 1e-5, 0.0], dtype=torch.float64, requires_grad=True)
    w = torch.tensor(1.5, dtype=torch.float64, requires_grad=True)
    J = rollout_objective(u, a, w, rc)
    J.backward()
    Jo, guo, gwo, gao = oracle.gradient(cfg, u0, T, kind)
    assert abs(J.item() - Jo) <= 1e-12 * abs(Jo)
    np.testing.assert_allclose(host(u.grad), guo, rtol=0, atol=1e-11 * np.abs(guo).max())
    np.testing.assert_allclose(a.grad.cpu().numpy(), gao, rtol=1e-10, atol=1e-14)
    assert abs(w.grad.item() - gwo) <= 1e-10 * abs(gwo)
