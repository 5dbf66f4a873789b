"""adjoint_solid = skip: the adjoint step leaves lambda at solid cells unwritten.

Fluid slots and the parameter gradient must equal those of the default
(copy), bit for bit; solid slots must keep what the buffer held; and a
checkpointed gradient rollout through a masked lattice, which never reads
lambda at solid cells, must give the same gradients either way."""
import numpy as np
import pytest
import torch

import oracle
from _helpers import case, dev, host, lattice, random_blobs, weights_for

pytestmark = pytest.mark.gpu


def _noisy(cfg, seed, amp=0.02, uamp=0.05):
    w = weights_for(cfg.q)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * w[:, None, None, None] * rng.standard_normal(f.shape)
    f[:, cfg.solid.astype(bool)] = w[:, None]
    return f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("stencil", [19, 27])
def test_skip_matches_copy_on_fluid_and_leaves_solid(dtype, stencil):
    solid = random_blobs((9, 14, 37), seed=150, frac=0.2)
    cfg, kw = case(37, 14, 9, periodic=(1, 0, 1), trt=True, omega=1.6, accel=(1e-4, 0, -2e-4),
                   solid=solid, stencil=stencil, improved=0 if stencil == 27 else 1)
    f = _noisy(cfg, 151)
    lam = np.random.default_rng(152).standard_normal(f.shape)
    out = {}
    for mode in ("copy", "skip"):
        lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype, adjoint_solid=mode)
        lat.set_pdfs(dev(f))
        ln, lp = lat.new_adjoint(), lat.new_adjoint()
        lat.state_view(ln).copy_(dev(lam, ln.dtype))
        lat.state_view(lp).fill_(7.0)
        grad = torch.zeros(4, dtype=torch.float64, device="cuda")
        lat.adjoint_step(lat.state, ln, lp, grad)
        out[mode] = (host(lat.state_view(lp)).astype(np.float64), host(grad))
        lat.close()
    s = solid.astype(bool)
    got_copy, g_copy = out["copy"]
    got_skip, g_skip = out["skip"]
    np.testing.assert_array_equal(got_skip[:, ~s], got_copy[:, ~s])
    np.testing.assert_array_equal(g_skip, g_copy)
    assert (got_skip[:, s] == 7.0).all()
    ldt = np.float64 if dtype == "f64" else np.float32
    np.testing.assert_array_equal(got_copy[:, s], lam[:, s].astype(ldt).astype(np.float64))


def test_rollout_gradient_same_with_skip():
    from paper_1803_04937_amd import RolloutConfig, rollout_objective
    nx, ny, nz, T = 24, 12, 10, 30
    solid = random_blobs((nz, ny, nx), seed=153, frac=0.15)
    sd = dev(solid, torch.uint8)
    u0 = np.random.default_rng(154).uniform(-0.03, 0.03, size=(3, nz, ny, nx))
    grads = {}
    for mode in ("copy", "skip"):
        rc = RolloutConfig(nx, ny, nz, steps=T, periodic=(1, 0, 1), collision="trt", dtype="f32",
                           objective=1, solid=sd, adjoint_solid=mode)
        u = dev(u0).requires_grad_(True)
        a = torch.tensor([2e-5, 0.0, 0.0], dtype=torch.float64, requires_grad=True)
        w = torch.tensor(1.7, dtype=torch.float64, requires_grad=True)
        J = rollout_objective(u, a, w, rc)
        J.backward()
        grads[mode] = (J.item(), host(u.grad), a.grad.numpy().copy(), w.grad.item())
    (Jc, uc, ac, wc), (Js, us, as_, ws) = grads["copy"], grads["skip"]
    assert Jc == Js and wc == ws
    np.testing.assert_array_equal(uc, us)
    np.testing.assert_array_equal(ac, as_)
