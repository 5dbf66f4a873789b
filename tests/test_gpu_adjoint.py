"""GPU parity of the adjoint path (lbm_adjoint_step, lbm_objective,
lbm_init_vjp and the checkpointed autograd rollout) against the FP64 oracle
and finite differences."""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from _helpers import W, assert_adjoint_parity, case, dev, host, lattice, random_blobs

pytestmark = pytest.mark.gpu

MODELS = [(False, False), (True, False), (False, True), (True, True)]
MODEL_IDS = ["S-SRT", "I-SRT", "S-TRT", "I-TRT"]


def _noisy(cfg, seed, amp=0.02, uamp=0.05):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * W[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = W[:, None]
    return f


def _load(lat, buf, arr):
    """Write a (19, nz, ny, nx) array into the cells of a buffer."""
    lat.state_view(buf).copy_(dev(arr, buf.dtype))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("improved,trt", MODELS, ids=MODEL_IDS)
def test_adjoint_step_matches_oracle(improved, trt, dtype):
    solid = random_blobs((17, 19, 41), seed=21)
    cfg, kw = case(41, 19, 17, periodic=(1, 0, 1), improved=improved, trt=trt, omega=1.7,
                   accel=(3e-4, -1e-4, 2e-4), solid=solid)
    f = _noisy(cfg, 22)
    rng = np.random.default_rng(23)
    lam = rng.standard_normal(f.shape)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype)
    lat.set_pdfs(dev(f))
    f_stored = host(lat.get_pdfs())       # the state as stored (FP32-rounded for f32)
    ln, lp = lat.new_adjoint(), lat.new_adjoint()
    _load(lat, ln, lam)
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    lat.adjoint_step(lat.state, ln, lp, grad)
    got = host(lat.state_view(lp)).astype(np.float64)
    want, gw = oracle.adjoint_step(cfg, f_stored, lam)
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert_adjoint_parity(got, want, dtype, "adjoint step")
    g = host(grad)
    np.testing.assert_allclose(g, gw, rtol=tol * 10, atol=tol * np.abs(gw).max())


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_objective_and_seed_match_oracle(kind, dtype):
    solid = random_blobs((11, 12, 13), seed=24)
    cfg, kw = case(13, 12, 11, periodic=(1, 0, 0), trt=True, omega=1.4, accel=(1e-4, 0, 0),
                   solid=solid)
    f = _noisy(cfg, 25)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype)
    lat.set_pdfs(dev(f))
    f_stored = host(lat.get_pdfs())
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    lam = lat.new_adjoint()
    lat.objective(kind, lat.state, out, lam)
    J, lam_o, da = oracle.objective(cfg, f_stored, kind)
    tol = 1e-12 if dtype == "f64" else 1e-6
    o = host(out)
    assert abs(o[0] - J) <= tol * max(abs(J), 1e-3)
    np.testing.assert_allclose(o[1:], da, rtol=tol, atol=1e-15)
    np.testing.assert_allclose(host(lat.state_view(lam)), lam_o, rtol=0, atol=tol)


@pytest.mark.parametrize("improved", [False, True], ids=["standard", "improved"])
def test_init_vjp_matches_oracle(improved):
    solid = random_blobs((9, 10, 11), seed=26)
    cfg, kw = case(11, 10, 9, improved=improved, solid=solid)
    rng = np.random.default_rng(27)
    u0 = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    lam = rng.standard_normal((19,) + cfg.shape)
    lat = lattice(cfg, kw, u0)
    l0 = lat.new_adjoint()
    _load(lat, l0, lam)
    gu = torch.empty((3,) + cfg.shape, dtype=torch.float64, device="cuda")
    lat.init_vjp(dev(u0), l0, gu)
    want = oracle.init_vjp(cfg, u0, lam)
    np.testing.assert_allclose(host(gu), want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("improved,trt", [(True, False), (False, True)], ids=["I-SRT", "S-TRT"])
def test_rollout_gradient_matches_oracle_fp64(improved, trt, kind):
    """Checkpointed autograd rollout (FP64, T = 13 steps, segments of 4) against
    the oracle's full-trajectory gradient."""
    from paper_1803_04937_amd import RolloutConfig, rollout_objective
    solid = random_blobs((10, 12, 16), seed=28)
    cfg, _ = case(16, 12, 10, periodic=(1, 0, 0), improved=improved, trt=trt, omega=1.5,
                  accel=(2e-4, 1e-5, 0), solid=solid)
    rng = np.random.default_rng(29)
    u0 = rng.uniform(-0.04, 0.04, size=(3,) + cfg.shape)
    T = 13
    rc = RolloutConfig(16, 12, 10, steps=T, periodic=(1, 0, 0),
                       equilibrium="improved" if improved else "standard",
                       collision="trt" if trt else "srt", dtype="f64", objective=kind,
                       checkpoint_every=4, solid=dev(solid, torch.uint8))
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


def test_rollout_gradient_fp32_against_finite_differences():
    """Duct (walls on y and z, periodic x), SRT, D3Q19-I, FP32 forward and
    adjoint, kinetic energy after T = 60 steps: the gradient with respect to
    a_x, omega and u_init along a random direction agrees with central
    differences of FP64 runs (relative step 1e-4) to the FP32 level."""
    from paper_1803_04937_amd import RolloutConfig, rollout_objective
    nx, ny, nz, T = 48, 24, 24, 60
    nu = (1 / 1.9 - 0.5) / 3
    u0 = lbm_inputs.duct_poiseuille(nx, ny, nz, 1e-5, nu) + lbm_inputs.perturbation(
        (nz, ny, nx), seed=30, amp=1e-3)
    rc = RolloutConfig(nx, ny, nz, steps=T, periodic=(1, 0, 0), dtype="f32", objective=0,
                       checkpoint_every=8)
    u = dev(u0).requires_grad_(True)
    a = torch.tensor([1e-5, 0.0, 0.0], dtype=torch.float64, requires_grad=True)
    w = torch.tensor(1.9, dtype=torch.float64, requires_grad=True)
    rollout_objective(u, a, w, rc).backward()
    rc64 = RolloutConfig(nx, ny, nz, steps=T, periodic=(1, 0, 0), dtype="f64", objective=0,
                         checkpoint_every=8)

    def J(uu, ax, om):
        with torch.no_grad():
            return rollout_objective(dev(uu), torch.tensor([ax, 0.0, 0.0], dtype=torch.float64),
                                     torch.tensor(om, dtype=torch.float64), rc64).item()

    h = 1e-4
    fd_a = (J(u0, 1e-5 * (1 + h), 1.9) - J(u0, 1e-5 * (1 - h), 1.9)) / (2e-5 * h)
    fd_w = (J(u0, 1e-5, 1.9 * (1 + h)) - J(u0, 1e-5, 1.9 * (1 - h))) / (2 * 1.9 * h)
    v = np.random.default_rng(31).standard_normal(u0.shape)
    hv = h * np.abs(u0).max() / np.abs(v).max()
    fd_u = (J(u0 + hv * v, 1e-5, 1.9) - J(u0 - hv * v, 1e-5, 1.9)) / (2 * hv)
    assert abs(a.grad[0].item() / fd_a - 1) < 2e-3, (a.grad[0].item(), fd_a)
    assert abs(w.grad.item() / fd_w - 1) < 2e-3, (w.grad.item(), fd_w)
    gu = (host(u.grad) * v).sum()
    assert abs(gu / fd_u - 1) < 2e-3, (gu, fd_u)
