"""Parity at full workload sizes, in the launch configurations the benchmark
times: one GPU step from a stored state against the FP64 oracle evaluated
cell by cell on a seeded sample (plus every corner and edge cell); the same
for one adjoint step, whose sampled cells' pushed values are compared at
their target slots."""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from _helpers import assert_adjoint_parity, case, host, lattice, push_targets, reduced_bound

pytestmark = pytest.mark.gpu


def _sample(shape, seed, k=4096):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    cells = set(rng.choice(nx * ny * nz, size=k, replace=False).tolist())
    for z in (0, nz - 1):
        for y in (0, ny - 1):
            for x in (0, 1, nx - 2, nx - 1):
                cells.add((z * ny + y) * nx + x)
    return np.array(sorted(cells), dtype=np.int64)


def _sampled_step(cfg, kw, u0, dtype, pattern, warm, seed):
    lat = lattice(cfg, kw, u0, dtype=dtype, pattern=pattern)
    lat.step(warm)
    f_in = host(lat.get_pdfs())
    lat.step(1)
    cells = _sample(cfg.shape, seed)
    got = lat.get_pdfs().view(19, -1)[:, torch.as_tensor(cells, device="cuda")]
    got = host(got)
    want = oracle.step_cells(cfg, f_in, cells).T
    del f_in
    return got, want, lat.scale


@pytest.mark.parametrize("pattern,warm", [("two_grid", 5), ("aa", 5), ("aa", 6)])
def test_bench_workload_256_f32(pattern, warm):
    """256^3 periodic D3Q19-I TRT, omega = 1.8, FP32 (the timed workload)."""
    n = 256
    cfg, kw = case(n, n, n, improved=True, trt=True, omega=1.8)
    u0 = lbm_inputs.shear_waves((n, n, n), seed=0)
    got, want, s = _sampled_step(cfg, kw, u0, "f32", pattern, warm, seed=1)
    assert np.all(np.abs(got - want) <= reduced_bound(want, "f32", s))


@pytest.mark.parametrize("dtype", ["f16s", "bf16s", "f32s", "f32"])
def test_512_reduced_precision(dtype):
    """512^3 periodic D3Q19-I TRT, omega = 1.98, shifted 16-bit and FP32 and
    plain FP32 storage."""
    n = 512
    cfg, kw = case(n, n, n, improved=True, trt=True, omega=1.98)
    u0 = lbm_inputs.shear_waves((n, n, n), seed=2, amax=0.04)
    got, want, s = _sampled_step(cfg, kw, u0, dtype, "two_grid", 3, seed=3)
    assert np.all(np.abs(got - want) <= reduced_bound(want, dtype, s))


def test_256_fp64_standard_srt():
    """256^3 FP64 D3Q19-S SRT, omega = 1.0: the oracle-matched precision."""
    n = 256
    cfg, kw = case(n, n, n, improved=False, trt=False, omega=1.0)
    u0 = lbm_inputs.shear_waves((n, n, n), seed=4)
    got, want, _ = _sampled_step(cfg, kw, u0, "f64", "two_grid", 4, seed=5)
    W = oracle.velocity_set()[1][:, None]
    assert np.all(np.abs(got - want) <= 1e-12 * np.maximum(np.abs(want), W))


def test_tube_192x192x768_f16_walls():
    """The constricted-tube geometry at full size (solid mask, TRT, body
    force), FP16 storage: sampled one-step parity including cells next to the
    wall."""
    nx, ny, nz = 768, 192, 192
    solid = lbm_inputs.tube_mask(nx, ny, nz)
    cfg, kw = case(nx, ny, nz, periodic=(1, 1, 1), improved=True, trt=True, omega=1.95,
                   accel=(2e-6, 0, 0), solid=solid)
    rng = np.random.default_rng(6)
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = 0.02 * (solid == 0)
    u0 += rng.uniform(-1e-3, 1e-3, size=u0.shape) * (solid == 0)
    got, want, s = _sampled_step(cfg, kw, u0, "f16s", "two_grid", 4, seed=7)
    assert np.all(np.abs(got - want) <= reduced_bound(want, "f16s", s))


def _sampled_adjoint(cfg, kw, u0, dtype, warm, seed):
    lat = lattice(cfg, kw, u0, dtype=dtype)
    lat.step(warm)
    f_in = host(lat.get_pdfs())            # the linearisation point, as stored
    lam = np.random.default_rng(seed).standard_normal(f_in.shape, dtype=np.float32)
    ln, lp = lat.new_adjoint(), lat.new_adjoint()
    lat.state_view(ln).copy_(torch.as_tensor(lam, device="cuda"))
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    lat.adjoint_step(lat.state, ln, lp, grad)
    cells = _sample(cfg.shape, seed + 1)
    if cfg.solid is not None:
        cells = cells[~np.asarray(cfg.solid).reshape(-1)[cells].astype(bool)]
    arr, tgt = push_targets(cfg, cells)
    flat = lat.state_view(lp).reshape(cfg.q, -1)
    got = host(flat[torch.as_tensor(arr, device="cuda"), torch.as_tensor(tgt, device="cuda")])
    g = host(grad)
    lat.close()
    want = oracle.adjoint_cells(cfg, f_in, lam.astype(np.float64), cells)
    return got.astype(np.float64), want, g


def test_bench_adjoint_256_f32():
    """The timed adjoint: 256^3 periodic D3Q19-I TRT, omega = 1.8, FP32 state
    and lambda, at the state after 5 steps."""
    n = 256
    cfg, kw = case(n, n, n, improved=True, trt=True, omega=1.8)
    u0 = lbm_inputs.shear_waves((n, n, n), seed=0)
    got, want, g = _sampled_adjoint(cfg, kw, u0, "f32", 5, seed=20)
    assert_adjoint_parity(got, want, "f32", "bench 256^3")
    assert np.isfinite(g).all()


def test_tube_adjoint_f16_state():
    """The tube's adjoint at full size: solid mask, walls of the mask next to
    fluid cells, FP16 state and FP32 lambda, body force."""
    nx, ny, nz = 768, 192, 192
    solid = lbm_inputs.tube_mask(nx, ny, nz)
    cfg, kw = case(nx, ny, nz, periodic=(1, 1, 1), improved=True, trt=True, omega=1.95,
                   accel=(2e-6, 0, 0), solid=solid)
    u0 = np.zeros((3, nz, ny, nx))
    u0[0] = 0.02 * (solid == 0)
    got, want, g = _sampled_adjoint(cfg, kw, u0, "f16s", 3, seed=21)
    assert_adjoint_parity(got, want, "f32", "tube")
    assert np.isfinite(g).all()


def test_periodic_adjoint_fields_over_4gib():
    """The planar adjoint of a periodic lattice keeps 64-bit plane bases: at
    1024 x 512 x 112 cells the FP32 state and lambda fields span 4.46 GB
    each, past 32-bit byte offsets.  Sampled cells against the oracle's
    per-cell adjoint."""
    nx, ny, nz = 1024, 512, 112
    assert nx * ny * nz * 19 * 4 > 2 ** 32
    cfg, kw = case(nx, ny, nz, improved=True, trt=True, omega=1.8, accel=(1e-5, 0, 0))
    u0 = lbm_inputs.perturbation((nz, ny, nx), seed=22, amp=0.03)
    got, want, g = _sampled_adjoint(cfg, kw, u0, "f32", 1, seed=23)
    assert_adjoint_parity(got, want, "f32", "periodic over 4 GiB")
    assert np.isfinite(g).all()
