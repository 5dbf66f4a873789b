"""The adjoint step's planar addressing (lattices whose planes hold a whole
number of 256-cell blocks, fields under 4 GiB): FP64 and FP32 parity with
the oracle's adjoint step for periodic lattices, walls, masks (lambda at
solid cells copied or left unwritten), every collision and both stencils."""
import numpy as np
import pytest
import torch

import oracle
from _helpers import assert_adjoint_parity, case, dev, host, lattice, random_blobs, weights_for

pytestmark = pytest.mark.gpu

# (nx, ny, nz), periodic, with a mask
# 64x16x19: 76 blocks, two whole groups of 32 taken four per XCD and a
# tail of 12 in dispatch order
SHAPES = [((32, 16, 12), (1, 0, 1), True), ((64, 4, 5), (0, 1, 1), False),
          ((16, 32, 7), (1, 1, 1), False), ((256, 2, 3), (1, 1, 1), True),
          ((512, 1, 3), (0, 1, 1), True), ((64, 16, 19), (1, 0, 1), True)]
SHAPE_IDS = ["32x16x12_mask", "64x4x5_walls", "16x32x7_periodic", "256x2x3_mask",
             "512x1x3_mask", "64x16x19_mask"]
MODELS = [dict(improved=0), dict(improved=1, trt=True), dict(improved=2, trt=True),
          dict(improved=1, mrt=(1.6, 1.1))]
MODEL_IDS = ["S-SRT", "I-TRT", "I3-TRT", "I-MRT"]


def _noisy(cfg, seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    w = weights_for(cfg.q)
    f = f + 0.02 * w[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = w[:, None]
    return f


def _adjoint(cfg, kw, dtype, seed, adjoint_solid="copy"):
    f = _noisy(cfg, seed)
    lam = np.random.default_rng(seed + 1).standard_normal(f.shape)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype, adjoint_solid=adjoint_solid)
    lat.set_pdfs(dev(f))
    f_stored = host(lat.get_pdfs())
    ln, lp = lat.new_adjoint(), lat.new_adjoint()
    lat.state_view(ln).copy_(dev(lam, ln.dtype))
    grad = torch.zeros(4, dtype=torch.float64, device="cuda")
    lat.adjoint_step(lat.state, ln, lp, grad)
    got = host(lat.state_view(lp)).astype(np.float64)
    g = host(grad)
    lat.close()
    want, gw = oracle.adjoint_step(cfg, f_stored, lam)
    return got, want, g, gw


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mi", range(len(MODELS)), ids=MODEL_IDS)
@pytest.mark.parametrize("si", range(len(SHAPES)), ids=SHAPE_IDS)
def test_planar_adjoint_matches_oracle(si, mi, dtype):
    (nx, ny, nz), per, mask = SHAPES[si]
    assert (nx * ny) % 256 == 0
    solid = random_blobs((nz, ny, nx), seed=31 + si) if mask else None
    cfg, kw = case(nx, ny, nz, periodic=per, omega=1.7, accel=(3e-4, -1e-4, 2e-4), solid=solid,
                   **MODELS[mi])
    got, want, g, gw = _adjoint(cfg, kw, dtype, 40 + si)
    assert_adjoint_parity(got, want, dtype, f"planar adjoint {SHAPE_IDS[si]}")
    tol = 1e-12 if dtype == "f64" else 2e-6
    np.testing.assert_allclose(g, gw, rtol=tol * 10, atol=tol * np.abs(gw).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_planar_adjoint_skip_leaves_solid_cells(dtype):
    nx, ny, nz = 32, 16, 12
    solid = random_blobs((nz, ny, nx), seed=51, frac=0.2)
    cfg, kw = case(nx, ny, nz, periodic=(1, 1, 0), improved=1, trt=True, omega=1.8,
                   accel=(1e-4, 0, 0), solid=solid)
    got, want, g, gw = _adjoint(cfg, kw, dtype, 52, adjoint_solid="skip")
    fl = solid == 0
    assert_adjoint_parity(got[:, fl], want[:, fl], dtype, "planar adjoint skip")
    tol = 1e-12 if dtype == "f64" else 2e-6
    np.testing.assert_allclose(g, gw, rtol=tol * 10, atol=tol * np.abs(gw).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mask", [False, True], ids=["walls", "mask"])
def test_planar_adjoint_d3q27(mask, dtype):
    nx, ny, nz = 32, 8, 6
    solid = random_blobs((nz, ny, nx), seed=61) if mask else None
    cfg, kw = case(nx, ny, nz, periodic=(1, 0, 1), improved=1, trt=True, omega=1.7,
                   accel=(2e-4, 1e-4, -1e-4), solid=solid, stencil=27)
    got, want, g, gw = _adjoint(cfg, kw, dtype, 62)
    assert_adjoint_parity(got, want, dtype, "planar adjoint d3q27")
    tol = 1e-12 if dtype == "f64" else 2e-6
    np.testing.assert_allclose(g, gw, rtol=tol * 10, atol=tol * np.abs(gw).max())
