"""GPU parity of the adjoint step for rows that do not match a 256-cell block.

The adjoint stages its x-shifted pushes in LDS and stores them at the
target cell's own x.  Whether a push is staged or stored directly depends on
how the rows of the lattice fall into 256-cell blocks: rows longer than a
block (a push crossing a block boundary inside a row, and the periodic wrap
from x = 0 to x = nx - 1 landing in another block), rows of exactly one
block, and rows that divide a block.  Each case is checked element by element
against the FP64 oracle, with and without walls along x and solid cells."""
import numpy as np
import pytest
import torch

import oracle
from _helpers import assert_adjoint_parity, case, dev, host, lattice, random_blobs, weights_for

pytestmark = pytest.mark.gpu

SHAPES = [(300, 3, 4), (256, 3, 2), (257, 2, 3), (64, 5, 2), (100, 4, 3)]


def _noisy(cfg, seed, amp=0.02, uamp=0.05):
    w = weights_for(cfg.q)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * w[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = w[:, None]
    return f


def _step(cfg, kw, dtype, seed):
    f = _noisy(cfg, seed)
    lam = np.random.default_rng(seed + 1).standard_normal(f.shape)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype)
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


@pytest.mark.parametrize("stencil", [19, 27])
@pytest.mark.parametrize("walls", ["periodic", "x_walls", "solid"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_adjoint_rows_match_oracle_f64(shape, walls, stencil):
    nx, ny, nz = shape
    periodic = (0, 1, 1) if walls == "x_walls" else (1, 1, 1)
    solid = random_blobs((nz, ny, nx), seed=120 + nx) if walls == "solid" else None
    cfg, kw = case(nx, ny, nz, periodic=periodic, trt=True, omega=1.7,
                   accel=(2e-4, -1e-4, 1e-4), solid=solid, stencil=stencil,
                   improved=0 if stencil == 27 else 1)
    got, want, g, gw = _step(cfg, kw, "f64", 130 + nx)
    assert_adjoint_parity(got, want, "f64", f"rows {shape} {walls} Q{stencil}")
    np.testing.assert_allclose(g, gw, rtol=1e-11, atol=1e-12 * np.abs(gw).max())


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_adjoint_rows_fast_path_f32(shape):
    """Fully periodic, no mask: the kernel without wall and mask tests."""
    nx, ny, nz = shape
    cfg, kw = case(nx, ny, nz, periodic=(1, 1, 1), trt=True, omega=1.8, improved=1)
    got, want, g, gw = _step(cfg, kw, "f32", 140 + nx)
    assert_adjoint_parity(got, want, "f32", f"rows {shape} fast path")
    np.testing.assert_allclose(g, gw, rtol=2e-5, atol=2e-6 * np.abs(gw).max())
