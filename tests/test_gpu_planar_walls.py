"""The two-grid step's planar addressing for walls and masks (lattices whose
planes hold a whole number of 256-cell blocks): FP64 parity with the oracle
for every collision, and bit-for-bit agreement with the AA step (which keeps
the general addressing) in every reduced storage format, with nearest and
stochastic rounding."""
import numpy as np
import pytest

import lbm_inputs
import oracle
from _helpers import assert_f64_parity, case, dev, host, lattice, random_blobs

pytestmark = pytest.mark.gpu

# the last shape has 76 blocks: two whole groups of 32 taken four per XCD
# and a tail of 12 in dispatch order
SHAPES = [((32, 16, 12), (1, 0, 1)), ((64, 4, 5), (0, 1, 1)), ((16, 32, 7), (1, 1, 0)),
          ((64, 16, 19), (1, 0, 1))]
COLL = [dict(trt=False), dict(trt=True), dict(mrt=(1.6, 1.1))]


@pytest.mark.parametrize("shape,per", SHAPES, ids=["32x16x12", "64x4x5", "16x32x7", "64x16x19"])
@pytest.mark.parametrize("improved", [0, 1, 2])
@pytest.mark.parametrize("ci", range(len(COLL)), ids=["srt", "trt", "mrt"])
def test_planar_walls_fp64(shape, per, improved, ci):
    nx, ny, nz = shape
    assert (nx * ny) % 256 == 0
    solid = random_blobs((nz, ny, nx), seed=nx + ny + nz)
    cfg, kw = case(nx, ny, nz, periodic=per, improved=improved, omega=1.7,
                   accel=(2e-4, -1e-4, 1e-4), solid=solid, **COLL[ci])
    rng = np.random.default_rng(3)
    u = rng.uniform(-0.05, 0.05, (3,) + cfg.shape)
    f0 = oracle.init(cfg, u)
    lat = lattice(cfg, kw, u)
    lat.step(4)
    assert_f64_parity(host(lat.get_pdfs()), oracle.step(cfg, f0, 4), f"planar walls {shape}")
    lat.close()


def test_planar_walls_kbc_fp64():
    nx, ny, nz = 32, 16, 12
    solid = random_blobs((nz, ny, nx), seed=9)
    cfg = oracle.Config(nx, ny, nz, periodic=(1, 0, 0), improved=1, kbc=True, omega=1.9,
                        accel=(1e-4, 0, 0), solid=solid)
    from paper_1803_04937_amd import Lattice
    import torch
    rng = np.random.default_rng(4)
    u = rng.uniform(-0.05, 0.05, (3,) + cfg.shape)
    lat = Lattice(nx, ny, nz, u=dev(u), solid=dev(solid, torch.uint8), periodic=(1, 0, 0),
                  equilibrium="improved", collision="kbc", omega=1.9, accel=(1e-4, 0, 0),
                  dtype="f64")
    lat.step(4)
    assert_f64_parity(host(lat.get_pdfs()), oracle.step(cfg, oracle.init(cfg, u), 4),
                      "planar walls kbc")
    lat.close()


@pytest.mark.parametrize("rounding", ["nearest", "stochastic"])
@pytest.mark.parametrize("dtype", ["f32", "f32s", "f16s", "bf16s"])
def test_planar_walls_equal_aa_bitwise(dtype, rounding):
    solid = random_blobs((10, 16, 48), seed=15)
    cfg, kw = case(48, 16, 10, periodic=(1, 0, 1), trt=True, omega=1.9, accel=(1e-5, 0, 0),
                   solid=solid)
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=16, amax=0.05)
    extra = dict(rounding=rounding, seed=11)
    a = lattice(cfg, kw, u0, dtype=dtype, pattern="two_grid", **extra)
    b = lattice(cfg, kw, u0, dtype=dtype, pattern="aa", **extra)
    for n in (1, 6):
        a.step(n)
        b.step(n)
        np.testing.assert_array_equal(host(a.get_pdfs()), host(b.get_pdfs()))
    a.close()
    b.close()


def test_walls_state_over_4gib_takes_the_general_kernel():
    """Walls on a lattice whose planes hold whole blocks but whose FP64 state
    spans more than 4 GiB (1024 x 512 x 56 cells, 4.46 GB): the 32-bit
    offsets of the planar kernel would not reach it, so the step takes the
    general kernel.  Sampled cells after one step against the oracle's
    per-cell step, including the wall rows and the last plane."""
    nx, ny, nz = 1024, 512, 56
    assert nx * ny % 256 == 0 and nx * ny * nz * 19 * 8 > 2 ** 32
    cfg, kw = case(nx, ny, nz, periodic=(1, 0, 1), trt=True, omega=1.7, accel=(1e-4, 0, 0))
    u0 = lbm_inputs.perturbation(cfg.shape, seed=41, amp=0.05)
    lat = lattice(cfg, kw, u0, dtype="f64")
    f0 = oracle.init(cfg, u0)
    del u0
    rng = np.random.default_rng(42)
    cells = rng.choice(nx * ny * nz, size=400, replace=False)
    edge = [(z * ny + y) * nx + x for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
    cells = np.unique(np.concatenate([cells, edge])).astype(np.int64)
    lat.step(1)
    got = host(lat.sample_pdfs(cells))
    lat.close()
    assert_f64_parity(got.T, oracle.step_cells(cfg, f0, cells).T, "walls over 4 GiB")
