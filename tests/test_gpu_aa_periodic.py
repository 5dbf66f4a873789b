"""The AA neighbour step on periodic lattices without a mask, whose x-shifted
stores go through LDS: rows longer than a block (edge values stored
directly), several rows per block, rows straddling blocks and a partial last
block.  AA equals two-grid bit for bit in every storage format, with nearest
and stochastic rounding, for D3Q19 and D3Q27, and matches the FP64 oracle."""
import numpy as np
import pytest

import lbm_inputs
import oracle
from _helpers import assert_f64_parity, case, host, lattice

pytestmark = pytest.mark.gpu

SHAPES = [(300, 4, 5), (64, 8, 6), (33, 18, 14), (256, 3, 4), (16, 5, 3)]
SHAPE_IDS = ["rows300", "rows64", "33x18x14", "rows256", "16x5x3"]


# stochastic rounding applies to the 16-bit formats only
STORAGE = [("f64", "nearest"), ("f32", "nearest"), ("f32s", "nearest"), ("f16s", "nearest"),
           ("bf16s", "nearest"), ("f16s", "stochastic"), ("bf16s", "stochastic")]


@pytest.mark.parametrize("dtype,rounding", STORAGE, ids=[f"{d}-{r}" for d, r in STORAGE])
@pytest.mark.parametrize("si", range(len(SHAPES)), ids=SHAPE_IDS)
def test_aa_periodic_equals_two_grid_bitwise(si, dtype, rounding):
    nx, ny, nz = SHAPES[si]
    cfg, kw = case(nx, ny, nz, trt=True, omega=1.9, accel=(1e-5, -2e-6, 3e-6))
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=17 + si, amax=0.05)
    extra = dict(rounding=rounding, seed=3)
    a = lattice(cfg, kw, u0, dtype=dtype, pattern="two_grid", **extra)
    b = lattice(cfg, kw, u0, dtype=dtype, pattern="aa", **extra)
    for n in (1, 1, 5):
        a.step(n)
        b.step(n)
        np.testing.assert_array_equal(host(a.get_pdfs()), host(b.get_pdfs()))
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f16s"])
@pytest.mark.parametrize("si", [0, 2], ids=["rows300", "33x18x14"])
def test_aa_periodic_d3q27_equals_two_grid_bitwise(si, dtype):
    nx, ny, nz = SHAPES[si]
    cfg, kw = case(nx, ny, nz, trt=True, omega=1.8, accel=(1e-5, 0, 0), stencil=27)
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=23 + si, amax=0.05)
    a = lattice(cfg, kw, u0, dtype=dtype, pattern="two_grid")
    b = lattice(cfg, kw, u0, dtype=dtype, pattern="aa")
    for n in (1, 4):
        a.step(n)
        b.step(n)
        np.testing.assert_array_equal(host(a.get_pdfs()), host(b.get_pdfs()))
    a.close()
    b.close()


@pytest.mark.parametrize("improved,trt", [(False, False), (True, True)], ids=["S-SRT", "I-TRT"])
@pytest.mark.parametrize("si", range(len(SHAPES)), ids=SHAPE_IDS)
def test_aa_periodic_fp64_matches_oracle(si, improved, trt):
    nx, ny, nz = SHAPES[si]
    cfg, kw = case(nx, ny, nz, improved=improved, trt=trt, omega=1.7, accel=(2e-4, 1e-4, -1e-4))
    rng = np.random.default_rng(29 + si)
    u0 = rng.uniform(-0.05, 0.05, (3,) + cfg.shape)
    lat = lattice(cfg, kw, u0, pattern="aa")
    lat.step(3)     # ends after a neighbour step
    assert_f64_parity(host(lat.get_pdfs()), oracle.step(cfg, oracle.init(cfg, u0), 3),
                      f"aa periodic {SHAPE_IDS[si]}")
    lat.close()
