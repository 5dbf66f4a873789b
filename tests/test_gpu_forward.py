"""GPU parity of the forward stream-collide path against the FP64 oracle.

Every GPU call goes through the C ABI (liblbm.so via capi / Lattice).  The
oracle runs the same seeded inputs on the CPU.  Tolerances are in
tests/_helpers.py.
"""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from _helpers import (W, assert_f64_parity, case, dev, host, lattice, random_blobs,
                      reduced_bound)

pytestmark = pytest.mark.gpu

MODELS = [(False, False), (True, False), (False, True), (True, True)]
MODEL_IDS = ["S-SRT", "I-SRT", "S-TRT", "I-TRT"]


def _noisy(cfg, seed, amp=0.02, uamp=0.05):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    rho = 1.0 + 0.01 * rng.standard_normal(cfg.shape)
    f = oracle.init(cfg, u, rho=rho)
    f = f + amp * W[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = W[:, None]
    return f


@pytest.mark.parametrize("improved", [False, True], ids=["standard", "improved"])
def test_taylor_green_32_fp64_every_10_steps(improved):
    """32^3 periodic Taylor-Green vortex, u0 = 0.05, tau = 0.8, SRT, FP64:
    PDFs and rho/u match the oracle after every 10 of 100 steps."""
    u0 = lbm_inputs.taylor_green(32, 0.05)
    cfg, kw = case(32, 32, 32, improved=improved, omega=1 / 0.8)
    lat = lattice(cfg, kw, u0)
    f = oracle.init(cfg, u0)
    assert_f64_parity(host(lat.get_pdfs()), f, "init")
    for k in range(10):
        lat.step(10)
        f = oracle.step(cfg, f, 10)
        assert_f64_parity(host(lat.get_pdfs()), f, f"step {10 * (k + 1)}")
        rho, u = lat.moments()
        rho_o, u_o = oracle.moments(cfg, f)
        np.testing.assert_allclose(host(rho), rho_o, rtol=1e-12, atol=0)
        np.testing.assert_allclose(host(u), u_o, rtol=0, atol=1e-13)


@pytest.mark.parametrize("pattern", ["two_grid", "aa"])
@pytest.mark.parametrize("improved,trt", MODELS, ids=MODEL_IDS)
def test_ragged_walls_obstacles_force_fp64(improved, trt, pattern):
    """37 x 29 x 23 (several blocks, ragged tail), periodic in x, walls in y
    and z, random solid blobs, body force; 11 and 12 steps (both AA
    parities)."""
    solid = random_blobs((23, 29, 37), seed=5)
    cfg, kw = case(37, 29, 23, periodic=(1, 0, 0), improved=improved, trt=trt, omega=1.6,
                   accel=(2e-4, -5e-5, 1e-4), solid=solid)
    rng = np.random.default_rng(6)
    u0 = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    lat = lattice(cfg, kw, u0, pattern=pattern)
    f = oracle.init(cfg, u0)
    lat.step(11)
    f = oracle.step(cfg, f, 11)
    assert_f64_parity(host(lat.get_pdfs()), f, "11 steps")
    lat.step(1)
    f = oracle.step(cfg, f, 1)
    assert_f64_parity(host(lat.get_pdfs()), f, "12 steps")


@pytest.mark.parametrize("shape,periodic", [
    ((1, 1, 1), (1, 1, 1)),
    ((5, 1, 1), (1, 1, 1)),
    ((1, 7, 3), (1, 0, 1)),
    ((300, 2, 3), (0, 1, 1)),
    ((3, 4, 5), (0, 0, 0)),
    ((64, 4, 1), (1, 1, 1)),
], ids=lambda v: str(v))
def test_degenerate_shapes_fp64(shape, periodic):
    """Single cells, one-cell-thick slabs, a grid smaller than one block and
    one that is a single row of several blocks, all-wall boxes."""
    nx, ny, nz = shape
    cfg, kw = case(nx, ny, nz, periodic=periodic, improved=True, trt=True, omega=1.3,
                   accel=(1e-4, 2e-4, -1e-4))
    f0 = _noisy(cfg, 7)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape))
    lat.set_pdfs(dev(f0))
    for pat_steps in (1, 2, 5):
        lat.step(pat_steps)
        f0 = oracle.step(cfg, f0, pat_steps)
        assert_f64_parity(host(lat.get_pdfs()), f0, f"{shape}")


@pytest.mark.parametrize("pattern", ["two_grid", "aa"])
def test_more_planes_than_planar_launch_fp64(pattern):
    """A periodic lattice without a mask normally runs the kernels launched
    one z-plane per grid row; with more planes than that grid dimension
    allows (65535) it takes the general kernels, whose neighbour links are
    then formed from the (periodic) walls in registers."""
    cfg, kw = case(2, 2, 65537, improved=True, trt=True, omega=1.3, accel=(1e-4, 0.0, 2e-4))
    f0 = _noisy(cfg, 8)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), pattern=pattern)
    lat.set_pdfs(dev(f0))
    lat.step(2)
    f0 = oracle.step(cfg, f0, 2)
    assert_f64_parity(host(lat.get_pdfs()), f0, f"nz = 65537, {pattern}")
    lat.close()


def test_all_solid_domain_is_inert():
    solid = np.ones((4, 5, 6), np.uint8)
    cfg, kw = case(6, 5, 4, solid=solid, accel=(1e-3, 0, 0))
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape))
    lat.step(3)
    f = host(lat.get_pdfs())
    np.testing.assert_array_equal(f, np.broadcast_to(W[:, None, None, None], f.shape))
    rho, u = lat.moments()
    assert not host(rho).any() and not host(u).any()
    assert lat.totals() == [0.0, 0.0, 0.0, 0.0]


@pytest.mark.parametrize("improved", [False, True], ids=["standard", "improved"])
def test_compressible_fp64(improved):
    cfg, kw = case(19, 11, 13, periodic=(1, 1, 0), improved=improved, trt=False, omega=1.1,
                   accel=(1e-4, 0, 0), compressible=True)
    rng = np.random.default_rng(8)
    u0 = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    rho0 = 1.0 + 0.05 * rng.standard_normal(cfg.shape)
    lat = lattice(cfg, kw, u0, rho=rho0)
    f = oracle.init(cfg, u0, rho=rho0)
    lat.step(7)
    f = oracle.step(cfg, f, 7)
    assert_f64_parity(host(lat.get_pdfs()), f, "compressible")
    rho, u = lat.moments()
    rho_o, u_o = oracle.moments(cfg, f)
    np.testing.assert_allclose(host(rho), rho_o, rtol=1e-12)
    np.testing.assert_allclose(host(u), u_o, rtol=0, atol=1e-13)


@pytest.mark.parametrize("pattern", ["two_grid", "aa"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s", "bf16s"])
def test_set_get_round_trip(dtype, pattern):
    """get(set(f)) is exact for FP64 and within half a storage ulp otherwise,
    in both AA layouts."""
    solid = random_blobs((9, 10, 11), seed=9)
    cfg, kw = case(11, 10, 9, periodic=(1, 0, 1), solid=solid)
    f = _noisy(cfg, 10)
    lat = lattice(cfg, kw, np.zeros((3,) + cfg.shape), dtype=dtype, pattern=pattern,
                  scale=2.0 ** 12 if dtype in ("f16s", "bf16s") else 0.0)
    for t in range(2):
        lat.set_pdfs(dev(f))
        got = host(lat.get_pdfs())
        if dtype == "f64":
            np.testing.assert_array_equal(got, f)
        else:
            bound = reduced_bound(f, dtype, lat.scale)
            assert np.all(np.abs(got - f) <= bound)
        lat.step(1)  # switch AA layout for the second round


def test_moments_and_totals_fp64():
    solid = random_blobs((12, 13, 14), seed=11)
    cfg, kw = case(14, 13, 12, periodic=(0, 1, 1), trt=True, omega=1.7, accel=(0, 1e-4, 0),
                   solid=solid)
    rng = np.random.default_rng(12)
    u0 = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    lat = lattice(cfg, kw, u0)
    lat.step(4)
    f = oracle.step(cfg, oracle.init(cfg, u0), 4)
    rho, u = lat.moments()
    rho_o, u_o = oracle.moments(cfg, f)
    np.testing.assert_allclose(host(rho), rho_o, rtol=1e-12)
    np.testing.assert_allclose(host(u), u_o, rtol=0, atol=1e-13)
    tot = lat.totals()
    fl = solid == 0
    j = np.einsum("qd,q...->d...", oracle.velocity_set()[0], f)
    want = [rho_o[fl].sum(), j[0][fl].sum(), j[1][fl].sum(), j[2][fl].sum()]
    np.testing.assert_allclose(tot, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dtype", ["f32", "f32s", "f16s", "bf16s"])
def test_aa_equals_two_grid_bitwise(dtype):
    """AA and two-grid apply the same arithmetic to the same values: the
    canonical states agree bit for bit."""
    solid = random_blobs((14, 18, 33), seed=13)
    cfg, kw = case(33, 18, 14, periodic=(1, 0, 1), trt=True, omega=1.9, accel=(1e-5, 0, 0),
                   solid=solid)
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=14, amax=0.05)
    a = lattice(cfg, kw, u0, dtype=dtype, pattern="two_grid")
    b = lattice(cfg, kw, u0, dtype=dtype, pattern="aa")
    for n in (1, 6):
        a.step(n)
        b.step(n)
        np.testing.assert_array_equal(host(a.get_pdfs()), host(b.get_pdfs()))


@pytest.mark.parametrize("pattern", ["two_grid", "aa"])
@pytest.mark.parametrize("dtype", ["f32", "f32s", "f16s", "bf16s"])
@pytest.mark.parametrize("improved,trt", [(True, True), (False, False)], ids=["I-TRT", "S-SRT"])
def test_reduced_precision_one_step(dtype, pattern, improved, trt):
    """One step from a stored reduced-precision state equals the FP64 oracle
    step from the same (dequantised) state within the storage rounding plus
    an FP32 arithmetic allowance."""
    solid = random_blobs((20, 24, 70), seed=15)
    cfg, kw = case(70, 24, 20, periodic=(1, 0, 1), improved=improved, trt=trt, omega=1.95,
                   accel=(2e-6, 0, 0), solid=solid)
    u0 = lbm_inputs.shear_waves(cfg.shape, seed=16, amax=0.08)
    lat = lattice(cfg, kw, u0, dtype=dtype, pattern=pattern)
    lat.step(3)
    f_in = host(lat.get_pdfs())
    lat.step(1)
    got = host(lat.get_pdfs())
    want = oracle.step(cfg, f_in, 1)
    bound = reduced_bound(want, dtype, lat.scale)
    ratio = np.abs(got - want) / bound
    assert ratio.max() <= 1.0, f"worst {ratio.max():.3f} of bound"


def test_watchdog_catches_nan_and_mass_drift():
    from paper_1803_04937_amd import LBMError, capi
    cfg, kw = case(16, 8, 8, trt=True, omega=1.5)
    lat = lattice(cfg, kw, lbm_inputs.shear_waves(cfg.shape, seed=17), dtype="f32")
    lat.step(5)
    lat.watchdog(1e-6)
    f = host(lat.get_pdfs())
    f[3, 2, 2, 2] += 0.5          # mass injection
    lat.set_pdfs(dev(f))
    with pytest.raises(LBMError) as e:
        lat.watchdog(1e-6)
    assert e.value.status == capi.LBM_EDIVERGED
    f[3, 2, 2, 2] = np.nan
    lat.set_pdfs(dev(f))
    with pytest.raises(LBMError) as e:
        lat.watchdog(1.0)
    assert "non-finite" in str(e.value)


def test_mass_conservation_fp64_long_run():
    """FP64 relative mass drift below 1e-13 over 1000 steps (walls, obstacles)."""
    solid = random_blobs((24, 24, 24), seed=18)
    cfg, kw = case(24, 24, 24, periodic=(1, 0, 0), trt=True, omega=1.95, accel=(1e-5, 0, 0),
                   solid=solid)
    lat = lattice(cfg, kw, lbm_inputs.shear_waves(cfg.shape, seed=19))
    m0 = lat.totals()[0]
    lat.step(1000)
    assert abs(lat.totals()[0] - m0) / m0 < 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f16s"])
def test_copy_state_is_exact(dtype):
    """lbm_copy_state copies a whole state buffer bit for bit (checkpoints)."""
    cfg, kw = case(21, 13, 9, trt=True, omega=1.3)
    lat = lattice(cfg, kw, lbm_inputs.shear_waves(cfg.shape, seed=20), dtype=dtype)
    lat.step(3)
    dst = lat.new_state()
    lat.copy_state(lat.state, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst.view(torch.uint8 if dtype == "f64" else torch.int16),
                       lat.state.view(torch.uint8 if dtype == "f64" else torch.int16))
