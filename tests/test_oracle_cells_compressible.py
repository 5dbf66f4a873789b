"""Pins of two oracle parts the GPU checks rely on (CPU only).

* ``oracle.step_cells``, the cell-by-cell step that serves as the reference
  of every full-size sampled check: it must give exactly the values of the
  whole-lattice ``oracle.step`` (pull gather with half-way bounce-back,
  Sec. 5.1; update of eq. lb_srt_with_forces, Sec. 2.3), on grids whose three
  extents differ, so that a slip in decoding a flat cell index shows.
* The compressible form rho0 = rho (Sec. 2.3 names rho0; the paper's runs use
  rho0 = 1): the collision conserves mass exactly and adds exactly a to the
  momentum (eqs. mass_conservation and macroscopic_vel_shift, with a the
  force density), a uniform flow at rho != 1 is a fixed point, the initial
  state f^eq(rho, u) reads back as (rho, u), and the read-out of a stored
  state returns the velocity the update used (the momentum identity:
  post-collision momentum is j + a, so (sum c f* - a/2) / rho equals
  (j + a/2) / rho).
"""
import numpy as np
import pytest

import oracle

C, W, OPP = oracle.velocity_set()


def _state(cfg, seed, rho_mean=1.0, amp=0.02, uamp=0.05):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    rho = rho_mean + 0.05 * rng.standard_normal(cfg.shape)
    f = oracle.init(cfg, u, rho=rho)
    f = f + amp * W[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = W[:, None]
    return f


def _solid(shape, seed):
    rng = np.random.default_rng(seed)
    m = (rng.random(shape) < 0.15).astype(np.uint8)
    return m


GRIDS = [
    # (nx, ny, nz, periodic): all extents distinct, walls on different axes
    (7, 5, 6, (1, 0, 1)),
    (5, 6, 7, (0, 1, 0)),
    (6, 7, 5, (1, 1, 0)),
    (9, 4, 3, (0, 0, 1)),
]


@pytest.mark.parametrize("nx,ny,nz,per", GRIDS, ids=[f"{g[0]}x{g[1]}x{g[2]}" for g in GRIDS])
@pytest.mark.parametrize("improved,trt", [(0, False), (1, True), (2, False)])
def test_step_cells_equals_full_step(nx, ny, nz, per, improved, trt):
    """oracle.step_cells at every cell, in a shuffled order, equals
    oracle.step bit for bit (solid cells keep their values)."""
    solid = _solid((nz, ny, nx), nx * 100 + ny * 10 + nz)
    cfg = oracle.Config(nx, ny, nz, periodic=per, improved=improved, trt=trt, omega=1.45,
                        accel=(2e-4, -1e-4, 5e-5), solid=solid)
    f = _state(cfg, 3)
    full = oracle.step(cfg, f).reshape(cfg.q, -1)
    cells = np.random.default_rng(4).permutation(cfg.ncells).astype(np.int64)
    got = oracle.step_cells(cfg, f, cells)
    np.testing.assert_array_equal(got, full[:, cells].T)


def test_step_cells_equals_full_step_d3q27_and_mrt():
    nx, ny, nz = 6, 4, 5
    solid = _solid((nz, ny, nx), 9)
    for cfg in (oracle.Config(nx, ny, nz, periodic=(0, 1, 1), stencil=27, trt=True, omega=1.3,
                              accel=(1e-4, 0, 2e-4), solid=solid),
                oracle.Config(nx, ny, nz, periodic=(1, 0, 1), improved=1, mrt=True, omega=1.3,
                              omega3=1.6, omega4=1.1, accel=(1e-4, 0, 2e-4), solid=solid)):
        f = _state(cfg, 5) if cfg.q == 19 else None
        if f is None:
            rng = np.random.default_rng(5)
            f = oracle.init(cfg, rng.uniform(-0.05, 0.05, (3,) + cfg.shape))
        full = oracle.step(cfg, f).reshape(cfg.q, -1)
        cells = np.arange(cfg.ncells, dtype=np.int64)[::-1].copy()
        np.testing.assert_array_equal(oracle.step_cells(cfg, f, cells), full[:, cells].T)


# --------------------------------------------------------------------------
# Compressible form
# --------------------------------------------------------------------------

MODELS = [(0, False), (1, False), (0, True), (1, True), (2, True)]


@pytest.mark.parametrize("improved,trt", MODELS)
def test_compressible_collision_conserves_mass_and_adds_a(improved, trt):
    """One periodic cell (streaming is the identity) at rho ~ 1.3: sum f* =
    sum f exactly, sum c f* = sum c f + a to rounding."""
    a = np.array([1e-3, -2e-3, 5e-4])
    cfg = oracle.Config(1, 1, 1, improved=improved, trt=trt, compressible=True, omega=1.7,
                        accel=tuple(a))
    for seed in range(5):
        f = _state(cfg, 10 + seed, rho_mean=1.3, amp=0.05)
        out = oracle.step(cfg, f)
        assert abs(out.sum() - f.sum()) <= 3e-15 * f.sum()
        j0 = C.T @ f.reshape(19)
        j1 = C.T @ out.reshape(19)
        np.testing.assert_allclose(j1 - j0, a, rtol=0, atol=2e-15)


@pytest.mark.parametrize("improved,trt", MODELS)
def test_compressible_mrt_collision_conserves_mass_and_adds_a(improved, trt):
    a = np.array([-1e-3, 2e-3, 1e-3])
    cfg = oracle.Config(1, 1, 1, improved=improved, mrt=True, compressible=True, omega=1.4,
                        omega3=1.7, omega4=0.9, accel=tuple(a))
    f = _state(cfg, 20, rho_mean=0.8, amp=0.05)
    out = oracle.step(cfg, f)
    assert abs(out.sum() - f.sum()) <= 3e-15 * f.sum()
    np.testing.assert_allclose(C.T @ out.reshape(19) - C.T @ f.reshape(19), a, rtol=0,
                               atol=2e-15)


@pytest.mark.parametrize("improved,trt", MODELS)
def test_compressible_uniform_flow_at_rho_not_one_is_a_fixed_point(improved, trt):
    cfg = oracle.Config(4, 3, 5, improved=improved, trt=trt, compressible=True, omega=1.6)
    u = np.zeros((3,) + cfg.shape)
    u[0], u[1], u[2] = 0.05, -0.03, 0.02
    f = oracle.init(cfg, u, rho=np.full(cfg.shape, 1.37))
    np.testing.assert_allclose(oracle.step(cfg, f, 20), f, rtol=0, atol=2e-15)


@pytest.mark.parametrize("improved", [0, 1, 2])
def test_compressible_init_reads_back_rho_and_u(improved):
    """f = f^eq(rho, rho0 = rho, u): its zeroth moment is rho and its first
    moment rho u, so the read-out (a = 0) returns the initial fields."""
    cfg = oracle.Config(5, 4, 3, improved=improved, compressible=True, omega=1.0)
    rng = np.random.default_rng(30)
    u = rng.uniform(-0.06, 0.06, (3,) + cfg.shape)
    rho = rng.uniform(0.7, 1.4, cfg.shape)
    f = oracle.init(cfg, u, rho=rho)
    r, v = oracle.moments(cfg, f)
    np.testing.assert_allclose(r, rho, rtol=2e-16 * 8, atol=0)
    np.testing.assert_allclose(v, u, rtol=0, atol=4e-16)
    # the zeroth and first moments of the stored state, by summation here
    np.testing.assert_allclose(f.sum(axis=0), rho, rtol=1e-15, atol=0)
    np.testing.assert_allclose(np.einsum("qd,q...->d...", C, f), rho * u, rtol=0, atol=1e-15)


@pytest.mark.parametrize("improved,trt", MODELS)
def test_compressible_readout_returns_the_update_velocity(improved, trt):
    """Momentum identity at rho != 1: after one step of a periodic cell, the
    read-out velocity (sum c f* - a/2) / rho equals (sum c f + a/2) / rho of
    the state the step started from, and the read-out density is sum f."""
    a = np.array([3e-3, 1e-3, -2e-3])
    cfg = oracle.Config(1, 1, 1, improved=improved, trt=trt, compressible=True, omega=1.2,
                        accel=tuple(a))
    f = _state(cfg, 40, rho_mean=1.25, amp=0.05).reshape(19)
    out = oracle.step(cfg, f.reshape(19, 1, 1, 1))
    r, v = oracle.moments(cfg, out)
    rho = f.sum()
    np.testing.assert_allclose(r.ravel(), [rho], rtol=4e-16, atol=0)
    np.testing.assert_allclose(v.ravel(), (C.T @ f + a / 2) / rho, rtol=0, atol=1e-16)


def test_compressible_differs_from_incompressible_at_rho_not_one():
    """The flag is not a no-op: at rho != 1 with a flow the two forms give
    different updates; at rho = 1 they start from the same initial state."""
    base = dict(nx=3, ny=3, nz=3, improved=1, trt=True, omega=1.3, accel=(1e-4, 0, 0))
    ci = oracle.Config(compressible=False, **base)
    cc = oracle.Config(compressible=True, **base)
    rng = np.random.default_rng(50)
    u = rng.uniform(-0.05, 0.05, (3, 3, 3, 3))
    f1 = oracle.init(ci, u)
    np.testing.assert_array_equal(oracle.init(cc, u), f1)
    f = oracle.init(cc, u, rho=np.full((3, 3, 3), 1.2))
    assert np.abs(oracle.step(cc, f) - oracle.step(ci, f)).max() > 1e-5
