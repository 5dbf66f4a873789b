"""Pins of the oracle's stream-collide step (CPU only).

The update is eq. lb_srt_with_forces (Sec. 2.3) with the Buick forcing term,
the force-shifted velocity of eq. macroscopic_vel_shift, half-way
bounce-back and periodic boundaries (Sec. 5.1).  Each test checks the oracle
against something it does not compute itself: numpy.roll, permutation
periods, conservation laws, closed-form Navier-Stokes solutions, symmetry.
"""
import numpy as np
import pytest

import lbm_inputs
import oracle

C, W, OPP = oracle.velocity_set()


def _noisy_state(cfg, seed, amp=0.02, uamp=0.05):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-uamp, uamp, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * W[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = W[:, None]
    return f


def _models():
    for improved in (False, True):
        for trt in (False, True):
            yield improved, trt


# --------------------------------------------------------------------------
# Streaming and boundaries
# --------------------------------------------------------------------------

def test_streaming_is_a_periodic_shift():
    """With omega = 0 and no force the update is pure streaming:
    f_q(x + c_q, t + 1) = f_q(x, t), i.e. numpy.roll by c_q."""
    cfg = oracle.Config(7, 5, 4, omega=0.0, trt=False)
    rng = np.random.default_rng(0)
    f = rng.uniform(0.0, 1.0, size=(19,) + cfg.shape)
    out = oracle.step(cfg, f)
    for q in range(19):
        want = np.roll(f[q], shift=(C[q][2], C[q][1], C[q][0]), axis=(0, 1, 2))
        np.testing.assert_array_equal(out[q], want)


def test_bounce_back_channel_period():
    """Free streaming between two half-way bounce-back walls (y) on a 1 x H x 1
    channel is a permutation whose period is 2H: a population travels to the
    wall, reverses in the wall-adjacent cell and comes back."""
    H = 5
    cfg = oracle.Config(1, H, 1, periodic=(1, 0, 1), omega=0.0)
    rng = np.random.default_rng(1)
    f = rng.uniform(0.0, 1.0, size=(19,) + cfg.shape)
    g = f.copy()
    for t in range(1, 2 * H + 1):
        g = oracle.step(cfg, g)
        if t < 2 * H:
            moving = [q for q in range(19) if C[q][1] != 0]
            assert not np.array_equal(g[moving], f[moving])
    np.testing.assert_array_equal(g, f)


def test_bounce_back_reflects_at_wall_cell():
    """Half-way bounce-back: at a wall-adjacent cell the population entering
    from the wall side is the one that left towards it, reversed."""
    cfg = oracle.Config(3, 4, 2, periodic=(1, 0, 1), omega=0.0)
    rng = np.random.default_rng(2)
    f = rng.uniform(0.0, 1.0, size=(19,) + cfg.shape)
    out = oracle.step(cfg, f)
    for q in range(19):
        if C[q][1] == 1:      # arrives at y = 0 from y = -1 (wall)
            np.testing.assert_array_equal(out[q][:, 0, :], f[OPP[q]][:, 0, :])
        if C[q][1] == -1:     # arrives at y = ny - 1 from y = ny (wall)
            np.testing.assert_array_equal(out[q][:, -1, :], f[OPP[q]][:, -1, :])


def test_solid_obstacle_free_streaming_period():
    """One solid cell in a periodic 1 x H x 1 column leaves a fluid segment of
    length L = H - 1 closed by the two faces of the obstacle: free streaming
    returns to the start after 2 L steps, and not before."""
    H = 7
    solid = np.zeros((1, H, 1), np.uint8)
    solid[0, 3, 0] = 1
    cfg = oracle.Config(1, H, 1, periodic=(1, 1, 1), omega=0.0, solid=solid)
    rng = np.random.default_rng(3)
    f = rng.uniform(0.0, 1.0, size=(19,) + cfg.shape)
    f[:, solid.astype(bool)] = W[:, None]
    g = f
    for t in range(1, 2 * (H - 1) + 1):
        g = oracle.step(cfg, g)
        if t < 2 * (H - 1):
            assert not np.array_equal(g, f)
    np.testing.assert_array_equal(g, f)


# --------------------------------------------------------------------------
# Conservation (eqs. mass_conservation, macroscopic_vel_shift)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("improved,trt", list(_models()))
def test_collision_conserves_mass_and_shifts_momentum(improved, trt):
    """One cell (periodic 1^3, so streaming is the identity): sum f* = sum f
    and sum c f* = sum c f + a."""
    a = (1e-3, -2e-3, 5e-4)
    cfg = oracle.Config(1, 1, 1, improved=improved, trt=trt, omega=1.7, accel=a)
    f = _noisy_state(cfg, 4, amp=0.05)
    out = oracle.step(cfg, f)
    assert abs(out.sum() - f.sum()) < 1e-15
    j0 = np.einsum("qd,q...->d...", C, f).ravel()
    j1 = np.einsum("qd,q...->d...", C, out).ravel()
    np.testing.assert_allclose(j1 - j0, a, rtol=0, atol=1e-16)


@pytest.mark.parametrize("improved,trt", list(_models()))
def test_global_mass_conserved_with_walls_and_obstacles(improved, trt):
    """Total mass is constant in a walled box with obstacles; periodic total
    momentum grows by N_cells a per step."""
    solid = np.zeros((6, 5, 8), np.uint8)
    solid[2:4, 1:3, 3:5] = 1
    cfg = oracle.Config(8, 5, 6, periodic=(1, 0, 1), improved=improved, trt=trt, omega=1.3,
                        accel=(1e-4, 0, 0), solid=solid)
    f = _noisy_state(cfg, 5)
    m0 = f[:, solid == 0].sum()
    g = oracle.step(cfg, f, 50)
    assert abs(g[:, solid == 0].sum() - m0) / m0 < 1e-13
    # fully periodic, no solid: momentum grows by N a each step
    cfg2 = oracle.Config(5, 4, 3, improved=improved, trt=trt, omega=0.9, accel=(1e-4, -3e-5, 2e-5))
    f2 = _noisy_state(cfg2, 6)
    g2 = oracle.step(cfg2, f2, 10)
    dj = np.einsum("qd,q...->d...", C, g2 - f2).reshape(3, -1).sum(axis=1)
    np.testing.assert_allclose(dj, 10 * cfg2.ncells * np.array(cfg2.accel), rtol=1e-11, atol=0)


# --------------------------------------------------------------------------
# Special cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("improved", [False, True])
def test_srt_omega_one_gives_equilibrium_plus_half_force(improved):
    a = np.array([2e-3, 1e-3, -1e-3])
    cfg = oracle.Config(1, 1, 1, improved=improved, omega=1.0, accel=tuple(a))
    f = _noisy_state(cfg, 7, amp=0.05)[:, 0, 0, 0]
    out = oracle.step(cfg, f.reshape(19, 1, 1, 1))[:, 0, 0, 0]
    rho = f.sum()
    u = C.T @ f + a / 2
    F = 3 * W * (C @ a)
    np.testing.assert_allclose(out, oracle.feq(cfg, rho, u) + F / 2, rtol=0, atol=1e-16)


@pytest.mark.parametrize("improved", [False, True])
def test_trt_with_equal_rates_is_srt(improved):
    """TRT with Lambda = (1/omega - 1/2)^2 has omega_minus = omega: it must equal
    SRT (with force) to rounding."""
    w = 1.37
    lam = (1 / w - 0.5) ** 2
    solid = np.zeros((4, 5, 6), np.uint8)
    solid[1, 2, 3] = 1
    base = dict(nx=6, ny=5, nz=4, periodic=(1, 0, 1), improved=improved, omega=w,
                accel=(1e-4, 2e-5, 0), solid=solid)
    srt = oracle.Config(trt=False, **base)
    trt = oracle.Config(trt=True, magic=lam, **base)
    f = _noisy_state(srt, 8)
    np.testing.assert_allclose(oracle.step(trt, f, 5), oracle.step(srt, f, 5), rtol=0,
                               atol=1e-15)


@pytest.mark.parametrize("improved,trt", list(_models()))
def test_uniform_flow_is_a_fixed_point(improved, trt):
    cfg = oracle.Config(4, 3, 5, improved=improved, trt=trt, omega=1.6)
    u = np.zeros((3,) + cfg.shape)
    u[0], u[1], u[2] = 0.05, -0.03, 0.02
    f = oracle.init(cfg, u)
    np.testing.assert_allclose(oracle.step(cfg, f, 20), f, rtol=0, atol=2e-16)


def _mirror_x(f):
    out = np.empty_like(f)
    for q in range(19):
        m = [p for p in range(19) if tuple(C[p]) == (-C[q][0], C[q][1], C[q][2])][0]
        out[q] = f[m][:, :, ::-1]
    return out


def _rotate_xyz(f):
    """Rotate a cubic box so that x' = z, y' = x, z' = y: c' = (c_z, c_x, c_y)
    and f'_{c'}(x') = f_c(x).  Arrays are indexed [z, y, x], so
    A'[y, x, z] = A[z, y, x]."""
    out = np.empty_like(f)
    for q in range(19):
        rotated = (C[q][2], C[q][0], C[q][1])
        p = [r for r in range(19) if tuple(C[r]) == rotated][0]
        out[p] = np.transpose(f[q], (1, 2, 0))
    return out


@pytest.mark.parametrize("improved,trt", list(_models()))
def test_mirror_symmetry(improved, trt):
    """Mirroring the initial state in x (with walls in y and an obstacle that
    is itself mirror-symmetric) mirrors the result."""
    solid = np.zeros((4, 6, 7), np.uint8)
    solid[1:3, 2:4, 3] = 1
    cfg = oracle.Config(7, 6, 4, periodic=(1, 0, 1), improved=improved, trt=trt, omega=1.4,
                        solid=solid)
    f = _noisy_state(cfg, 9)
    a = oracle.step(cfg, f, 8)
    b = oracle.step(cfg, _mirror_x(f), 8)
    np.testing.assert_allclose(b, _mirror_x(a), rtol=0, atol=1e-15)


@pytest.mark.parametrize("improved,trt", list(_models()))
def test_axis_rotation_symmetry(improved, trt):
    """The update treats the three axes alike: rotating x -> y -> z -> x of
    the initial state of a periodic cube rotates the result."""
    cfg = oracle.Config(5, 5, 5, improved=improved, trt=trt, omega=1.2)
    f = _noisy_state(cfg, 10)
    a = oracle.step(cfg, f, 6)
    b = oracle.step(cfg, _rotate_xyz(f), 6)
    np.testing.assert_allclose(b, _rotate_xyz(a), rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# Closed-form Navier-Stokes solutions
# --------------------------------------------------------------------------

def _shear_decay_error(n, omega, improved, amp=1e-3):
    nu = (1 / omega - 0.5) / 3
    k = 2 * np.pi / n
    steps = int(round(0.5 / (nu * k * k)))
    cfg = oracle.Config(1, n, 1, improved=improved, omega=omega)
    f = oracle.init(cfg, lbm_inputs.shear_wave(cfg.shape, amp))
    f = oracle.step(cfg, f, steps)
    _, u = oracle.moments(cfg, f)
    y = np.arange(n)
    A = 2 * (u[0][0, :, 0] * np.sin(k * y)).mean()
    return abs(A / amp - np.exp(-nu * k * k * steps))


@pytest.mark.parametrize("improved", [False, True])
def test_shear_wave_decay_converges_second_order(improved):
    """u_x = A sin(k y) decays as exp(-nu k^2 t), nu = (1/omega - 1/2)/3.
    Under diffusive scaling (steps ~ N^2) the error falls ~4x per doubling."""
    errs = [_shear_decay_error(n, 1.3, improved) for n in (16, 32, 64)]
    assert errs[0] < 2e-2
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_taylor_green_2d_decay():
    """z-invariant Taylor-Green vortex, tau = 0.8 on a 32^2 box: the amplitude
    after 100 steps is exp(-2 nu k^2 t) = 0.4625 to within 1 %."""
    n, tau, steps = 32, 0.8, 100
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / n
    for improved in (False, True):
        cfg = oracle.Config(n, n, 1, improved=improved, omega=1 / tau)
        f = oracle.init(cfg, lbm_inputs.taylor_green_2d(n, 0.01))
        f = oracle.step(cfg, f, steps)
        _, u = oracle.moments(cfg, f)
        ref = lbm_inputs.taylor_green_2d(n, 0.01)
        amp = (u[0] * ref[0]).sum() / (ref[0] * ref[0]).sum()
        want = np.exp(-2 * nu * k * k * steps)
        assert abs(want - 0.4625) < 1e-3
        assert abs(amp / want - 1) < 1e-2


@pytest.mark.parametrize("improved", [False, True])
def test_plane_poiseuille_is_exact_at_magic_lambda(improved):
    """Force-driven flow between half-way bounce-back walls at y = -1/2 and
    H - 1/2: u_x(y) = a/(2 nu) (y + 1/2)(H - 1/2 - y).  With TRT at Lambda =
    3/16 the discrete steady state is this parabola to rounding error."""
    H, a, omega = 12, 1e-5, 1.1
    nu = (1 / omega - 0.5) / 3
    y = np.arange(H)
    exact = a / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    cfg = oracle.Config(1, H, 1, periodic=(1, 0, 1), improved=improved, trt=True,
                        magic=3 / 16, omega=omega, accel=(a, 0, 0))
    u0 = np.zeros((3,) + cfg.shape)
    u0[0] = exact[None, :, None]
    f = oracle.step(cfg, oracle.init(cfg, u0), 4000)
    _, u = oracle.moments(cfg, f)
    np.testing.assert_allclose(u[0][0, :, 0], exact, rtol=1e-9, atol=0)
    assert np.abs(u[1:]).max() < 1e-15


def test_plane_poiseuille_srt_wall_slip_depends_on_lambda():
    """For SRT the half-way wall sits exactly at -1/2 only where
    (1/omega - 1/2)^2 = 3/16; elsewhere the profile slips."""
    H, a = 12, 1e-5
    y = np.arange(H)
    errs = {}
    for omega in (1 / (0.5 + np.sqrt(3) / 4), 1.8):
        nu = (1 / omega - 0.5) / 3
        exact = a / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
        cfg = oracle.Config(1, H, 1, periodic=(1, 0, 1), omega=omega, accel=(a, 0, 0))
        u0 = np.zeros((3,) + cfg.shape)
        u0[0] = exact[None, :, None]
        f = oracle.step(cfg, oracle.init(cfg, u0), 6000)
        _, u = oracle.moments(cfg, f)
        errs[omega] = np.abs(u[0][0, :, 0] / exact - 1).max()
    magic, other = errs.values()
    assert magic < 1e-9 and other > 1e-3, errs


def test_duct_transverse_velocity_vanishes_only_for_improved():
    """Square duct, periodic in x, half-way walls on y and z, body force along
    x (Sec. 5.1).  D3Q19-I keeps u_y = u_z = 0 to rounding; D3Q19-S develops
    spurious transverse currents."""
    D, omega = 9, 1.0
    nu = (1 / omega - 0.5) / 3
    a = 10 * nu * nu / (0.07 * D ** 3)   # max u ~ Re nu / D with Re ~ 10
    out = {}
    for improved in (True, False):
        cfg = oracle.Config(1, D, D, periodic=(1, 0, 0), improved=improved, omega=omega,
                            accel=(a, 0, 0))
        f = oracle.init(cfg, np.zeros((3,) + cfg.shape))
        f = oracle.step(cfg, f, 1500)
        _, u = oracle.moments(cfg, f)
        out[improved] = np.abs(u[1:]).max() / np.abs(u[0]).max()
    assert out[True] < 1e-13, out
    assert out[False] > 1e-7, out


def test_duct_third_order_improved_has_no_transverse_current():
    """The third-order D3Q19-I equilibrium keeps the duct invariant as well."""
    D, omega = 9, 1.0
    nu = (1 / omega - 0.5) / 3
    a = 10 * nu * nu / (0.07 * D ** 3)
    cfg = oracle.Config(1, D, D, periodic=(1, 0, 0), improved=2, omega=omega, accel=(a, 0, 0))
    f = oracle.step(cfg, oracle.init(cfg, np.zeros((3,) + cfg.shape)), 1500)
    _, u = oracle.moments(cfg, f)
    assert np.abs(u[1:]).max() / np.abs(u[0]).max() < 1e-13


# --------------------------------------------------------------------------
# MRT with Maxwellian equilibrium moments (Sec. 3.2)
# --------------------------------------------------------------------------

def _mrt_base(**kw):
    solid = np.zeros((4, 5, 6), np.uint8)
    solid[1, 2, 2:4] = 1
    d = dict(nx=6, ny=5, nz=4, periodic=(1, 0, 1), omega=1.4, accel=(2e-4, -1e-4, 5e-5),
             solid=solid)
    d.update(kw)
    return d


@pytest.mark.parametrize("improved", [0, 1, 2])
def test_mrt_with_equal_rates_is_srt(improved):
    """C_MRT with S = omega I is the BGK operator with f^eq = M^-1 m_eq."""
    srt = oracle.Config(improved=improved, **_mrt_base())
    mrt = oracle.Config(improved=improved, mrt=True, omega3=1.4, omega4=1.4, **_mrt_base())
    f = _noisy_state(srt, 80)
    np.testing.assert_allclose(oracle.step(mrt, f, 4), oracle.step(srt, f, 4), rtol=0,
                               atol=1e-15)


@pytest.mark.parametrize("improved", [0, 1])
def test_mrt_with_trt_rates_is_trt(improved):
    """Third-order moments at omega_minus and fourth-order at omega: the even
    and odd moment groups relax like TRT's even and odd parts."""
    w, lam = 1.4, 3 / 16
    wm = 1 / (0.5 + lam / (1 / w - 0.5))
    trt = oracle.Config(improved=improved, trt=True, magic=lam, **_mrt_base())
    mrt = oracle.Config(improved=improved, mrt=True, omega3=wm, omega4=w, **_mrt_base())
    f = _noisy_state(trt, 81)
    np.testing.assert_allclose(oracle.step(mrt, f, 4), oracle.step(trt, f, 4), rtol=0,
                               atol=1e-15)


def test_mrt_conservation_and_viscosity():
    """Mass and momentum (+a) are conserved whatever the free rates; the shear
    wave decays with nu = (1/omega - 1/2)/3 whatever omega3, omega4."""
    cfg = oracle.Config(1, 1, 1, improved=1, mrt=True, omega=1.3, omega3=1.7, omega4=0.9,
                        accel=(1e-3, 2e-4, -5e-4))
    f = _noisy_state(cfg, 82, amp=0.05)
    out = oracle.step(cfg, f)
    assert abs(out.sum() - f.sum()) < 1e-15
    dj = np.einsum("qd,q...->d...", C, out - f).ravel()
    np.testing.assert_allclose(dj, cfg.accel, rtol=0, atol=1e-16)
    n, omega = 32, 1.3
    nu = (1 / omega - 0.5) / 3
    k = 2 * np.pi / n
    steps = int(round(0.5 / (nu * k * k)))
    amps = []
    for w3, w4 in ((1.3, 1.3), (1.8, 0.7)):
        c2 = oracle.Config(1, n, 1, improved=1, mrt=True, omega=omega, omega3=w3, omega4=w4)
        f2 = oracle.step(c2, oracle.init(c2, lbm_inputs.shear_wave(c2.shape, 1e-3)), steps)
        _, u = oracle.moments(c2, f2)
        amps.append(2 * (u[0][0, :, 0] * np.sin(k * np.arange(n))).mean() / 1e-3)
    for a in amps:
        assert abs(a - np.exp(-nu * k * k * steps)) < 5e-3


@pytest.mark.parametrize("w3,w4", [(1.7, 0.8), (0.6, 1.5)])
def test_mrt_maxwellian_moments_keep_the_duct_invariant(w3, w4):
    """Sec. 3.3: the construction generalises to MRT.  With Maxwellian
    equilibrium moments (D3Q19-I) the duct keeps u_y = u_z = 0 for any free
    rates; with the standard equilibrium's moments it does not."""
    D, omega = 9, 1.0
    nu = (1 / omega - 0.5) / 3
    a = 10 * nu * nu / (0.07 * D ** 3)
    ratios = {}
    for improved in (1, 0):
        cfg = oracle.Config(1, D, D, periodic=(1, 0, 0), improved=improved, omega=omega,
                            accel=(a, 0, 0), mrt=True, omega3=w3, omega4=w4)
        f = oracle.step(cfg, oracle.init(cfg, np.zeros((3,) + cfg.shape)), 1500)
        _, u = oracle.moments(cfg, f)
        ratios[improved] = np.abs(u[1:]).max() / np.abs(u[0]).max()
    assert ratios[1] < 1e-13 and ratios[0] > 1e-5, ratios
