"""Pins of the oracle's adjoint (CPU only).

The adjoint is not in the paper: it is the exact transpose of the discrete
update of eq. lb_srt_with_forces (Sec. 2.3) with pull streaming and half-way
bounce-back.  With rho0 = 1 one step is a quadratic polynomial in the PDFs,
in a and (for SRT) linear in omega, so central differences are exact up to
rounding for those derivatives; multi-step and TRT-omega derivatives are
checked against central differences with an O(h^2) error.
"""
import numpy as np
import pytest

import lbm_inputs
import oracle

C, W, OPP = oracle.velocity_set()


def _state(cfg, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * W[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = W[:, None]
    return f


def _cfgs():
    solid = np.zeros((4, 5, 6), np.uint8)
    solid[1:3, 2, 2:4] = 1
    for improved in (False, True):
        for trt in (False, True):
            yield oracle.Config(6, 5, 4, periodic=(1, 0, 1), improved=improved, trt=trt,
                                omega=1.45, magic=3 / 16, accel=(2e-4, -1e-4, 5e-5),
                                solid=solid)


def _replace(cfg, **kw):
    d = dict(nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, periodic=cfg.periodic, improved=cfg.improved,
             trt=cfg.trt, compressible=cfg.compressible, omega=cfg.omega, magic=cfg.magic,
             accel=cfg.accel, solid=cfg.solid)
    d.update(kw)
    return oracle.Config(**d)


@pytest.mark.parametrize("cfg", list(_cfgs()), ids=lambda c: f"I{int(c.improved)}T{int(c.trt)}")
def test_adjoint_step_dot_product(cfg):
    """<step'(f) v, lam> = <v, step'(f)^T lam> with the directional derivative
    taken by central differences (exact for a quadratic map)."""
    rng = np.random.default_rng(11)
    f = _state(cfg, 12)
    v = W[:, None, None, None] * rng.standard_normal(f.shape)
    lam = rng.standard_normal(f.shape)
    h = 1e-3
    jvp = (oracle.step(cfg, f + h * v) - oracle.step(cfg, f - h * v)) / (2 * h)
    lam_prev, _ = oracle.adjoint_step(cfg, f, lam)
    lhs = (jvp * lam).sum()
    rhs = (v * lam_prev).sum()
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + np.abs(v).sum()), (lhs, rhs)


@pytest.mark.parametrize("cfg", list(_cfgs()), ids=lambda c: f"I{int(c.improved)}T{int(c.trt)}")
def test_adjoint_step_parameter_gradients(cfg):
    """dJ/da (and dJ/domega) of J = <lam, step(f)> against central
    differences."""
    rng = np.random.default_rng(13)
    f = _state(cfg, 14)
    lam = rng.standard_normal(f.shape)
    _, grad = oracle.adjoint_step(cfg, f, lam)

    def J(c):
        return (oracle.step(c, f) * lam).sum()

    h = 1e-4
    for b in range(3):
        ap = list(cfg.accel)
        am = list(cfg.accel)
        ap[b] += h
        am[b] -= h
        fd = (J(_replace(cfg, accel=tuple(ap))) - J(_replace(cfg, accel=tuple(am)))) / (2 * h)
        assert abs(fd - grad[1 + b]) <= 1e-9 * max(1.0, abs(fd)), (b, fd, grad[1 + b])
    hw = 1e-5
    fd = (J(_replace(cfg, omega=cfg.omega + hw)) - J(_replace(cfg, omega=cfg.omega - hw))) / (2 * hw)
    tol = 1e-9 if not cfg.trt else 1e-6   # TRT: omega_minus(omega) is not polynomial
    assert abs(fd - grad[0]) <= tol * max(1.0, abs(fd)), (fd, grad[0])


def test_adjoint_solid_cells_pass_through():
    cfg = list(_cfgs())[0]
    rng = np.random.default_rng(15)
    f = _state(cfg, 16)
    lam = rng.standard_normal(f.shape)
    lam_prev, _ = oracle.adjoint_step(cfg, f, lam)
    s = cfg.solid.astype(bool)
    np.testing.assert_array_equal(lam_prev[:, s], lam[:, s])


@pytest.mark.parametrize("kind", [0, 1])
def test_objective_seed_is_its_gradient(kind):
    """lam_T = dJ/df and the explicit dJ/da of both objectives."""
    cfg = list(_cfgs())[3]
    rng = np.random.default_rng(17)
    f = _state(cfg, 18)
    J0, lam, da = oracle.objective(cfg, f, kind)
    v = rng.standard_normal(f.shape)
    h = 1e-4
    fd = (oracle.objective(cfg, f + h * v, kind)[0] - oracle.objective(cfg, f - h * v, kind)[0]) / (2 * h)
    assert abs(fd - (lam * v).sum()) < 1e-9 * max(1, abs(fd))
    for b in range(3):
        ap = list(cfg.accel)
        am = list(cfg.accel)
        ap[b] += h
        am[b] -= h
        fd = (oracle.objective(_replace(cfg, accel=tuple(ap)), f, kind)[0]
              - oracle.objective(_replace(cfg, accel=tuple(am)), f, kind)[0]) / (2 * h)
        assert abs(fd - da[b]) < 1e-9 * max(1, abs(fd))


def _fd4(fun, h):
    """Fourth-order central difference of a scalar function of one step h."""
    return (-fun(2 * h) + 8 * fun(h) - 8 * fun(-h) + fun(-2 * h)) / (12 * h)


@pytest.mark.parametrize("cfg", list(_cfgs()), ids=lambda c: f"I{int(c.improved)}T{int(c.trt)}")
@pytest.mark.parametrize("kind", [0, 1])
def test_rollout_gradient_against_finite_differences(cfg, kind):
    """Full gradient of J(f_T), T = 6 steps from f_0 = f^eq(1, u_init), with
    respect to u_init (along a random direction), a and omega."""
    T = 6
    rng = np.random.default_rng(19)
    u0 = rng.uniform(-0.04, 0.04, size=(3,) + cfg.shape)
    J, gu, gw, ga = oracle.gradient(cfg, u0, T, kind)
    v = rng.standard_normal(u0.shape)
    h = 1e-5
    fd = _fd4(lambda s: oracle.run_objective(cfg, u0 + s * v, T, kind), h)
    assert abs(fd - (gu * v).sum()) <= 1e-8 * max(1e-3, abs(fd)), (fd, (gu * v).sum())
    for b in range(3):
        def shifted(s, b=b):
            a = list(cfg.accel)
            a[b] += s
            return oracle.run_objective(_replace(cfg, accel=tuple(a)), u0, T, kind)
        fd = _fd4(shifted, h)
        assert abs(fd - ga[b]) <= 1e-8 * max(1e-3, abs(fd)), (b, fd, ga[b])
    fd = _fd4(lambda s: oracle.run_objective(_replace(cfg, omega=cfg.omega + s), u0, T, kind), h)
    assert abs(fd - gw) <= 1e-8 * max(1e-3, abs(fd)), (fd, gw)


def test_shear_wave_energy_gradient_matches_viscous_decay():
    """Kinetic energy of a decaying shear wave, E(T) ~ E(0) exp(-2 nu k^2 T),
    so dE/domega ~ E (-2 k^2 T) dnu/domega with dnu/domega = -1/(3 omega^2).
    Holds to the discretisation error of the decay rate."""
    n, omega, T = 32, 1.2, 200
    cfg = oracle.Config(1, n, 1, improved=True, omega=omega)
    u0 = lbm_inputs.shear_wave(cfg.shape, 1e-3)
    J, _, gw, _ = oracle.gradient(cfg, u0, T, 0)
    k = 2 * np.pi / n
    want = J * (-2 * k * k * T) * (-1 / (3 * omega ** 2))
    assert abs(gw / want - 1) < 0.03, (gw, want)


def test_compressible_adjoint_is_refused():
    cfg = oracle.Config(2, 2, 2, compressible=True, omega=1.0)
    f = _state(oracle.Config(2, 2, 2, omega=1.0), 1)
    with pytest.raises(ValueError):
        oracle.adjoint_step(cfg, f, f)


# --------------------------------------------------------------------------
# The adjoint of the widened forward path: D3Q27 (Sec. 2.3, 3.1), the
# third-order D3Q19-I (Sec. 3.2 carried to O(u^3)) and MRT with Maxwellian
# moments (Sec. 3.2).  The third-order step is not quadratic in f and a, so
# these pins use fourth-order central differences throughout.
# --------------------------------------------------------------------------

def _wide_cfgs():
    solid = np.zeros((4, 5, 6), np.uint8)
    solid[1:3, 2, 2:4] = 1
    base = dict(nx=6, ny=5, nz=4, periodic=(1, 0, 1), omega=1.45, magic=3 / 16,
                accel=(2e-4, -1e-4, 5e-5), solid=solid)
    return [
        ("Q27-SRT", oracle.Config(stencil=27, improved=0, **base)),
        ("Q27-TRT", oracle.Config(stencil=27, improved=0, trt=True, **base)),
        ("I3-SRT", oracle.Config(improved=2, **base)),
        ("I3-TRT", oracle.Config(improved=2, trt=True, **base)),
        ("MRT-S", oracle.Config(improved=0, mrt=True, omega3=1.7, omega4=0.9, **base)),
        ("MRT-I", oracle.Config(improved=1, mrt=True, omega3=1.7, omega4=0.9, **base)),
        ("MRT-I3", oracle.Config(improved=2, mrt=True, omega3=0.8, omega4=1.6, **base)),
    ]


def _wstate(cfg, seed, amp=0.02):
    w = oracle.velocity_set(cfg.stencil)[1]
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.05, 0.05, size=(3,) + cfg.shape)
    f = oracle.init(cfg, u, rho=1.0 + 0.01 * rng.standard_normal(cfg.shape))
    f = f + amp * w[:, None, None, None] * rng.standard_normal(f.shape)
    if cfg.solid is not None:
        f[:, cfg.solid.astype(bool)] = w[:, None]
    return f, w


def _wreplace(cfg, **kw):
    d = dict(nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, periodic=cfg.periodic, improved=cfg.improved,
             trt=cfg.trt, compressible=cfg.compressible, omega=cfg.omega, magic=cfg.magic,
             accel=cfg.accel, solid=cfg.solid, stencil=cfg.stencil, mrt=cfg.mrt,
             omega3=cfg.omega3, omega4=cfg.omega4)
    d.update(kw)
    return oracle.Config(**d)


WIDE = _wide_cfgs()


@pytest.mark.parametrize("name,cfg", WIDE, ids=[n for n, _ in WIDE])
def test_wide_adjoint_step_dot_product(name, cfg):
    rng = np.random.default_rng(31)
    f, w = _wstate(cfg, 32)
    v = w[:, None, None, None] * rng.standard_normal(f.shape)
    lam = rng.standard_normal(f.shape)
    jvp = _fd4(lambda s: (oracle.step(cfg, f + s * v) * lam).sum(), 1e-3)
    lam_prev, _ = oracle.adjoint_step(cfg, f, lam)
    rhs = (v * lam_prev).sum()
    assert abs(jvp - rhs) <= 1e-10 * (abs(jvp) + np.abs(v).sum()), (jvp, rhs)


@pytest.mark.parametrize("name,cfg", WIDE, ids=[n for n, _ in WIDE])
def test_wide_adjoint_step_parameter_gradients(name, cfg):
    rng = np.random.default_rng(33)
    f, _ = _wstate(cfg, 34)
    lam = rng.standard_normal(f.shape)
    _, grad = oracle.adjoint_step(cfg, f, lam)

    def J(c):
        return (oracle.step(c, f) * lam).sum()

    for b in range(3):
        def shifted(s, b=b):
            a = list(cfg.accel)
            a[b] += s
            return J(_wreplace(cfg, accel=tuple(a)))
        fd = _fd4(shifted, 1e-4)
        assert abs(fd - grad[1 + b]) <= 1e-9 * max(1.0, abs(fd)), (b, fd, grad[1 + b])
    fd = _fd4(lambda s: J(_wreplace(cfg, omega=cfg.omega + s)), 1e-4)
    assert abs(fd - grad[0]) <= 1e-9 * max(1.0, abs(fd)), (fd, grad[0])


@pytest.mark.parametrize("name,cfg", WIDE, ids=[n for n, _ in WIDE])
def test_wide_rollout_gradient_against_finite_differences(name, cfg):
    """Gradient of the kinetic energy after T = 5 steps from f^eq(1, u_init)
    with respect to u_init (random direction), a and omega: the init VJP,
    the adjoint steps and the objective seed of the widened path together."""
    T, kind = 5, 0
    rng = np.random.default_rng(35)
    u0 = rng.uniform(-0.04, 0.04, size=(3,) + cfg.shape)
    J, gu, gw, ga = oracle.gradient(cfg, u0, T, kind)
    v = rng.standard_normal(u0.shape)
    fd = _fd4(lambda s: oracle.run_objective(cfg, u0 + s * v, T, kind), 1e-5)
    assert abs(fd - (gu * v).sum()) <= 1e-8 * max(1e-3, abs(fd)), (fd, (gu * v).sum())
    for b in range(3):
        def shifted(s, b=b):
            a = list(cfg.accel)
            a[b] += s
            return oracle.run_objective(_wreplace(cfg, accel=tuple(a)), u0, T, kind)
        fd = _fd4(shifted, 1e-5)
        assert abs(fd - ga[b]) <= 1e-8 * max(1e-3, abs(fd)), (b, fd, ga[b])
    fd = _fd4(lambda s: oracle.run_objective(_wreplace(cfg, omega=cfg.omega + s), u0, T, kind),
              1e-5)
    assert abs(fd - gw) <= 1e-8 * max(1e-3, abs(fd)), (fd, gw)


def test_third_order_dfeq_du_against_differences():
    """d f^eq / d u of the third-order D3Q19-I: the oracle differentiates its
    moments; compare with central differences of the equilibrium itself."""
    cfg = oracle.Config(1, 1, 1, improved=2)
    rng = np.random.default_rng(36)
    for _ in range(5):
        u = rng.uniform(-0.2, 0.2, 3)
        D = oracle.dfeq_du(cfg, u)
        for b in range(3):
            e = np.zeros(3)
            e[b] = 1.0
            fd = _fd4(lambda s: oracle.feq(cfg, 1.0, u + s * e), 1e-4)
            np.testing.assert_allclose(D[:, b], fd, rtol=0, atol=1e-12)


@pytest.mark.parametrize("cfg", list(_cfgs()) + [c for _, c in _wide_cfgs()],
                         ids=lambda c: f"Q{c.stencil}I{int(c.improved)}T{int(c.trt)}M{int(c.mrt)}")
def test_adjoint_cells_match_full_adjoint(cfg):
    """The per-cell adjoint (for sampled checks of large grids) gives, for
    every fluid cell, exactly the values the full adjoint pushes to its
    targets; solid cells report lam_next."""
    from _helpers import push_targets
    f = _wstate(cfg, 40)[0]
    lam = np.random.default_rng(41).standard_normal(f.shape)
    lp, _ = oracle.adjoint_step(cfg, f, lam)
    cells = np.arange(cfg.ncells)
    mu = oracle.adjoint_cells(cfg, f, lam, cells)
    fluid = ~cfg.solid.reshape(-1).astype(bool)
    arr, tgt = push_targets(cfg, cells[fluid])
    np.testing.assert_array_equal(mu[fluid], lp.reshape(cfg.q, -1)[arr, tgt])
    np.testing.assert_array_equal(mu[~fluid], lam.reshape(cfg.q, -1)[:, ~fluid].T)
