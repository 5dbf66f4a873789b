"""Pins of the oracle's D3Q27 mode (CPU only).

D3Q27 (Sec. 2.3) is the full-neighbourhood stencil; by Sec. 3.1 matching all
27 Maxwellian moments on it gives the standard equilibrium with the D3Q27
weights, and its duct flow has no spurious transverse currents (Sec. 5.1).
"""
import numpy as np
import pytest
import sympy as sp

import lbm_inputs
import oracle
from oracle import moment_matching as mm

C, W, OPP = oracle.velocity_set(27)


def _cfg(**kw):
    kw.setdefault("stencil", 27)
    return oracle.Config(**kw)


def test_d3q27_velocity_set_is_the_gauss_hermite_product_rule():
    assert len({tuple(c) for c in C}) == 27
    np.testing.assert_array_equal(C[:19], oracle.velocity_set(19)[0])
    n1 = np.abs(C).sum(axis=1)
    expect = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for q in range(27):
        assert W[q] == expect[n1[q]]
        np.testing.assert_array_equal(C[OPP[q]], -C[q])
    cs = mm.stencil("D3Q27")
    gh = mm.gauss_hermite_weights("D3Q27")
    for c, w in zip(cs, gh):
        q = [i for i in range(27) if tuple(C[i]) == tuple(c)][0]
        assert abs(W[q] - float(w)) < 1e-17
    cs2 = 1 / 3
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", W, C, C), cs2 * np.eye(3), atol=1e-16)


def test_d3q27_equilibrium_is_the_moment_matched_one():
    cs, f = mm.construct("D3Q27", order=2)
    fn = mm.lambdify(f)
    idx = [cs.index(tuple(int(v) for v in c)) for c in C]
    rng = np.random.default_rng(40)
    for improved in (False, True):       # D3Q27 has a single equilibrium
        cfg = _cfg(nx=1, ny=1, nz=1, improved=improved)
        for _ in range(10):
            rho, rho0 = 1 + 0.2 * rng.standard_normal(2)
            u = 0.3 * rng.standard_normal(3)
            np.testing.assert_allclose(oracle.feq(cfg, rho, u, rho0=rho0),
                                       np.array(fn(rho, rho0, *u))[idx], rtol=0, atol=2e-16)


def test_d3q27_streaming_is_a_periodic_shift():
    cfg = _cfg(nx=6, ny=5, nz=4, omega=0.0)
    f = np.random.default_rng(41).uniform(size=(27,) + cfg.shape)
    out = oracle.step(cfg, f)
    for q in range(27):
        np.testing.assert_array_equal(
            out[q], np.roll(f[q], shift=(C[q][2], C[q][1], C[q][0]), axis=(0, 1, 2)))


@pytest.mark.parametrize("trt", [False, True])
def test_d3q27_conservation_and_fixed_point(trt):
    a = (1e-3, -5e-4, 2e-4)
    cfg = _cfg(nx=1, ny=1, nz=1, trt=trt, omega=1.6, accel=a)
    rng = np.random.default_rng(42)
    f = oracle.init(cfg, rng.uniform(-0.05, 0.05, (3, 1, 1, 1)))
    f = f + 0.02 * W[:, None, None, None] * rng.standard_normal(f.shape)
    out = oracle.step(cfg, f)
    assert abs(out.sum() - f.sum()) < 1e-15
    dj = np.einsum("qd,q...->d...", C, out - f).ravel()
    np.testing.assert_allclose(dj, a, rtol=0, atol=1e-16)
    cfg2 = _cfg(nx=3, ny=4, nz=2, trt=trt, omega=1.3)
    u = np.zeros((3,) + cfg2.shape)
    u[0], u[1], u[2] = 0.04, -0.02, 0.03
    f2 = oracle.init(cfg2, u)
    np.testing.assert_allclose(oracle.step(cfg2, f2, 10), f2, rtol=0, atol=2e-16)


def test_d3q27_trt_with_equal_rates_is_srt():
    w = 1.2
    base = dict(nx=5, ny=4, nz=3, periodic=(1, 0, 1), omega=w, accel=(1e-4, 0, 2e-5))
    srt = _cfg(trt=False, **base)
    trt = _cfg(trt=True, magic=(1 / w - 0.5) ** 2, **base)
    f = oracle.init(srt, np.random.default_rng(43).uniform(-0.05, 0.05, (3,) + srt.shape))
    np.testing.assert_allclose(oracle.step(trt, f, 4), oracle.step(srt, f, 4), rtol=0, atol=1e-15)


def test_d3q27_shear_wave_decay_second_order():
    errs = []
    for n in (16, 32, 64):
        omega = 1.3
        nu = (1 / omega - 0.5) / 3
        k = 2 * np.pi / n
        steps = int(round(0.5 / (nu * k * k)))
        cfg = _cfg(nx=1, ny=n, nz=1, omega=omega)
        f = oracle.step(cfg, oracle.init(cfg, lbm_inputs.shear_wave(cfg.shape, 1e-3)), steps)
        _, u = oracle.moments(cfg, f)
        A = 2 * (u[0][0, :, 0] * np.sin(k * np.arange(n))).mean()
        errs.append(abs(A / 1e-3 - np.exp(-nu * k * k * steps)))
    assert errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs


def test_d3q27_duct_has_no_transverse_current():
    """Sec. 5.1: the D3Q27 duct keeps u_y = u_z = 0 to machine precision."""
    D, omega = 9, 1.0
    nu = (1 / omega - 0.5) / 3
    a = 10 * nu * nu / (0.07 * D ** 3)
    cfg = _cfg(nx=1, ny=D, nz=D, periodic=(1, 0, 0), omega=omega, accel=(a, 0, 0))
    f = oracle.step(cfg, oracle.init(cfg, np.zeros((3,) + cfg.shape)), 1500)
    _, u = oracle.moments(cfg, f)
    assert np.abs(u[1:]).max() / np.abs(u[0]).max() < 1e-13


def test_d3q27_table1_column_second_order():
    """All 27 moments of the D3Q27 equilibrium equal the D3Q27 column of
    Table 1 truncated at O(u^2)."""
    from test_oracle_equilibrium import _discrete_moment, _expand_table1, _truncate_num
    table = _expand_table1(3)
    cfg = _cfg(nx=1, ny=1, nz=1)
    rng = np.random.default_rng(44)
    for _ in range(3):
        rho, rho0 = 1 + 0.2 * rng.standard_normal(2)
        u = 0.2 * rng.standard_normal(3)
        f = oracle.feq(cfg, rho, u, rho0=rho0)
        for e, expr in table.items():
            assert abs(_discrete_moment(f, C, e) - _truncate_num(expr, 2, rho, rho0, u)) < 1e-15
