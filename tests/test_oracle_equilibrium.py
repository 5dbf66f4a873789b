"""Pins of the oracle's velocity set and equilibria (CPU only).

Velocity set and weights: Sec. 2.3; Gauss-Hermite weights: Sec. 2.2.
Equilibria: Sec. 2.2 (standard, eq. discreteEquilibriumStandard) and Sec. 3.2
(improved, eq. new_d3q19_equilibrium).  The pins are Table 1 (transcribed in
tests/golden/table1_moments.txt) and the moment-matching construction of
Sec. 3.1-3.2 done in exact rationals.
"""
import itertools
import os

import numpy as np
import pytest
import sympy as sp

import oracle
from oracle import moment_matching as mm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_moments.txt")


def _cfg(improved):
    return oracle.Config(1, 1, 1, improved=improved)


# --------------------------------------------------------------------------
# Velocity set
# --------------------------------------------------------------------------

def test_velocity_set_groups_and_weights():
    c, w, opp = oracle.velocity_set()
    n2 = (c * c).sum(axis=1)
    # Sec. 2.3: one rest, six axis and twelve edge directions, all distinct.
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(x) for x in c}) == 19
    assert n2[0] == 0 and all(n2[1:7] == 1) and all(n2[7:] == 2)
    np.testing.assert_array_equal(w[n2 == 0], 1 / 3)
    np.testing.assert_array_equal(w[n2 == 1], 1 / 18)
    np.testing.assert_array_equal(w[n2 == 2], 1 / 36)
    for q in range(19):
        np.testing.assert_array_equal(c[opp[q]], -c[q])


def test_velocity_set_isotropy():
    """The lattice sums that the moment conditions of Sec. 3.1 rely on:
    sum w = 1, sum w c_a c_b = c_s^2 delta_ab, odd sums vanish, and the
    fourth-order sum is c_s^4 (dd + dd + dd)."""
    c, w, _ = oracle.velocity_set()
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("q,qa->a", w, c), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", w, c, c), cs2 * np.eye(3), atol=1e-16)
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc->abc", w, c, c, c), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c), iso4,
                               atol=1e-16)


def test_gauss_hermite_weights_d3q27():
    """Sec. 2.2-2.3: D3Q27 weights are products of the 1-D weights 1/6, 2/3,
    1/6, giving 8/27, 2/27, 1/54 and 1/216 by the number of nonzero
    components; the 1-D rule integrates polynomials up to degree five."""
    ws = mm.gauss_hermite_weights("D3Q27")
    cs = mm.stencil("D3Q27")
    expect = {0: sp.Rational(8, 27), 1: sp.Rational(2, 27), 2: sp.Rational(1, 54),
              3: sp.Rational(1, 216)}
    for c, wv in zip(cs, ws):
        assert wv == expect[sum(abs(x) for x in c)]
    # 1-D Gauss-Hermite exactness (abscissae scaled to 0, +-sqrt(3)):
    # integral of W(xi) xi^n = 0, 1, 0, 3, 0, 15 for n = 0..5 (n = 0..5).
    x = [0, sp.sqrt(3), -sp.sqrt(3)]
    w1 = [sp.Rational(2, 3), sp.Rational(1, 6), sp.Rational(1, 6)]
    gauss = [1, 0, 1, 0, 3, 0]
    for n in range(6):
        assert sp.simplify(sum(wi * xi ** n for wi, xi in zip(w1, x)) - gauss[n]) == 0


# --------------------------------------------------------------------------
# Table 1
# --------------------------------------------------------------------------

def _table1():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split(";")]
            rows.append((parts[0], tuple(int(v) for v in parts[1].split()), parts[2:]))
    return rows


def _expand_table1(column):
    """{exponent tuple (e_x, e_y, e_z): sympy expr} for one table column."""
    ui, uj, uk = sp.symbols("u_i u_j u_k")
    loc = {"rho": mm.RHO, "rho0": mm.RHO0, "u_i": ui, "u_j": uj, "u_k": uk}
    out = {}
    for name, pat, cols in _table1():
        expr = sp.sympify(cols[column], locals=loc)
        for perm in itertools.permutations(range(3)):
            e = [0, 0, 0]
            for slot, axis in enumerate(perm):
                e[axis] = pat[slot]
            val = sp.expand(expr.subs({ui: mm.U[perm[0]], uj: mm.U[perm[1]],
                                       uk: mm.U[perm[2]]}, simultaneous=True))
            key = tuple(e)
            if key in out:
                # the same moment reached through another labelling must agree
                assert sp.expand(out[key] - val) == 0, (name, key)
            out[key] = val
    assert len(out) == 27
    return out


def _discrete_moment(fvals, cs, e):
    return sum(fv * np.prod([ci ** ei for ci, ei in zip(c, e)]) for fv, c in zip(fvals, cs))


def _truncate_num(expr, order, rho, rho0, u):
    t = mm._truncate(expr, order)
    return float(t.subs({mm.RHO: rho, mm.RHO0: rho0, mm.U[0]: u[0], mm.U[1]: u[1],
                         mm.U[2]: u[2]}))


@pytest.mark.parametrize("improved,column", [(False, 1), (True, 2)])
def test_oracle_equilibrium_moments_match_table1(improved, column):
    """All 27 non-aliased moments of the oracle's second-order equilibria equal
    the D3Q19-S / D3Q19-I columns of Table 1 truncated at O(u^2)."""
    table = _expand_table1(column)
    c, _, _ = oracle.velocity_set()
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = 1.0 + 0.2 * rng.standard_normal()
        rho0 = 1.0 + 0.2 * rng.standard_normal()
        u = 0.2 * rng.standard_normal(3)
        f = oracle.feq(_cfg(improved), rho, u, rho0=rho0)
        for e, expr in table.items():
            got = _discrete_moment(f, c, e)
            want = _truncate_num(expr, 2, rho, rho0, u)
            assert abs(got - want) < 1e-15, (e, got, want)


def test_table1_d3q27_column_is_the_moment_matched_d3q27_equilibrium():
    """Sec. 3.1: the D3Q27 equilibrium matches all 27 Maxwellian moments.  The
    O(u^3) moment-matched D3Q27 equilibrium reproduces the transcribed D3Q27
    and Maxwellian columns up to third order (checks the transcription)."""
    cs, f = mm.construct("D3Q27", order=3)
    for col in (0, 3):
        table = _expand_table1(col)
        for e, expr in table.items():
            m = sp.expand(sum(fi * sp.prod([sp.Integer(ci) ** ei for ci, ei in zip(c, e)])
                              for fi, c in zip(f, cs)))
            assert sp.expand(mm._truncate(m, 3) - mm._truncate(expr, 3)) == 0, e


def test_table1_standard_column_is_third_order_hermite_on_d3q19():
    """The D3Q19-S column of Table 1 is the moment set of the third-order
    Hermite equilibrium with D3Q19 weights (reading of the garbled
    third-order term of eq. discreteEquilibriumStandard: 9/2[(c.u)^3 -
    (c.u) u^2])."""
    cs = mm.stencil("D3Q19")
    w = {0: sp.Rational(1, 3), 1: sp.Rational(1, 18), 2: sp.Rational(1, 36)}
    f = [mm.standard_equilibrium(c, w[sum(abs(x) for x in c)], order=3) for c in cs]
    table = _expand_table1(1)
    for e, expr in table.items():
        m = sp.expand(sum(fi * sp.prod([sp.Integer(ci) ** ei for ci, ei in zip(c, e)])
                          for fi, c in zip(f, cs)))
        assert sp.expand(mm._truncate(m, 3) - mm._truncate(expr, 3)) == 0, e


# --------------------------------------------------------------------------
# Moment-matching construction (Sec. 3.1-3.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_moment_matching_reproduces_standard_equilibrium(name):
    """Sec. 3.1: on D2Q9 and D3Q27, matching all 3^d Maxwellian moments
    truncated at O(u^2) gives the standard second-order equilibrium."""
    cs, f = mm.construct(name, order=2)
    ws = mm.gauss_hermite_weights(name)
    for c, fi, wi in zip(cs, f, ws):
        c3 = tuple(c) + (0,) * (3 - len(c))
        want = mm.standard_equilibrium(c3, wi)
        if len(c) == 2:
            want = want.subs(mm.U[2], 0)  # two-dimensional velocity
        assert sp.expand(fi - want) == 0, c


def test_moment_matching_d3q19_gives_oracle_improved_equilibrium():
    """Sec. 3.2: matching the 19 moments left after dropping those of eq.
    dropped_d3q19_moments gives D3Q19-I.  Compared with the oracle's literal
    transcription of eq. new_d3q19_equilibrium at random (rho, rho0, u)."""
    cs, f = mm.construct("D3Q19", order=2)
    fn = mm.lambdify(f)
    c, _, _ = oracle.velocity_set()
    idx = [cs.index(tuple(int(v) for v in ci)) for ci in c]
    rng = np.random.default_rng(2)
    for _ in range(20):
        rho = 1.0 + 0.2 * rng.standard_normal()
        rho0 = 1.0 + 0.2 * rng.standard_normal()
        u = 0.3 * rng.standard_normal(3)
        want = np.array(fn(rho, rho0, *u))[idx]
        got = oracle.feq(_cfg(True), rho, u, rho0=rho0)
        np.testing.assert_allclose(got, want, rtol=0, atol=2e-16 * 8)


def test_moment_matching_d3q19_differs_from_standard():
    """The two D3Q19 equilibria differ by w rho0 delta s with s = u^2 -
    sum_i c_i^2 u_i^2: +u^2/6 at rest, -(u_y^2 + u_z^2)/12 on (1,0,0),
    +u_z^2/24 on (1,1,0) (with rho0 = 1)."""
    u = np.array([0.07, -0.05, 0.11])
    fs = oracle.feq(_cfg(False), 1.0, u)
    fi = oracle.feq(_cfg(True), 1.0, u)
    c, _, _ = oracle.velocity_set()
    q100 = [q for q in range(19) if tuple(c[q]) == (1, 0, 0)][0]
    q110 = [q for q in range(19) if tuple(c[q]) == (1, 1, 0)][0]
    uu = (u * u).sum()
    assert abs((fi - fs)[0] - uu / 6) < 2e-16  # rounding of O(1/3) values
    assert abs((fi - fs)[q100] + (u[1] ** 2 + u[2] ** 2) / 12) < 1e-16
    assert abs((fi - fs)[q110] - u[2] ** 2 / 24) < 1e-16
    assert abs((fi - fs).sum()) < 5e-16
    np.testing.assert_allclose(((fi - fs)[:, None] * c).sum(axis=0), 0.0, atol=5e-16)


def test_projection_property_of_improved_equilibrium():
    """Summing D3Q19-I over c_x for each (c_y, c_z) gives the D2Q9 equilibrium
    of (rho, u_y, u_z) whatever u_x is; D3Q19-S carries a u_x^2 defect.
    This is the mechanism behind the duct results of Sec. 5.1."""
    c, _, _ = oracle.velocity_set()
    rng = np.random.default_rng(3)
    for improved in (True, False):
        base = None
        for ux in (0.0, 0.13, -0.21):
            u = np.array([ux, 0.04, -0.06])
            f = oracle.feq(_cfg(improved), 1.07, u)
            proj = {}
            for q in range(19):
                key = (int(c[q][1]), int(c[q][2]))
                proj[key] = proj.get(key, 0.0) + f[q]
            vec = np.array([proj[k] for k in sorted(proj)])
            if base is None:
                base = vec
            elif improved:
                np.testing.assert_allclose(vec, base, rtol=0, atol=1e-16)
            else:
                assert np.abs(vec - base).max() > 1e-4


# --------------------------------------------------------------------------
# Third-order D3Q19-I (the Sec. 3.2 construction carried to O(u^3))
# --------------------------------------------------------------------------

def test_third_order_improved_matches_table1_to_third_order():
    """All 27 moments of the third-order D3Q19-I equilibrium equal the D3Q19-I
    column of Table 1 (which lists terms up to O(u^3))."""
    table = _expand_table1(2)
    c, _, _ = oracle.velocity_set()
    cfg = oracle.Config(1, 1, 1, improved=2)
    rng = np.random.default_rng(30)
    for _ in range(5):
        rho, rho0 = 1.0 + 0.2 * rng.standard_normal(2)
        u = 0.2 * rng.standard_normal(3)
        f = oracle.feq(cfg, rho, u, rho0=rho0)
        for e, expr in table.items():
            got = _discrete_moment(f, c, e)
            want = _truncate_num(expr, 3, rho, rho0, u)
            assert abs(got - want) < 1e-15, (e, got, want)


def test_third_order_improved_adds_only_cubic_odd_terms():
    """f3(t u) - f2(t u) scales as t^3 and is odd in c (the second-order part
    is the paper's eq. new_d3q19_equilibrium)."""
    c, _, opp = oracle.velocity_set()
    u = np.array([0.07, -0.04, 0.05])
    d = []
    for t in (1.0, 2.0):
        f3 = oracle.feq(oracle.Config(1, 1, 1, improved=2), 1.1, t * u)
        f2 = oracle.feq(oracle.Config(1, 1, 1, improved=1), 1.1, t * u)
        d.append(f3 - f2)
    # rounding of O(1/3) values: 1e-15
    np.testing.assert_allclose(d[1], 8 * d[0], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(d[0] + d[0][opp], 0.0, atol=1e-15)
    assert np.abs(d[0]).max() > 1e-6
