"""Exact-rational equilibrium construction by moment matching (Sec. 3.1-3.2).

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

The paper builds a discrete equilibrium by choosing Q linearly independent
velocity moments xi_0^e0 xi_1^e1 xi_2^e2, e_i in {0, 1, 2} (only these are
independent on single-speed stencils, because xi^3 = xi there), setting each
one to the matching moment of the continuous Maxwellian truncated in u, and
solving the Q x Q moment system for f^eq.  For D3Q27 all 27 moments are used;
for D3Q19 the eight moments of eq. dropped_d3q19_moments are left out.

Everything here is exact (sympy rationals).  The Maxwellian moment of
exponent e factorises into one-dimensional Gaussian moments with variance
c_s^2 = 1/3: 1, u_i, u_i^2 + 1/3 for e_i = 0, 1, 2.  As in Table 1 and in
the moment conditions of Sec. 3.1, the velocity-free part of each moment
carries rho and every velocity-dependent part carries rho0.
"""
from __future__ import annotations

import itertools

import sympy as sp

RHO, RHO0 = sp.symbols("rho rho0")
U = sp.symbols("u_x u_y u_z")
CS2 = sp.Rational(1, 3)

# Moments left out for D3Q19-I (eq. dropped_d3q19_moments).
DROPPED_D3Q19 = [(1, 2, 2), (2, 1, 2), (2, 2, 1), (1, 1, 2), (1, 2, 1), (2, 1, 1),
                 (1, 1, 1), (2, 2, 2)]


def stencil(name: str):
    """Integer velocities of D2Q9, D3Q27 or D3Q19 (Sec. 2.3), as tuples."""
    if name == "D2Q9":
        return [c for c in itertools.product((0, 1, -1), repeat=2)]
    full = [c for c in itertools.product((0, 1, -1), repeat=3)]
    if name == "D3Q27":
        return full
    if name == "D3Q19":
        return [c for c in full if sum(x * x for x in c) <= 2]
    raise ValueError(name)


def exponents(name: str):
    dim = 2 if name == "D2Q9" else 3
    es = list(itertools.product((0, 1, 2), repeat=dim))
    if name == "D3Q19":
        es = [e for e in es if e not in DROPPED_D3Q19]
    return es


def _truncate(expr, order: int):
    """Drop every term whose total degree in u exceeds ``order``."""
    poly = sp.Poly(sp.expand(expr), *U)
    keep = 0
    for monom, coeff in poly.terms():
        if sum(monom) <= order:
            keep += coeff * sp.prod([U[i] ** monom[i] for i in range(3)])
    return sp.expand(keep)


def maxwellian_moment(e, order: int = 2):
    """Moment xi^e of the Maxwellian, truncated at O(u^order): velocity-free
    part times rho, the rest times rho0."""
    one_d = {0: lambda u: sp.Integer(1), 1: lambda u: u, 2: lambda u: u ** 2 + CS2}
    m = sp.expand(sp.prod([one_d[ei](U[i]) for i, ei in enumerate(e)]))
    m = _truncate(m, order)
    free = m.subs({U[0]: 0, U[1]: 0, U[2]: 0})
    return sp.expand(free * RHO + (m - free) * RHO0)


def construct(name: str, order: int = 2):
    """Equilibrium by moment matching: returns (velocities, [f^eq_q expr])."""
    cs = stencil(name)
    es = exponents(name)
    assert len(es) == len(cs)
    M = sp.Matrix([[sp.prod([sp.Integer(c[i]) ** e[i] for i in range(len(e))]) for c in cs]
                   for e in es])
    m = sp.Matrix([maxwellian_moment(e + (0,) * (3 - len(e)), order) for e in es])
    f = M.LUsolve(m)
    return cs, [sp.expand(fi) for fi in f]


def gauss_hermite_weights(name: str):
    """Product weights of the three-point Gauss-Hermite rule (Sec. 2.2):
    2/3 at abscissa 0 and 1/6 at +-sqrt(3), multiplied over dimensions."""
    w1 = {0: sp.Rational(2, 3), 1: sp.Rational(1, 6), -1: sp.Rational(1, 6)}
    return [sp.prod([w1[ci] for ci in c]) for c in stencil(name)]


def standard_equilibrium(c, w, order: int = 2):
    """Textbook Hermite equilibrium w[rho + rho0(3 c.u + 9/2 (c.u)^2 - 3/2 u^2)]
    (plus 9/2[(c.u)^3 - (c.u) u^2] at third order) for velocity c, weight w."""
    cu = sum(ci * ui for ci, ui in zip(c, U))
    uu = sum(ui * ui for ui in U)
    poly = 3 * cu + sp.Rational(9, 2) * cu ** 2 - sp.Rational(3, 2) * uu
    if order >= 3:
        poly += sp.Rational(9, 2) * (cu ** 3 - cu * uu)
    return sp.expand(w * RHO + w * RHO0 * poly)


def lambdify(exprs):
    """Numeric callable f(rho, rho0, ux, uy, uz) -> list of values."""
    return sp.lambdify((RHO, RHO0) + U, exprs, modules="math")
