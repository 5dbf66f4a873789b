"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of oracle/oracle.c (a wrong
coefficient, sign, index, weight or transposed operand), builds it into a
separate library and runs the oracle pin suite against that library in a
fresh process: the suite must fail.  The unmodified oracle passes the same
suite (the other test files).
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PIN_FILES = ["tests/test_oracle_equilibrium.py", "tests/test_oracle_step.py",
             "tests/test_oracle_adjoint.py", "tests/test_oracle_d3q27.py",
             "tests/test_oracle_cells_compressible.py", "tests/test_oracle_kbc_open.py"]

# The per-cell step's index decoding (the full-size checks' reference).
_CELLS_DECODE = ("        int x = (int)(c % cfg->nx), y = (int)((c / cfg->nx) % cfg->ny),\n"
                 "            z = (int)(c / ((int64_t)cfg->nx * cfg->ny));\n"
                 "        if (solid && solid[c]) {\n"
                 "            for (int q = 0; q < QN(cfg); ++q) out[k * QN(cfg) + q] = fin[q * n + c];")

MUTANTS = [
    ("standard: 9/2 -> 4", "(3.0 * first + 4.5 * second)", "(3.0 * first + 4.0 * second)"),
    ("standard: trace term dropped", "(a == b ? 1.0 / 3.0 : 0.0)", "(a == b ? 0.0 : 0.0)"),
    ("improved rest: -u^2 -> -3/2 u^2", "bracket = -uu;", "bracket = -1.5 * uu;"),
    ("improved axis: 6 (c.u)^2 -> 9/2", "6.0 * cu * cu;", "4.5 * cu * cu;"),
    ("improved edge: unsummed u^2", "3.0 * cu - 1.5 * uc2", "3.0 * cu - 1.5 * uu"),
    ("edge weight 1/36 -> 1/18", "return 1.0 / 36.0;", "return 1.0 / 18.0;"),
    ("streaming sign", "int p[3] = {x + s * C[q][0],", "int p[3] = {x - s * C[q][0],"),
    ("bounce-back reads own direction",
     "if (is_solid(solid, src))\n            g[q] = f[(int64_t)qb * n + here];",
     "if (is_solid(solid, src))\n            g[q] = f[(int64_t)q * n + here];"),
    ("velocity shift a/2 -> a", "u[d] = (j[d] + 0.5 * cfg->accel[d]) / *rho0;",
     "u[d] = (j[d] + 1.0 * cfg->accel[d]) / *rho0;"),
    ("SRT force factor (1 - w/2) -> (1 - w)",
     "out[q] = g[q] - w * (g[q] - fe[q]) + (1.0 - w / 2.0) * force_term(cfg, q);",
     "out[q] = g[q] - w * (g[q] - fe[q]) + (1.0 - w) * force_term(cfg, q);"),
    ("TRT force relaxed with the even rate",
     "out[q] = g[q] - w * (gp - ep) - wm * (gm - em) + (1.0 - wm / 2.0) * force_term(cfg, q);",
     "out[q] = g[q] - w * (gp - ep) - wm * (gm - em) + (1.0 - w / 2.0) * force_term(cfg, q);"),
    ("TRT Lambda inverted", "return 1.0 / (0.5 + cfg->magic / tau_plus);",
     "return 1.0 / (0.5 + tau_plus / cfg->magic);"),
    ("forcing weight / c_s^2 dropped", "return weight(q) / (1.0 / 3.0) * ca;",
     "return weight(q) * ca;"),
    ("read-out velocity shift dropped",
     "u[d * n + c] = (j[d] - 0.5 * cfg->accel[d]) / rho0;", "u[d * n + c] = j[d] / rho0;"),
    ("adjoint push to the opposite array", "lam_prev[(int64_t)r * n + src] = mu;",
     "lam_prev[(int64_t)opposite(r) * n + src] = mu;"),
    ("adjoint Jacobian transposed", "for (int r = 0; r < QN(cfg); ++r) {\n            double v = weight(q);\n            for (int b = 0; b < 3; ++b) v += D[q][b] * C[r][b];",
     "for (int r = 0; r < QN(cfg); ++r) {\n            double v = weight(q);\n            for (int b = 0; b < 3; ++b) v += D[q][b] * C[q][b];"),
    ("d feq/du improved axis 12 -> 9", "(3.0 * cb - 6.0 * u[b] + 12.0 * cu * cb)",
     "(3.0 * cb - 6.0 * u[b] + 9.0 * cu * cb)"),
    ("objective dJ/da sign", "da[d] += -0.5 * u[d];", "da[d] += 0.5 * u[d];"),
    ("TRT d omega_minus / d omega sign",
     "double dwm_dwp = -wm * wm * cfg->magic / (tau_p * tau_p * wp * wp);",
     "double dwm_dwp = wm * wm * cfg->magic / (tau_p * tau_p * wp * wp);"),
    ("D3Q27 corner weight 1/216 -> 1/108", "return 1.0 / 216.0;", "return 1.0 / 108.0;"),
    ("D3Q27 takes the D3Q19-I form",
     "if (cfg->stencil == 27) return feq_standard(cfg, q, rho, rho0, u);",
     "if (cfg->stencil == 27) return feq_improved(cfg, q, rho, rho0, u);"),
    ("third-order construction truncated at O(u^2)", "if (a + b + c == 0 || a + b + c > 3) continue;",
     "if (a + b + c == 0 || a + b + c > 2) continue;"),
    ("third-order construction drops the wrong moment", "{1, 2, 1}, {2, 1, 1}, {1, 1, 1}, {2, 2, 2}};",
     "{1, 2, 1}, {2, 1, 1}, {1, 1, 1}, {0, 2, 2}};"),
    ("MRT force without (1 - s/2)", "mnew[k] = m[k] - s * (m[k] - meq[k]) + (1.0 - s / 2.0) * mF[k];",
     "mnew[k] = m[k] - s * (m[k] - meq[k]) + mF[k];"),
    ("MRT third-order moments take the fourth-order rate",
     "(order == 3 ? cfg->omega3 : cfg->omega4)", "(order == 3 ? cfg->omega4 : cfg->omega4)"),
    ("init VJP reads the rest population only", "v += lam0[q * n + c] * D[q][b];",
     "v += lam0[c] * D[q][b];"),
    ("MRT adjoint force term without (I - R/2)",
     "v -= 0.5 * R[q][s] * 3.0 * weight(s) * C[s][b];", "v -= 0.0 * R[q][s] * 3.0 * weight(s) * C[s][b];"),
    ("MRT d/domega moves the third-order rate", "p2 += order == 2 ? mk : 0.0;",
     "p2 += order == 3 ? mk : 0.0;"),
    ("third-order moment derivative drops the power factor",
     "t *= i == d ? pw[i] * ipow(u[i], pw[i] - 1) : ipow(u[i], pw[i]);",
     "t *= i == d ? ipow(u[i], pw[i] - 1) : ipow(u[i], pw[i]);"),
    ("per-cell step decodes y modulo nx", _CELLS_DECODE,
     _CELLS_DECODE.replace("(c / cfg->nx) % cfg->ny", "(c / cfg->nx) % cfg->nx")),
    ("per-cell step decodes z with nx nz", _CELLS_DECODE,
     _CELLS_DECODE.replace("(int64_t)cfg->nx * cfg->ny", "(int64_t)cfg->nx * cfg->nz")),
    ("compressible velocity: force shift outside the division",
     "u[d] = (j[d] + 0.5 * cfg->accel[d]) / *rho0;", "u[d] = j[d] / *rho0 + 0.5 * cfg->accel[d];"),
    ("compressible flag ignored in the update", "*rho0 = cfg->compressible ? r : 1.0;",
     "*rho0 = 1.0;"),
    ("compressible flag ignored in the initial state", "double rho0 = cfg->compressible ? rho : 1.0;",
     "double rho0 = 1.0;"),
    ("compressible flag ignored in the read-out", "double rho0 = cfg->compressible ? r : 1.0;",
     "double rho0 = 1.0;"),
    ("KBC shear part takes the fourth order", "} else if (order <= 3) {",
     "} else if (order <= 4) {"),
    ("KBC shear part without the third order", "} else if (order <= 3) {",
     "} else if (order <= 2) {"),
    ("KBC shear force without (1 - beta)", "+ Fk[q] + (1.0 - beta) * Fs[q] +",
     "+ Fk[q] + Fs[q] +"),
    ("KBC stabiliser ratio inverted", "(2.0 - 1.0 / beta) * sh / hh, 0.0)",
     "(2.0 - 1.0 / beta) * hh / sh, 0.0)"),
    ("KBC stabiliser sign", "1.0 / beta - (2.0 - 1.0 / beta) * sh / hh",
     "1.0 / beta + (2.0 - 1.0 / beta) * sh / hh"),
    ("KBC entropic metric weights w instead of f^eq",
     "sh += ds[q] * dh[q] / fe[q];\n        hh += dh[q] * dh[q] / fe[q];",
     "sh += ds[q] * dh[q] / weight(q);\n        hh += dh[q] * dh[q] / weight(q);"),
    ("KBC stabiliser unbounded", "fmin(fmax(1.0 / beta - (2.0 - 1.0 / beta) * sh / hh, 0.0), 2.0)",
     "(1.0 / beta - (2.0 - 1.0 / beta) * sh / hh)"),
    ("KBC stabiliser bounded by the marginal rate", "sh / hh, 0.0), 2.0)",
     "sh / hh, 0.0), 2.0 / beta)"),
    ("inlet moving-wall term 6 -> 3", "+ 6.0 * weight(q) * cu;", "+ 3.0 * weight(q) * cu;"),
    ("inlet rule one cell too far", "if (cfg->open_x && px < 0) {", "if (cfg->open_x && px <= 0) {"),
    ("outlet bounce-back instead of anti-bounce-back",
     "g[q] = -f[(int64_t)qb * n + here] + (fe[q] + fe[qb]);",
     "g[q] = f[(int64_t)qb * n + here] + (fe[q] + fe[qb]) - 2.0 * weight(q) * cfg->rho_out;"),
    ("outlet equilibrium at the inflow density", "feq_all(cfg, cfg->rho_out, 1.0, ub, fe);",
     "feq_all(cfg, 1.0, 1.0, ub, fe);"),
    ("outlet velocity from the rest population only",
     "for (int d = 0; d < 3; ++d) ub[d] += C[q][d] * f[(int64_t)q * n + here];",
     "for (int d = 0; d < 3; ++d) ub[d] += C[q][d] * f[here];"),
]


def _caught(name, old, new, workdir):
    """Build the oracle with one planted mistake and run the pin suite
    against it in a fresh process; True when the suite fails."""
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    d = os.path.join(workdir, re.sub(r"[^A-Za-z0-9]+", "_", name))
    os.makedirs(d, exist_ok=True)
    mutant = os.path.join(d, "oracle_mutant.c")
    with open(mutant, "w") as fh:
        fh.write(src.replace(old, new))
    lib = oracle.build(force=True, src=mutant, out=os.path.join(d, "liboracle_mutant.so"))
    env = dict(os.environ, LBM_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *PIN_FILES], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=900)
    return res.returncode != 0, res.stdout[-1500:]


def test_mutation_sites_are_unique():
    src = open(SRC).read()
    for name, old, _ in MUTANTS:
        assert src.count(old) == 1, f"{name}: mutation site not unique: {old!r}"


def test_planted_mistakes_are_caught(tmp_path):
    """Every planted mistake makes the pin suite fail (mutants run four at a
    time, each in its own process with two threads)."""
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {ex.submit(_caught, n, o, w, str(tmp_path)): n for n, o, w in MUTANTS}
        results = {futs[f]: f.result() for f in futs}
    escaped = [n for n, (caught, _) in results.items() if not caught]
    for n in escaped:
        print(f"not caught: {n}\n{results[n][1]}")
    assert not escaped, escaped
