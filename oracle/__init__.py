"""FP64 CPU oracle for the D3Q19 stream-collide update and its adjoint.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library (``paper_1803_04937_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP over z); this
module only loads it with ctypes and marshals numpy arrays.  The exact-rational
equilibrium construction of Sec. 3 lives in ``oracle.moment_matching``.

Array conventions: PDFs are float64 arrays of shape (Q, nz, ny, nx), Q = 19
(D3Q19) or 27 (D3Q27), x fastest; velocities (3, nz, ny, nx); densities and
masks (nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The pin suite can be pointed at another build of oracle.c (a deliberately
# broken copy, to show that the pins catch the mistake).
_LIB_OVERRIDE = os.environ.get("LBM_ORACLE_LIB")


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile oracle.c (or another source) with gcc into a shared library."""
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
               "-fPIC", "-std=c99", src, "-o", out + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("periodic", ctypes.c_int * 3),
        ("improved", ctypes.c_int), ("trt", ctypes.c_int), ("compressible", ctypes.c_int),
        ("omega", ctypes.c_double), ("magic", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("stencil", ctypes.c_int),
        ("mrt", ctypes.c_int),
        ("omega3", ctypes.c_double), ("omega4", ctypes.c_double),
        ("kbc", ctypes.c_int), ("kbc_fixed", ctypes.c_int), ("kbc_gamma", ctypes.c_double),
        ("open_x", ctypes.c_int), ("rho_out", ctypes.c_double),
        ("inlet", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB
        if not _LIB_OVERRIDE and not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        cfgp = ctypes.POINTER(_Cfg)
        lib.oracle_velocity_set.argtypes = [ctypes.c_int, P, P, P]
        lib.oracle_feq.argtypes = [cfgp, ctypes.c_double, ctypes.c_double, P, P]
        lib.oracle_dfeq_du.argtypes = [cfgp, ctypes.c_double, P, P]
        lib.oracle_init.argtypes = [cfgp, P, P, P, P]
        lib.oracle_step.argtypes = [cfgp, P, P, P]
        lib.oracle_run.argtypes = [cfgp, P, P, P, ctypes.c_int]
        lib.oracle_step_cells.argtypes = [cfgp, P, P, P, ctypes.c_int64, P]
        lib.oracle_moments.argtypes = [cfgp, P, P, P, P]
        lib.oracle_adjoint_step.argtypes = [cfgp, P, P, P, P, P]
        lib.oracle_adjoint_step.restype = ctypes.c_int
        lib.oracle_adjoint_cells.argtypes = [cfgp, P, P, P, P, ctypes.c_int64, P]
        lib.oracle_adjoint_cells.restype = ctypes.c_int
        lib.oracle_objective.argtypes = [cfgp, P, ctypes.c_int, P, P, P]
        lib.oracle_objective.restype = ctypes.c_double
        lib.oracle_init_vjp.argtypes = [cfgp, P, P, P, P]
        lib.oracle_init_vjp.restype = ctypes.c_int
        lib.oracle_kbc_collide.argtypes = [cfgp, P, P]
        lib.oracle_kbc_collide.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


@dataclass
class Config:
    """Lattice and model parameters of one oracle run."""
    nx: int
    ny: int
    nz: int
    periodic: tuple = (1, 1, 1)
    improved: int = 1          # 0: D3Q19-S, 1: D3Q19-I, 2: D3Q19-I to O(u^3)
    trt: bool = False
    compressible: bool = False
    omega: float = 1.0
    magic: float = 3.0 / 16.0
    accel: tuple = (0.0, 0.0, 0.0)
    solid: np.ndarray | None = field(default=None, repr=False)
    stencil: int = 19
    mrt: bool = False
    omega3: float = 1.0
    omega4: float = 1.0
    kbc: bool = False          # KBC entropic collision (D3Q19)
    kbc_gamma: float | None = None   # None: entropic stabiliser; else this fixed value
    open_x: bool = False       # velocity inlet at x = -1/2, pressure outlet at nx - 1/2
    rho_out: float = 1.0
    inlet: np.ndarray | None = field(default=None, repr=False)   # [3, nz, ny]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def q(self):
        return 27 if self.stencil == 27 else 19

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    def _c(self):
        c = _Cfg()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        for d in range(3):
            c.periodic[d] = int(self.periodic[d])
            c.accel[d] = float(self.accel[d])
        c.improved = int(self.improved)
        c.trt = int(self.trt)
        c.compressible = int(self.compressible)
        c.omega = float(self.omega)
        c.magic = float(self.magic)
        c.stencil = int(self.stencil)
        c.mrt = int(self.mrt)
        c.omega3 = float(self.omega3)
        c.omega4 = float(self.omega4)
        c.kbc = int(self.kbc)
        c.kbc_fixed = int(self.kbc_gamma is not None)
        c.kbc_gamma = 0.0 if self.kbc_gamma is None else float(self.kbc_gamma)
        c.open_x = int(self.open_x)
        c.rho_out = float(self.rho_out)
        keep = None
        if self.open_x:
            if self.periodic[0]:
                raise ValueError("open x faces need a non-periodic x axis")
            keep = (np.zeros((3, self.nz, self.ny)) if self.inlet is None
                    else _f64(self.inlet, (3, self.nz, self.ny)))
            c.inlet = keep.ctypes.data
        return ctypes.byref(c), (c, keep)

    def _solid(self):
        if self.solid is None:
            return None
        s = np.ascontiguousarray(self.solid, dtype=np.uint8).reshape(self.shape)
        self.solid = s
        return s


def velocity_set(stencil: int = 19):
    """(c [Q,3] int, w [Q] float, opposite [Q] int) as the oracle encodes them."""
    lib = _load()
    qn = 27 if stencil == 27 else 19
    c = np.zeros((qn, 3), dtype=np.int32)
    w = np.zeros(qn, dtype=np.float64)
    o = np.zeros(qn, dtype=np.int32)
    lib.oracle_velocity_set(int(stencil), _ptr(c), _ptr(w), _ptr(o))
    return c.astype(np.int64), w, o.astype(np.int64)


def feq(cfg: Config, rho: float, u, rho0: float | None = None):
    """Equilibrium f^eq_q(rho, u) for one cell; rho0 defaults to 1 or rho."""
    lib = _load()
    if rho0 is None:
        rho0 = rho if cfg.compressible else 1.0
    uu = _f64(u, (3,))
    out = np.zeros(cfg.q)
    ref, _keep = cfg._c()
    lib.oracle_feq(ref, float(rho), float(rho0), _ptr(uu), _ptr(out))
    return out


def kbc_collide(cfg: Config, g):
    """(post-collision f*, stabiliser gamma) of the KBC collision of one
    gathered state g (19 values), without streaming."""
    lib = _load()
    gg = _f64(g, (19,))
    out = np.zeros(19)
    ref, _keep = cfg._c()
    gamma = lib.oracle_kbc_collide(ref, _ptr(gg), _ptr(out))
    return out, gamma


def dfeq_du(cfg: Config, u, rho0: float = 1.0):
    lib = _load()
    uu = _f64(u, (3,))
    out = np.zeros((cfg.q, 3))
    ref, _keep = cfg._c()
    lib.oracle_dfeq_du(ref, float(rho0), _ptr(uu), _ptr(out))
    return out


def init(cfg: Config, u, rho=None):
    """Initial PDFs f = f^eq(rho, u); u has shape (3, nz, ny, nx)."""
    lib = _load()
    u = _f64(u, (3,) + cfg.shape)
    r = None if rho is None else _f64(rho, cfg.shape)
    f = np.empty((cfg.q,) + cfg.shape)
    ref, _keep = cfg._c()
    lib.oracle_init(ref, _ptr(cfg._solid()), _ptr(r), _ptr(u), _ptr(f))
    return f


def step(cfg: Config, f, nsteps: int = 1):
    """Advance a copy of f by nsteps two-grid pull steps; returns the result."""
    lib = _load()
    f = _f64(f, (cfg.q,) + cfg.shape).copy()
    tmp = np.empty_like(f)
    ref, _keep = cfg._c()
    lib.oracle_run(ref, _ptr(cfg._solid()), _ptr(f), _ptr(tmp), int(nsteps))
    return f


def step_cells(cfg: Config, f, cells):
    """Post-step PDFs at the listed flat cell indices: array (len(cells), 19)."""
    lib = _load()
    f = _f64(f, (cfg.q,) + cfg.shape)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((cells.size, cfg.q))
    ref, _keep = cfg._c()
    lib.oracle_step_cells(ref, _ptr(cfg._solid()), _ptr(f), _ptr(cells), cells.size, _ptr(out))
    return out


def moments(cfg: Config, f):
    """(rho (nz,ny,nx), u (3,nz,ny,nx)) of a stored post-collision state."""
    lib = _load()
    f = _f64(f, (cfg.q,) + cfg.shape)
    rho = np.empty(cfg.shape)
    u = np.empty((3,) + cfg.shape)
    ref, _keep = cfg._c()
    lib.oracle_moments(ref, _ptr(cfg._solid()), _ptr(f), _ptr(rho), _ptr(u))
    return rho, u


def adjoint_step(cfg: Config, f_t, lam_next):
    """(lam_prev, grad[4] = [dJ/domega, dJ/da_x, dJ/da_y, dJ/da_z]) of one step."""
    lib = _load()
    f_t = _f64(f_t, (cfg.q,) + cfg.shape)
    lam_next = _f64(lam_next, (cfg.q,) + cfg.shape)
    lam_prev = np.empty_like(lam_next)
    grad = np.zeros(4)
    ref, _keep = cfg._c()
    rc = lib.oracle_adjoint_step(ref, _ptr(cfg._solid()), _ptr(f_t), _ptr(lam_next),
                                 _ptr(lam_prev), _ptr(grad))
    if rc != 0:
        raise ValueError("the oracle adjoint covers the incompressible form with SRT, TRT or "
                         "MRT and without open faces only")
    return lam_prev, grad


def adjoint_cells(cfg: Config, f_t, lam_next, cells):
    """mu = J_C^T lam_next at the listed flat cell indices: array (len(cells), Q).
    mu[k, r] is what adjoint_step pushes to lam_prev[r] at x - c_r (or to
    lam_prev[rbar] at x when x - c_r is a wall or solid), x = cells[k]."""
    lib = _load()
    f_t = _f64(f_t, (cfg.q,) + cfg.shape)
    lam_next = _f64(lam_next, (cfg.q,) + cfg.shape)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((cells.size, cfg.q))
    ref, _keep = cfg._c()
    rc = lib.oracle_adjoint_cells(ref, _ptr(cfg._solid()), _ptr(f_t), _ptr(lam_next),
                                  _ptr(cells), cells.size, _ptr(out))
    if rc != 0:
        raise ValueError("the oracle adjoint covers the incompressible form only")
    return out


def objective(cfg: Config, f, kind: int):
    """(J, lam_seed, dJ/da explicit) for kind 0 (kinetic energy) or 1 (outlet flux)."""
    lib = _load()
    f = _f64(f, (cfg.q,) + cfg.shape)
    lam = np.empty_like(f)
    da = np.zeros(3)
    ref, _keep = cfg._c()
    J = lib.oracle_objective(ref, _ptr(cfg._solid()), int(kind), _ptr(f), _ptr(lam), _ptr(da))
    return J, lam, da


def init_vjp(cfg: Config, u_init, lam0):
    lib = _load()
    u = _f64(u_init, (3,) + cfg.shape)
    lam0 = _f64(lam0, (cfg.q,) + cfg.shape)
    g = np.empty((3,) + cfg.shape)
    ref, _keep = cfg._c()
    rc = lib.oracle_init_vjp(ref, _ptr(cfg._solid()), _ptr(u), _ptr(lam0), _ptr(g))
    if rc != 0:
        raise ValueError("oracle_init_vjp failed")
    return g


def gradient(cfg: Config, u_init, nsteps: int, kind: int, rho=None):
    """Reference gradient of J(f_T) by full-trajectory storage.

    Returns (J, dJ/du_init (3,nz,ny,nx), dJ/domega, dJ/da (3,)).
    """
    states = [init(cfg, u_init, rho)]
    for _ in range(nsteps):
        states.append(step(cfg, states[-1]))
    J, lam, da = objective(cfg, states[-1], kind)
    grad = np.zeros(4)
    grad[1:] += da
    for t in range(nsteps - 1, -1, -1):
        lam, g = adjoint_step(cfg, states[t], lam)
        grad += g
    gu = init_vjp(cfg, u_init, lam)
    return J, gu, grad[0], grad[1:]


def run_objective(cfg: Config, u_init, nsteps: int, kind: int, rho=None):
    """J(f_T) of a forward run, for finite differences."""
    f = step(cfg, init(cfg, u_init, rho), nsteps)
    return objective(cfg, f, kind)[0]
