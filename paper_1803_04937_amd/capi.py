"""ctypes binding of liblbm.so: the C ABI of include/lbm.h, one Python function
per C entry point, same names, argument marshalling only.

Device buffers are passed as torch CUDA tensors (their data_ptr()) or raw
integer addresses; host outputs come back as Python values.  Every function
raises LBMError on a non-zero status with the library's message.  There is
no fallback: if liblbm.so is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_EQ_STANDARD, LBM_EQ_IMPROVED, LBM_EQ_IMPROVED3 = 0, 1, 2
LBM_SRT, LBM_TRT, LBM_MRT, LBM_KBC = 0, 1, 2, 3
LBM_ROUND_NEAREST, LBM_ROUND_STOCHASTIC = 0, 1
LBM_CACHE_AUTO, LBM_CACHE_STREAM, LBM_CACHE_KEEP = 0, 1, 2
LBM_ADJ_SOLID_COPY, LBM_ADJ_SOLID_SKIP = 0, 1
LBM_F64, LBM_F32, LBM_F32_SHIFTED, LBM_F16_SHIFTED, LBM_BF16_SHIFTED = 0, 1, 2, 3, 4
LBM_TWO_GRID, LBM_AA = 0, 1
LBM_OBJ_KINETIC_ENERGY, LBM_OBJ_OUTLET_FLUX = 0, 1

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP",
                -4: "LBM_EDIVERGED", -5: "LBM_ESTATE"}

# Every entry point declared in include/lbm.h.
EXPORTS = [
    "lbm_version", "lbm_velocity_set", "lbm_qstride", "lbm_state_bytes", "lbm_adjoint_bytes",
    "lbm_validate", "lbm_links_bytes", "lbm_choose_scale", "lbm_init", "lbm_destroy", "lbm_last_error", "lbm_step",
    "lbm_stream_collide", "lbm_current_state", "lbm_copy_state", "lbm_time", "lbm_scale", "lbm_moments",
    "lbm_get_pdfs", "lbm_sample_pdfs", "lbm_set_pdfs", "lbm_watchdog", "lbm_set_rates",
    "lbm_set_inlet", "lbm_adjoint_step",
    "lbm_objective", "lbm_init_vjp", "lbm_moments_noalloc",
]


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("equilibrium", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("dtype", ctypes.c_int32), ("pattern", ctypes.c_int32),
        ("compressible", ctypes.c_int32), ("adjoint_dtype", ctypes.c_int32),
        ("stencil", ctypes.c_int32),
        ("omega", ctypes.c_double), ("trt_magic", ctypes.c_double),
        ("accel", ctypes.c_double * 3), ("scale", ctypes.c_double),
        ("mrt_omega3", ctypes.c_double), ("mrt_omega4", ctypes.c_double),
        ("rounding", ctypes.c_int32), ("seed", ctypes.c_uint32),
        ("cache_policy", ctypes.c_int32),
        ("adjoint_solid", ctypes.c_int32),
        ("open_x", ctypes.c_int32),
        ("rho_out", ctypes.c_double),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_1803_04937_amd.build` "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    pp = ctypes.POINTER(lbm_params)
    sig = {
        "lbm_version": ([], ctypes.c_char_p),
        "lbm_velocity_set": ([ctypes.c_int32, P, P, P], None),
        "lbm_qstride": ([pp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "lbm_state_bytes": ([pp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_adjoint_bytes": ([pp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_validate": ([pp, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
        "lbm_links_bytes": ([pp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "lbm_choose_scale": ([ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
                             ctypes.c_int),
        "lbm_init": ([ctypes.POINTER(P), pp, P, P, P, P, P, P, P], ctypes.c_int),
        "lbm_destroy": ([P], None),
        "lbm_last_error": ([P], ctypes.c_char_p),
        "lbm_step": ([P, ctypes.c_int64], ctypes.c_int),
        "lbm_stream_collide": ([P, P, P, ctypes.c_int64], ctypes.c_int),
        "lbm_current_state": ([P], P),
        "lbm_copy_state": ([P, P, P], ctypes.c_int),
        "lbm_time": ([P], ctypes.c_int64),
        "lbm_scale": ([P], ctypes.c_double),
        "lbm_moments": ([P, P, P, P], ctypes.c_int),
        "lbm_get_pdfs": ([P, P], ctypes.c_int),
        "lbm_sample_pdfs": ([P, P, ctypes.c_int64, P], ctypes.c_int),
        "lbm_set_pdfs": ([P, P], ctypes.c_int),
        "lbm_watchdog": ([P, ctypes.c_double], ctypes.c_int),
        "lbm_set_rates": ([P, ctypes.c_double, P], ctypes.c_int),
        "lbm_set_inlet": ([P, P], ctypes.c_int),
        "lbm_adjoint_step": ([P, P, P, P, P], ctypes.c_int),
        "lbm_objective": ([P, ctypes.c_int, P, P, P], ctypes.c_int),
        "lbm_init_vjp": ([P, P, P, P], ctypes.c_int),
        "lbm_moments_noalloc": ([pp, P, P, ctypes.c_int64, ctypes.c_double, P, P, P, P],
                                ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _addr(x):
    """Device/host address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(rc: int, ctx=None):
    if rc != LBM_OK:
        msg = _lib.lbm_last_error(ctx)
        raise LBMError(rc, msg.decode() if msg else "")


def make_params(nx, ny, nz, periodic=(1, 1, 1), equilibrium=LBM_EQ_IMPROVED, collision=LBM_SRT,
                dtype=LBM_F32, pattern=LBM_TWO_GRID, compressible=0, adjoint_dtype=None,
                omega=1.0, trt_magic=3.0 / 16.0, accel=(0.0, 0.0, 0.0), scale=0.0,
                stencil=19, mrt_omega3=1.0, mrt_omega4=1.0, rounding=0,
                seed=0, cache_policy=0, adjoint_solid=0, open_x=0, rho_out=1.0) -> lbm_params:
    p = lbm_params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    for d in range(3):
        p.periodic[d] = int(periodic[d])
        p.accel[d] = float(accel[d])
    p.equilibrium = int(equilibrium)
    p.collision = int(collision)
    p.dtype = int(dtype)
    p.pattern = int(pattern)
    p.compressible = int(compressible)
    if adjoint_dtype is None:
        adjoint_dtype = LBM_F64 if dtype == LBM_F64 else LBM_F32
    p.adjoint_dtype = int(adjoint_dtype)
    p.stencil = int(stencil)
    p.omega = float(omega)
    p.trt_magic = float(trt_magic)
    p.scale = float(scale)
    p.mrt_omega3 = float(mrt_omega3)
    p.mrt_omega4 = float(mrt_omega4)
    p.rounding = int(rounding)
    p.seed = int(seed) & 0xFFFFFFFF
    p.cache_policy = int(cache_policy)
    p.adjoint_solid = int(adjoint_solid)
    p.open_x = int(open_x)
    p.rho_out = float(rho_out)
    return p


# ---------------------------------------------------------------------------
# One wrapper per entry point
# ---------------------------------------------------------------------------

def lbm_version() -> str:
    return _lib.lbm_version().decode()


def lbm_velocity_set(stencil: int = 19):
    qn = 27 if stencil == 27 else 19
    c = (ctypes.c_int32 * (3 * qn))()
    w = (ctypes.c_double * qn)()
    o = (ctypes.c_int32 * qn)()
    _lib.lbm_velocity_set(int(stencil), ctypes.addressof(c), ctypes.addressof(w),
                          ctypes.addressof(o))
    return ([tuple(c[3 * q:3 * q + 3]) for q in range(qn)], list(w), list(o))


def lbm_qstride(p: lbm_params) -> int:
    v = ctypes.c_int64()
    _check(_lib.lbm_qstride(ctypes.byref(p), ctypes.byref(v)))
    return v.value


def lbm_state_bytes(p: lbm_params) -> int:
    v = ctypes.c_size_t()
    _check(_lib.lbm_state_bytes(ctypes.byref(p), ctypes.byref(v)))
    return v.value


def lbm_adjoint_bytes(p: lbm_params) -> int:
    v = ctypes.c_size_t()
    _check(_lib.lbm_adjoint_bytes(ctypes.byref(p), ctypes.byref(v)))
    return v.value


def lbm_validate(p: lbm_params):
    buf = ctypes.create_string_buffer(512)
    rc = _lib.lbm_validate(ctypes.byref(p), buf, 512)
    return rc, buf.value.decode()


def lbm_links_bytes(p: lbm_params) -> int:
    v = ctypes.c_size_t()
    _check(_lib.lbm_links_bytes(ctypes.byref(p), ctypes.byref(v)))
    return v.value


def lbm_choose_scale(dtype: int, maxdev: float) -> float:
    v = ctypes.c_double()
    _check(_lib.lbm_choose_scale(int(dtype), float(maxdev), ctypes.byref(v)))
    return v.value


def lbm_init(p: lbm_params, solid, links, pdf0, pdf1, stream, rho_init, u_init) -> int:
    ctx = ctypes.c_void_p()
    rc = _lib.lbm_init(ctypes.byref(ctx), ctypes.byref(p), _addr(solid), _addr(links),
                       _addr(pdf0), _addr(pdf1), _addr(stream), _addr(rho_init),
                       _addr(u_init))
    _check(rc, None)
    return ctx.value


def lbm_destroy(ctx) -> None:
    _lib.lbm_destroy(ctx)


def lbm_last_error(ctx) -> str:
    m = _lib.lbm_last_error(ctx)
    return m.decode() if m else ""


def lbm_step(ctx, nsteps: int) -> None:
    _check(_lib.lbm_step(ctx, int(nsteps)), ctx)


def lbm_stream_collide(ctx, src, dst, t) -> None:
    _check(_lib.lbm_stream_collide(ctx, _addr(src), _addr(dst), int(t)), ctx)


def lbm_current_state(ctx) -> int:
    return _lib.lbm_current_state(ctx)


def lbm_copy_state(ctx, src, dst) -> None:
    _check(_lib.lbm_copy_state(ctx, _addr(src), _addr(dst)), ctx)


def lbm_time(ctx) -> int:
    return _lib.lbm_time(ctx)


def lbm_scale(ctx) -> float:
    return _lib.lbm_scale(ctx)


def lbm_moments(ctx, rho=None, u=None, want_sums: bool = False):
    sums = (ctypes.c_double * 4)() if want_sums else None
    _check(_lib.lbm_moments(ctx, _addr(rho), _addr(u),
                            ctypes.addressof(sums) if want_sums else None), ctx)
    return list(sums) if want_sums else None


def lbm_get_pdfs(ctx, canonical) -> None:
    _check(_lib.lbm_get_pdfs(ctx, _addr(canonical)), ctx)


def lbm_sample_pdfs(ctx, cells, n: int, out) -> None:
    _check(_lib.lbm_sample_pdfs(ctx, _addr(cells), int(n), _addr(out)), ctx)


def lbm_set_pdfs(ctx, canonical) -> None:
    _check(_lib.lbm_set_pdfs(ctx, _addr(canonical)), ctx)


def lbm_watchdog(ctx, rel_tol: float) -> None:
    _check(_lib.lbm_watchdog(ctx, float(rel_tol)), ctx)


def lbm_set_rates(ctx, omega: float, accel=None) -> None:
    a = None
    if accel is not None:
        a = (ctypes.c_double * 3)(*[float(v) for v in accel])
    _check(_lib.lbm_set_rates(ctx, float(omega), ctypes.addressof(a) if a is not None else None),
           ctx)


def lbm_set_inlet(ctx, u_in) -> None:
    _check(_lib.lbm_set_inlet(ctx, _addr(u_in)), ctx)


def lbm_adjoint_step(ctx, state_t, lam_next, lam_prev, grad=None) -> None:
    _check(_lib.lbm_adjoint_step(ctx, _addr(state_t), _addr(lam_next), _addr(lam_prev),
                                 _addr(grad)), ctx)


def lbm_objective(ctx, kind: int, state, out, lam) -> None:
    _check(_lib.lbm_objective(ctx, int(kind), _addr(state), _addr(out), _addr(lam)), ctx)


def lbm_init_vjp(ctx, u_init, lam0, grad_u) -> None:
    _check(_lib.lbm_init_vjp(ctx, _addr(u_init), _addr(lam0), _addr(grad_u)), ctx)


def lbm_moments_noalloc(p: lbm_params, links, state, t: int, scale: float, rho, u, sums,
                        stream) -> None:
    _check(_lib.lbm_moments_noalloc(ctypes.byref(p), _addr(links), _addr(state), int(t),
                                    float(scale), _addr(rho), _addr(u), _addr(sums),
                                    _addr(stream)), None)
