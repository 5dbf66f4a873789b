"""Shared helpers of the GPU parity tests: build the same case for the oracle
and for the GPU library, move arrays between numpy and the device, and the
tolerances used throughout.

Tolerances (per PDF value, f = post-collision PDF, w_q its weight):
  FP64 storage      |f_gpu - f_oracle| <= 1e-12 max(|f_oracle|, w_q)
  reduced storage   one step from the same stored state:
                    |f_gpu - f_oracle| <= half a storage ulp of the stored
                    quantity (f, or s (f - w) for the shifted formats; a
                    whole ulp with stochastic rounding)
                    + an FP32 arithmetic allowance of 2^-18 max(|f - w|, w_q / 8)
                    (about 64 rounding errors of the largest term of the
                    shifted update).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle

C, W, OPP = oracle.velocity_set()
W27 = oracle.velocity_set(27)[1]


def weights_for(nq):
    return W27 if nq == 27 else W

DTYPE_NAMES = {"f64": 0, "f32": 1, "f32s": 2, "f16s": 3, "bf16s": 4}


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def case(nx, ny, nz, periodic=(1, 1, 1), improved=True, trt=False, omega=1.2, magic=3 / 16,
         accel=(0.0, 0.0, 0.0), solid=None, compressible=False, stencil=19, mrt=None):
    """(oracle.Config, Lattice keyword arguments) of one case.  mrt: None or
    the MRT rates (omega3, omega4) of the third- and fourth-order moments."""
    cfg = oracle.Config(nx, ny, nz, periodic=tuple(periodic), improved=improved, trt=trt,
                        compressible=compressible, omega=omega, magic=magic, accel=tuple(accel),
                        solid=solid, stencil=stencil)
    eq_name = {0: "standard", 1: "improved", 2: "improved3"}[int(improved)]
    kw = dict(periodic=tuple(periodic), equilibrium=eq_name,
              collision="trt" if trt else "srt", compressible=compressible, omega=omega,
              trt_magic=magic, accel=tuple(accel), stencil=stencil)
    if mrt is not None:
        cfg = oracle.Config(nx, ny, nz, periodic=tuple(periodic), improved=improved,
                            compressible=compressible, omega=omega, accel=tuple(accel),
                            solid=solid, mrt=True, omega3=mrt[0], omega4=mrt[1])
        kw.update(collision="mrt", mrt_omega3=mrt[0], mrt_omega4=mrt[1])
    if solid is not None:
        kw["solid"] = dev(solid, torch.uint8)
    return cfg, kw


def lattice(cfg, kw, u, rho=None, dtype="f64", pattern="two_grid", scale=0.0, **extra):
    from paper_1803_04937_amd import Lattice
    return Lattice(cfg.nx, cfg.ny, cfg.nz, u=dev(u), rho=None if rho is None else dev(rho),
                   dtype=dtype, pattern=pattern, scale=scale, **kw, **extra)


def random_blobs(shape, seed, frac=0.08):
    """Seeded solid mask of random boxes covering roughly frac of the cells."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    m = np.zeros(shape, np.uint8)
    while m.mean() < frac:
        z, y, x = rng.integers(0, nz), rng.integers(0, ny), rng.integers(0, nx)
        dz, dy, dx = rng.integers(1, 4, size=3)
        m[z:z + dz, y:y + dy, x:x + dx] = 1
    return m


def assert_f64_parity(f_gpu, f_ref, what=""):
    nq = f_ref.shape[0]
    bound = 1e-12 * np.maximum(np.abs(f_ref), weights_for(nq).reshape((nq,) + (1,) * (f_ref.ndim - 1)))
    err = np.abs(f_gpu - f_ref)
    worst = np.max(err / bound)
    assert worst <= 1.0, f"{what}: max error {err.max():.3e}, {worst:.2f} x bound"


def ulp_half(x, dtype):
    """Half a unit in the last place of |x| in the storage format."""
    x = np.abs(x)
    if dtype == "f16s":
        e = np.floor(np.log2(np.maximum(x, 2.0 ** -14)))
        return 0.5 * 2.0 ** (e - 10)
    if dtype == "bf16s":
        e = np.floor(np.log2(np.maximum(x, 2.0 ** -126)))
        return 0.5 * 2.0 ** (e - 7)
    e = np.floor(np.log2(np.maximum(x, 2.0 ** -126)))
    return 0.5 * 2.0 ** (e - 23)


def reduced_bound(f_ref, dtype, scale, rounding="nearest"):
    """Per-value error bound of one reduced-precision step (see module doc).
    Stochastic rounding of the 16-bit formats may land on either neighbour:
    a whole ulp instead of half."""
    nq = f_ref.shape[0]
    wq = weights_for(nq).reshape((nq,) + (1,) * (f_ref.ndim - 1))
    d = f_ref - wq
    arith = 2.0 ** -18 * np.maximum(np.abs(d), wq / 8)
    if dtype == "f32":
        return ulp_half(np.abs(f_ref) + arith, "f32") + arith
    if dtype == "f32s":
        return ulp_half(np.abs(d) + arith, "f32") + arith
    s = scale
    k = 2.0 if rounding == "stochastic" else 1.0
    return k * ulp_half(s * (np.abs(d) + arith), dtype) / s + arith


def push_targets(cfg, cells):
    """Where the adjoint of one pull step writes mu_r of cell x (flat index):
    slot (r, x - c_r) when that cell is inside (periodic wrap) and fluid,
    else (rbar, x) (half-way bounce-back).  Returns (direction, cell) index
    arrays of shape (len(cells), Q), from the definition of the pull."""
    import oracle
    c, _, opp = oracle.velocity_set(cfg.stencil)
    cells = np.asarray(cells, dtype=np.int64)
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    x, y, z = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    arr = np.empty((cells.size, cfg.q), np.int64)
    tgt = np.empty((cells.size, cfg.q), np.int64)
    solid = None if cfg.solid is None else np.asarray(cfg.solid).reshape(-1).astype(bool)
    for r in range(cfg.q):
        xs, ys, zs = x - c[r, 0], y - c[r, 1], z - c[r, 2]
        inside = np.ones(cells.size, bool)
        for v, n, per in ((xs, nx, cfg.periodic[0]), (ys, ny, cfg.periodic[1]),
                          (zs, nz, cfg.periodic[2])):
            if per:
                v %= n
            else:
                inside &= (v >= 0) & (v < n)
        src = (np.clip(zs, 0, nz - 1) * ny + np.clip(ys, 0, ny - 1)) * nx + np.clip(xs, 0, nx - 1)
        fluid = inside if solid is None else inside & ~solid[src]
        arr[:, r] = np.where(fluid, r, opp[r])
        tgt[:, r] = np.where(fluid, src, cells)
    return arr, tgt


# Per-element bound of an adjoint field (lambda) against the oracle:
# |got - want| <= tol * max(|want|, floor * max|want|).  The floor covers
# values that are small because their terms cancel: their rounding error
# scales with the terms (about max|lambda|), not with the value.
ADJ_TOL = {"f64": (1e-12, 1e-2), "f32": (2e-6, 0.25)}


def assert_adjoint_parity(got, want, dtype, what=""):
    tol, floor = ADJ_TOL["f64" if dtype == "f64" else "f32"]
    m = np.abs(want).max()
    bound = tol * np.maximum(np.abs(want), floor * m)
    err = np.abs(got - want)
    worst = (err / bound).max()
    # error profile for the record: worst error relative to the largest value,
    # and among the values below a tenth of it
    small = np.abs(want) < 0.1 * m
    prof = (err.max() / m, (err[small].max() / m) if small.any() else 0.0)
    print(f"adjoint parity {what} {dtype}: worst {worst:.3f} x bound, "
          f"max err / max {prof[0]:.2e}, small-value err / max {prof[1]:.2e}")
    assert worst <= 1.0, f"{what}: {worst:.2f} x bound"
