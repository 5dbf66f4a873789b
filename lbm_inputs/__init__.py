"""Seeded synthetic inputs: initial velocity fields and solid masks.

This module is shared by the tests (which feed the same inputs to the oracle
and to the GPU library) and by the benchmark.  It holds none of the lattice
Boltzmann arithmetic: it only produces velocity fields u (shape (3, nz, ny,
nx), float64, x fastest) and uint8 solid masks (shape (nz, ny, nx), 1 =
solid).  Coordinates are integer cell indices.

Fields:
  taylor_green      3-D Taylor-Green vortex (periodic box)
  taylor_green_2d   z-invariant 2-D Taylor-Green vortex (exact decaying
                    Navier-Stokes solution)
  shear_wave        single z-invariant shear wave u_x = A sin(2 pi y / ny)
  shear_waves       superposition of seeded random-phase shear waves
  spectrum_field    seeded isotropic field with E(k) ~ k^4 exp(-2 (k/k0)^2)
  duct_poiseuille   series solution of the square-duct Poiseuille flow
  perturbation      seeded uniform noise
  tube_mask         axisymmetric constricted tube along x
"""
from __future__ import annotations

import numpy as np


def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def taylor_green(n: int, u0: float):
    """u = u0 (sin X cos Y cos Z, -cos X sin Y cos Z, 0), X = 2 pi i / n."""
    x, y, z = _grid((n, n, n))
    X, Y, Z = (2 * np.pi * v / n for v in (x, y, z))
    u = np.zeros((3, n, n, n))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    return u


def taylor_green_2d(n: int, u0: float, nz: int = 1):
    """u = u0 (sin X cos Y, -cos X sin Y, 0) on an n x n x nz box."""
    x, y, _ = _grid((nz, n, n))
    X, Y = 2 * np.pi * x / n, 2 * np.pi * y / n
    u = np.zeros((3, nz, n, n))
    u[0] = u0 * np.sin(X) * np.cos(Y)
    u[1] = -u0 * np.cos(X) * np.sin(Y)
    return u


def shear_wave(shape, amp: float, mode: int = 1):
    """u_x = amp sin(2 pi mode y / ny), other components zero."""
    x, y, z = _grid(shape)
    u = np.zeros((3,) + tuple(shape))
    u[0] = amp * np.sin(2 * np.pi * mode * y / shape[1])
    return u


def shear_waves(shape, seed: int, nmodes: int = 8, kmax: float = 4.0, amax: float = 0.03):
    """Sum over m of A_m e_m sin(2 pi k_m . x / N + phi_m).

    k_m is drawn uniformly from the integer vectors with 0 < |k| <= kmax,
    e_m is a random unit vector orthogonal to k_m (so every mode is
    divergence-free), A_m ~ U(0, amax), phi_m ~ U(0, 2 pi).  N is the box
    length along each axis, so every mode is periodic.
    """
    rng = np.random.default_rng(seed)
    r = int(np.floor(kmax))
    ks = [np.array(k) for k in np.ndindex(2 * r + 1, 2 * r + 1, 2 * r + 1)]
    ks = [k - r for k in ks]
    ks = [k for k in ks if 0 < np.dot(k, k) <= kmax * kmax]
    x, y, z = _grid(shape)
    nz, ny, nx = shape
    u = np.zeros((3,) + tuple(shape))
    for _ in range(nmodes):
        k = ks[rng.integers(len(ks))].astype(np.float64)
        v = rng.standard_normal(3)
        e = v - np.dot(v, k) / np.dot(k, k) * k
        e /= np.linalg.norm(e)
        a = rng.uniform(0.0, amax)
        phi = rng.uniform(0.0, 2 * np.pi)
        phase = 2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + phi
        s = a * np.sin(phase)
        for d in range(3):
            u[d] += e[d] * s
    return u


def spectrum_field(n: int, seed: int, k0: float = 8.0, umax: float = 0.08, dtype=np.float64):
    """Isotropic random field with energy spectrum E(k) ~ k^4 exp(-2 (k/k0)^2).

    Each integer mode 0 < |k| <= n/2 gets a complex Gaussian vector projected
    orthogonal to k with amplitude sqrt(E(|k|) / (4 pi |k|^2)); the real
    field comes from an inverse real FFT and is rescaled to max |u| = umax.
    """
    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(n, 1.0 / n)
    ky = np.fft.fftfreq(n, 1.0 / n)
    kx = np.fft.rfftfreq(n, 1.0 / n)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    kk = np.sqrt(k2)
    spec = kk ** 4 * np.exp(-2.0 * (kk / k0) ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where((kk > 0) & (kk <= n / 2), np.sqrt(spec / (4 * np.pi * k2)), 0.0)
    comps = []
    for _ in range(3):
        comps.append(rng.standard_normal(KX.shape) + 1j * rng.standard_normal(KX.shape))
    kvec = (KX, KY, KZ)
    with np.errstate(divide="ignore", invalid="ignore"):
        dot = sum(c * k for c, k in zip(comps, kvec)) / np.where(k2 > 0, k2, 1.0)
    u = np.empty((3, n, n, n), dtype=dtype)
    for d in range(3):
        hat = (comps[d] - dot * kvec[d]) * amp
        u[d] = np.fft.irfftn(hat, s=(n, n, n), axes=(0, 1, 2))
    del comps, dot
    mag = np.sqrt((u.astype(np.float64) ** 2).sum(axis=0)).max()
    u *= umax / mag
    return u


def duct_poiseuille(nx: int, ny: int, nz: int, accel: float, nu: float, nterms: int = 200):
    """Square-duct Poiseuille flow along x, walls at y, z = -1/2 and n - 1/2.

    u_x(y, z) = 16 a b^2 / (nu pi^3) sum_{n odd} (-1)^((n-1)/2)
                [1 - cosh(n pi z' / 2b) / cosh(n pi / 2)] cos(n pi y' / 2b) / n^3
    with half-width b = ny / 2 and y', z' measured from the duct centre.
    Requires ny == nz.
    """
    assert ny == nz
    b = ny / 2.0
    yc = (np.arange(ny) - (ny - 1) / 2.0)
    zc = (np.arange(nz) - (nz - 1) / 2.0)
    Z, Y = np.meshgrid(zc, yc, indexing="ij")
    s = np.zeros_like(Y)
    for m in range(nterms):
        k = 2 * m + 1
        arg = k * np.pi / (2 * b)
        # cosh(k pi z/2b)/cosh(k pi/2), written with exponentials to avoid overflow
        ratio = (np.exp(arg * Z - k * np.pi / 2) + np.exp(-arg * Z - k * np.pi / 2)) / (
            1.0 + np.exp(-k * np.pi))
        s += (-1) ** m * (1.0 - ratio) * np.cos(arg * Y) / k ** 3
    ux = 16.0 * accel * b * b / (nu * np.pi ** 3) * s
    u = np.zeros((3, nz, ny, nx))
    u[0] = ux[:, :, None]
    return u


def perturbation(shape, seed: int, amp: float):
    """Uniform noise U(-amp, amp) per component, shape (3,) + shape."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(3,) + tuple(shape))


def tube_mask(nx: int, ny: int, nz: int, r0: float = 80.0, depth: float = 0.5,
              centre: float | None = None, width: float = 60.0):
    """Axisymmetric constricted tube along x.

    Radius r(x) = r0 (1 - depth exp(-((x - centre) / width)^2)); a cell is
    solid when its distance from the tube axis (at the cross-section centre)
    exceeds r(x).
    """
    if centre is None:
        centre = nx / 2.0
    x = np.arange(nx, dtype=np.float64)
    r = r0 * (1.0 - depth * np.exp(-((x - centre) / width) ** 2))
    yc, zc = (ny - 1) / 2.0, (nz - 1) / 2.0
    Z, Y = np.meshgrid(np.arange(nz) - zc, np.arange(ny) - yc, indexing="ij")
    rc = np.sqrt(Y * Y + Z * Z)
    return (rc[:, :, None] > r[None, None, :]).astype(np.uint8)
