"""Python-side owner of one lattice: allocates the caller-owned device buffers
with torch and drives the C ABI through ``capi``.  Every step of the update
runs in the HIP kernels of liblbm.so; torch is used only for device memory
and the current stream.
"""
from __future__ import annotations

import torch

from . import capi
from .capi import LBMError

EQUILIBRIA = {"standard": capi.LBM_EQ_STANDARD, "improved": capi.LBM_EQ_IMPROVED,
              "improved3": capi.LBM_EQ_IMPROVED3}
COLLISIONS = {"srt": capi.LBM_SRT, "trt": capi.LBM_TRT, "mrt": capi.LBM_MRT,
              "kbc": capi.LBM_KBC}
DTYPES = {"f64": capi.LBM_F64, "f32": capi.LBM_F32, "f32s": capi.LBM_F32_SHIFTED,
          "f16s": capi.LBM_F16_SHIFTED, "bf16s": capi.LBM_BF16_SHIFTED}
PATTERNS = {"two_grid": capi.LBM_TWO_GRID, "aa": capi.LBM_AA}
ROUNDINGS = {"nearest": capi.LBM_ROUND_NEAREST, "stochastic": capi.LBM_ROUND_STOCHASTIC}
CACHE_POLICIES = {"auto": capi.LBM_CACHE_AUTO, "stream": capi.LBM_CACHE_STREAM,
                  "keep": capi.LBM_CACHE_KEEP}
ADJOINT_SOLID = {"copy": capi.LBM_ADJ_SOLID_COPY, "skip": capi.LBM_ADJ_SOLID_SKIP}
STORAGE_TORCH = {capi.LBM_F64: torch.float64, capi.LBM_F32: torch.float32,
                 capi.LBM_F32_SHIFTED: torch.float32, capi.LBM_F16_SHIFTED: torch.float16,
                 capi.LBM_BF16_SHIFTED: torch.bfloat16}
ADJ_TORCH = {capi.LBM_F64: torch.float64, capi.LBM_F32: torch.float32}


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


def require_gpu(device=None):
    if not torch.cuda.is_available():
        raise LBMError(capi.LBM_EHIP, "no ROCm GPU visible: the library runs on gfx950 only")
    return torch.device(device or "cuda")


class Lattice:
    """A D3Q19 or D3Q27 lattice (shape nz x ny x nx, x fastest) with its PDF
    buffers.

    u: initial velocity, tensor (3, nz, ny, nx); rho: optional density
    (nz, ny, nx); solid: optional mask (nz, ny, nx), nonzero = solid.
    adjoint_solid: "copy" (adjoint_step copies lambda through solid cells)
    or "skip" (leaves it unwritten there).
    inlet: with open_x, the inflow velocity (3, nz, ny) of the inlet cells
    (x = 0); rho_out: the outlet density.
    """

    def __init__(self, nx, ny, nz, *, u, rho=None, solid=None, periodic=(1, 1, 1),
                 equilibrium="improved", collision="srt", dtype="f32", pattern="two_grid",
                 compressible=False, omega=1.0, trt_magic=3.0 / 16.0, accel=(0.0, 0.0, 0.0),
                 scale=0.0, stencil=19, mrt_omega3=1.0, mrt_omega4=1.0, rounding="nearest",
                 seed=0, cache_policy="auto", adjoint_solid="copy", open_x=False, inlet=None,
                 rho_out=1.0, device=None, stream=None):
        self.device = require_gpu(device)
        self.params = capi.make_params(
            nx, ny, nz, periodic=periodic, equilibrium=_code(EQUILIBRIA, equilibrium),
            collision=_code(COLLISIONS, collision), dtype=_code(DTYPES, dtype),
            pattern=_code(PATTERNS, pattern), compressible=int(bool(compressible)), omega=omega,
            trt_magic=trt_magic, accel=accel, scale=scale, stencil=stencil,
            mrt_omega3=mrt_omega3, mrt_omega4=mrt_omega4,
            rounding=_code(ROUNDINGS, rounding), seed=seed,
            cache_policy=_code(CACHE_POLICIES, cache_policy),
            adjoint_solid=_code(ADJOINT_SOLID, adjoint_solid), open_x=int(bool(open_x)),
            rho_out=rho_out)
        rc, why = capi.lbm_validate(self.params)
        if rc != capi.LBM_OK:
            raise LBMError(rc, why)
        self.shape = (int(nz), int(ny), int(nx))
        self.q = int(stencil)
        self.ncells = int(nx) * int(ny) * int(nz)
        self.qstride = capi.lbm_qstride(self.params)
        self.storage_dtype = STORAGE_TORCH[self.params.dtype]
        self.adjoint_dtype = ADJ_TORCH[self.params.adjoint_dtype]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.solid = None
        self.links = None
        if solid is not None:
            self.solid = torch.as_tensor(solid).to(self.device, torch.uint8).contiguous()
            assert self.solid.shape == self.shape
            # uint32 link words (one per cell) and the list of blocks with a
            # fluid cell, written by lbm_init (held as int32)
            nbytes = capi.lbm_links_bytes(self.params)
            self.links = torch.empty(nbytes // 4, dtype=torch.int32, device=self.device)
        u = torch.as_tensor(u).to(self.device, torch.float64).contiguous()
        assert u.shape == (3,) + self.shape, u.shape
        if rho is not None:
            rho = torch.as_tensor(rho).to(self.device, torch.float64).contiguous()
            assert rho.shape == self.shape
        self.buffers = [self.new_state()]
        if self.params.pattern == capi.LBM_TWO_GRID:
            self.buffers.append(self.new_state())
        self._ctx = None
        self._ctx = capi.lbm_init(self.params, self.solid, self.links, self.buffers[0],
                                  self.buffers[1] if len(self.buffers) > 1 else None,
                                  self.stream.cuda_stream, rho, u)
        self.inlet = None
        if open_x:
            self.set_inlet(torch.zeros((3, self.shape[0], self.shape[1])) if inlet is None
                           else inlet)

    # -- buffers -------------------------------------------------------------
    def new_state(self) -> torch.Tensor:
        """A state buffer of this lattice's layout: tensor (nz, Q, qstride),
        the Q direction arrays of each z-plane contiguous."""
        return torch.empty((self.shape[0], self.q, self.qstride), dtype=self.storage_dtype,
                           device=self.device)

    def new_adjoint(self, zero: bool = True) -> torch.Tensor:
        """An adjoint field: tensor (nz, Q, qstride) of the adjoint dtype."""
        f = torch.zeros if zero else torch.empty
        return f((self.shape[0], self.q, self.qstride), dtype=self.adjoint_dtype,
                 device=self.device)

    def state_view(self, buf: torch.Tensor) -> torch.Tensor:
        """(Q, nz, ny, nx) view (not a copy) of the cells of a state or adjoint
        buffer."""
        nz, ny, nx = self.shape
        planes = buf.view(nz, self.q, self.qstride)[:, :, :ny * nx]
        return planes.unflatten(2, (ny, nx)).permute(1, 0, 2, 3)

    @property
    def ctx(self):
        if self._ctx is None:
            raise LBMError(capi.LBM_ESTATE, "lattice is closed")
        return self._ctx

    @property
    def state(self) -> torch.Tensor:
        """The buffer holding the current state."""
        ptr = capi.lbm_current_state(self.ctx)
        for b in self.buffers:
            if b.data_ptr() == ptr:
                return b
        raise LBMError(capi.LBM_ESTATE, "current state buffer not found")

    @property
    def time(self) -> int:
        return capi.lbm_time(self.ctx)

    @property
    def scale(self) -> float:
        return capi.lbm_scale(self.ctx)

    # -- forward -------------------------------------------------------------
    def step(self, n: int = 1) -> None:
        capi.lbm_step(self.ctx, n)

    def stream_collide(self, src: torch.Tensor, dst: torch.Tensor, t: int = 0) -> None:
        """One two-grid step from src (the state at time t) into dst."""
        capi.lbm_stream_collide(self.ctx, src, dst, t)

    def copy_state(self, src: torch.Tensor, dst: torch.Tensor) -> None:
        capi.lbm_copy_state(self.ctx, src, dst)

    def moments(self):
        """(rho (nz,ny,nx), u (3,nz,ny,nx)) FP64 device tensors."""
        rho = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        capi.lbm_moments(self.ctx, rho, u)
        return rho, u

    def totals(self):
        """FP64 [mass, momentum_x, momentum_y, momentum_z] over fluid cells."""
        return capi.lbm_moments(self.ctx, None, None, want_sums=True)

    def get_pdfs(self) -> torch.Tensor:
        out = torch.empty((self.q,) + self.shape, dtype=torch.float64, device=self.device)
        capi.lbm_get_pdfs(self.ctx, out)
        return out

    def sample_pdfs(self, cells) -> torch.Tensor:
        """Canonical f*_q at the given flat cell indices: tensor (n, Q) FP64."""
        cells = torch.as_tensor(cells, dtype=torch.int64).to(self.device).contiguous()
        out = torch.empty((cells.numel(), self.q), dtype=torch.float64, device=self.device)
        capi.lbm_sample_pdfs(self.ctx, cells, cells.numel(), out)
        return out

    def set_pdfs(self, f) -> None:
        f = torch.as_tensor(f).to(self.device, torch.float64).contiguous()
        assert f.shape == (self.q,) + self.shape
        capi.lbm_set_pdfs(self.ctx, f)

    def watchdog(self, rel_tol: float = 1e-6) -> None:
        capi.lbm_watchdog(self.ctx, rel_tol)

    def set_rates(self, omega: float, accel=None) -> None:
        capi.lbm_set_rates(self.ctx, omega, accel)

    def set_inlet(self, u_in) -> None:
        """Inflow velocity (3, nz, ny) of the inlet cells of an open lattice;
        kept on the device as long as the lattice uses it."""
        u_in = torch.as_tensor(u_in).to(self.device, torch.float64).contiguous()
        assert u_in.shape == (3, self.shape[0], self.shape[1]), u_in.shape
        capi.lbm_set_inlet(self.ctx, u_in)
        self.inlet = u_in

    # -- adjoint -------------------------------------------------------------
    def adjoint_step(self, state_t, lam_next, lam_prev, grad=None) -> None:
        capi.lbm_adjoint_step(self.ctx, state_t, lam_next, lam_prev, grad)

    def objective(self, kind: int, state, out, lam) -> None:
        capi.lbm_objective(self.ctx, kind, state, out, lam)

    def init_vjp(self, u_init, lam0, grad_u) -> None:
        capi.lbm_init_vjp(self.ctx, u_init, lam0, grad_u)

    # -- lifetime ------------------------------------------------------------
    def close(self) -> None:
        if self._ctx is not None:
            capi.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
