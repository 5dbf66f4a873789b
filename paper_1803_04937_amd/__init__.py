"""MI355X (gfx950) D3Q19 lattice Boltzmann stream-collide library.

Implements the fused D3Q19 update of Bauer & Ruede (arXiv:1803.04937) with
the standard and the improved (moment-matched) equilibrium, SRT/TRT
collision, body force, half-way bounce-back, two-grid and AA streaming, FP64
/ FP32 / shifted FP32 / FP16 / BF16 storage, and a hand-written adjoint.

Layout of the package:
  csrc/        HIP kernels and the C ABI (include/lbm.h), built into liblbm.so
  build.py     hipcc build of liblbm.so
  capi.py      ctypes binding, one function per C entry point
  lattice.py   Lattice: torch-allocated buffers + the C ABI
  autograd.py  torch.autograd.Function over a rollout, checkpointed adjoint

Importing ``capi``, ``Lattice`` or ``rollout_objective`` loads liblbm.so and
raises if it is not built.  There is no CPU fallback.
"""
from __future__ import annotations

__all__ = ["capi", "Lattice", "LBMError", "rollout_objective", "RolloutConfig"]


def __getattr__(name):
    import importlib
    if name in ("capi", "lattice", "autograd", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    if name == "Lattice":
        return importlib.import_module(f"{__name__}.lattice").Lattice
    if name == "LBMError":
        return importlib.import_module(f"{__name__}.capi").LBMError
    if name in ("rollout_objective", "RolloutConfig"):
        return getattr(importlib.import_module(f"{__name__}.autograd"), name)
    raise AttributeError(name)
