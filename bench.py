"""Benchmark of the D3Q19 stream-collide + adjoint hot path on one MI355X.

Workload (default): 256^3 periodic lattice, improved equilibrium (D3Q19-I),
TRT with Lambda = 3/16, omega = 1.8, FP32 storage, two-grid pull streaming,
seeded random-phase shear-wave initial field (8 modes, |k| <= 4, amplitudes
U(0, 0.03)).  One timed step = one fused forward stream-collide update of
every cell followed by one adjoint update of every cell (FP32 adjoint field,
FP64 parameter-gradient reduction): the full differentiable lattice update.

Printed: one JSON line with MLUPS (million lattice-cell updates per second,
one update = forward + adjoint of one cell), the roofline of the dominant
kernel from HIP events, per-kernel breakdowns, a few secondary
configurations, and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 256


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip secondary configurations")
    ap.add_argument("--n", type=int, default=N, help="cube edge (default 256)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run one plain device copy of 19 n^3 floats (profiler reference)")
    return ap.parse_args()


def kernel_source_hash():
    """sha256 over the HIP sources, to tell whether recorded counters are current."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1803_04937_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel_name):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by the plain-copy calibration), or
    None if absent or taken from different kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("per_launch", {}).get(kernel_name)
    return None if k is None else int(round(k["bytes"]))


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _events(torch, k):
    return [torch.cuda.Event(enable_timing=True) for _ in range(k)]


def timed_forward(torch, lat, steps, warmup):
    """Average duration (ms) of one fused forward step launched by lbm_step."""
    lat.step(warmup)
    e0, e1 = _events(torch, 2)
    torch.cuda.synchronize()
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def timed_adjoint(torch, lat, steps, warmup):
    """Average duration (ms) of one adjoint step with parameter gradients,
    linearised at the lattice's current state."""
    lam = [lat.new_adjoint(), lat.new_adjoint()]
    grad = torch.zeros(4, dtype=torch.float64, device=lat.device)
    out = torch.zeros(4, dtype=torch.float64, device=lat.device)
    lat.objective(0, lat.state, out, lam[0])
    for i in range(warmup):
        lat.adjoint_step(lat.state, lam[i % 2], lam[1 - i % 2], grad)
    e0, e1 = _events(torch, 2)
    torch.cuda.synchronize()
    e0.record()
    for i in range(steps):
        lat.adjoint_step(lat.state, lam[i % 2], lam[1 - i % 2], grad)
    e1.record()
    torch.cuda.synchronize()
    if not torch.isfinite(grad).all():
        raise RuntimeError("non-finite adjoint gradient")
    return e0.elapsed_time(e1) / steps


def _rate(ms, cells, bytes_per_cell):
    gbs = bytes_per_cell * cells / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 5), "mlups": round(cells / (ms * 1e-3) / 1e6, 1),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def timed_fwd_adj(torch, lat, steps, warmup):
    """Average durations (ms) of one forward step (lbm_stream_collide) and one
    adjoint step with parameter gradients, alternating as in a rollout."""
    A, B = lat.buffers
    lam = [lat.new_adjoint(), lat.new_adjoint()]
    grad = torch.zeros(4, dtype=torch.float64, device=lat.device)
    out = torch.zeros(4, dtype=torch.float64, device=lat.device)
    lat.objective(1, A, out, lam[0])
    ev = [_events(torch, 3) for _ in range(steps)]
    for i in range(warmup + steps):
        src, dst = (A, B) if i % 2 == 0 else (B, A)
        e = ev[i - warmup] if i >= warmup else None
        if e:
            e[0].record()
        lat.stream_collide(src, dst, i)
        if e:
            e[1].record()
        lat.adjoint_step(src, lam[i % 2], lam[1 - i % 2], grad)
        if e:
            e[2].record()
    torch.cuda.synchronize()
    if not torch.isfinite(grad).all():
        raise RuntimeError("non-finite adjoint gradient")
    return (sum(e[0].elapsed_time(e[1]) for e in ev) / steps,
            sum(e[1].elapsed_time(e[2]) for e in ev) / steps)


def workload_extras(torch, Lattice, lbm_inputs, dev):
    """The other configured workloads, timed outside the main region."""
    out = {}
    # 512^3 periodic D3Q19-I TRT omega = 1.98 in every storage format (the
    # FP16-storage speedup at its configured size); the rate does not depend
    # on the field, so these start from seeded noise
    n = 512
    cells = n ** 3
    u = torch.tensor(lbm_inputs.perturbation((n, n, n), seed=3, amp=0.02), device=dev)
    ms512 = {}
    for dt, size in (("f32", 4), ("f32s", 4), ("f16s", 2), ("bf16s", 2)):
        _log(f"extra 512^3 {dt}")
        lat = Lattice(n, n, n, u=u, equilibrium="improved", collision="trt", omega=1.98,
                      dtype=dt, device=dev)
        ms512[dt] = timed_forward(torch, lat, 20, 3)
        out[f"fwd_512_{dt}_I_trt"] = _rate(ms512[dt], cells, 2 * 19 * size)
        lat.close()
        del lat
        torch.cuda.empty_cache()
    del u
    torch.cuda.empty_cache()
    out["fwd_512_f16s_speedup_vs_f32"] = round(ms512["f32"] / ms512["f16s"], 3)
    # 512 x 128 x 128 duct (walls on y, z), D3Q19-I SRT omega = 1.9, g_x = 1e-6,
    # FP32 forward + FP32 adjoint
    nx, ny, nz = 512, 128, 128
    nu = (1 / 1.9 - 0.5) / 3
    u = torch.tensor(lbm_inputs.duct_poiseuille(nx, ny, nz, 1e-6, nu), device=dev)
    _log("extra duct forward + adjoint")
    lat = Lattice(nx, ny, nz, u=u, periodic=(1, 0, 0), equilibrium="improved",
                  collision="srt", omega=1.9, accel=(1e-6, 0, 0), dtype="f32", device=dev)
    fms, ams = timed_fwd_adj(torch, lat, 20, 3)
    c = nx * ny * nz
    out["duct_512x128x128_srt_f32"] = {"fwd": _rate(fms, c, 152), "adj": _rate(ams, c, 228),
                                       "step_mlups": round(c / ((fms + ams) * 1e-3) / 1e6, 1)}
    lat.close()
    del lat, u
    torch.cuda.empty_cache()
    # 768 x 192 x 192 constricted tube (mask), D3Q19-I TRT omega = 1.95,
    # FP16 state + FP32 adjoint (lambda at solid cells skipped); bytes per
    # fluid cell (every cell also reads its 4-byte link word)
    nx, ny, nz = 768, 192, 192
    solid = lbm_inputs.tube_mask(nx, ny, nz)
    nfluid = int((solid == 0).sum())
    sd = torch.tensor(solid, dtype=torch.uint8, device=dev)
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float64, device=dev)
    _log("extra tube forward + adjoint")
    lat = Lattice(nx, ny, nz, u=u, solid=sd, equilibrium="improved", collision="trt",
                  omega=1.95, accel=(2e-6, 0, 0), dtype="f16s", adjoint_solid="skip",
                  device=dev)
    fms, ams = timed_fwd_adj(torch, lat, 20, 3)
    c = nx * ny * nz
    link = 4 * c / nfluid
    out["tube_768x192x192_trt_f16"] = {
        "fluid_cells": nfluid, "fwd": _rate(fms, nfluid, 76 + link),
        "adj": _rate(ams, nfluid, 190 + link),
        "step_mflups": round(nfluid / ((fms + ams) * 1e-3) / 1e6, 1)}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    # the same tube opened at both x faces (Sec. 5.2): parabolic inflow at
    # x = -1/2, constant pressure at x = nx - 1/2, KBC with Maxwellian moments,
    # FP32 forward
    _log("extra open tube (KBC)")
    yc, zc = (ny - 1) / 2, (nz - 1) / 2
    yy, zz = np.meshgrid(np.arange(ny) - yc, np.arange(nz) - zc)
    r2 = (yy ** 2 + zz ** 2) / 80.0 ** 2
    inlet = np.zeros((3, nz, ny))
    inlet[0] = np.where(r2 < 1, 0.02 * (1 - r2), 0.0)
    lat = Lattice(nx, ny, nz, u=u, solid=sd, periodic=(0, 1, 1), equilibrium="improved",
                  collision="kbc", omega=1.98, dtype="f32", open_x=True, rho_out=1.0,
                  inlet=torch.tensor(inlet, device=dev), device=dev)
    ms = timed_forward(torch, lat, 20, 3)
    out["open_tube_768x192x192_kbc_f32"] = _rate(ms, nfluid, 152 + link)
    lat.close()
    del lat, u, sd
    torch.cuda.empty_cache()
    return out


def cpu_oracle_baseline(lbm_inputs, n, steps=4):
    """The FP64 oracle timed on the host cores: `steps` forward steps and
    `steps` adjoint steps of the n^3 bench workload, MLUPS of forward +
    adjoint cell updates (the unit of the GPU value)."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    _log(f"cpu oracle sample on {cores} threads")
    cfg = oracle.Config(n, n, n, improved=True, trt=True, omega=1.8, magic=3.0 / 16.0)
    f = oracle.init(cfg, lbm_inputs.shear_waves((n, n, n), seed=0))
    t0 = time.perf_counter()
    g = oracle.step(cfg, f, steps)
    t_fwd = time.perf_counter() - t0
    lam = oracle.objective(cfg, g, 0)[1]
    t0 = time.perf_counter()
    for _ in range(steps):
        lam, _ = oracle.adjoint_step(cfg, f, lam)
    t_adj = time.perf_counter() - t0
    cells = n ** 3
    return {"value": round(steps * cells / (t_fwd + t_adj) / 1e6, 3),
            "unit": "MLUPS (forward + adjoint)", "cores": cores, "kind": "oracle",
            "forward_only_mlups": round(steps * cells / t_fwd / 1e6, 3),
            "adjoint_only_mlups": round(steps * cells / t_adj / 1e6, 3),
            "sample": f"FP64 C oracle, {n}^3 D3Q19-I TRT: {steps} forward steps "
                      f"({t_fwd:.1f} s) and {steps} adjoint steps ({t_adj:.1f} s), "
                      f"{platform.processor() or platform.machine()}"}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import lbm_inputs
    from paper_1803_04937_amd import Lattice, capi

    dev = torch.device("cuda:0")
    n = a.n
    ncells = n ** 3
    _log(f"inputs {n}^3 shear waves")
    u0 = torch.tensor(lbm_inputs.shear_waves((n, n, n), seed=0), device=dev)
    common = dict(periodic=(1, 1, 1), equilibrium="improved", collision="trt", omega=1.8,
                  trt_magic=3.0 / 16.0, device=dev)

    # ---- main timed region: forward + adjoint per step -------------------
    lat = Lattice(n, n, n, u=u0, dtype="f32", pattern="two_grid", **common)
    A, B = lat.buffers
    lam = [lat.new_adjoint(), lat.new_adjoint()]
    grad = torch.zeros(4, dtype=torch.float64, device=dev)
    # adjoint seed: kinetic-energy objective of the initial state
    jout = torch.zeros(4, dtype=torch.float64, device=dev)
    lat.objective(capi.LBM_OBJ_KINETIC_ENERGY, A, jout, lam[0])

    def one_step(i, ev=None):
        src, dst = (A, B) if i % 2 == 0 else (B, A)
        ln, lp = (lam[0], lam[1]) if i % 2 == 0 else (lam[1], lam[0])
        if ev is not None:
            ev[0].record()
        lat.stream_collide(src, dst, i)
        if ev is not None:
            ev[1].record()
        lat.adjoint_step(src, ln, lp, grad)
        if ev is not None:
            ev[2].record()

    _log(f"warmup {a.warmup}")
    for i in range(a.warmup):
        one_step(i)
    torch.cuda.synchronize()
    evs = [_events(torch, 3) for _ in range(a.steps)]
    _log(f"timed {a.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        one_step(a.warmup + i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / a.steps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / a.steps
    step_ms = evs[0][0].elapsed_time(evs[-1][2]) / a.steps
    if not np.isfinite(grad.cpu().numpy()).all():
        raise RuntimeError("non-finite adjoint gradient in the timed loop")

    bytes_fwd = 2 * 19 * 4 * ncells          # read + write every PDF once (FP32)
    bytes_adj = 3 * 19 * 4 * ncells          # state + lam_next read, lam_prev written
    fwd_gbs = bytes_fwd / (fwd_ms * 1e-3) / 1e9
    adj_gbs = bytes_adj / (adj_ms * 1e-3) / 1e9
    kernels = {
        "stream_collide_f32": {"ms": fwd_ms, "bytes_per_cell": 152, "GBs": fwd_gbs,
                               "frac": fwd_gbs / HBM_PEAK_GBS,
                               "mlups": ncells / (fwd_ms * 1e-3) / 1e6},
        "adjoint_f32": {"ms": adj_ms, "bytes_per_cell": 228, "GBs": adj_gbs,
                        "frac": adj_gbs / HBM_PEAK_GBS,
                        "mlups": ncells / (adj_ms * 1e-3) / 1e6},
    }
    dom = "adjoint_f32" if adj_ms >= fwd_ms else "stream_collide_f32"
    kernel_symbol = {"adjoint_f32": "k_adjoint_planar", "stream_collide_f32": "k_step_tg"}

    # plain copy of one state buffer with the library's copy kernel: the
    # achievable-bandwidth reference, and the byte-count reference of the
    # profiler's FETCH_SIZE / WRITE_SIZE runs
    state_bytes = A.numel() * A.element_size()
    copy_ms = None
    if a.copy_ref or not a.no_extras:
        lat.copy_state(A, B)
        e0, e1 = _events(torch, 2)
        torch.cuda.synchronize()
        e0.record()
        reps = 1 if a.copy_ref else 20
        for _ in range(reps):
            lat.copy_state(A, B)
        e1.record()
        torch.cuda.synchronize()
        copy_ms = e0.elapsed_time(e1) / reps
    del lam, A, B
    lat.close()
    del lat

    # ---- secondary configurations (outside the timed region) --------------
    extras = {}
    if not a.no_extras:
        for name, kw in [("fwd_f64_I_trt", dict(dtype="f64")),
                         ("fwd_f32s_I_trt", dict(dtype="f32s")),
                         ("fwd_f16s_I_trt", dict(dtype="f16s")),
                         ("fwd_bf16s_I_trt", dict(dtype="bf16s")),
                         ("fwd_f32_I_trt_aa", dict(dtype="f32", pattern="aa")),
                         ("fwd_f16s_I_trt_aa", dict(dtype="f16s", pattern="aa")),
                         ("fwd_f16s_I_trt_stochastic",
                          dict(dtype="f16s", rounding="stochastic", seed=1))]:
            _log(f"extra {name}")
            c = dict(common)
            lat2 = Lattice(n, n, n, u=u0, **c, **kw)
            ms = timed_forward(torch, lat2, 50, 5)
            size = {"f64": 8, "f32": 4, "f32s": 4, "f16s": 2, "bf16s": 2}[kw["dtype"]]
            gbs = 2 * 19 * size * ncells / (ms * 1e-3) / 1e9
            extras[name] = {"ms": round(ms, 5), "mlups": round(ncells / (ms * 1e-3) / 1e6, 1),
                            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
            lat2.close()
            del lat2
            torch.cuda.empty_cache()
        c = dict(common)
        c.update(equilibrium="standard", collision="srt")
        lat2 = Lattice(n, n, n, u=u0, dtype="f32", **c)
        ms = timed_forward(torch, lat2, 50, 5)
        extras["fwd_f32_S_srt"] = {"ms": round(ms, 5),
                                   "mlups": round(ncells / (ms * 1e-3) / 1e6, 1)}
        lat2.close()
        del lat2
        # D3Q27 (Sec. 1 and Sec. 6: D3Q19 moves 19/27 of the data)
        lat2 = Lattice(n, n, n, u=u0, dtype="f32", stencil=27, **common)
        ms27 = timed_forward(torch, lat2, 50, 5)
        gbs = 2 * 27 * 4 * ncells / (ms27 * 1e-3) / 1e9
        extras["fwd_f32_d3q27_trt"] = {
            "ms": round(ms27, 5), "mlups": round(ncells / (ms27 * 1e-3) / 1e6, 1),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "time_ratio_vs_d3q19": round(ms27 / fwd_ms, 3)}
        lat2.close()
        del lat2
        # MRT (Sec. 3.2) in the 19 kept moments, same second-order rate
        c = dict(common)
        c.update(collision="mrt", mrt_omega3=1.6, mrt_omega4=1.2)
        lat2 = Lattice(n, n, n, u=u0, dtype="f32", **c)
        msm = timed_forward(torch, lat2, 50, 5)
        gbs = 2 * 19 * 4 * ncells / (msm * 1e-3) / 1e9
        extras["fwd_f32_I_mrt"] = {
            "ms": round(msm, 5), "mlups": round(ncells / (msm * 1e-3) / 1e6, 1),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "time_ratio_vs_trt": round(msm / fwd_ms, 3)}
        lat2.close()
        del lat2
        # adjoint of other configurations: bytes = Q (sizeof(state) + 2 sizeof(lam))
        for name, kw, q, size in [
                ("adj_f16s_I_trt", dict(dtype="f16s"), 19, 2 + 2 * 4),
                ("adj_f64_I_trt", dict(dtype="f64"), 19, 3 * 8),
                ("adj_f32_I_mrt", dict(dtype="f32", collision="mrt", mrt_omega3=1.6,
                                       mrt_omega4=1.2), 19, 3 * 4),
                ("adj_f32_I3_trt", dict(dtype="f32", equilibrium="improved3"), 19, 3 * 4),
                ("adj_f32_d3q27_trt", dict(dtype="f32", stencil=27), 27, 3 * 4)]:
            _log(f"extra {name}")
            c = dict(common)
            c.update(kw)
            lat2 = Lattice(n, n, n, u=u0, **c)
            ms = timed_adjoint(torch, lat2, 20, 3)
            gbs = q * size * ncells / (ms * 1e-3) / 1e9
            extras[name] = {"ms": round(ms, 5), "mlups": round(ncells / (ms * 1e-3) / 1e6, 1),
                            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
            lat2.close()
            del lat2
            torch.cuda.empty_cache()
        # KBC (Sec. 3.3) in the 19 kept moments, 256^3 FP32
        c = dict(common)
        c.update(collision="kbc")
        lat2 = Lattice(n, n, n, u=u0, dtype="f32", **c)
        msk = timed_forward(torch, lat2, 50, 5)
        gbs = 2 * 19 * 4 * ncells / (msk * 1e-3) / 1e9
        extras["fwd_f32_I_kbc"] = {
            "ms": round(msk, 5), "mlups": round(ncells / (msk * 1e-3) / 1e6, 1),
            "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "time_ratio_vs_trt": round(msk / fwd_ms, 3)}
        lat2.close()
        del lat2
        torch.cuda.empty_cache()
        extras.update(workload_extras(torch, Lattice, lbm_inputs, dev))
    if copy_ms is not None:
        extras["copy_state_f32"] = {"ms": round(copy_ms, 5), "bytes": 2 * state_bytes,
                                    "GBs": round(2 * state_bytes / (copy_ms * 1e-3) / 1e9, 1)}

    # ---- CPU oracle baseline (bounded sample) -----------------------------
    cpu = None
    if not a.no_cpu:
        cpu = cpu_oracle_baseline(lbm_inputs, n)

    ms_step = step_ms
    out = {
        "metric": "MLUPS & % HBM roofline, D3Q19 256^3 FP32/FP16 fwd + adjoint vs FP64",
        "value": round(ncells / (ms_step * 1e-3) / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic D3Q19-I TRT(Lambda=3/16) omega=1.8, FP32 "
                               "two-grid; step = forward stream-collide + adjoint update",
                   "cells": ncells, "init": "8 seeded shear waves |k|<=4, A~U(0,0.03)"},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(kernels[dom]["GBs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(kernels[dom]["frac"], 4),
                     "traffic": recorded_traffic(kernel_symbol[dom]),
                     "algorithmic_bytes": kernels[dom]["bytes_per_cell"] * ncells},
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in kernels.items()},
        "extras": extras,
        "cpu_baseline": cpu,
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
