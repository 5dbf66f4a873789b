"""Duct-flow experiment of Sec. 5.1 on the GPU path: spurious transverse
currents of the standard and the improved D3Q19 equilibrium.

Set-up (Sec. 5.1): a square duct of D x D cells, one cell long and periodic
along the flow axis x, half-way bounce-back walls on y and z, driven by the
Buick body force along x, SRT collision with a fixed relaxation rate under
diffusive scaling, Re = 10, run to a steady state.  Error measure:
max |u_y| / max u_x.  Lambda = 1/omega - 1/2 (Sec. 4).

Readings: Re = u_max D / nu with u_max the centre velocity of the
square-duct Poiseuille solution, u_max = K a (D/2)^2 / nu, K = 0.29468...;
the run starts from that solution and stops after `sweeps` viscous times
D^2 / nu.

Also here: a flow driven from rest by a small body force in every storage
type, which measures how the rounding of the stored f - w treats a per-step
force increment near its half-ulp (`driven_flow`).

And the forward throughput against the lattice size (`size_sweep`), and one
checkpointed gradient rollout of the constricted tube with 16-bit storage
(`tube_rollout`), timed as a whole.

Usage: python -m paper_1803_04937_amd.experiments [--dtype f64] [--sizes 15,25,45]
       python -m paper_1803_04937_amd.experiments --driven-flow
       python -m paper_1803_04937_amd.experiments --size-sweep
"""
from __future__ import annotations

import argparse
import json
import math
import time

import torch

from .lattice import Lattice


def _square_duct_centre_constant(nterms: int = 200) -> float:
    """u(0, 0) a^-1 b^-2 nu of the square-duct Poiseuille series."""
    s = 0.0
    for m in range(nterms):
        k = 2 * m + 1
        s += (-1) ** m * (1.0 - 1.0 / math.cosh(k * math.pi / 2)) / k ** 3
    return 16.0 / math.pi ** 3 * s


K_CENTRE = _square_duct_centre_constant()


def duct_spurious_current(D: int, lam2: float, equilibrium: str, dtype: str = "f64",
                          re: float = 10.0, sweeps: float = 3.0, stencil: int = 19,
                          mrt=None, device=None) -> dict:
    """Steady-state max |u_y| / max u_x of the duct for one resolution D,
    one Lambda^2 and one equilibrium ("standard" or "improved"; D3Q27 has a
    single equilibrium).  SRT, or with mrt = (omega3, omega4) the MRT
    collision whose second-order moments relax at the same omega."""
    import lbm_inputs
    lam = math.sqrt(lam2)
    omega = 1.0 / (lam + 0.5)
    nu = lam / 3.0
    a = re * nu * nu / (K_CENTRE * (D / 2.0) ** 2 * D)
    u0 = torch.as_tensor(lbm_inputs.duct_poiseuille(1, D, D, a, nu))
    coll = dict(collision="srt")
    if mrt is not None:
        coll = dict(collision="mrt", mrt_omega3=mrt[0], mrt_omega4=mrt[1])
    lat = Lattice(1, D, D, u=u0, periodic=(1, 0, 0), equilibrium=equilibrium, dtype=dtype,
                  omega=omega, accel=(a, 0.0, 0.0), stencil=stencil, device=device, **coll)
    steps = int(math.ceil(sweeps * D * D / nu))
    chunks = 10
    per = max(1, steps // chunks)
    history = []
    for _ in range(chunks):
        lat.step(per)
        _, u = lat.moments()
        ux = u[0].abs().max().item()
        uy = torch.maximum(u[1].abs().max(), u[2].abs().max()).item()
        history.append(uy / ux)
    lat.close()
    last, prev = history[-1], history[-2]
    return {"D": D, "lambda2": lam2, "omega": omega, "stencil": stencil,
            "equilibrium": equilibrium if stencil == 19 else "d3q27", "dtype": dtype,
            "collision": "srt" if mrt is None else f"mrt{tuple(mrt)}",
            "steps": per * chunks, "ratio": last, "ux_max": ux,
            "last_chunk_rel_change": abs(last - prev) / max(abs(last), 1e-300)}


def convergence_order(results):
    """Least-squares slope of log(ratio) against log(D)."""
    xs = [math.log(r["D"]) for r in results]
    ys = [math.log(r["ratio"]) for r in results]
    n = len(xs)
    mx, my = sum(xs) / n, sum(ys) / n
    return sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs)


def driven_flow(dtype: str, shape=(32, 32, 32), walls: bool = False, g: float = 2e-6,
                omega: float = 1.95, times=(2000, 20000), rounding: str = "nearest",
                seed: int = 0, device=None) -> dict:
    """Flow driven from rest by a small body force g along x (D3Q19-I TRT,
    Lambda = 3/16), stored in one storage type: the mean u_x over the fluid
    at each time in `times`.  In a periodic box every cell stays identical and
    the exact answer is u_x = (t - 1/2) g (the momentum grows by g per step,
    the read-out subtracts g/2), so the relative deviation measures how much
    of the per-step force increment, 3 w_q c_q.g, survives the rounding of the
    stored f - w.  With walls on y and z (a duct) compare with an FP64 run."""
    nz, ny, nx = shape
    u0 = torch.zeros((3, nz, ny, nx), dtype=torch.float64)
    lat = Lattice(nx, ny, nz, u=u0, periodic=(1, 0, 0) if walls else (1, 1, 1),
                  equilibrium="improved", collision="trt", dtype=dtype, omega=omega,
                  accel=(g, 0.0, 0.0), rounding=rounding, seed=seed, device=device)
    rows, done = [], 0
    for t in times:
        lat.step(t - done)
        done = t
        _, u = lat.moments()
        ux = u[0].mean().item()
        row = {"t": t, "mean_ux": ux}
        if not walls:
            row["rel_dev"] = ux / ((t - 0.5) * g) - 1.0
        rows.append(row)
    scale = lat.scale
    lat.close()
    return {"dtype": dtype, "rounding": rounding, "shape": list(shape), "walls": walls, "g": g,
            "omega": omega, "scale": scale, "rows": rows}


def size_sweep(sizes=(16, 32, 64, 96, 128, 160, 192, 256, 384), dtypes=("f32", "f16s"),
               policies=("auto",), min_updates: float = 4e9, device=None) -> list:
    """Forward throughput of the periodic D3Q19-I TRT update against the
    lattice size n^3: the launch-latency regime of small lattices, the regime
    where the two state buffers fit the last-level cache, and the HBM
    regime.  Each point times enough steps for about `min_updates` cell
    updates (at least 50 steps)."""
    import lbm_inputs
    rows = []
    for dt, n, policy in ((dt, n, pol) for dt in dtypes for n in sizes for pol in policies):
        u0 = torch.as_tensor(lbm_inputs.shear_waves((n, n, n), seed=1, amax=0.03))
        lat = Lattice(n, n, n, u=u0, equilibrium="improved", collision="trt", omega=1.8,
                      dtype=dt, cache_policy=policy, device=device)
        steps = max(50, int(min_updates / n ** 3))
        lat.step(10)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        lat.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        size = {"f64": 8, "f32": 4, "f32s": 4, "f16s": 2, "bf16s": 2}[dt]
        state_mb = 2 * 19 * size * n ** 3 / 1e6
        rows.append({"dtype": dt, "n": n, "policy": policy, "steps": steps,
                     "us_per_step": round(ms * 1e3, 2),
                     "glups": round(n ** 3 / (ms * 1e-3) / 1e9, 2),
                     "GBs": round(2 * 19 * size * n ** 3 / (ms * 1e-3) / 1e9, 1),
                     "two_states_MB": round(state_mb, 1)})
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return rows


def tube_rollout(steps: int = 2000, dtype: str = "f16s", nx: int = 768, ny: int = 192,
                 nz: int = 192, omega: float = 1.95, gx: float = 2e-6):
    """One gradient of the outlet flux J(f_T) through the constricted tube
    (D3Q19-I TRT, solid mask, periodic box, body force along x), with respect
    to g_x, omega and the initial velocity, by the checkpointed adjoint:
    ceil(sqrt(T)) checkpoints, each segment recomputed into a ring before its
    adjoint steps.  Returns wall times and update counts."""
    import lbm_inputs
    from .autograd import RolloutConfig, rollout_objective
    solid = torch.as_tensor(lbm_inputs.tube_mask(nx, ny, nz, r0=80.0 * ny / 192, depth=0.5,
                                                 centre=nx / 2, width=60.0 * nx / 768),
                            dtype=torch.uint8).cuda()
    rc = RolloutConfig(nx, ny, nz, steps=steps, periodic=(1, 1, 1), collision="trt",
                       dtype=dtype, objective=1, solid=solid)
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor([gx, 0.0, 0.0], dtype=torch.float64, requires_grad=True)
    w = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = rollout_objective(u, a, w, rc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cells = nx * ny * nz
    fwd, bwd = t1 - t0, t2 - t1
    return {"shape": [nx, ny, nz], "steps": steps, "dtype": dtype, "segment": rc.segment,
            "J": J.item(), "dJ/dgx": a.grad[0].item(), "dJ/domega": w.grad.item(),
            "forward_s": round(fwd, 3), "backward_s": round(bwd, 3),
            "forward_glups": round(cells * steps / fwd / 1e9, 2),
            "backward_glups": round(cells * steps / bwd / 1e9, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--sizes", default="15,25,35,45,65")
    ap.add_argument("--lambda2", default="0.16,0.0833333333333333")
    ap.add_argument("--d3q27", action="store_true", help="also run the D3Q27 stencil")
    ap.add_argument("--sweep", type=int, default=0,
                    help="also sweep Lambda^2 at this D for the standard equilibrium")
    ap.add_argument("--driven-flow", action="store_true",
                    help="only run the small-force driven flow in every storage type")
    ap.add_argument("--size-sweep", action="store_true",
                    help="only run the forward throughput sweep over lattice sizes")
    ap.add_argument("--mrt", default="",
                    help="omega3,omega4: run the duct study with the MRT collision")
    ap.add_argument("--tube-rollout", type=int, default=0, metavar="T",
                    help="only run one checkpointed gradient rollout of T steps through "
                         "the constricted tube (768 x 192 x 192, --dtype, default f16s)")
    a = ap.parse_args()
    if a.tube_rollout:
        dt = a.dtype if a.dtype != "f64" else "f16s"
        print(json.dumps(tube_rollout(a.tube_rollout, dt)), flush=True)
        return
    if a.size_sweep:
        for row in size_sweep(policies=("stream", "keep")):
            print(json.dumps(row), flush=True)
        return
    if a.driven_flow:
        runs = [(dt, "nearest") for dt in ("f64", "f32", "f32s", "f16s", "bf16s")]
        runs += [("f16s", "stochastic"), ("bf16s", "stochastic")]
        for walls in (False, True):
            ref = None
            for dt, rnd in runs:
                r = driven_flow(dt, walls=walls, rounding=rnd)
                if walls:
                    ref = ref or r
                    for row, r64 in zip(r["rows"], ref["rows"]):
                        row["rel_dev_vs_f64"] = row["mean_ux"] / r64["mean_ux"] - 1.0
                print(json.dumps(r), flush=True)
        return
    sizes = [int(v) for v in a.sizes.split(",")]
    mrt = tuple(float(v) for v in a.mrt.split(",")) if a.mrt else None
    out = {}
    for lam2 in [float(v) for v in a.lambda2.split(",")]:
        for eq in ("standard", "improved"):
            rows = [duct_spurious_current(D, lam2, eq, a.dtype, mrt=mrt) for D in sizes]
            key = f"{eq}_lambda2={lam2:.4f}" + (f"_mrt={a.mrt}" if mrt else "")
            out[key] = {"rows": rows}
            if eq == "standard":
                out[key]["order"] = convergence_order(rows)
            print(json.dumps({key: out[key]}), flush=True)
    if a.d3q27:
        for lam2 in [float(v) for v in a.lambda2.split(",")]:
            rows = [duct_spurious_current(D, lam2, "standard", a.dtype, stencil=27) for D in sizes]
            print(json.dumps({f"d3q27_lambda2={lam2:.4f}": {"rows": rows}}), flush=True)
    if a.sweep:
        lams = [0.01, 0.02, 0.04, 0.06, 1.0 / 12.0, 0.1, 0.12, 0.16, 0.25]
        sweep = [(l2, duct_spurious_current(a.sweep, l2, "standard", a.dtype)["ratio"])
                 for l2 in lams]
        print(json.dumps({f"standard_sweep_D={a.sweep}": sweep}), flush=True)


if __name__ == "__main__":
    main()
