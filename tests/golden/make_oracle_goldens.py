"""Write the oracle-made reference values of the full-size GPU checks.

Calls only the FP64 CPU oracle (``oracle``) and the seeded input generators
(``lbm_inputs``); nothing here touches the GPU library.  Each part writes one
file next to this script:

  shear256   sampled post-collision PDFs after 1000 FP64 steps of the 256^3
             random-phase shear-wave field (8 modes, |k| <= 4, A ~ U(0, 0.03),
             seed 4) at omega = 1.95, for D3Q19-S SRT and D3Q19-I TRT
             (Lambda = 3/16): c2_256_w195_<model>.npz with the flat cell
             indices, the PDFs [k, 19] and the run's parameters.
  duct       the 512 x 128 x 128 duct (x periodic, half-way walls on y and z),
             D3Q19-I SRT, omega = 1.9, g_x = 1e-6, square-duct Poiseuille
             start plus U(-1e-3, 1e-3) noise (seed 9), T = 500: the kinetic
             energy J and its central differences (relative step 1e-4) in
             g_x, omega and along the seeded direction v (seed 10) of the
             initial velocity: c4_duct_fd.json.
  tube       the 768 x 192 x 192 constricted tube (periodic box, solid where
             r_cell > 80 (1 - 0.5 exp(-((x - 384)/60)^2))), D3Q19-I TRT
             (Lambda = 3/16), omega = 1.95, g_x = 2e-6, from rest, T = 500:
             the outlet flux J (the plane x = nx - 1) and its central
             differences in g_x (relative step 1e-4) and along the seeded
             per-cell direction v (seed 11, fluid cells) of the initial
             velocity (step 1e-6): c5_tube_fd_T500.json.  (The configured
             horizon is T = 2000; at the oracle's speed a run of it takes
             hours, so the reference stops at T = 500.)

Usage: python tests/golden/make_oracle_goldens.py shear256|duct|tube [model] [--out DIR]
(DIR defaults to this folder.)
The runs are long (the oracle is plain C): about 15 min per shear-wave model
and 15 min for the duct on 16 host cores; the tube's five runs take about
35 min each on 8 cores.  Progress goes to stdout; the tube file is rewritten
after each run, with "complete" false until the last.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = HERE
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import lbm_inputs  # noqa: E402
import oracle  # noqa: E402

SHEAR_MODELS = {
    "S_srt": dict(improved=0, trt=False),
    "I_trt": dict(improved=1, trt=True),
}


def _say(msg):
    print(f"[golden {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _advance(cfg, f, nsteps, chunk, label):
    done = 0
    t0 = time.perf_counter()
    while done < nsteps:
        k = min(chunk, nsteps - done)
        f = oracle.step(cfg, f, k)
        done += k
        rate = done * cfg.ncells / (time.perf_counter() - t0) / 1e6
        _say(f"{label}: step {done}/{nsteps} ({rate:.1f} MLUPS)")
    return f


def sample_cells(shape, seed, k=512):
    """Seeded cell sample plus every corner cell and its x-neighbours."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    cells = set(rng.choice(nx * ny * nz, size=k, replace=False).tolist())
    for z in (0, nz - 1):
        for y in (0, ny - 1):
            for x in (0, 1, nx - 2, nx - 1):
                cells.add((z * ny + y) * nx + x)
    return np.array(sorted(cells), dtype=np.int64)


def shear256(model: str):
    n, T, omega = 256, 1000, 1.95
    kw = SHEAR_MODELS[model]
    cfg = oracle.Config(n, n, n, omega=omega, magic=3.0 / 16.0, **kw)
    u0 = lbm_inputs.shear_waves((n, n, n), seed=4)
    f = oracle.init(cfg, u0)
    del u0
    f = _advance(cfg, f, T, 25, f"shear256 {model}")
    cells = sample_cells(cfg.shape, seed=12)
    flat = f.reshape(cfg.q, -1)
    pdfs = np.ascontiguousarray(flat[:, cells].T)
    meta = dict(n=n, steps=T, omega=omega, magic=3.0 / 16.0, model=model,
                init="lbm_inputs.shear_waves((256, 256, 256), seed=4)",
                equilibrium="improved" if kw["improved"] else "standard",
                collision="trt" if kw["trt"] else "srt")
    out = os.path.join(OUT, f"c2_256_w195_{model}.npz")
    np.savez(out, cells=cells, pdfs=pdfs, meta=np.array(json.dumps(meta)))
    _say(f"wrote {out}")


def duct():
    nx, ny, nz, T = 512, 128, 128, 500
    gx, omega, h = 1e-6, 1.9, 1e-4
    nu = (1 / omega - 0.5) / 3
    u0 = lbm_inputs.duct_poiseuille(nx, ny, nz, gx, nu) + lbm_inputs.perturbation(
        (nz, ny, nx), seed=9, amp=1e-3)
    v = lbm_inputs.perturbation((nz, ny, nx), seed=10, amp=1.0)
    hv = h * float(np.abs(u0).max())

    def J(accel_x, w, u):
        cfg = oracle.Config(nx, ny, nz, periodic=(1, 0, 0), improved=1, trt=False, omega=w,
                            accel=(accel_x, 0.0, 0.0))
        f = _advance(cfg, oracle.init(cfg, u), T, 50, f"duct g={accel_x:.9e} w={w:.9f}")
        return oracle.objective(cfg, f, 0)[0]

    rec = {"nx": nx, "ny": ny, "nz": nz, "steps": T, "gx": gx, "omega": omega, "h": h,
           "hv": hv, "objective": "kinetic energy 1/2 sum |u|^2",
           "init": "duct_poiseuille(512,128,128,gx,nu) + perturbation(seed=9, amp=1e-3)",
           "direction": "perturbation((128,128,512), seed=10, amp=1)"}
    rec["J"] = J(gx, omega, u0)
    rec["J_gx_plus"] = J(gx * (1 + h), omega, u0)
    rec["J_gx_minus"] = J(gx * (1 - h), omega, u0)
    rec["J_omega_plus"] = J(gx, omega * (1 + h), u0)
    rec["J_omega_minus"] = J(gx, omega * (1 - h), u0)
    rec["J_u_plus"] = J(gx, omega, u0 + hv * v)
    rec["J_u_minus"] = J(gx, omega, u0 - hv * v)
    rec["dJ_dgx"] = (rec["J_gx_plus"] - rec["J_gx_minus"]) / (2 * gx * h)
    rec["dJ_domega"] = (rec["J_omega_plus"] - rec["J_omega_minus"]) / (2 * omega * h)
    rec["dJ_du_dot_v"] = (rec["J_u_plus"] - rec["J_u_minus"]) / (2 * hv)
    out = os.path.join(OUT, "c4_duct_fd.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    _say(f"wrote {out}: {json.dumps(rec)}")


def tube():
    nx, ny, nz, T = 768, 192, 192, 500
    gx, omega, h, hv = 2e-6, 1.95, 1e-4, 1e-6
    solid = lbm_inputs.tube_mask(nx, ny, nz, r0=80.0, depth=0.5, centre=384.0, width=60.0)
    v = lbm_inputs.perturbation((nz, ny, nx), seed=11, amp=1.0) * (solid == 0)
    u0 = np.zeros((3, nz, ny, nx))

    def J(accel_x, u):
        cfg = oracle.Config(nx, ny, nz, periodic=(1, 1, 1), improved=1, trt=True, omega=omega,
                            magic=3.0 / 16.0, accel=(accel_x, 0.0, 0.0), solid=solid)
        f = _advance(cfg, oracle.init(cfg, u), T, 25, f"tube g={accel_x:.9e}")
        return oracle.objective(cfg, f, 1)[0]

    rec = {"nx": nx, "ny": ny, "nz": nz, "steps": T, "gx": gx, "omega": omega, "magic": 3 / 16,
           "h": h, "hv": hv, "objective": "outlet flux: sum of u_x over the fluid cells of x = nx - 1",
           "mask": "tube_mask(768, 192, 192, r0=80, depth=0.5, centre=384, width=60)",
           "init": "rest", "direction": "perturbation((192,192,768), seed=11, amp=1) * fluid",
           "complete": False}
    out = os.path.join(OUT, "c5_tube_fd_T500.json")
    runs = [("J", gx, u0), ("J_gx_plus", gx * (1 + h), u0), ("J_gx_minus", gx * (1 - h), u0),
            ("J_u_plus", gx, hv * v), ("J_u_minus", gx, -hv * v)]
    for name, a, u in runs:
        rec[name] = J(a, u)
        with open(out, "w") as fh:
            json.dump(rec, fh, indent=1)
        _say(f"{name} = {rec[name]!r}")
    rec["dJ_dgx"] = (rec["J_gx_plus"] - rec["J_gx_minus"]) / (2 * gx * h)
    rec["dJ_du_dot_v"] = (rec["J_u_plus"] - rec["J_u_minus"]) / (2 * hv)
    rec["complete"] = True
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    _say(f"wrote {out}: {json.dumps(rec)}")


if __name__ == "__main__":
    args = sys.argv[1:]
    if "--out" in args:
        i = args.index("--out")
        OUT = args[i + 1]
        del args[i:i + 2]
        os.makedirs(OUT, exist_ok=True)
    what = args[0] if args else ""
    if what == "shear256":
        for m in (args[1:] or list(SHEAR_MODELS)):
            shear256(m)
    elif what == "duct":
        duct()
    elif what == "tube":
        tube()
    else:
        print(__doc__)
        sys.exit(2)
