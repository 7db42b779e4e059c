"""Precision study: the 3-D LWFA physics at 8 particles per cell
(256 x 256 x 512 cells, 268,435,456 electrons at load) run in the three
particle/field precision modes of the library:

  fp64     every particle and field quantity in FP64 (the reference);
  fp32abs  FP32 absolute positions (24 B per particle), FP32 fields;
  fp32     int32 cell + FP32 offsets, FP32 fields, FP64 tau, window
           thresholds and diagnostics.

At each checkpoint the on-axis E_z(zeta) (node Nx/2, Ny/2), the charge on the
grid (sum rho V after the move), the charge of the pushed macro-particles and
the field energy are recorded; the FP32 modes are reported against the FP64
run: relative L2 difference of on-axis E_z and relative differences of the
charge and energy.  Every step runs in the HIP library; this module orders the
calls and reads results.

    python -m paper_2509_16793_amd.precision_study --steps 200 --out study.json
"""
import argparse
import json
import sys
import time

import numpy as np


def run_mode(mode, steps, checkpoints, log=print):
    import torch
    import workloads
    from .gempic import Sim

    cfg = workloads.precision_study(mode)
    t0 = time.perf_counter()
    sim = Sim(cfg, deposit_rho=True)
    log(f"{mode}: created in {time.perf_counter() - t0:.1f} s")
    dt = torch.float64 if mode == "fp64" else torch.float32
    ez = torch.empty((1, sim.Nz, sim.Ny, sim.Nx), dtype=dt, device="cuda")
    rec = {"mode": mode, "checkpoints": []}
    k = 0
    t_run = 0.0
    for c in checkpoints:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = sim.step(c - k, diag=True)
        torch.cuda.synchronize()
        t_run += time.perf_counter() - t1
        k = c
        sim.fields_device(("Ez",), ez)
        axis = ez[0, :, sim.Ny // 2, sim.Nx // 2].double().cpu().numpy()
        rec["checkpoints"].append(dict(step=c, ez_axis=axis.tolist(), charge_grid=d["charge_grid"],
                                       charge_particles=d["charge_particles"],
                                       field_energy=d["field_energy"],
                                       continuity_rel=d["continuity_rel"],
                                       n_particles=d["n_particles"]))
        log(f"{mode}: step {c}, energy {d['field_energy']:.6g}, charge {d['charge_grid']:.9g}")
    rec["ms_per_step"] = 1e3 * t_run / k
    sim.close()
    return rec


def compare(ref, run):
    out = []
    for a, b in zip(ref["checkpoints"], run["checkpoints"]):
        ea, eb = np.asarray(a["ez_axis"]), np.asarray(b["ez_axis"])
        out.append(dict(step=a["step"],
                        ez_axis_rel_l2=float(np.linalg.norm(eb - ea) / np.linalg.norm(ea)),
                        charge_grid_rel=abs(b["charge_grid"] - a["charge_grid"]) / abs(a["charge_grid"]),
                        charge_particles_rel=abs(b["charge_particles"] - a["charge_particles"])
                        / abs(a["charge_particles"]),
                        field_energy_rel=abs(b["field_energy"] - a["field_energy"]) / a["field_energy"],
                        continuity_rel=b["continuity_rel"]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--checkpoints", default="50,100,200")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import torch     # the library shares torch's HIP runtime: load torch first
    if not torch.cuda.is_available():
        raise RuntimeError("the precision study needs a GPU")
    cps = sorted({int(v) for v in a.checkpoints.split(",") if int(v) <= a.steps} | {a.steps})

    def log(m):
        print(m, flush=True)

    runs = {m: run_mode(m, a.steps, cps, log) for m in ("fp64", "fp32abs", "fp32")}
    res = {"workload": "lwfa3d_fp32 physics at 8 ppc (2,2,2), 256x256x512, 268,435,456 electrons",
           "steps": a.steps,
           "ms_per_step": {m: r["ms_per_step"] for m, r in runs.items()},
           "fp64_reference": [{k: v for k, v in c.items() if k != "ez_axis"}
                              for c in runs["fp64"]["checkpoints"]],
           "fp32abs_vs_fp64": compare(runs["fp64"], runs["fp32abs"]),
           "fp32_vs_fp64": compare(runs["fp64"], runs["fp32"])}
    print(json.dumps({k: v for k, v in res.items()}), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(dict(res, runs=runs), f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
