"""The paper's example (Sec. 6) scaled down to one GPU, without ionisation:
a laser (a0 = 2) in a Gaussian plasma channel, integrated with the zeta
march (GT2, Delta = 40 lambda = 32 um; workloads.lwfa_channel).

Every `every` slow steps it prints, as one JSON line:
  * the laser: peak |E_x| (the polarisation component), the zeta plane where
    it sits, and the rms width of |E_x| across x through the axis at that
    plane (w0 / 2 for a Gaussian spot of waist w0);
  * the wake: peak |E_z| on the axis;
  * the field energy and the macro-particles left in the box (in GT2 only
    those whose slow budget ran out inside it, i.e. electrons pushed
    forwards);
  * witness diagnostics in the style of Table 1 for the electrons with
    gamma >= gamma_min (charge, mean gamma and its spread, centroid, rms
    sizes, normalised emittances).
Every step runs in the HIP library; this module only orders the calls.

    python -m paper_2509_16793_amd.channel_example --steps 60 --every 10
"""
import argparse
import json
import math
import sys

import numpy as np


def diagnostics(sim, cfg, gamma_min):
    nx, ny, nz = cfg["n"]
    F = sim.fields(("Ex", "Ez"))
    ex, ez = F["Ex"], F["Ez"]
    amp = np.abs(ex).max(axis=(1, 2))
    iz = int(np.argmax(amp))
    prof = np.abs(ex[iz, ny // 2, :]).astype(np.float64)
    xs = (np.arange(nx) - nx // 2) * cfg["d"][0]
    width = math.sqrt(float(np.sum(prof ** 2 * xs ** 2) / np.sum(prof ** 2)))
    d = sim.step(0, diag=True)
    return {"laser_peak_ex": float(amp[iz]), "laser_plane": iz, "laser_rms_x_lambda": width,
            "wake_peak_ez_axis": float(np.abs(ez[:, ny // 2, nx // 2]).max()),
            "field_energy": d["field_energy"], "n_particles": d["n_particles"],
            "witness": sim.bunch(gamma_min)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--gamma-min", type=float, default=2.0)
    ap.add_argument("--nz", type=int, default=4096)
    args = ap.parse_args(argv)
    import workloads
    from .gempic import Sim
    cfg = workloads.lwfa_channel(nz=args.nz)
    sim = Sim(cfg)
    k = 0
    while True:
        rec = {"slow_step": k, "s_lambda": k * cfg["delta"]}
        rec.update(diagnostics(sim, cfg, args.gamma_min))
        print(json.dumps(rec), flush=True)
        if k >= args.steps:
            break
        n = min(args.every, args.steps - k)
        sim.step(n)
        k += n
    sim.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
