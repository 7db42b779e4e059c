"""Benchmark of the Galilean PIC step on one MI355X.

Workload: the 3-D LWFA setup -- 256 x 256 x 512 cells, dx = dy = 0.4,
dzeta = 0.05 (laser wavelengths), n_e = 0.001 n_c, 2 particles per cell
(67,108,864 electrons plus window inflow), a0 = 2 laser, FP32 cell + offset
particles -- synthetic and seeded.  One step = gather + push + deposit, stable
sort + window injection, and the field update (FFT, march, inverse FFT).

--workload pwfa runs the PWFA setup instead (512 x 512 x 1024 cells, 4 ppc,
1e7-particle driver, plasma units).

Prints one JSON line.  value = particle updates per second of the
gather + push + deposit kernel (HIP events around its launches, on the stream
the library runs on); ms_per_step = wall time per whole step over the timed
region.  roofline = that kernel's algorithmic bytes (2 x 28 B particle state,
24 B of fields and 12 B of current per cell) per launch over its average
duration, against 8 TB/s.  cpu_baseline = the FP64 CPU oracle's gather + push
+ deposit on a bounded crop of the same workload, timed on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle updates/s (gather+push+deposit), % HBM roofline; 1ppc+CNN vs 16ppc"
# HBM bytes per k_push_deposit launch from rocprofv3 FETCH_SIZE / WRITE_SIZE on this
# workload, scaled by a plain-copy calibration (profiles/k_push_deposit_lwfa3d_*.md);
# valid only for the kernel source it was measured on.
MEASURED_TRAFFIC = {"push_h_sha256_prefix": "48b9e47424576003", "bytes_per_launch": 5.778e+09}
HBM_PEAK_GBS = 8000.0
WORKLOAD_TEXT = {
    "lwfa": "lwfa3d_fp32: 3-D LWFA 256x256x512, dx=dy=0.4, dzeta=0.05 (lambda_L), n_e=0.001 n_c, "
            "2 ppc, a0=2, waist 8, FWHM 8, FP32 cell+offset particles, 8x8x4 tiles",
    "pwfa": "pwfa3d_fp32: 3-D PWFA 512x512x1024, dx=dy=0.1, dzeta=0.05 (c/omega_p), n_e=1, 4 ppc, "
            "Gaussian driver sigma_r=0.5, sigma_zeta=1, peak 10 n_e, gamma 2000 +- 0.1 %, "
            "1e7 macro-particles, FP32 cell+offset particles, 8x8x4 tiles",
}
STATE_BYTES = 28          # int32 cell + 3 x FP32 offset + 3 x FP32 momentum


def algorithmic_bytes_per_update(ppc):
    """Particle state read + written once, 6 FP32 fields read once per cell,
    3 FP32 currents written once per cell."""
    return 2 * STATE_BYTES + (24.0 + 12.0) / ppc


def cpu_baseline(workload="lwfa", seconds_budget=30.0):
    """FP64 oracle gather + push + deposit on a transverse crop of the workload:
    LWFA 32 x 32 x 512 cells (same steps, density, ppc; laser waist scaled to
    the crop); PWFA 16 x 16 x 512 cells of its plasma (same steps, density,
    ppc; the driver is left out: its 1e7 particles do not fit a crop)."""
    import numpy as np
    import workloads
    from oracle.sim import Simulation
    from oracle.push import push_and_move
    from oracle.deposit import deposit

    if workload == "pwfa":
        cfg = workloads.pwfa3d_fp32()
        cfg["n"] = [16, 16, 512]
        cfg["beam"] = None
        crop = "16x16x512 crop of the PWFA plasma (no driver)"
    else:
        cfg = workloads.lwfa3d_fp32()
        cfg["n"] = [32, 32, 512]
        cfg["waist"] = 2.0
        crop = "32x32x512 crop of the workload"
    cfg["precision"] = "fp64"
    s = Simulation(cfg)
    p = s.p
    done = 0
    t_used = 0.0
    steps = 0
    P = s.P
    while steps < 3 and t_used < seconds_budget:
        t0 = time.perf_counter()
        old, st, vy = push_and_move(p, P, s.F)
        deposit(p, old, (P.ix, P.iy, P.iz, P.dx, P.dy, P.dz), st, vy)
        t_used += time.perf_counter() - t0
        done += len(P)
        steps += 1
        P = P.take(P.iz >= 0)          # particles that left the box (untimed)
    return {"value": done / t_used, "unit": "particle updates/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 numpy oracle, gather+push+deposit, {steps} steps of a "
                      f"{crop} ({len(s.P)} particles), single thread",
            "seconds": t_used}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("lwfa", "pwfa"), default="lwfa",
                    help="lwfa: 3-D LWFA 256x256x512 at 2 ppc (default); pwfa: 3-D PWFA "
                         "512x512x1024 at 4 ppc with a 1e7-particle driver")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 28                      # 2^28 floats = 1 GiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2509_16793_amd.gempic import Sim

    torch.cuda.init()
    dev = torch.cuda.current_device()
    stream = torch.cuda.current_stream(dev).cuda_stream
    cfg = workloads.pwfa3d_fp32() if args.workload == "pwfa" else workloads.lwfa3d_fp32()
    ppc = cfg["ppc"][0] * cfg["ppc"][1] * cfg["ppc"][2]
    sim = Sim(cfg, stream=stream)
    print(f"[bench] created {cfg['n']} ppc={ppc}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    n0 = sim._count()
    print(f"[bench] warmup {args.warmup} steps done, {n0} particles", file=sys.stderr, flush=True)

    sim.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ph, nt = sim.get_timing()
    n1 = sim._count()
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)

    import hashlib
    src = open(os.path.join(ROOT, "paper_2509_16793_amd", "csrc", "push.h"), "rb").read()
    same_kernel = hashlib.sha256(src).hexdigest()[:16] == MEASURED_TRAFFIC["push_h_sha256_prefix"]
    traffic = MEASURED_TRAFFIC["bytes_per_launch"] if same_kernel and args.workload == "lwfa" else None
    n_avg = 0.5 * (n0 + n1)
    push_s = ph["push_deposit"] / 1e3
    value = n_avg * args.steps / push_s
    launch_s = push_s / args.steps
    bpu = algorithmic_bytes_per_update(ppc)
    achieved = n_avg * bpu / launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "grid": cfg["n"], "ppc": ppc, "particles": int(n_avg)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_push_deposit", "bytes_per_update": bpu,
                     "avg_launch_ms": launch_s * 1e3},
        "phase_ms_per_step": {k: v / args.steps for k, v in ph.items()},
        "step_updates_per_s": n_avg * args.steps / (t1 - t0),
    }
    sim.close()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a crop", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
