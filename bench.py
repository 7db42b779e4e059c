"""Benchmark of the Galilean PIC step on one MI355X.

Workload: the 3-D LWFA setup -- 256 x 256 x 512 cells, dx = dy = 0.4,
dzeta = 0.05 (laser wavelengths), n_e = 0.001 n_c, 2 particles per cell
(67,108,864 electrons plus window inflow), a0 = 2 laser, FP32 cell + offset
particles -- synthetic and seeded.  One step = gather + push + deposit, stable
sort + window injection, and the field update (FFT, march, inverse FFT).

--workload pwfa runs the PWFA setup instead (512 x 512 x 1024 cells, 4 ppc,
1e7-particle driver, plasma units).

Prints one JSON line.  value = particle updates per second of the
gather + push + deposit kernel: particles over the median of its per-step
durations (HIP events on the stream the library runs on); ms_per_step = wall
time per whole step over the timed region.  roofline = that kernel's
algorithmic bytes (2 x 28 B particle state, 24 B of fields and 12 B of current
per cell) per launch over its median duration, against 8 TB/s; traffic = the
HBM bytes per launch that rocprofv3 counted on this kernel source (null for
another source), and traffic_achieved / traffic_frac = those over the same
median duration.
cpu_baseline = the FP64 CPU oracle's gather + push + deposit on bounded
transverse crops of the same workload, on every host core (one crop per
process) and on one core; and, as lwfa2d_full_step, the small 2-D FP64 case
run in full (100 whole steps) on the GPU and by the oracle on one core.

Extra objects on the same line:
  march   -- the paper's own slow step (the zeta march, GT1) on the same
             physics at 1 particle per transverse cell per batch and
             Delta = 8 lambda (320 times the tau scheme's dtau), its median
             wall time per slow step, the time the tau scheme needs for the
             same Delta, and the oracle's march on crops beside it; and the
             paper's example scaled down to one GPU (Gaussian channel,
             128 x 128 x 4096, Delta = 32 um, GT2).
  denoise -- wall time per whole step at 1 ppc with the committed network
             against 16 ppc without it (the same LWFA physics, a seed held
             out from training), and at step 500 the relative L2 difference
             of on-axis E_z from the 16-ppc run, with the network and for
             plain 1 ppc (the 2 % accuracy condition of the comparison).
  pwfa    -- the push kernel's throughput and roofline fraction, and the
             whole step, on the PWFA setup (5 timed steps after 2).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle updates/s (gather+push+deposit), % HBM roofline; 1ppc+CNN vs 16ppc"
# HBM bytes per k_push_deposit launch from rocprofv3 FETCH_SIZE / WRITE_SIZE on this
# workload, scaled by a plain-copy calibration (profiles/k_push_deposit_lwfa3d_*.md);
# valid only for the kernel source it was measured on.
MEASURED_TRAFFIC = {"push_h_sha256_prefix": "632fbbfc27b15b7e", "bytes_per_launch": 5.740e+09}
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


def _oracle_crop(args):
    """One process: FP64 oracle gather + push + deposit on a crop (seeded by
    its index), `steps` steps or until `budget` seconds; returns (particle
    updates, seconds)."""
    workload, nx, index, steps, budget = args
    import workloads
    from oracle.sim import Simulation
    from oracle.push import push_and_move
    from oracle.deposit import deposit
    if workload == "pwfa":
        cfg = workloads.pwfa3d_fp32()
        cfg["beam"] = None
    else:
        cfg = workloads.lwfa3d_fp32()
        cfg["waist"] = 2.0 * nx / 32
    cfg["n"] = [nx, nx, 512]
    cfg["precision"] = "fp64"
    cfg["seed"] = index
    s = Simulation(cfg)
    p = s.p
    P = s.P
    done, used, k = 0, 0.0, 0
    while k < steps and used < budget:
        t0 = time.perf_counter()
        old, st, vy = push_and_move(p, P, s.F)
        deposit(p, old, (P.ix, P.iy, P.iz, P.dx, P.dy, P.dz), st, vy)
        used += time.perf_counter() - t0
        done += len(P)
        k += 1
        P = P.take(P.iz >= 0)          # particles that left the box (untimed)
    return done, used, len(s.P)


def cpu_baseline(workload="lwfa"):
    """The FP64 oracle (as it stands) on every host core: one transverse crop
    of 16 x 16 x 512 cells of the workload per process (same cell sizes,
    density, ppc; the LWFA laser waist scaled to the crop; PWFA without the
    driver, whose 1e7 particles do not fit a crop), 3 steps each; aggregate
    updates over the slowest process's time.  Plus one process alone."""
    import multiprocessing as mp
    import platform
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ncpu = os.cpu_count() or 1
    try:
        ncpu = min(ncpu, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    nproc = max(1, min(ncpu, 16))
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    one_done, one_s, one_n = _oracle_crop((workload, 16, 0, 3, 20.0))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(nproc) as pool:
        res = pool.map(_oracle_crop, [(workload, 16, i, 3, 20.0) for i in range(nproc)])
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    slowest = max(r[1] for r in res)
    return {"value": done / slowest, "unit": "particle updates/s", "cores": nproc, "kind": "oracle",
            "sample": f"FP64 numpy oracle, gather+push+deposit, 3 steps of {nproc} independent 16x16x512 "
                      f"transverse crops of the workload ({res[0][2]} particles each), one process per "
                      f"core (slowest process's compute time); wall {wall:.1f} s with start-up",
            "single_thread": {"value": one_done / one_s, "cores": 1, "seconds": one_s},
            "host_cpu": model, "os_cpu_count": os.cpu_count()}


def full_step_2d(stream, steps=100, warmup=5):
    """The small 2-D (x, zeta) LWFA case in full (64 x 256 cells, 2 ppc, FP64,
    100 steps): wall time per whole step (gather, push, deposit, sort,
    window, field update) on the GPU and of the FP64 oracle on one host core,
    on the same configuration."""
    import torch
    import workloads
    from oracle.sim import Simulation
    from paper_2509_16793_amd.gempic import Sim
    cfg = workloads.lwfa2d_fp64()
    g = Sim(cfg, stream=stream)
    g.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    n = g._count()
    g.close()
    o = Simulation(cfg)
    o.run(warmup)
    t0 = time.perf_counter()
    o.run(steps)
    cpu_s = time.perf_counter() - t0
    return {"workload": "lwfa2d_fp64: 2-D LWFA 64x256, dx=0.25, dzeta=0.05, n_e=0.01 n_c, 2 ppc, a0=1, "
                        "FP64, whole step", "steps": steps, "particles": n,
            "gpu_ms_per_step": 1e3 * gpu_s / steps, "oracle_ms_per_step": 1e3 * cpu_s / steps,
            "oracle_cores": 1}


def _oracle_march_crop(args):
    """One process: the FP64 oracle's zeta march (GT1, Delta = 8 lambda) on an
    nx x nx x 512 crop of the LWFA physics (laser waist scaled to the crop),
    one untimed slow step after creation, then one timed; returns (transverse
    column slow steps, seconds, particles)."""
    nx, index = args
    import workloads
    from oracle.march import MarchSim
    cfg = workloads.lwfa3d_fp32(ppc=(1, 1, 1))
    cfg.update(scheme=1, delta=8.0, n=[nx, nx, 512], precision="fp64", waist=2.0 * nx / 32, seed=index)
    s = MarchSim(cfg)
    s.step()
    t0 = time.perf_counter()
    s.step()
    return nx * nx, time.perf_counter() - t0, len(s.P)


def cpu_baseline_march(nx=32):
    """The oracle's zeta march on every host core (<= 16 processes), one
    nx x nx x 512 crop per process; aggregate column slow steps over the
    slowest process's time."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    try:
        ncpu = min(ncpu, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    nproc = max(1, min(ncpu, 16))
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    with mp.get_context("spawn").Pool(nproc) as pool:
        res = pool.map(_oracle_march_crop, [(nx, i) for i in range(nproc)])
    cols = sum(r[0] for r in res)
    slowest = max(r[1] for r in res)
    return {"value": cols / slowest, "unit": "transverse-column slow steps/s", "cores": nproc, "kind": "oracle",
            "sample": f"FP64 numpy oracle zeta march (GT1, Delta = 8 lambda), one slow step of {nproc} "
                      f"independent {nx}x{nx}x512 crops of the LWFA physics ({res[0][2]} particles each), "
                      f"one process per core (slowest process's time)"}


def median_step_phases(sim, steps):
    """Per-step HIP-event phases (ms) of `steps` single steps."""
    rows = []
    for _ in range(steps):
        sim.timing(True)
        sim.step(1)
        ph, n = sim.get_timing()
        rows.append(ph)
    return {k: statistics.median(r[k] for r in rows) for k in rows[0]}, rows


def bench_pwfa(stream, steps=5, warmup=2):
    """The PWFA setup (512 x 512 x 1024 cells, 4 ppc, 1e7-particle driver):
    the push kernel's throughput and roofline fraction, and the whole step,
    over a few steps (its creation samples the driver on the host)."""
    import workloads
    from paper_2509_16793_amd.gempic import Sim
    cfg = workloads.pwfa3d_fp32()
    ppc = cfg["ppc"][0] * cfg["ppc"][1] * cfg["ppc"][2]
    g = Sim(cfg, stream=stream)
    g.step(warmup)
    n0 = g._count()
    med, _ = median_step_phases(g, steps)
    n_avg = 0.5 * (n0 + g._count())
    g.close()
    launch_s = med["push_deposit"] / 1e3
    bpu = algorithmic_bytes_per_update(ppc)
    achieved = n_avg * bpu / launch_s / 1e9
    return {"workload": WORKLOAD_TEXT["pwfa"], "particles": int(n_avg), "steps": steps, "warmup": warmup,
            "value": n_avg / launch_s, "unit": "particle updates/s",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "kernel": "k_push_deposit", "bytes_per_update": bpu,
                         "median_launch_ms": launch_s * 1e3},
            "ms_per_step": med["step"], "phase_ms_per_step": med}


def bench_march(stream, steps=5, cpu=True):
    """The zeta march on the LWFA physics, and the paper's example scaled down."""
    import workloads
    from paper_2509_16793_amd.gempic import Sim
    out = {}
    cfg = workloads.lwfa3d_fp32(ppc=(1, 1, 1))
    cfg.update(scheme=1, delta=8.0)
    g = Sim(cfg, stream=stream)
    g.step(1)
    med, _ = median_step_phases(g, steps)
    d = g.step(1, diag=True)
    nz, ncol = cfg["n"][2], cfg["n"][0] * cfg["n"][1]
    # in a zeta-march step the second timing phase is the stage loop (stage
    # kernel, per-plane transforms, node solve), the third the parking sort
    out["lwfa"] = {"workload": "lwfa3d physics (256x256x512, dx=dy=0.4, dzeta=0.05 lambda, n_e=0.001, a0=2), "
                               "zeta march GT1, 1 particle per transverse cell per batch, Delta = 8 lambda",
                   "ms_per_slow_step": med["step"], "value": ncol / (med["step"] / 1e3),
                   "unit": "transverse-column slow steps/s",
                   "us_per_stage": med["push_deposit"] * 1e3 / nz, "ms_parking_sort": med["sort_window"],
                   "delta_over_dtau": 8.0 / 0.025, "particles_in_box": d["n_particles"]}
    g.close()
    if cpu:
        print("[bench] timing the CPU oracle's zeta march on crops", file=sys.stderr, flush=True)
        cb = cpu_baseline_march()
        out["lwfa"]["cpu_baseline"] = cb
        out["lwfa"]["gpu_over_cpu"] = out["lwfa"]["value"] / cb["value"]
    cfg = workloads.lwfa_channel()
    g = Sim(cfg, stream=stream)
    g.step(1)
    med2, _ = median_step_phases(g, 3)
    n_steps_paper = 31.8e-2 / 32e-6          # 31.8 cm at Delta = 32 um
    out["paper_example"] = {
        "workload": "Sec. 6 example scaled down: Gaussian channel n1/n0 = 0.25, R_ch 95.5 lambda, "
                    "n0 = 2.9e-4 n_c, a0 = 2, 128x128x4096 cells over 187.5x187.5x225 lambda, "
                    "zeta march GT2, Delta = 32 um (40 lambda)",
        "ms_per_slow_step": med2["step"],
        "hours_for_31.8_cm": med2["step"] * n_steps_paper / 3.6e6,
        "paper_context": "GEM-PIC: 12 h on 432 Xeon E5-2697 v2 cores for 31.8 cm (150x150x180 um window, "
                         "4+4 macro-atoms per cell, ionisation) -- other hardware and physics, not a target"}
    g.close()
    return out, med


def bench_denoise(stream, steps=16, acc_steps=500, seed=64):
    """1 ppc + the committed network against 16 ppc on the LWFA physics, with a
    seed the network was not trained on: median whole-step times over `steps`
    steps after 3 warm-up steps (also for plain 1 ppc), then, at step
    `acc_steps`, the relative L2 difference of on-axis E_z (node column Nx/2,
    Ny/2, over zeta) from the 16-ppc run, with the network and for plain 1 ppc."""
    import numpy as np
    import workloads
    from paper_2509_16793_amd.gempic import Denoiser, Sim
    theta = np.load(os.path.join(ROOT, "paper_2509_16793_amd", "weights", "denoiser_lwfa.npy"))

    def run(ppc, dn=None):
        sim = Sim(dict(workloads.denoiser_lwfa(ppc=ppc), seed=seed), stream=stream)
        if dn is not None:
            sim.set_denoiser(dn, 1e-3)
        sim.step(3)
        t, _ = median_step_phases(sim, steps)
        sim.timing(False)
        sim.step(acc_steps - sim.step(0, diag=True)["step"])
        ez = sim.axis_field("Ez")
        fb = sim.step(0, diag=True)["fallbacks"]
        sim.close()
        return t, ez, fb

    dn = Denoiser(theta, stream=stream)
    t_lo, ez_net, fallbacks = run((1, 1, 1), dn)
    dn.close()
    t_plain, ez_plain, _ = run((1, 1, 1))
    t_hi, ez_ref, _ = run((2, 2, 4))
    nr = float(np.linalg.norm(ez_ref))
    return {"workload": "lwfa3d physics at 1 ppc + network (3->16->32->16->3 BF16 MFMA) against 16 ppc, "
                        f"seed {seed} (held out from training)",
            "ms_per_step_1ppc_net": t_lo["step"], "ms_per_step_16ppc": t_hi["step"],
            "ratio": t_hi["step"] / t_lo["step"],
            "ms_per_step_1ppc_plain": t_plain["step"],
            "ez_axis_steps": acc_steps,
            "ez_axis_rel_err_net": float(np.linalg.norm(ez_net - ez_ref)) / nr,
            "ez_axis_rel_err_plain_1ppc": float(np.linalg.norm(ez_plain - ez_ref)) / nr,
            "fallbacks": fallbacks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the march, denoise and pwfa objects")
    ap.add_argument("--march-only", action="store_true",
                    help="only the zeta-march object (no CPU oracle), for profiling")
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
    if args.march_only:
        m, _ = bench_march(stream, cpu=False)
        print(json.dumps({"march": m}), flush=True)
        return
    cfg = workloads.pwfa3d_fp32() if args.workload == "pwfa" else workloads.lwfa3d_fp32()
    ppc = cfg["ppc"][0] * cfg["ppc"][1] * cfg["ppc"][2]
    sim = Sim(cfg, stream=stream)
    print(f"[bench] created {cfg['n']} ppc={ppc}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    n0 = sim._count()
    print(f"[bench] warmup {args.warmup} steps done, {n0} particles", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    med, rows = median_step_phases(sim, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n1 = sim._count()
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)

    import hashlib
    src = open(os.path.join(ROOT, "paper_2509_16793_amd", "csrc", "push.h"), "rb").read()
    same_kernel = hashlib.sha256(src).hexdigest()[:16] == MEASURED_TRAFFIC["push_h_sha256_prefix"]
    traffic = MEASURED_TRAFFIC["bytes_per_launch"] if same_kernel and args.workload == "lwfa" else None
    n_avg = 0.5 * (n0 + n1)
    launch_s = med["push_deposit"] / 1e3
    value = n_avg / launch_s
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
                     "traffic_achieved": traffic / launch_s / 1e9 if traffic else None,
                     "traffic_frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS if traffic else None,
                     "kernel": "k_push_deposit", "bytes_per_update": bpu,
                     "median_launch_ms": launch_s * 1e3,
                     "mean_launch_ms": statistics.fmean(r["push_deposit"] for r in rows)},
        "phase_ms_per_step": med,
        "step_updates_per_s": n_avg / (med["step"] / 1e3),
    }
    sim.close()
    if args.workload == "lwfa" and not args.no_extras:
        print("[bench] zeta march", file=sys.stderr, flush=True)
        m, _ = bench_march(stream, cpu=not args.no_cpu_baseline)
        m["lwfa"]["tau_ms_for_same_delta"] = med["step"] * m["lwfa"]["delta_over_dtau"]
        m["lwfa"]["speedup_over_tau"] = m["lwfa"]["tau_ms_for_same_delta"] / m["lwfa"]["ms_per_slow_step"]
        out["march"] = m
        print("[bench] denoiser", file=sys.stderr, flush=True)
        out["denoise"] = bench_denoise(stream)
        print("[bench] pwfa", file=sys.stderr, flush=True)
        out["pwfa"] = bench_pwfa(stream)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on crops", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
        if args.workload == "lwfa":
            print("[bench] the 2-D case in full, GPU and oracle", file=sys.stderr, flush=True)
            out["cpu_baseline"]["lwfa2d_full_step"] = full_step_2d(stream)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
