"""Training and evaluation of the learned current denoiser.

Every step runs in the HIP library (gempic_* and gempic_dn_* entry points);
this module only orders the calls and keeps the sampled currents on the
device (torch supplies the memory).

Training data: pairs of runs with the same physics and seed at 1 and 16
macro-particles per cell (the LWFA setup in a 64 x 64 cell periodic
transverse box, workloads.denoiser_train).  Every `every` steps the raw
deposited currents of both runs are captured and `crops` zeta-windows of
64 planes plus a halo of 5 planes on each side are cut from them (the full
periodic cross-section, so every crop is a 64^3 training region whose
network receptive field, 4 voxels, plus the curl, 1 voxel, stays inside the
window).  The loss region is the central 64 planes.

Evaluation: the full-size 1-ppc run with and without the network against
the 16-ppc run of the same seed: relative L2 difference of on-axis E_z over
zeta after given steps, and wall time per step.

    python -m paper_2509_16793_amd.denoiser_study train --seeds 0-63 --out W.npy
    python -m paper_2509_16793_amd.denoiser_study eval --weights W.npy --seeds 64-67
    python -m paper_2509_16793_amd.denoiser_study step --weights W.npy --steps 5
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HALO = 5
CROP = 64


def _seeds(spec):
    if "-" in spec:
        a, b = spec.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in spec.split(",")]


def _ctx():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the denoiser study needs a GPU")
    return torch


def grid_steps(cfg):
    """(h_x, h_y, h_zeta) in the library's normalised units."""
    lu = cfg["length_unit"]
    return tuple(float(v) * lu for v in cfg["d"])


def capture_pairs(seeds, steps, every, crops, first, rng, log=print):
    """Sampled (raw 1-ppc current, raw 16-ppc current) crops, each a device
    tensor [3, CROP + 2 HALO, Ny, Nx]."""
    torch = _ctx()
    import workloads
    from .gempic import Sim
    X, T = [], []
    for s in seeds:
        lo = Sim(workloads.denoiser_train(ppc=(1, 1, 1), seed=s))
        hi = Sim(workloads.denoiser_train(ppc=(2, 2, 4), seed=s))
        shape = (3, lo.NPJ, lo.Ny, lo.Nx)
        jl = torch.empty(shape, dtype=torch.float32, device="cuda")
        jh = torch.empty(shape, dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        for k in range(every, steps + 1, every):
            lo.step(every)
            hi.step(every)
            if k < first:
                continue
            lo.fields_device(("Jx", "Jy", "Jz"), jl)
            hi.fields_device(("Jx", "Jy", "Jz"), jh)
            w = CROP + 2 * HALO
            for _ in range(crops):
                z0 = int(rng.integers(0, lo.NPJ - w + 1))
                X.append(jl[:, z0:z0 + w].contiguous())
                T.append(jh[:, z0:z0 + w].contiguous())
        torch.cuda.synchronize()
        log(f"seed {s}: {len(X)} crops so far, {time.perf_counter() - t0:.1f} s")
        lo.close()
        hi.close()
    return X, T


def train(X, T, n_e, h, iters, batch, lr, rng, theta=None, log=print, log_every=100):
    """Adam with cosine decay over ``iters`` steps of ``batch`` crops."""
    torch = _ctx()
    import workloads
    from .gempic import Denoiser
    if theta is None:
        theta = workloads.denoiser_init(seed=0, last_scale=0.0)
    d = Denoiser(theta)
    region = (HALO, HALO + CROP)
    hist = []
    for it in range(iters):
        idx = rng.integers(0, len(X), batch)
        jr = torch.stack([X[i] for i in idx])
        jt = torch.stack([T[i] for i in idx])
        lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * it / iters))
        loss = d.train(jr, jt, n_e, h, region, lr_t)
        hist.append(loss)
        if it % log_every == 0 or it == iters - 1:
            log(f"iter {it}: loss {loss:.5g} (lr {lr_t:.3g})")
    return d, hist


def plain_loss(X, T, n_e, h, n=64, rng=None):
    """Mean loss of the filtered current alone (a network with zero output)
    over up to n crops: the baseline the training has to beat."""
    import workloads
    from .gempic import Denoiser
    d = Denoiser(workloads.denoiser_init(seed=0, last_scale=0.0))
    torch = _ctx()
    ls = []
    for i in range(min(n, len(X))):
        ls.append(d.train(X[i][None], T[i][None], n_e, h, (HALO, HALO + CROP), 0.0))
    d.close()
    return float(np.mean(ls))


def on_axis_ez(sim):
    """E_z along the axis node column (Nx/2, Ny/2), FP64, one value per plane."""
    return sim.axis_field("Ez")


def run_timed(sim, nsteps):
    torch = _ctx()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(nsteps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def evaluate(theta, seeds, checkpoints, cfg_fn, threshold=1e-3, log=print):
    """Per seed: on-axis E_z of 1 ppc plain / 1 ppc + network against 16 ppc
    at each checkpoint, and seconds per step of each run."""
    from .gempic import Denoiser, Sim
    out = []
    d = Denoiser(theta)
    for s in seeds:
        rec = dict(seed=s)
        ez = {}
        for name, ppc, den in (("ppc16", (2, 2, 4), False), ("ppc1", (1, 1, 1), False),
                               ("ppc1_net", (1, 1, 1), True)):
            sim = Sim(cfg_fn(ppc, s))
            if den:
                sim.set_denoiser(d, threshold)
            t, k = 0.0, 0
            ez[name] = []
            for c in checkpoints:
                t += run_timed(sim, c - k)
                k = c
                ez[name].append(on_axis_ez(sim))
            rec[f"ms_per_step_{name}"] = 1e3 * t / k
            if den:
                rec["fallbacks"] = sim.step(0, diag=True)["fallbacks"]
            sim.close()
        for i, c in enumerate(checkpoints):
            ref = ez["ppc16"][i]
            nr = np.linalg.norm(ref)
            rec[f"err_plain_{c}"] = float(np.linalg.norm(ez["ppc1"][i] - ref) / nr)
            rec[f"err_net_{c}"] = float(np.linalg.norm(ez["ppc1_net"][i] - ref) / nr)
        rec["speedup_vs_ppc16"] = rec["ms_per_step_ppc16"] / rec["ms_per_step_ppc1_net"]
        log(json.dumps(rec))
        out.append(rec)
    d.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--seeds", default="0-63")
    tr.add_argument("--steps", type=int, default=1000)
    tr.add_argument("--every", type=int, default=50)
    tr.add_argument("--first", type=int, default=100)
    tr.add_argument("--crops", type=int, default=2)
    tr.add_argument("--iters", type=int, default=2000)
    tr.add_argument("--batch", type=int, default=8)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--out", required=True)
    tr.add_argument("--log", default=None)
    ev = sub.add_parser("eval")
    ev.add_argument("--weights", required=True)
    ev.add_argument("--seeds", default="64-67")
    ev.add_argument("--checkpoints", default="500,1000")
    ev.add_argument("--narrow", action="store_true", help="64 x 64 transverse box")
    ev.add_argument("--threshold", type=float, default=1e-3)
    ev.add_argument("--out", default=None)
    st = sub.add_parser("step", help="time steps of the full-size 1-ppc run with the network")
    st.add_argument("--weights", required=True)
    st.add_argument("--steps", type=int, default=5)
    st.add_argument("--warmup", type=int, default=3)
    a = ap.parse_args(argv)
    # torch carries its own HIP runtime: load it before the library so that
    # both share one runtime in this process
    _ctx()

    logf = open(a.log, "a") if getattr(a, "log", None) else None

    def log(msg):
        print(msg, flush=True)
        if logf:
            logf.write(msg + "\n")
            logf.flush()

    import workloads
    if a.cmd == "step":
        from .gempic import Denoiser, Sim
        d = Denoiser(np.load(a.weights))
        sim = Sim(workloads.denoiser_lwfa(ppc=(1, 1, 1)))
        sim.set_denoiser(d, 1e-3)
        sim.step(a.warmup)
        sim.timing(True)
        t = run_timed(sim, a.steps)
        ph, n = sim.get_timing()
        log(json.dumps(dict(ms_per_step=1e3 * t / a.steps,
                            phase_ms_per_step={k: v / n for k, v in ph.items()},
                            fallbacks=sim.step(0, diag=True)["fallbacks"])))
        sim.close()
        d.close()
        return 0
    if a.cmd == "train":
        rng = np.random.default_rng(1234)
        cfg = workloads.denoiser_train()
        h = grid_steps(cfg)
        n_e = cfg["n_e"]
        X, T = capture_pairs(_seeds(a.seeds), a.steps, a.every, a.crops, a.first, rng, log)
        base = plain_loss(X, T, n_e, h)
        log(f"plain (filter only) loss: {base:.5g}")
        d, hist = train(X, T, n_e, h, a.iters, a.batch, a.lr, rng, log=log)
        theta = d.params()
        np.save(a.out, theta)
        tail = float(np.mean(hist[-50:]))
        log(json.dumps(dict(plain_loss=base, final_loss=tail, crops=len(X), iters=a.iters)))
    else:
        theta = np.load(a.weights)
        cps = [int(v) for v in a.checkpoints.split(",")]
        if a.narrow:
            fn = lambda ppc, s: workloads.denoiser_train(ppc=ppc, seed=s)
        else:
            fn = lambda ppc, s: dict(workloads.denoiser_lwfa(ppc=ppc), seed=s)
        res = evaluate(theta, _seeds(a.seeds), cps, fn, a.threshold, log)
        summ = {k: float(np.mean([r[k] for r in res])) for k in res[0] if k != "seed"}
        log(json.dumps(dict(mean=summ)))
        if a.out:
            with open(a.out, "w") as f:
                json.dump(dict(runs=res, mean=summ), f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
