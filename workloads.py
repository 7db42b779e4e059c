"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and bench.py.

This module only holds parameter sets (plain numbers in the units the workload
is stated in).  It contains none of the method's arithmetic: unit conversion,
particle loading, random offsets and every other derived quantity are computed
independently by the oracle (``oracle/``) and by the HIP library.

Lengths and times are in laser wavelengths (lambda_L = 1, c = 1) unless
``length_unit`` says otherwise; ``length_unit`` is the factor that turns them
into the paper's normalised units c/omega_0 (2*pi for lambda_L units, 1 when
the workload is already in c/omega_0).  Densities are in units of the critical
density of omega_0 (so omega_p^2 = n_e).
"""
import math

TWO_PI = 2.0 * math.pi


def _base(**kw):
    cfg = dict(
        dims=3, n=[64, 64, 64], d=[0.4, 0.4, 0.05], length_unit=TWO_PI,
        dtau=0.0,             # 0 -> half the zeta step
        precision="fp32",     # "fp64" | "fp32" (cell+offset) | "fp32abs"
        tile=[8, 8, 8],
        n_e=0.0, ppc=[1, 1, 2], load=0,   # load 0 = stratified random, 1 = quiet lattice
        a0=0.0, waist=0.0, fwhm=0.0, zeta_c=None, pol=0,
        seed=0, filter_passes=1, steps=1,
        beam=None,
    )
    cfg.update(kw)
    return cfg


def lwfa2d_fp64():
    """2-D (x, zeta) LWFA, 64 x 256, dx = 0.25, dzeta = 0.05, n_e = 0.01, 2 ppc,
    a0 = 1, FWHM 5, waist 4, laser centred at zeta = 200 dzeta; 100 steps, FP64."""
    return _base(dims=2, n=[64, 1, 256], d=[0.25, 1.0, 0.05], precision="fp64",
                 tile=[8, 1, 8], n_e=0.01, ppc=[1, 1, 2], a0=1.0, waist=4.0,
                 fwhm=5.0, zeta_c=200 * 0.05, steps=100)


def lwfa3d_fp32(ppc=(1, 1, 2), steps=1000):
    """3-D LWFA, 256 x 256 x 512, dx = dy = 0.4, dzeta = 0.05, n_e = 0.001, 2 ppc
    (67,108,864 electrons), a0 = 2, waist 8, FWHM 8; FP32 cell + offset,
    8 x 8 x 4 particle tiles."""
    return _base(dims=3, n=[256, 256, 512], d=[0.4, 0.4, 0.05], precision="fp32",
                 tile=[8, 8, 4], n_e=0.001, ppc=list(ppc), a0=2.0, waist=8.0,
                 fwhm=8.0, zeta_c=None, steps=steps)


def precision_study(mode):
    """As lwfa3d_fp32 at 8 ppc (268,435,456 electrons), 200 steps, in one of the
    three precision modes."""
    c = lwfa3d_fp32(ppc=(2, 2, 2), steps=200)
    c["precision"] = mode
    return c


def pwfa3d_fp32():
    """3-D PWFA in plasma units: 512 x 512 x 1024, dx = dy = 0.1, dzeta = 0.05,
    n_e = 1, 4 ppc (1,073,741,824 electrons at load), Gaussian driver
    sigma_r = 0.5, sigma_zeta = 1, peak 10 n_e, gamma = 2000 with 0.1 % spread,
    1e7 macro-particles; 500 steps; FP32 cell + offset, 8 x 8 x 4 tiles."""
    return _base(dims=3, n=[512, 512, 1024], d=[0.1, 0.1, 0.05], length_unit=1.0,
                 precision="fp32", tile=[8, 8, 4], n_e=1.0, ppc=[1, 2, 2],
                 steps=500, a0=0.0,
                 beam=dict(n=10.0, sr=0.5, sz=1.0, zc=None, gamma=2000.0,
                           dgamma=2.0, np=10_000_000))


def pwfa_small(precision="fp64", n=(32, 32, 64), tile=(8, 8, 8), ppc=(1, 1, 1),
               np_beam=3000, seed=5, steps=4):
    """Small PWFA case for parity tests: the plasma-unit physics of pwfa3d_fp32
    with a shorter, narrower driver (sigma_r = sigma_zeta = 0.3) that fits the
    small box."""
    return _base(dims=3, n=list(n), d=[0.1, 0.1, 0.05], length_unit=1.0,
                 precision=precision, tile=list(tile), n_e=1.0, ppc=list(ppc),
                 steps=steps, a0=0.0, seed=seed,
                 beam=dict(n=10.0, sr=0.3, sz=0.3, zc=None, gamma=2000.0,
                           dgamma=2.0, np=np_beam))


def denoiser_lwfa(ppc=(1, 1, 1)):
    """lwfa3d_fp32 at 1 ppc (the network's input) or 16 ppc (its reference)."""
    return lwfa3d_fp32(ppc=ppc, steps=1000)


def denoiser_train(ppc=(1, 1, 1), seed=0, n=(64, 64, 512)):
    """Training runs of the denoiser: the physics of denoiser_lwfa in a
    64 x 64 cell transverse box (periodic), so that every 64^3 training crop
    spans the full periodic cross-section and needs a halo only in zeta."""
    cfg = lwfa3d_fp32(ppc=ppc, steps=1000)
    cfg.update(n=list(n), seed=seed)
    return cfg


def denoiser_init(seed=0, last_scale=1.0, bias_scale=0.0):
    """Initial FP32 weights of the 3 -> 16 -> 32 -> 16 -> 3 denoiser, flat,
    layer by layer as (W[Cout][Cin][kz][ky][kx], b[Cout]): He-uniform bounds
    sqrt(6 / (27 Cin)), the last layer scaled by ``last_scale`` (0 starts the
    network as the plain filter), biases uniform in +-bias_scale."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    layers = ((3, 16), (16, 32), (32, 16), (16, 3))
    for l, (ci, co) in enumerate(layers):
        bound = math.sqrt(6.0 / (27 * ci))
        W = rng.uniform(-bound, bound, size=co * ci * 27)
        if l == len(layers) - 1:
            W = W * last_scale
        parts += [W, rng.uniform(-bias_scale, bias_scale, size=co)]
    return np.concatenate(parts).astype(np.float32)


def small3d(precision="fp64", n=(32, 32, 64), tile=(8, 8, 8), ppc=(1, 1, 2),
            steps=4, a0=1.0, seed=3, n_e=0.01):
    """Small 3-D LWFA-like case: several tiles in every direction, a laser strong
    enough to move particles across cells, finishes in seconds on a CPU."""
    return _base(dims=3, n=list(n), d=[0.4, 0.4, 0.05], precision=precision,
                 tile=list(tile), n_e=n_e, ppc=list(ppc), a0=a0, waist=3.0,
                 fwhm=1.5, zeta_c=None, steps=steps, seed=seed)


def lwfa_channel(nz=4096, delta=40.0, scheme=2, nodes=None):
    """The paper's example (Sec. 6) scaled down to one GPU and without
    ionisation: hydrogen plasma in a Gaussian channel, n_e = n_0 [1 + (n_1 -
    n_0) / n_0 exp(-r^2 / R_ch^2)] with n_0 = 5e17 cm^-3 (2.9e-4 of the
    critical density at 0.8 um), n_1 / n_0 = 0.25 on the axis, R_ch = 76.4 um
    (95.5 lambda); laser a0 = 2, T = 50.9 fs in exp(-phi^2 / T^2) (19.1
    lambda, intensity FWHM 22.5 lambda), R = 22.9 um (28.6 lambda); window
    150 x 150 x 180 um (187.5 x 187.5 x 225 lambda) at h_x = h_y = 1.46
    lambda (128 x 128) and h = 50 nm (0.0549 lambda, 4096 nodes); zeta march
    with Delta = 32 um (40 lambda), in GT2: with GT1 and Delta < L the
    parked plasma stitches the density every Delta (Sec. 5), which the
    temporal transformation avoids.  Lengths in lambda = 0.8 um.
    nodes: optional zeta node positions (a refined rear, as the paper's
    6.3 nm rear third)."""
    cfg = _base(dims=3, n=[128, 128, nz], d=[187.5 / 128, 187.5 / 128, 225.0 / nz], precision="fp32",
                tile=[8, 8, 4], n_e=2.9e-4, ppc=[1, 1, 1], a0=2.0, waist=28.6, fwhm=22.5,
                zeta_c=225.0 - 40.0, steps=20)
    cfg.update(scheme=scheme, delta=delta, ch_ratio=0.25, ch_radius=95.5)
    if nodes is not None:
        cfg["zeta_nodes"] = list(nodes)
    return cfg


def channel_small(precision="fp64", scheme=1, delta=0.5):
    """A small 3-D zeta-march case with the Gaussian channel, for parity tests."""
    cfg = small3d(precision=precision, n=(32, 32, 64), tile=(8, 8, 4))
    cfg.update(scheme=scheme, delta=delta, ch_ratio=0.25, ch_radius=3.0)
    return cfg


CONFIGS = {
    "lwfa2d_fp64": lwfa2d_fp64,
    "lwfa3d_fp32": lwfa3d_fp32,
    "precision_study": precision_study,
    "pwfa3d_fp32": pwfa3d_fp32,
    "denoiser_lwfa": denoiser_lwfa,
    "lwfa_channel": lwfa_channel,
}
