"""Linear wake behind a plane-wave Gaussian laser pulse in a cold uniform
plasma (test helper, shared by the oracle and the GPU tests): the
configuration, and on-axis E_z against linear theory.

Pulse a0 = 0.1, T = 4.247 lambda in exp(-phi^2 / T^2), centred 12 lambda
behind the front of a 51.2 lambda box; plasma n_e = 0.01 n_c.  For a0 << 1
the wake behind a Gaussian pulse has the amplitude
E_max = k_p^2 (a0^2 / 4) T sqrt(pi / 2) exp(-k_p^2 T^2 / 8) and
half-periods lambda_p / 2 (units c / omega_0, k_p^2 = n_e / n_c)."""
import numpy as np

import workloads
from oracle.params import from_config

A0, N_E, T_LAMBDA = 0.1, 0.01, 4.247


def wake_cfg(nz, delta, scheme, nx=2, tile=(2, 1, 8), precision="fp64"):
    """2-D (x, zeta) box of nx x nz cells, transversally uniform plasma and
    pulse; zeta march with slow step delta (lambda) in scheme 1 (GT1) or 2
    (GT2)."""
    cfg = workloads._base(dims=2, n=[nx, 1, nz], d=[0.25, 1.0, 51.2 / nz], n_e=N_E, ppc=[1, 1, 1], load=1,
                          a0=A0, waist=0.0, fwhm=T_LAMBDA * np.sqrt(2 * np.log(2)), zeta_c=51.2 - 12.0,
                          tile=list(tile), precision=precision)
    cfg.update(scheme=scheme, delta=delta)
    return cfg


def wake_measure(cfg, ez_axis):
    """Peak |E_z| over the first plasma period behind the pulse (from 2.6 T
    behind its centre) in units of linear theory, and the distances between
    the zero crossings there (interpolated between nodes) in units of
    lambda_p / 2.  ez_axis: E_z on the
    nodes zeta_n = n h, n = 0 .. Nz - 1."""
    p = from_config(cfg)
    kp, T = np.sqrt(N_E), p.T
    amp = kp ** 2 * (A0 ** 2 / 4) * T * np.sqrt(np.pi / 2) * np.exp(-kp ** 2 * T ** 2 / 8)
    lam = 2 * np.pi / kp
    zeta = np.arange(p.Nz) * p.h
    win = (zeta < p.zeta_c - 2.6 * T) & (zeta > p.zeta_c - 2.6 * T - 1.2 * lam)
    e = np.asarray(ez_axis, float)[win]
    z = zeta[win]
    # zero crossings, linearly interpolated between the nodes around each
    i = np.nonzero(np.sign(e[:-1]) != np.sign(e[1:]))[0]
    zc = z[i] - e[i] * (z[i + 1] - z[i]) / (e[i + 1] - e[i])
    return np.abs(e).max() / amp, np.diff(zc) / (lam / 2)
