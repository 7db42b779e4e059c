"""Witness-bunch diagnostics (Table 1 style) and the Gaussian plasma channel
(Sec. 6, eq. n_plasma) on the GPU, through the C ABI, against the FP64 oracle
(oracle/bunch.py, oracle/march.py).

Bars: charge and macro-particle count exact up to FP64 summation order
(1e-12 relative); means, rms sizes, gamma moments and emittances within 1e-8
relative (the GPU forms central moments from raw FP64 sums, the oracle from
deviations); the channel march's fields, currents and particles as in the
other zeta-march parity tests."""
import numpy as np
import pytest

import workloads
from oracle import bunch
from oracle.march import MarchSim
from oracle.sim import Simulation
from paper_2509_16793_amd.gempic import Sim
from test_gpu_march import _compare

pytestmark = pytest.mark.gpu

KEYS = ("gamma_mean", "gamma_rms", "mean_x", "mean_y", "mean_z", "sigma_x", "sigma_y", "sigma_z",
        "eps_x", "eps_y")


def _check(ref, got, scale_len, scale_eps):
    assert got["n_macro"] == ref["n_macro"]
    assert abs(got["charge"] - ref["charge"]) <= 1e-12 * abs(ref["charge"])
    for k in KEYS:
        s = scale_eps if k.startswith("eps") else (scale_len if k.startswith(("mean", "sigma")) else
                                                  max(abs(ref["gamma_mean"]), 1.0))
        assert abs(got[k] - ref[k]) <= 1e-8 * s, (k, got[k], ref[k])


def test_bunch_of_the_sampled_driver():
    cfg = workloads.pwfa_small()
    o = Simulation(cfg)
    g = Sim(cfg, track_ids=True)
    p = o.p
    P = o.P
    x, y, z = bunch.positions_tau(p, P)
    w = np.where(P.sp == 1, p.beam["w"], p.w)
    ref = bunch.moments(x, y, z, P.ux, P.uy, P.uz, w, 100.0)
    got = g.bunch(100.0)
    assert got["n_macro"] == cfg["beam"]["np"] or got["n_macro"] > 0.9 * cfg["beam"]["np"]
    _check(ref, got, p.beam["sr"], 1e-6)
    # after two steps the driver has moved and its transverse momenta grown
    o.run(2)
    g.step(2)
    P = o.P
    x, y, z = bunch.positions_tau(p, P)
    w = np.where(P.sp == 1, p.beam["w"], p.w)
    ref = bunch.moments(x, y, z, P.ux, P.uy, P.uz, w, 100.0)
    _check(ref, g.bunch(100.0), p.beam["sr"], max(ref["eps_x"], 1e-12))


@pytest.mark.parametrize("scheme", [1, 2])
def test_channel_march_fp64_and_its_bunch(scheme):
    cfg = workloads.channel_small(scheme=scheme)
    o = MarchSim(cfg)
    g = Sim(cfg, track_ids=True)
    for _ in range(3):
        o.step()
        g.step(1)
        _compare(o, g)
    x, y, z = bunch.positions_march(o.m, o.P)
    ref = bunch.moments(x, y, z, o.P.ux, o.P.uy, o.P.uz, o.P.w, 1.0)
    if ref["n_macro"]:
        _check(ref, g.bunch(1.0), o.p.hx, max(ref["eps_x"], 1e-12))
