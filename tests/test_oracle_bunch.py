"""Pins of the witness-bunch diagnostics (Table 1 style, oracle/bunch.py) and
of the Gaussian plasma channel (Sec. 6, eq. n_plasma) of the zeta march.

* Closed forms: a four-particle set with uncorrelated x and u_x has
  emittance a b; a laminar (fully correlated) set has zero emittance; weights
  act as multiplicities; particles below gamma_min are not counted.
* The host-sampled Gaussian driver (oracle/plasma.py) reproduces the requested
  rms sizes, mean and spread of gamma within five standard errors, has zero
  emittance (u_perp = 0) and the bunch charge.
* Channel: every fresh particle's weight is the closed-form density at its
  transverse position times h_x h_y Delta / ppc; a batch holds
  n_e Delta [A + (ratio - 1) pi R^2] electrons to O(h^2) when the channel lies
  inside the box; ratio 1 is the uniform plasma bit for bit."""
import math

import numpy as np

import workloads
from oracle import bunch
from oracle.march import MarchParams, batch
from oracle.plasma import load_beam
from oracle import params


def test_closed_form_moments_and_emittance():
    a, b = 0.7, 0.3
    x = np.array([a, -a, a, -a])
    ux = np.array([b, -b, -b, b])
    z = np.zeros(4)
    uz = np.full(4, 100.0)
    r = bunch.moments(x, z, z, ux, z, uz, np.ones(4), 10.0)
    assert r["n_macro"] == 4 and r["charge"] == -4.0
    assert abs(r["sigma_x"] - a) < 1e-15 and abs(r["eps_x"] - a * b) < 1e-15 and r["eps_y"] == 0.0
    # laminar: u_x proportional to x
    r = bunch.moments(x, z, z, 2.0 * x, z, uz, np.ones(4), 10.0)
    assert r["eps_x"] < 1e-15
    # weights are multiplicities; slow particles are not counted
    x5 = np.r_[x, 5.0]
    ux5 = np.r_[ux, 0.0]
    uz5 = np.r_[uz, 0.0]
    w = np.array([2.0, 2.0, 2.0, 2.0, 7.0])
    r2 = bunch.moments(x5, np.zeros(5), np.zeros(5), ux5, np.zeros(5), uz5, w, 10.0)
    assert r2["n_macro"] == 4 and r2["charge"] == -8.0 and abs(r2["eps_x"] - a * b) < 1e-15
    g = math.sqrt(1 + 100.0 ** 2 + b * b)
    assert abs(r2["gamma_mean"] - g) < 1e-12 and r2["gamma_rms"] < 1e-12


def test_sampled_driver_reproduces_its_parameters():
    cfg = workloads.pwfa_small(np_beam=20000)
    p = params.from_config(cfg)
    B = load_beam(p)
    x, y, z = bunch.positions_tau(p, B)
    r = bunch.moments(x, y, z, B.ux, B.uy, B.uz, np.full(len(B), p.beam["w"]), 100.0)
    n = len(B)
    sr, sz = p.beam["sr"], p.beam["sz"]
    assert abs(r["sigma_x"] - sr) < 5 * sr / math.sqrt(2 * n)
    assert abs(r["sigma_y"] - sr) < 5 * sr / math.sqrt(2 * n)
    assert abs(r["sigma_z"] - sz) < 5 * sz / math.sqrt(2 * n)
    assert abs(r["mean_z"] - p.beam["zc"]) < 5 * sz / math.sqrt(n)
    assert abs(r["gamma_mean"] - 2000.0) < 5 * 2.0 / math.sqrt(n)
    assert abs(r["gamma_rms"] - 2.0) < 5 * 2.0 / math.sqrt(2 * n)
    assert r["eps_x"] == 0.0 and r["eps_y"] == 0.0
    assert abs(r["charge"] + n * p.beam["w"]) < 1e-9 * n * p.beam["w"]


def test_channel_weights():
    cfg = workloads.channel_small()
    m = MarchParams(cfg)
    p = m.p
    B = batch(m, 3, m.L)
    X, Y = (B.ix + B.dx) * p.hx, (B.iy + B.dy) * p.hy
    r2 = (X - (p.Nx // 2) * p.hx) ** 2 + (Y - (p.Ny // 2) * p.hy) ** 2
    n = p.n_e * (1.0 + (m.ratio - 1.0) * np.exp(-r2 / (m.R * m.R)))
    assert np.max(np.abs(B.w - n * p.hx * p.hy * m.Delta)) < 1e-15 * np.max(B.w)
    A = p.Nx * p.hx * p.Ny * p.hy
    want = p.n_e * m.Delta * (A + (m.ratio - 1.0) * math.pi * m.R ** 2)
    assert abs(np.sum(B.w) - want) < 2e-3 * want
    # ratio 1: the uniform plasma
    c1 = dict(cfg)
    c1["ch_ratio"] = 1.0
    m1 = MarchParams(c1)
    u = batch(m1, 3, m1.L)
    c0 = dict(cfg)
    c0.pop("ch_ratio")
    c0.pop("ch_radius")
    m0 = MarchParams(c0)
    assert np.array_equal(u.w, batch(m0, 3, m0.L).w)
