"""Pins of the zeta-march oracle (oracle/march.py): the paper's slow step with
the particles integrated along zeta (Sec. 5, eq:trap1 / eq:trap2), fresh
macro-particles of charge Q_f (Sec. 5.1) and the interleaved right-to-left
march (Sec. 4.1).

* The Sec. 2 / Fig. 1 electron in a plane wave E_x = B_y = A'(zeta),
  integrated in zeta: u_x equals -q times the trapezoid integral of the node
  E_x from the right edge exactly (du_x / d zeta = -q E_x when E_x = B_y, and the midpoint rule is
  exact on the linear interpolant), u_x = A + O(h^2), gamma - u_z = 1 and the
  elapsed slow time int gamma d zeta to second order, at rest after the pulse.
* A fresh plasma drifting at v deposits j = q n v / (1 - v_z) (Sec. 5.1).
* Charge conservation: cell charges, transverse currents and node fluxes
  satisfy the discrete continuity equation to roundoff (GT1 with and without
  parked particles, GT2, 2-D and 3-D, laser-driven).
* In vacuum the stage-by-stage march equals the all-nodes march of
  oracle/fields.py (a second route), and creation equals laser_state.
* Delta <= h: the scheme reduces to the tau push, converging at second order
  to a reference integration (and to the Higuera-Cary tau trajectory).
* GT2 stop rule: a particle at rest streams through the whole box in one step
  (GT1 parks it after Delta); a forward-moving one stops after its lab z has
  advanced by Delta, i.e. at zeta displacement -(1 - v_z) Delta / v_z."""
import math

import numpy as np
import pytest

import workloads
from oracle import fields as ofields
from oracle.march import MarchSim, continuity_residual, init_state, velocity
from oracle.push import higuera_cary


def _cfg(n=(2, 2, 200), d=(0.5, 0.5, 0.1), **kw):
    c = workloads._base(dims=3, n=list(n), d=list(d), length_unit=1.0, precision="fp64",
                        tile=[n[0], n[1], 4], n_e=1e-6, ppc=[1, 1, 1], load=1, a0=0.0, seed=7)
    c.update(delta=1000.0, scheme=1)
    c.update(kw)
    return c


def _pulse(zeta, a0=1.0, zc=12.8, sig=1.5):
    ph = zeta - zc
    A = a0 * np.cos(ph) * np.exp(-ph * ph / (2 * sig * sig))
    dA = a0 * (-np.sin(ph) - ph / (sig * sig) * np.cos(ph)) * np.exp(-ph * ph / (2 * sig * sig))
    return A, dA


def _plane_wave_run(h):
    Nz = int(round(25.6 / h))
    s = MarchSim(_cfg(n=(2, 2, Nz), d=(0.5, 0.5, h)), solver=False)
    zn = s.m.zn[:Nz]
    _, dA = _pulse(zn)
    s.F0[:] = 0.0
    s.F0[0, :Nz] = dA[:, None, None]
    s.F0[4, :Nz] = dA[:, None, None]
    s.trace = []
    s.step()
    E = np.r_[dA, 0.0]
    # trapezoid integral of the node E_x from the right edge to node n
    trap = np.r_[np.cumsum((0.5 * h * (E[:-1] + E[1:]))[::-1])[::-1], 0.0]
    return s, trap


def test_plane_wave_electron_integrated_in_zeta():
    errs = []
    for h in (0.1, 0.05):
        s, trap = _plane_wave_run(h)
        zn = s.m.zn
        A, _ = _pulse(zn)
        e_g, e_s, e_a = 0.0, 0.0, 0.0
        # elapsed slow time to node n: int gamma d zeta with gamma = 1 + A^2 / 2
        fine = np.linspace(0.0, 25.6, 256001)
        Af, _ = _pulse(fine)
        g_int = np.cumsum(((1 + 0.5 * Af ** 2)[1:] + (1 + 0.5 * Af ** 2)[:-1]) * 0.5 * (fine[1] - fine[0]))
        g_int = np.r_[0.0, g_int]
        for n, P in s.trace:
            assert len(P) == 4
            # exact: u_x = -q times the integral of the interpolated E_x
            # from the right edge down to node n (trapezoid sum, q = -1)
            assert np.max(np.abs(P.ux + trap[n])) < 1e-11
            g, _, _, _, _ = velocity(P.ux, P.uy, P.uz)
            e_g = max(e_g, np.max(np.abs(g - P.uz - 1.0)))
            e_a = max(e_a, np.max(np.abs(P.ux - A[n])))
            want = g_int[-1] - np.interp(zn[n], fine, g_int)
            e_s = max(e_s, np.max(np.abs((s.m.Delta - P.b) - want)) / want)
        errs.append((e_g, e_a, e_s))
        # after the pulse (node 0): at rest up to the scheme's error
        n0, P0 = s.trace[-1]
        assert n0 == 0 and np.max(np.abs(P0.ux)) < 1e-8 and np.max(np.abs(P0.uz)) < 5 * h * h
        assert e_g < 5 * h * h and e_a < 5 * h * h and e_s < 5 * h * h
    for a, b in zip(errs[0], errs[1]):
        assert 3.0 < a / b < 5.0, errs       # second order


def test_fresh_drifting_plasma_deposits_qnv_over_one_minus_vz():
    n_e = 0.01
    cfg = _cfg(n=(4, 4, 32), d=(0.5, 0.5, 0.1), n_e=n_e, delta=100.0)
    s = MarchSim(cfg, solver=False, record=True)
    u0 = (0.3, 0.2, 0.4)
    s.inject_u0 = u0
    s.step()
    g = math.sqrt(1 + sum(u * u for u in u0))
    v = [u / g for u in u0]
    J = s.J
    q = -1.0
    for c in range(3):
        want = q * n_e * v[c] / (1.0 - v[2])
        assert np.max(np.abs(J[c] - want)) < 1e-12 * abs(want), c
    assert len(s.left) == 16 and len(s.P) == 0


@pytest.mark.parametrize("dims,scheme,delta", [(3, 1, 0.5), (3, 1, 50.0), (3, 2, 0.5), (2, 1, 0.7)],
                         ids=["gt1_parked", "gt1_through", "gt2", "gt1_2d"])
def test_discrete_continuity_to_roundoff(dims, scheme, delta):
    if dims == 3:
        cfg = workloads.small3d(precision="fp64", n=(16, 16, 64), tile=(8, 8, 4))
    else:
        cfg = workloads.lwfa2d_fp64()
        cfg["n"] = [32, 1, 128]
    cfg.update(delta=delta, scheme=scheme)
    s = MarchSim(cfg, record=True)
    for _ in range(3):
        s.step()
        r = continuity_residual(s.m, s.rho0, s.rho1, s.J, s.flux)
        scale = np.abs(s.rho0).max() / s.m.Delta
        assert np.abs(r).max() < 1e-12 * scale
    # the laser moved particles: the check is not of a plasma at rest
    assert np.abs(np.r_[s.P.ux, s.left.ux]).max() > 1e-3


def test_vacuum_stage_march_equals_full_march():
    cfg = workloads.small3d(precision="fp64", n=(16, 8, 64), tile=(8, 8, 4), n_e=0.0)
    cfg.update(delta=3.0)
    s = MarchSim(cfg)
    p = s.p
    ref0 = ofields.laser_state(p)
    init = init_state(s.m)
    for nm in ofields.SpectralState.NAMES:
        a, b = getattr(init, nm), getattr(ref0, nm)
        assert np.max(np.abs(a - b)) <= 1e-13 * max(np.abs(b).max(), 1.0)
    s.step()
    z = np.zeros((p.Nz + 1, p.Ny, p.Nx), complex)
    ref1 = ofields.march(p, ref0, (z, z, z), s.m.Delta)
    for nm in ofields.SpectralState.NAMES:
        a, b = getattr(s.state, nm), getattr(ref1, nm)
        assert np.max(np.abs(a - b)) <= 1e-12 * max(np.abs(b).max(), 1.0), nm


def _rk4_reference(E, B, T, dt=1e-4):
    u = np.zeros(3)

    def f(u):
        g = math.sqrt(1 + u @ u)
        return -1.0 * (E + np.cross(u / g, B))
    for _ in range(int(round(T / dt))):
        k1 = f(u)
        k2 = f(u + 0.5 * dt * k1)
        k3 = f(u + 0.5 * dt * k2)
        k4 = f(u + dt * k3)
        u = u + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u


def test_small_delta_reduces_to_tau_push():
    E = np.array([0.05, 0.0, 0.02])
    B = np.array([0.0, 0.01, 0.3])
    T = 8.0
    ref = _rk4_reference(E, B, T)
    errs, diffs = [], []
    for N in (32, 64):
        D = T / N
        cfg = _cfg(n=(2, 2, 64), d=(2.0, 2.0, 0.5), delta=D)
        s = MarchSim(cfg, solver=False)
        s.F0[:] = 0.0
        for c in range(3):
            s.F0[c, :64] = E[c]
            s.F0[3 + c, :64] = B[c]
        # the ghost node above the last cell carries zero fields: follow the
        # initial batch that starts at rest at zeta = L - 2 (batch m = 2 / D)
        s.run(N)
        m = int(round(2.0 / D))
        first = (s.P.pid >= 4 * (m - 1)) & (s.P.pid < 4 * m)
        u = np.stack([s.P.ux[first], s.P.uy[first], s.P.uz[first]])
        assert u.shape[1] == 4
        errs.append(np.max(np.abs(u - ref[:, None])))
        ux, uy, uz = np.zeros(1), np.zeros(1), np.zeros(1)
        for _ in range(N):
            ux, uy, uz = higuera_cary(ux, uy, uz, E[:, None], B[:, None], -0.5 * D)
        diffs.append(np.max(np.abs(u - np.array([ux, uy, uz]))))
    assert 3.0 < errs[0] / errs[1] < 5.5, errs
    assert 3.0 < diffs[0] / diffs[1] < 5.5, diffs


@pytest.mark.parametrize("scheme", [1, 2])
def test_stop_rules(scheme):
    D = 0.5
    cfg = _cfg(n=(2, 2, 64), d=(0.5, 0.5, 0.1), n_e=0.01, delta=D, scheme=scheme)
    s = MarchSim(cfg, solver=False)
    s.P = s.P.take(np.zeros(0, np.int64))        # only the fresh batch
    s.step()
    if scheme == 2:
        assert len(s.P) == 0 and len(s.left) == 4     # streams through the box
    else:
        assert len(s.P) == 4                         # parked after Delta
        zeta = s.m.zn[s.P.iz] + s.P.dz * s.m.hz[s.P.iz]
        assert np.max(np.abs(zeta - (s.m.L - D))) < 1e-12
    # a forward-moving particle (u_z = 0.6)
    s = MarchSim(cfg, solver=False)
    s.P = s.P.take(np.zeros(0, np.int64))
    s.inject_u0 = (0.0, 0.0, 0.6)
    s.step()
    vz = 0.6 / math.sqrt(1.36)
    zeta = s.m.zn[s.P.iz] + s.P.dz * s.m.hz[s.P.iz]
    want = s.m.L - (1 - vz) * D / (vz if scheme == 2 else 1.0)
    assert len(s.P) == 4 and np.max(np.abs(zeta - want)) < 1e-12
