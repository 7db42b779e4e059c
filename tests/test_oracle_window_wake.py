"""Pins of the moving window, the loader and the coupled step.

* Quiet lattice at rest: the particle count after k steps equals the closed-form
  lattice count, and the charge density in the refilled box is exactly flat.
* Stratified loading: every lab lattice particle enters exactly once.
* Linear wake (a0 << 1): behind a plane Gaussian pulse the on-axis E_z has the
  1-D linear cold-fluid amplitude
      E_max = k_p^2 (a0^2 / 4) T sqrt(pi/2) exp(-k_p^2 T^2 / 8)
  (psi'' + k_p^2 psi = k_p^2 <a^2>/2 with <a^2> = (a0^2/2) exp(-2 zeta^2/T^2)),
  times the factor (2 + cos(k0 h)) / 3 by which linear (CIC) interpolation of a
  wave sampled on nodes lowers the mean square field a particle sees; and the
  plasma wavelength 2 pi / k_p.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle.sim import Simulation
from oracle.plasma import inject_batch
from oracle.deposit import deposit_rho, G


def _quiet_cfg(**kw):
    cfg = dict(dims=3, n=[4, 4, 32], d=[0.25, 0.25, 0.05], length_unit=2 * np.pi, n_e=0.01,
               ppc=[1, 2, 2], load=1, tile=[4, 4, 4])
    cfg.update(kw)
    return cfg


def test_quiet_lattice_particle_count_closed_form():
    s = Simulation(_quiet_cfg())
    p = s.p
    per_row = p.Nx * p.Ny * p.ppc[0] * p.ppc[1]
    a = Fraction(1, 2)                         # dtau / h
    for k in range(0, 12):
        if k:
            s.step()
        # lab sub-row m sits at z_m / h = (m + 1/2) / ppc_z; it is present when
        # k dtau <= z_m < L + (k + 1) dtau
        lo, hi = k * a, (p.Nzp - 1) + (k + 1) * a
        cnt = sum(1 for m in range(0, 4 * (p.Nzp + k + 2))
                  if lo <= Fraction(2 * m + 1, 2 * p.ppc[2]) < hi)
        assert len(s.P) == per_row * cnt


def test_quiet_lattice_density_flat():
    s = Simulation(_quiet_cfg())
    s.run(9)
    p = s.p
    P = s.P
    rho = deposit_rho(p, P.ix, P.iy, P.iz, P.dx, P.dy, P.dz)
    # nodes 6 .. N_zeta - 1: away from the exit boundary, where the first nodes
    # see the (small) field of the currents of particles leaving the box
    inner = rho[G + 6:G + p.Nz]
    assert np.allclose(inner, p.q * p.n_e, rtol=1e-12, atol=0)


def test_every_lattice_particle_enters_once():
    cfg = _quiet_cfg(load=0, seed=11, n=[4, 4, 16])
    s = Simulation(cfg)
    p = s.p
    hz = p.h / p.ppc[2]
    nb = 40
    zs = []
    for b in range(nb):
        B = inject_batch(p, b)
        zs.append(((B.iz + B.dz) * p.h + b * p.dtau, B.ix, B.iy, B.dx, B.dy))
    # lab positions of all injected particles, keyed by transverse identity
    z = np.concatenate([a[0] for a in zs])
    key = np.stack([np.concatenate([a[i] for a in zs]) for i in (1, 2, 3, 4)], axis=1)
    # no lattice particle twice: (transverse identity, z) pairs are distinct
    order = np.lexsort((z, key[:, 3], key[:, 2], key[:, 1], key[:, 0]))
    ks, zz = key[order], z[order]
    same = np.all(ks[1:] == ks[:-1], axis=1) & (np.abs(zz[1:] - zz[:-1]) < 0.5 * hz)
    assert not np.any(same)
    # count equals the lattice sub-rows between L and L + nb dtau (each sub-row
    # holds one particle per transverse sub-column)
    lo = p.L
    hi = p.L + nb * p.dtau
    m0 = (p.Nzp - 1) * p.ppc[2]
    per_row = p.Nx * p.Ny * p.ppc[0] * p.ppc[1]
    assert abs(len(z) - per_row * (hi - lo) / hz) <= per_row
    assert np.all(z >= lo - 1e-12) and np.all(z < hi + 1e-12)


@pytest.mark.slow
def test_linear_wake_amplitude_and_wavelength():
    a0, n = 0.1, 0.01
    T_lambda = 4.247
    cfg = dict(dims=2, n=[2, 1, 512], d=[0.25, 1.0, 0.1], length_unit=2 * np.pi, n_e=n,
               ppc=[1, 1, 4], load=1, a0=a0, waist=0.0,
               fwhm=T_lambda * np.sqrt(2 * np.log(2)), zeta_c=51.1 - 12.0,
               tile=[2, 1, 8], filter_passes=1)
    s = Simulation(cfg)
    p = s.p
    s.run(700)
    ez = s.F[2, :p.Nz, 0, 0]
    zeta = np.arange(p.Nz) * p.h
    kp = np.sqrt(n)
    T = p.T
    amp = kp ** 2 * (a0 ** 2 / 4) * T * np.sqrt(np.pi / 2) * np.exp(-kp ** 2 * T ** 2 / 8)
    amp *= (2.0 + np.cos(p.h)) / 3.0
    lam = 2 * np.pi / kp
    win = (zeta < p.zeta_c - 2.6 * T) & (zeta > p.zeta_c - 2.6 * T - 1.2 * lam)
    assert abs(np.abs(ez[win]).max() - amp) < 0.02 * amp
    e = ez[win]
    zc = zeta[win][:-1][np.sign(e[:-1]) != np.sign(e[1:])]
    assert len(zc) >= 2
    assert np.all(np.abs(np.diff(zc) - lam / 2) < 0.01 * lam / 2)


def test_load_box_is_the_subset_of_the_full_load():
    """The sampled-cell loader used at full size reproduces the full load's
    particles (positions and load-order ids) cell by cell."""
    import workloads
    from oracle import params, plasma
    cfg = workloads.small3d(precision="fp64", ppc=(1, 2, 2))
    p = params.from_config(cfg)
    full = plasma.load_full_cells(p)
    full.pid = np.arange(len(full))
    xs, ys, zs = [30, 31, 0, 1], [5, 6], [0, 13, 14, 66]
    B = plasma.load_box(p, xs, ys, zs)
    sel = np.isin(full.ix, xs) & np.isin(full.iy, ys) & np.isin(full.iz, zs)
    F = full.take(np.nonzero(sel)[0])
    assert len(B) == len(F) > 0
    for k in plasma.Particles.FIELDS:
        assert np.array_equal(getattr(B, k), getattr(F, k)), k
