"""Pins of the oracle's Galilean field update.

* App. B closed form (with the readings named in oracle/fields.py) equals the
  oracle's direct solve of the node system; the printed text does not.
* Vacuum: every transverse/longitudinal Fourier mode of R rotates per step by
  exp(-i Omega Delta) with the scheme's dispersion relation
      tan(Omega Delta / 2) = Delta h (K^2 + w_p^2) sin(kh) /
                             (16 sin^2(kh/2) - h^2 w_p^2 - h^2 K^2 cos^2(kh/2)),
  derived from the node equations with the ansatz exp(-i Omega s + i k zeta);
  it reduces to the paper's 1-D relation (Sec. 4.2) at K = 0, to the universal
  relation (Sec. 3.2, eq. fu) as h, Delta -> 0, and further to App. A's
  Omega = (K^2 + w_p^2) / (2 k) in the paraxial limit; all three are checked.
* A plane (K = 0) pulse in vacuum is frozen exactly.
* The laser initialisation reproduces Sec. 6's pulse on the nodes.
"""
import numpy as np

from oracle import params
from oracle.fields import (laser_state, march, wavenumbers, node_matrix, node_rhs,
                           real_fields)


def _appb(kx, ky, h, D, Rx00, Ry00, Ez00, Bz00, Rx1, Ry1, Lx1, Ly1, Ez1, Bz1, jm, jp):
    """App. B (analytic solution of the node system) with j^0 = j^1."""
    K2 = kx * kx + ky * ky
    Dd = 16 + h * (2 * D + h) * K2
    Jx = 2 * (jm[0] + jp[0])
    Jy = 2 * (jm[1] + jp[1])
    Wx = -2 * Lx1 + Rx00 + Rx1
    Wy = -2 * Ly1 + Ry00 + Ry1
    T = (Ez1 * (16 - h * h * K2), -16 * h * jp[2], -1j * h * D * (kx * Jx + ky * Jy),
         -2 * h * D * Ez00 * K2,                       # reading: printed with +
         2j * h * h * (kx * jp[0] + ky * jp[1]), 4j * h * (kx * Wx + ky * Wy))
    Ux = 2 * Lx1 + Rx00 + Rx1
    Uy = 2 * Ly1 + Ry00 + Ry1
    Q = (Bz1 * (16 - h * h * K2), 2j * h * h * (kx * jp[1] - ky * jp[0]),
         1j * h * D * (kx * Jy - ky * Jx), -2 * h * D * Bz00 * K2, 4j * h * (ky * Ux - kx * Uy))
    return sum(T) / Dd, sum(Q) / Dd


def test_appendix_b_equals_node_solve():
    rs = np.random.default_rng(3)
    n = 500
    kx, ky = rs.normal(size=n) * 2, rs.normal(size=n) * 2
    h = 0.05 + abs(rs.normal()) * 0.3
    D = 0.1 + abs(rs.normal()) * 2
    c = lambda: rs.normal(size=n) + 1j * rs.normal(size=n)
    old = [c() for _ in range(4)]
    right = [c() for _ in range(6)]
    jm = [c() for _ in range(3)]
    jp = [c() for _ in range(3)]
    A = node_matrix(kx, ky, h, D)
    sol = np.linalg.solve(A, node_rhs(kx, ky, h, D, old, right, jm, jp)[..., None])[..., 0]
    Ez, Bz = _appb(kx, ky, h, D, *old, *right, jm, jp)
    assert np.max(np.abs(Ez - sol[:, 4]) / np.abs(sol[:, 4])) < 1e-12
    assert np.max(np.abs(Bz - sol[:, 5]) / np.abs(sol[:, 5])) < 1e-12
    # R from (RxN) once E_z, B_z are known
    Rx = old[0] + 0.5 * D * (1j * kx * (Ez + old[2]) + 1j * ky * (Bz + old[3])) - D * 0.5 * (jm[0] + jp[0])
    assert np.max(np.abs(Rx - sol[:, 0]) / np.abs(sol[:, 0])) < 1e-12


def test_printed_t4_sign_disagrees():
    """Documents the garble: with the printed +2 h Delta E_z0^0 K^2 the closed
    form does not solve the node system."""
    rs = np.random.default_rng(4)
    kx, ky, h, D = np.array([1.3]), np.array([-0.7]), 0.2, 1.1
    old = [np.array([1.0 + 0.5j]), np.array([0.3j]), np.array([0.8 - 0.1j]), np.array([0.2])]
    right = [np.array([rs.normal() + 1j * rs.normal()]) for _ in range(6)]
    z = [np.zeros(1, complex)] * 3
    sol = np.linalg.solve(node_matrix(kx, ky, h, D), node_rhs(kx, ky, h, D, old, right, z, z)[..., None])[..., 0]
    Ez, _ = _appb(kx, ky, h, D, *old, *right, z, z)
    Ez_printed = Ez + 4 * h * D * old[2] * (kx * kx + ky * ky) / (16 + h * (2 * D + h) * (kx * kx + ky * ky))
    assert abs(Ez - sol[:, 4])[0] < 1e-13
    assert abs(Ez_printed - sol[:, 4])[0] > 1e-2


def dispersion_factor(K2, kap, h, D, wp2=0.0):
    """exp(-i Omega Delta) of the scheme's numerical dispersion relation."""
    num = D * h * (K2 + wp2) * np.sin(kap * h)
    den = 16 * np.sin(kap * h / 2) ** 2 - h * h * wp2 - K2 * h * h * np.cos(kap * h / 2) ** 2
    zero = (num == 0) & (den == 0)
    return np.where(zero, 1.0, (den - 1j * num) / np.where(zero, 1.0, den + 1j * num))


def test_dispersion_relation_limits():
    h, D, wp2 = 0.1, 0.3, 0.04
    kap = np.linspace(0.2, 3.0, 50)
    # K = 0: the paper's 1-D relation tan(wD/2) = -wp^2 D h sin(kh) / (wp^2 h^2 + 8 cos(kh) - 8)
    tan_paper = -wp2 * D * h * np.sin(kap * h) / (wp2 * h * h + 8 * np.cos(kap * h) - 8)
    f = dispersion_factor(0.0, kap, h, D, wp2)
    tan_here = np.tan(-np.angle(f) / 2)
    assert np.allclose(tan_here, tan_paper, rtol=1e-12)
    # continuum limit (h, Delta -> 0): the universal relation of Sec. 3.2 (eq. fu,
    # omega = 2 kappa wp^2 / (4 kappa^2 - wp^2), quoted again in Sec. 4.2) with
    # wp^2 -> K^2 + wp^2
    K2 = 0.09
    kap = np.linspace(0.5, 3.0, 50)
    S = K2 + wp2
    Om_u = 2 * kap * S / (4 * kap * kap - S)
    e = []
    for hh in (1e-2, 1e-3):
        f = dispersion_factor(K2, kap, hh, hh, wp2)
        e.append(np.max(np.abs(-np.angle(f) / hh - Om_u) / Om_u))
    assert e[1] < 1e-5
    # second order: error ratio 100 for a 10x smaller step
    assert 80 < e[0] / e[1] < 120
    # paraxial limit K^2 + wp^2 << kappa^2: App. A's Omega = (K^2 + wp^2) / (2 kappa)
    kap = np.linspace(20.0, 40.0, 11)
    f = dispersion_factor(K2, kap, 1e-4, 1e-4, wp2)
    Om = -np.angle(f) / 1e-4
    assert np.max(np.abs(Om - S / (2 * kap)) / (S / (2 * kap))) < 1e-3


def _vacuum_run(dims, pol, N):
    if dims == 2:
        cfg = dict(dims=2, n=[32, 1, 1024], d=[4.0, 1.0, 0.2])
    else:
        cfg = dict(dims=3, n=[16, 16, 512], d=[4.0, 4.0, 0.25])
    T = 12.0
    cfg.update(length_unit=1.0, n_e=0.0, a0=1.0, waist=10.0,
               fwhm=T * np.sqrt(2 * np.log(2)), pol=pol,
               tile=[8, 8 if dims == 3 else 1, 8])
    cfg["zeta_c"] = cfg["n"][2] * cfg["d"][2] / 2
    p = params.from_config(cfg)
    s0 = laser_state(p)
    s = s0
    zero = np.zeros((p.Nz + 1, p.Ny, p.Nx), complex)
    for _ in range(N):
        s = march(p, s, (zero, zero, zero), p.dtau)
    KX, KY, _ = wavenumbers(p)
    kap = 2 * np.pi * np.fft.fftfreq(p.Nz, d=p.h)[:, None, None]
    f = dispersion_factor(KX ** 2 + KY ** 2, kap, p.h, p.dtau)
    err = nrm = moved = 0.0
    for a, b in ((s0.Rx, s.Rx), (s0.Ry, s.Ry)):
        pred = np.fft.ifft(np.fft.fft(a, axis=0) * f ** N, axis=0)
        err += np.sum(np.abs(pred - b) ** 2)
        nrm += np.sum(np.abs(b) ** 2)
        moved += np.sum(np.abs(b - a) ** 2)
    return np.sqrt(err / nrm), np.sqrt(moved / nrm)


def test_vacuum_pulse_follows_numerical_dispersion_2d():
    # broad waist, long pulse: no spectral content near kappa = K/2, where the
    # zeta recursion's undamped homogeneous solution would make the
    # right-boundary condition differ from a periodic zeta
    err, moved = _vacuum_run(2, 0, 50)
    assert moved > 0.03
    assert err < 1e-9


def test_vacuum_pulse_follows_numerical_dispersion_3d():
    for pol in (0, 1):
        err, moved = _vacuum_run(3, pol, 12)
        assert moved > 0.02
        assert err < 1e-9


def test_plane_pulse_frozen_exactly():
    cfg = dict(dims=3, n=[8, 8, 256], d=[0.4, 0.4, 0.05], length_unit=2 * np.pi, a0=1.5,
               waist=0.0, fwhm=2.0, zeta_c=6.0, tile=[8, 8, 8])
    p = params.from_config(cfg)
    s0 = laser_state(p)
    s = s0
    zero = np.zeros((p.Nz + 1, p.Ny, p.Nx), complex)
    for _ in range(10):
        s = march(p, s, (zero, zero, zero), p.dtau)
    assert np.array_equal(s.Rx, s0.Rx) and np.array_equal(s.Ry, s0.Ry)
    F = real_fields(p, s)
    # forward wave: E_x = B_y, nothing else
    assert np.allclose(F[0], F[4], atol=1e-14)
    assert np.abs(F[[1, 2, 3, 5]]).max() < 1e-14


def test_laser_initialisation_on_axis():
    cfg = dict(dims=2, n=[64, 1, 256], d=[0.25, 1.0, 0.05], length_unit=2 * np.pi,
               a0=1.0, waist=4.0, fwhm=5.0, zeta_c=10.0, tile=[8, 1, 8])
    p = params.from_config(cfg)
    F = real_fields(p, laser_state(p))
    zeta = np.arange(p.Nz) * p.h
    phi = zeta - p.zeta_c
    T = 5.0 * 2 * np.pi / np.sqrt(2 * np.log(2))
    want = np.cos(phi) * np.exp(-phi ** 2 / T ** 2)
    got = F[0, :p.Nz, 0, p.Nx // 2]
    # on axis, E_x = (R + L)/2 with R = 2 E_laser and a small L from the finite waist
    assert np.max(np.abs(got - want)) < 2e-2
    # R/2 = E_laser up to the zeroed transverse Nyquist column
    assert np.max(np.abs(0.5 * (got + F[4, :p.Nz, 0, p.Nx // 2]) - want)) < 1e-4
