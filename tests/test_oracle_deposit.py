"""Pins of the oracle's charge-conserving deposition.

* Discrete Galilean continuity (rho^{k+1} - rho^k)/dtau - D_zeta rhobar + D.J = 0
  at every node, to roundoff, for random moves of up to one cell per axis
  (the residual is written here from the equation, with rho from the plain
  CIC definition).
* Totals: sum_nodes J_d V dtau = sum_p q w (lab displacement)_d.
* A hand-expanded single particle.
* A quiet plasma at rest in the lab deposits zero lab current.
"""
import numpy as np

from oracle import params
from oracle.deposit import deposit, nplanes, G
from oracle.sim import Simulation


def _params(dims):
    if dims == 3:
        cfg = dict(dims=3, n=[8, 8, 16], d=[0.4, 0.3, 0.05], n_e=0.01, ppc=[1, 1, 2],
                   tile=[4, 4, 4], length_unit=2 * np.pi)
    else:
        cfg = dict(dims=2, n=[8, 1, 16], d=[0.4, 1.0, 0.05], n_e=0.01, ppc=[1, 1, 2],
                   tile=[4, 1, 4], length_unit=2 * np.pi)
    return params.from_config(cfg)


def _cic_rho(p, ix, iy, iz, dx, dy, dz):
    """rho on nodes from the CIC definition, written out node by node."""
    rho = np.zeros((nplanes(p), p.Ny, p.Nx))
    qwV = p.q * p.w / (p.hx * p.hy_eff * p.h)
    for k in range(len(ix)):
        for c, wz in ((0, 1 - dz[k]), (1, dz[k])):
            for a, wx in ((0, 1 - dx[k]), (1, dx[k])):
                if p.dims == 3:
                    for b, wy in ((0, 1 - dy[k]), (1, dy[k])):
                        rho[iz[k] + c + G, (iy[k] + b) % p.Ny, (ix[k] + a) % p.Nx] += qwV * wx * wy * wz
                else:
                    rho[iz[k] + c + G, 0, (ix[k] + a) % p.Nx] += qwV * wx * wz
    return rho


def _random_moves(p, n, seed):
    rs = np.random.default_rng(seed)
    ix = rs.integers(0, p.Nx, n)
    iy = rs.integers(0, p.Ny, n) if p.dims == 3 else np.zeros(n, np.int64)
    iz = rs.integers(1, p.Nz - 1, n)
    d0 = rs.random((3, n))
    # displacement in cells: x, y in (-0.9, 0.9), zeta in (-0.95, 0)
    s = np.stack([rs.uniform(-0.9, 0.9, n), rs.uniform(-0.9, 0.9, n), rs.uniform(-0.95, 0, n)])
    if p.dims == 2:
        d0[1] = 0
        s[1] = 0
    t = d0 + s
    k = np.floor(t).astype(np.int64)
    d1 = t - k
    old = (ix, iy, iz, d0[0], d0[1], d0[2])
    new = ((ix + k[0]) % p.Nx, (iy + k[1]) % p.Ny, iz + k[2], d1[0], d1[1], d1[2])
    return old, new, (k[0], k[1], k[2]), s


def _residual(p, rho0, rho1, J):
    Jx, Jy, Jz = J
    rbar = np.zeros_like(rho0)
    rbar[:-1] = 0.25 * (rho0[:-1] + rho0[1:] + rho1[:-1] + rho1[1:])
    rbar[-1] = 0.25 * (rho0[-1] + rho1[-1])
    def back(A, axis):
        B = np.zeros_like(A)
        if axis == 0:
            B[1:] = A[:-1]
        else:
            B = np.roll(A, 1, axis=axis)
        return B
    r = (rho1 - rho0) / p.dtau - (rbar - back(rbar, 0)) / p.h \
        + (Jx - back(Jx, 2)) / p.hx + (Jz - back(Jz, 0)) / p.h
    if p.dims == 3:
        r += (Jy - back(Jy, 1)) / p.hy
    return r


def _check_continuity(dims):
    p = _params(dims)
    old, new, steps, s = _random_moves(p, 300, 5 + dims)
    vy = np.random.default_rng(1).uniform(-0.5, 0.5, 300)
    J = deposit(p, old, new, steps, vy)
    rho0 = _cic_rho(p, *old)
    rho1 = _cic_rho(p, *new)
    r = _residual(p, rho0, rho1, J)
    scale = np.abs((rho1 - rho0) / p.dtau).max()
    assert np.abs(r).max() < 1e-12 * scale
    return p, old, new, steps, s, J, vy


def test_continuity_3d():
    _check_continuity(3)


def test_continuity_2d():
    _check_continuity(2)


def test_totals_equal_charge_times_displacement():
    for dims in (2, 3):
        p, old, new, steps, s, J, vy = _check_continuity(dims)
        V = p.hx * p.hy_eff * p.h
        qw = p.q * p.w
        # lab displacements: grid-frame displacement, plus dtau along z
        dx = s[0] * p.hx
        dz = s[2] * p.h + p.dtau
        assert abs(J[0].sum() * V * p.dtau - qw * dx.sum()) < 1e-12 * abs(qw) * np.abs(dx).sum()
        assert abs(J[2].sum() * V * p.dtau - qw * dz.sum()) < 1e-12 * abs(qw) * np.abs(dz).sum()
        if dims == 3:
            dy = s[1] * p.hy
            assert abs(J[1].sum() * V * p.dtau - qw * dy.sum()) < 1e-12 * abs(qw) * np.abs(dy).sum()
        else:
            # out-of-plane current of the 2-D model: q w v_y per particle
            assert abs(J[1].sum() * V - qw * vy.sum()) < 1e-12 * abs(qw) * np.abs(vy).sum()


def test_single_particle_hand_expanded():
    p = _params(2)
    qw = p.q * p.w
    V = p.hx * p.h
    # x: cell 2, offset 0.7 -> cell 3, offset 0.2 (half a cell); zeta fixed at
    # node 4 + 0.3 (no zeta motion)
    old = (np.array([2]), np.array([0]), np.array([4]), np.array([0.7]), np.array([0.0]), np.array([0.3]))
    new = (np.array([3]), np.array([0]), np.array([4]), np.array([0.2]), np.array([0.0]), np.array([0.3]))
    Jx, Jy, Jz = deposit(p, old, new, (np.array([1]), np.array([0]), np.array([0])), np.zeros(1))
    c = qw / (p.dtau * p.h)
    # charge that crosses x = 2.5 is the part (1 - 0.7) on node 2; across 3.5 the part 0.2
    expect_x = {(4, 2): 0.3 * 0.7 * c, (5, 2): 0.3 * 0.3 * c, (4, 3): 0.2 * 0.7 * c, (5, 3): 0.2 * 0.3 * c}
    got = {(n - G, i): Jx[n, 0, i] for n, i in zip(*np.nonzero(Jx[:, 0, :]))}
    assert set(got) == set(expect_x)
    for key, v in expect_x.items():
        assert abs(got[key] - v) < 1e-15 * abs(c)
    # lab J_z = rhobar only: (qw/V)/4 [S0x (S0z(n) + S0z(n+1)) + S1x (S1z(n) + S1z(n+1))]
    S0x = {2: 0.3, 3: 0.7}
    S1x = {3: 0.8, 4: 0.2}
    Sz = {4: 0.7, 5: 0.3}
    for n in range(2, 7):
        for i in range(0, 6):
            sz = Sz.get(n, 0.0) + Sz.get(n + 1, 0.0)
            e = 0.25 * qw / V * (S0x.get(i, 0.0) * sz + S1x.get(i, 0.0) * sz)
            assert abs(Jz[n + G, 0, i] - e) < 1e-15 * abs(qw / V)
    assert not np.any(Jy)


def test_quiet_plasma_at_rest_has_zero_lab_current():
    for dims in (2, 3):
        if dims == 2:
            cfg = dict(dims=2, n=[8, 1, 64], d=[0.25, 1, 0.05], n_e=0.01, ppc=[1, 1, 4],
                       load=1, tile=[8, 1, 8], length_unit=2 * np.pi)
        else:
            cfg = dict(dims=3, n=[4, 4, 32], d=[0.25, 0.25, 0.05], n_e=0.01, ppc=[1, 2, 2],
                       load=1, tile=[4, 4, 4], length_unit=2 * np.pi)
        s = Simulation(cfg)
        s.step()
        p = s.p
        Jx, Jy, Jz = s.J
        scale = abs(p.q * p.w / (p.hx * p.hy_eff * p.h))
        # every plane the field solver uses, away from the exit boundary
        used = slice(G + 3, G + p.Nz + 1)
        for A in (Jx, Jy, Jz):
            assert np.abs(A[used]).max() < 1e-13 * scale
        # and the fields stay zero away from the exit boundary
        assert np.abs(s.F[:, 3:]).max() < 1e-15
