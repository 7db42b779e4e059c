"""Charge-conserving current deposition on the Galilean grid (oracle side).

The paper's macro-particle carrying Q_b = q n h_x h_y h deposits the current
j = q n v of a beam particle (Sec. 5.1).  This module deposits that current
so that the discrete Galilean continuity equation
    (rho^{k+1} - rho^k)/dtau - D_zeta rhobar + D_x J_x + D_y J_y + D_zeta J_z = 0
holds to roundoff at every node:

* In the grid frame the particle moves by (dx, dy, (v_z - 1) dtau); the
  Esirkepov decomposition (Comput. Phys. Commun. 135, 144, 2001) of that move
  with linear (CIC) shapes gives the frame current W on the staggered grid:
  W_x at (i+1/2, j, n), W_y at (i, j+1/2, n), W_zeta at (i, j, n+1/2).
* The lab current adds the frame velocity c = 1 of the grid:
  J_z = W_zeta + rhobar with rhobar(n+1/2) = (rho^k_n + rho^k_{n+1} +
  rho^{k+1}_n + rho^{k+1}_{n+1}) / 4 (time- and zeta-centred charge).
  J_x = W_x, J_y = W_y.
In 2-D (x, zeta) the out-of-plane J_y is q w v_y times the time-averaged
shape S0 S0 + DS S0 / 2 + S0 DS / 2 + DS DS / 3 on nodes.

Storage: every array has N_zeta + ext + 4 planes, plane p = n + 2 for node
(or half-node n + 1/2) index n = -2 .. N_zeta + ext + 1, enough for every
particle of the box (cells 0 .. N_zeta + ext - 1) and one filter pass beyond;
J_x(i+1/2) is stored at x index i, J_y(j+1/2) at y index j, J_z(n+1/2) at
plane n + 2.  The two planes below n = 0 receive the currents of particles
leaving at zeta < 0.
"""
import numpy as np

G = 2  # ghost planes below n = 0


def _window(c0, k, d0, d1):
    """3-node window of one axis.  Returns (base, S0[3], S1[3])."""
    base = c0 + np.minimum(k, 0)
    off0 = (k < 0).astype(np.int64)
    off1 = (k > 0).astype(np.int64)
    a = np.arange(3)[:, None]
    S0 = np.where(a == off0, 1.0 - d0, 0.0) + np.where(a == off0 + 1, d0, 0.0)
    S1 = np.where(a == off1, 1.0 - d1, 0.0) + np.where(a == off1 + 1, d1, 0.0)
    return base, S0, S1


def nplanes(p):
    return p.Nz + p.ext + 4


class _Acc:
    def __init__(self, p):
        self.p = p
        self.size = nplanes(p) * p.Ny * p.Nx
        self.idx = []
        self.val = []

    def add(self, plane, y, x, v):
        p = self.p
        i = ((plane * p.Ny + (y % p.Ny)) * p.Nx + (x % p.Nx))
        self.idx.append(i)
        self.val.append(v)

    def result(self):
        p = self.p
        shape = (nplanes(p), p.Ny, p.Nx)
        if not self.idx:
            return np.zeros(shape)
        idx = np.concatenate(self.idx)
        val = np.concatenate(self.val)
        # The last rhobar half-node of a particle that did not cross a zeta
        # boundary lies one plane beyond the range and always carries zero.
        out = (idx < 0) | (idx >= self.size)
        if np.any(out & (val != 0.0)):
            raise IndexError("deposit outside the ghost layers")
        idx, val = idx[~out], val[~out]
        return np.bincount(idx, weights=val, minlength=self.size).reshape(shape)


def deposit(p, old, new, steps, vy, wr=None):
    """Currents of one step.  ``old``/``new`` = (ix, iy, iz, dx, dy, dz) before
    and after the move, ``steps`` = per-axis cell steps, ``vy`` = v_y (used in
    2-D only), ``wr`` = per-particle weight over p.w (None: all 1, the
    plasma).  Returns (Jx, Jy, Jz) each of shape (nplanes, Ny, Nx)."""
    ix0, iy0, iz0, dx0, dy0, dz0 = old
    ix1, iy1, iz1, dx1, dy1, dz1 = new
    kx, ky, kz = steps
    qw = p.q * p.w if wr is None else p.q * p.w * wr
    V = p.hx * p.hy_eff * p.h
    bx, S0x, S1x = _window(ix0, kx, dx0, dx1)
    bz, S0z, S1z = _window(iz0, kz, dz0, dz1)
    DSx = S1x - S0x
    DSz = S1z - S0z
    third = 1.0 / 3.0
    ax, ay, az = _Acc(p), _Acc(p), _Acc(p)
    if p.dims == 3:
        by, S0y, S1y = _window(iy0, ky, dy0, dy1)
        DSy = S1y - S0y
        cx = -qw / (p.dtau * p.hy * p.h)
        cy = -qw / (p.dtau * p.hx * p.h)
        cz = -qw / (p.dtau * p.hx * p.hy)
        for b in range(3):
            for c in range(3):
                acc = 0.0
                for a in range(2):
                    acc = acc + DSx[a] * (S0y[b] * S0z[c] + 0.5 * DSy[b] * S0z[c]
                                          + 0.5 * S0y[b] * DSz[c] + third * DSy[b] * DSz[c])
                    ax.add(bz + c + G, by + b, bx + a, cx * acc)
        for a in range(3):
            for c in range(3):
                acc = 0.0
                for b in range(2):
                    acc = acc + DSy[b] * (S0x[a] * S0z[c] + 0.5 * DSx[a] * S0z[c]
                                          + 0.5 * S0x[a] * DSz[c] + third * DSx[a] * DSz[c])
                    ay.add(bz + c + G, by + b, bx + a, cy * acc)
        for a in range(3):
            for b in range(3):
                acc = 0.0
                for c in range(2):
                    acc = acc + DSz[c] * (S0x[a] * S0y[b] + 0.5 * DSx[a] * S0y[b]
                                          + 0.5 * S0x[a] * DSy[b] + third * DSx[a] * DSy[b])
                    az.add(bz + c + G, by + b, bx + a, cz * acc)
                # time- and zeta-centred charge on the half-nodes n + 1/2,
                # n = bz - 1 .. bz + 2
                t0 = S0x[a] * S0y[b]
                t1 = S1x[a] * S1y[b]
                for e in range(4):
                    s0 = (S0z[e - 1] if 1 <= e else 0.0) + (S0z[e] if e <= 2 else 0.0)
                    s1 = (S1z[e - 1] if 1 <= e else 0.0) + (S1z[e] if e <= 2 else 0.0)
                    az.add(bz + e - 1 + G, by + b, bx + a, (qw / V) * 0.25 * (t0 * s0 + t1 * s1))
    else:
        cx = -qw / (p.dtau * p.h)
        cz = -qw / (p.dtau * p.hx)
        cyv = qw * vy / (p.hx * p.h)
        y0 = np.zeros_like(ix0)
        for c in range(3):
            acc = 0.0
            for a in range(2):
                acc = acc + DSx[a] * (S0z[c] + 0.5 * DSz[c])
                ax.add(bz + c + G, y0, bx + a, cx * acc)
        for a in range(3):
            for c in range(3):
                wt = (S0x[a] * S0z[c] + 0.5 * DSx[a] * S0z[c] + 0.5 * S0x[a] * DSz[c]
                      + third * DSx[a] * DSz[c])
                ay.add(bz + c + G, y0, bx + a, cyv * wt)
        for a in range(3):
            acc = 0.0
            for c in range(2):
                acc = acc + DSz[c] * (S0x[a] + 0.5 * DSx[a])
                az.add(bz + c + G, y0, bx + a, cz * acc)
            for e in range(4):
                s0 = (S0z[e - 1] if 1 <= e else 0.0) + (S0z[e] if e <= 2 else 0.0)
                s1 = (S1z[e - 1] if 1 <= e else 0.0) + (S1z[e] if e <= 2 else 0.0)
                az.add(bz + e - 1 + G, y0, bx + a, (qw / V) * 0.25 * (S0x[a] * s0 + S1x[a] * s1))
    return ax.result(), ay.result(), az.result()


def deposit_rho(p, ix, iy, iz, dx, dy, dz, wr=None):
    """Charge density (linear shape) on nodes, same plane layout as the currents;
    ``wr`` as in deposit."""
    qw = p.q * p.w if wr is None else p.q * p.w * wr
    V = p.hx * p.hy_eff * p.h
    acc = _Acc(p)
    wx = (1.0 - dx, dx)
    wz = (1.0 - dz, dz)
    if p.dims == 3:
        wy = (1.0 - dy, dy)
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    acc.add(iz + c + G, iy + b, ix + a, (qw / V) * (wx[a] * wy[b] * wz[c]))
    else:
        for c in range(2):
            for a in range(2):
                acc.add(iz + c + G, np.zeros_like(ix), ix + a, (qw / V) * (wx[a] * wz[c]))
    return acc.result()


def continuity_residual(p, rho0, rho1, Jx, Jy, Jz):
    """Residual of (rho1 - rho0)/dtau - D_zeta rhobar + D.J at every node of the
    stored range (half-node quantities beyond the range count as zero).
    rhobar is rebuilt from the node charges exactly as the deposit defines it."""
    rbar = np.zeros_like(rho0)
    rbar[:-1] = 0.25 * (rho0[:-1] + rho0[1:] + rho1[:-1] + rho1[1:])
    rbar[-1] = 0.25 * (rho0[-1] + rho1[-1])
    def dz_half(A):   # (A(n+1/2) - A(n-1/2)) / h at node n
        out = A.copy()
        out[1:] = A[1:] - A[:-1]
        return out / p.h
    r = (rho1 - rho0) / p.dtau - dz_half(rbar) + (Jx - np.roll(Jx, 1, axis=2)) / p.hx \
        + dz_half(Jz)
    if p.dims == 3:
        r = r + (Jy - np.roll(Jy, 1, axis=1)) / p.hy
    return r
