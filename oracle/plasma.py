"""Plasma macro-particles: loading and moving-window injection (oracle side).

Particles are stored as an integer cell (ix, iy, iz) and an offset in [0, 1)
per axis, plus the momentum u = gamma v.  Node (i, j, n) sits at
(i h_x, j h_y, n h); the plasma box is zeta in [0, L) with
L = (N_zeta - 1 + ext) h (see params), and the cell N_zeta + ext - 1 is the
entry cell that fresh plasma crosses during its first step.

Lattice (reading): every transverse cell (i, j) is split into ppc_x x ppc_y
sub-columns and the lab z axis into sub-rows of length h / ppc_z indexed by
m >= 0.  Lab particle (i, j, sx, sy, m) sits at offsets (sx + xi_x)/ppc_x,
(sy + xi_y)/ppc_y and lab z_m = (m + xi_z) h / ppc_z, with xi uniform in
[0,1) from SplitMix64 (stratified random) or 1/2 (quiet lattice).  Ions are
immobile and neutralising: they are not simulated.

Window (reading, Sec. 5.1 "fresh" plasma that the domain sweeps over): the
lab plasma is at rest, so a lab particle has zeta = z_m - tau.  Batch b
holds the lattice particles with L + b dtau <= z_m < L + (b + 1) dtau; it is
placed at tau_b = b dtau, i.e. at zeta in [L, L + dtau) inside the entry
cell.  Batch 0 joins the initial load (together with every full cell
m < (N_zeta + ext - 1) ppc_z); batch k + 1 is appended at the end of step k.
Thresholds are computed once per batch in FP64 so that every lattice
particle enters exactly once.
"""
import math

import numpy as np

from . import rng

ONE_MINUS = np.nextafter(1.0, 0.0)


class Particles:
    """Structure of arrays; every array has one entry per macro-particle."""

    FIELDS = ("ix", "iy", "iz", "dx", "dy", "dz", "ux", "uy", "uz", "pid", "sp")

    def __init__(self, **arrays):
        for k in self.FIELDS:
            v = arrays.get(k)
            if v is None and k == "sp":
                # species: 0 plasma electron, 1 driver-beam electron
                v = np.zeros(len(arrays["ix"]), np.int64)
            setattr(self, k, v)

    def __len__(self):
        return len(self.ix)

    @staticmethod
    def empty():
        i = np.zeros(0, np.int64)
        f = np.zeros(0, np.float64)
        return Particles(ix=i, iy=i.copy(), iz=i.copy(), dx=f, dy=f.copy(), dz=f.copy(),
                         ux=f.copy(), uy=f.copy(), uz=f.copy(), pid=i.copy(), sp=i.copy())

    def take(self, idx):
        return Particles(**{k: getattr(self, k)[idx] for k in self.FIELDS})

    @staticmethod
    def concat(a, b):
        return Particles(**{k: np.concatenate([getattr(a, k), getattr(b, k)])
                            for k in Particles.FIELDS})

    def weight_ratio(self, p):
        """Macro-particle weight over the plasma weight p.w."""
        if p.beam is None:
            return np.ones(len(self))
        return np.where(self.sp == 1, p.beam["rb"], 1.0)

    def cell(self, p):
        """Linear node/cell index (n * Ny + j) * Nx + i."""
        return (self.iz * p.Ny + self.iy) * p.Nx + self.ix


def _xi(p, key, m, j, i, sy, sx, axis):
    if p.load == 1:
        return np.full(m.shape, 0.5)
    c = ((((m.astype(np.uint64) * np.uint64(p.Ny) + j.astype(np.uint64)) * np.uint64(p.Nx)
           + i.astype(np.uint64)) * np.uint64(p.ppc[1]) + sy.astype(np.uint64))
         * np.uint64(p.ppc[0]) + sx.astype(np.uint64)) * np.uint64(3) + np.uint64(axis)
    return rng.uniform(key, c)


def _lattice(p, m_values, j_values=None, i_values=None):
    """Lattice particles of the given sub-rows (and transverse cells, default
    all), in (m, j, i, sy, sx) order."""
    jv = np.arange(p.Ny) if j_values is None else np.asarray(j_values, np.int64)
    iv = np.arange(p.Nx) if i_values is None else np.asarray(i_values, np.int64)
    m, j, i, sy, sx = np.meshgrid(np.asarray(m_values, np.int64), jv, iv,
                                  np.arange(p.ppc[1]), np.arange(p.ppc[0]), indexing="ij")
    m, j, i, sy, sx = (a.ravel() for a in (m, j, i, sy, sx))
    key = rng.stream_key(p.seed, 0)
    xi_x = _xi(p, key, m, j, i, sy, sx, 0)
    xi_z = _xi(p, key, m, j, i, sy, sx, 2)
    if p.dims == 3:
        xi_y = _xi(p, key, m, j, i, sy, sx, 1)
    else:
        xi_y = np.zeros_like(xi_x)
    dx = np.minimum((sx + xi_x) / p.ppc[0], ONE_MINUS)
    dy = np.minimum((sy + xi_y) / p.ppc[1], ONE_MINUS) if p.dims == 3 else np.zeros_like(dx)
    return m, j, i, dx, dy, xi_z


def _make(p, ix, iy, iz, dx, dy, dz):
    z = np.zeros(len(ix))
    return Particles(ix=ix.astype(np.int64), iy=iy.astype(np.int64), iz=iz.astype(np.int64),
                     dx=dx, dy=dy, dz=dz, ux=z, uy=z.copy(), uz=z.copy(),
                     pid=np.zeros(len(ix), np.int64))


def threshold(p, b):
    """Lab-z threshold L + b dtau of window batch b (FP64)."""
    return p.L + float(b) * p.dtau


def load_full_cells(p):
    """Every sub-row of the cells 0 .. N_zeta + ext - 2 at tau = 0."""
    if p.n_e <= 0.0:
        return Particles.empty()
    m_all = np.arange((p.Nzp - 1) * p.ppc[2], dtype=np.int64)
    m, j, i, dx, dy, xi_z = _lattice(p, m_all)
    iz = m // p.ppc[2]
    dz = np.minimum(((m % p.ppc[2]) + xi_z) / p.ppc[2], ONE_MINUS)
    return _make(p, i, j, iz, dx, dy, dz)


def load_box(p, i_values, j_values, iz_values):
    """The particles that load_full_cells puts in the given cells (i, j
    periodic indices, iz < N_zeta + ext - 1), with pid = their index in the
    full load, in load order."""
    if p.n_e <= 0.0:
        return Particles.empty()
    iv = np.asarray(i_values, np.int64) % p.Nx
    jv = np.asarray(j_values, np.int64) % p.Ny
    izv = np.asarray(iz_values, np.int64)
    if np.any(izv < 0) or np.any(izv >= p.Nzp - 1):
        raise ValueError("iz outside the fully loaded cells")
    m_vals = (izv[:, None] * p.ppc[2] + np.arange(p.ppc[2])[None, :]).ravel()
    m_vals = np.unique(m_vals)
    m, j, i, dx, dy, xi_z = _lattice(p, m_vals, np.sort(np.unique(jv)), np.sort(np.unique(iv)))
    iz = m // p.ppc[2]
    dz = np.minimum(((m % p.ppc[2]) + xi_z) / p.ppc[2], ONE_MINUS)
    P = _make(p, i, j, iz, dx, dy, dz)
    n = len(i)
    ppcy, ppcx = p.ppc[1], p.ppc[0]
    sub = np.arange(n) % (ppcy * ppcx)
    P.pid = ((m * p.Ny + j) * p.Nx + i) * (ppcy * ppcx) + sub
    return P


def inject_batch(p, b):
    """Window batch b placed at tau_b = b dtau (zeta in the entry cell)."""
    if p.n_e <= 0.0:
        return Particles.empty()
    hz = p.h / p.ppc[2]
    m0 = (p.Nzp - 1) * p.ppc[2]
    lo, hi = threshold(p, b), threshold(p, b + 1)
    m_lo = max(m0, int(np.floor(lo / hz)) - 1) if b > 0 else m0
    m_hi = int(np.floor(hi / hz)) + 1
    m, j, i, dx, dy, xi_z = _lattice(p, np.arange(m_lo, m_hi + 1, dtype=np.int64))
    z = (m + xi_z) * hz
    sel = z < hi
    if b > 0:
        sel &= z >= lo
    zeta = z[sel] - float(b) * p.dtau
    s = zeta / p.h
    iz = np.floor(s)
    dz = s - iz
    iz = iz.astype(np.int64)
    # Rounding can put zeta a hair below L: keep the particle in the entry cell.
    low = iz < p.Nzp - 1
    iz[low] = p.Nzp - 1
    dz[low] = 0.0
    return _make(p, i[sel], j[sel], iz, dx[sel], dy[sel], dz)


def load_beam(p):
    """Driver-beam macro-particles (species 1) in sample order.

    Particle i takes four SplitMix64 uniforms u_k = uniform(key, 4 i + k) with
    the beam's own stream key; the Box-Muller transform (Box & Muller 1958) of
    (1 - u_0, u_1) gives the transverse normal pair, of (1 - u_2, u_3) the zeta
    and gamma deviates:
        x = x_c + sr r_1 cos(2 pi u_1),  y = y_c + sr r_1 sin(2 pi u_1),
        zeta = zc + sz r_2 cos(2 pi u_3), gamma = gamma_0 + dgamma r_2 sin(2 pi u_3),
    r = sqrt(-2 ln(1 - u)), axis at node (Nx/2, Ny/2), u_z = sqrt(gamma^2 - 1).
    Positions wrap transversally; particles outside 0 <= zeta < (N_zeta - 1) h
    are dropped.  Scalar FP64 arithmetic with the C library's log, cos, sin
    and sqrt, one particle at a time, so that any implementation doing the
    same operations gets the same bits."""
    b = p.beam
    if b is None:
        return Particles.empty()
    key = rng.stream_key(p.seed, 1)
    Lx, Ly = p.Nx * p.hx, p.Ny * p.hy
    xc, yc = (p.Nx // 2) * p.hx, (p.Ny // 2) * p.hy
    zmax = (p.Nz - 1) * p.h
    below1 = float(ONE_MINUS)
    out = {k: [] for k in ("ix", "iy", "iz", "dx", "dy", "dz", "uz")}
    u = rng.uniform(key, np.arange(4 * b["np"], dtype=np.uint64))
    for i in range(b["np"]):
        u0, u1, u2, u3 = 1.0 - float(u[4 * i]), float(u[4 * i + 1]), 1.0 - float(u[4 * i + 2]), float(u[4 * i + 3])
        r1 = math.sqrt(-2.0 * math.log(u0))
        r2 = math.sqrt(-2.0 * math.log(u2))
        a1 = 2.0 * math.pi * u1
        a2 = 2.0 * math.pi * u3
        x = xc + b["sr"] * r1 * math.cos(a1)
        y = yc + b["sr"] * r1 * math.sin(a1)
        zeta = b["zc"] + b["sz"] * r2 * math.cos(a2)
        gam = b["gamma"] + b["dgamma"] * r2 * math.sin(a2)
        if not (0.0 <= zeta < zmax):
            continue
        x = math.fmod(x, Lx)
        if x < 0.0:
            x += Lx
        y = math.fmod(y, Ly)
        if y < 0.0:
            y += Ly
        fx, fy, fz = x / p.hx, y / p.hy, zeta / p.h
        ix = min(math.floor(fx), p.Nx - 1)
        iy = min(math.floor(fy), p.Ny - 1)
        iz = math.floor(fz)
        out["ix"].append(ix)
        out["iy"].append(iy)
        out["iz"].append(iz)
        out["dx"].append(min(fx - ix, below1))
        out["dy"].append(min(fy - iy, below1))
        out["dz"].append(min(fz - iz, below1))
        out["uz"].append(math.sqrt(gam * gam - 1.0) if gam > 1.0 else 0.0)
    n = len(out["ix"])
    i64 = lambda k: np.asarray(out[k], np.int64).reshape(n)
    f64 = lambda k: np.asarray(out[k], np.float64).reshape(n)
    return Particles(ix=i64("ix"), iy=i64("iy"), iz=i64("iz"), dx=f64("dx"), dy=f64("dy"),
                     dz=f64("dz"), ux=np.zeros(n), uy=np.zeros(n), uz=f64("uz"),
                     pid=np.zeros(n, np.int64), sp=np.ones(n, np.int64))
