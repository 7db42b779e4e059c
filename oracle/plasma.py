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
import numpy as np

from . import rng

ONE_MINUS = np.nextafter(1.0, 0.0)


class Particles:
    """Structure of arrays; every array has one entry per macro-particle."""

    FIELDS = ("ix", "iy", "iz", "dx", "dy", "dz", "ux", "uy", "uz", "pid")

    def __init__(self, **arrays):
        for k in self.FIELDS:
            setattr(self, k, arrays[k])

    def __len__(self):
        return len(self.ix)

    @staticmethod
    def empty():
        i = np.zeros(0, np.int64)
        f = np.zeros(0, np.float64)
        return Particles(ix=i, iy=i.copy(), iz=i.copy(), dx=f, dy=f.copy(), dz=f.copy(),
                         ux=f.copy(), uy=f.copy(), uz=f.copy(), pid=i.copy())

    def take(self, idx):
        return Particles(**{k: getattr(self, k)[idx] for k in self.FIELDS})

    @staticmethod
    def concat(a, b):
        return Particles(**{k: np.concatenate([getattr(a, k), getattr(b, k)])
                            for k in Particles.FIELDS})

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
