"""Helpers shared by the GPU parity tests (no tests here).  They convert the
oracle's state to the library's layout and measure agreement; they do no
arithmetic of the method."""
import numpy as np

from oracle.plasma import Particles

SPEC_NAMES = ("Rx", "Ry", "Lx", "Ly", "Ez", "Bz")
FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


BEAM_BIT = 1 << 30   # the library's marker of driver-beam particles in a cell word


def oracle_particles(o):
    P, p = o.P, o.p
    cell = ((P.iz * p.Ny + P.iy) * p.Nx + P.ix).astype(np.int64) | (P.sp.astype(np.int64) << 30)
    return cell, np.stack([P.dx, P.dy, P.dz]), np.stack([P.ux, P.uy, P.uz]), P.pid


def oracle_half_spectrum(o):
    nxh = o.p.Nx // 2
    return np.stack([getattr(o.state, nm)[:, :, :nxh] for nm in SPEC_NAMES])


def upload(gpu, o, with_fields=False):
    """Give the GPU handle the oracle's particles and spectral state."""
    cell, off, u, pid = oracle_particles(o)
    gpu.set_state(o.k, cell, off, u, oracle_half_spectrum(o), ids=pid)
    if with_fields:
        gpu.set_fields(o.F[:, :o.p.Nz])


def gpu_particles_to_oracle(p, d, dtype=np.float64):
    word = d["cell"].astype(np.int64)
    sp = (word >> 30) & 1
    cell = word & ~BEAM_BIT
    ix = cell % p.Nx
    iy = (cell // p.Nx) % p.Ny
    iz = cell // (p.Nx * p.Ny)
    off, u = d["off"].astype(dtype), d["u"].astype(dtype)
    return Particles(ix=ix, iy=iy, iz=iz, dx=off[0], dy=off[1], dz=off[2], ux=u[0], uy=u[1],
                     uz=u[2], pid=d.get("id", np.zeros(len(cell), np.int64)), sp=sp)


def rel_errors(ref, got, floor=1e-6):
    """Relative L2 error per component; a component whose reference norm is
    below floor times the largest component norm is measured against the
    largest norm instead."""
    norms = {k: np.linalg.norm(np.asarray(ref[k], np.float64)) for k in ref}
    big = max(norms.values()) if norms else 0.0
    out = {}
    for k in ref:
        n = norms[k] if norms[k] >= floor * big else big
        d = np.linalg.norm(np.asarray(got[k], np.float64) - np.asarray(ref[k], np.float64))
        out[k] = d / n if n > 0 else d
    return out


def check_fp32_fields(ref, got, rel=2e-4, ulps=30):
    """FP32 fields against the FP64 oracle, every component against its own
    norm: relative L2 error at most max(rel, ulps 2^-24 |largest| / |own|).
    FP32 roundoff of the largest fields leaves an error of a few units of
    2^-24 of them in every component, which is a large fraction of a
    component 1e-3 of the largest (observed: 2 to 3 units); the bar allows
    ten times that and no more."""
    norms = {k: np.linalg.norm(np.asarray(ref[k], np.float64)) for k in ref}
    big = max(norms.values())
    for k in ref:
        d = np.linalg.norm(np.asarray(got[k], np.float64) - np.asarray(ref[k], np.float64))
        bar = max(rel * norms[k], ulps * 2.0 ** -24 * big)
        assert d <= bar, (k, d / max(norms[k], 1e-300), bar / max(norms[k], 1e-300))


def oracle_fields(o):
    return {nm: o.F[c, :o.p.Nz] for c, nm in enumerate(FIELDS)}


def oracle_currents(o, nplanes):
    return {"Jx": o.J[0][:nplanes], "Jy": o.J[1][:nplanes], "Jz": o.J[2][:nplanes]}
