"""Normalisation and derived parameters (oracle side).

Paper, Sec. 3 (normalisation): time in 1/omega_0, length in c/omega_0, fields
in m c omega_0 / e, so c = 1.  Densities are given in units of the critical
density of omega_0, hence omega_p^2 = n_e.  Electrons: q = -1, m = 1.

Plasma box (reading): the field grid has nodes n = 0 .. N_zeta - 1 and a
ghost node N_zeta with zero fields where the right-to-left march starts.
Unperturbed plasma lies ahead of the window, so the simulated plasma extends
E = filter_passes + 3 cells past the last field node (fields are zero there):
then every current on the half-nodes and nodes the march uses (after the
binomial filter) is the complete sum over all particles that reach it, and a
quiet plasma at rest deposits exactly zero lab current.  The plasma edge is
L = (N_zeta - 1 + E) h; particles occupy cells 0 .. N_zeta + E - 1.

Slow step (reading): the paper's particle rule limits the zeta sub-step to
min(h, Delta (1 - v_z)) (Sec. 5, stop rule eq:trap1), and the beam-particle
current of Sec. 5.1 needs Delta (1 - v_z) < h.  Pushing every particle in
tau, |d zeta| = (1 - v_z) d tau < 2 d tau, so d tau = h / 2 keeps every
particle within one cell crossing per step; larger steps are rejected.  The
scheme's own stability estimate Delta * h <= 4 / omega_p^2 (Sec. 4.2) is
checked as well.
"""
import math
from dataclasses import dataclass, field


class ConfigError(ValueError):
    pass


@dataclass
class Params:
    dims: int
    Nx: int
    Ny: int
    Nz: int
    hx: float
    hy: float
    h: float
    dtau: float
    n_e: float
    ppc: tuple
    load: int
    a0: float
    waist: float
    T: float
    zeta_c: float
    pol: int
    seed: int
    tile: tuple
    filter_passes: int
    q: float = -1.0
    w: float = 0.0          # physical electrons per macro-particle (number weight)
    L: float = 0.0          # right edge of the plasma box: (Nz - 1 + ext) h
    ext: int = 0            # plasma cells beyond the last field node
    beam: dict = field(default=None)

    @property
    def ppc_total(self):
        return self.ppc[0] * self.ppc[1] * self.ppc[2]

    @property
    def hy_eff(self):
        """Transverse y extent of a cell; 1 in 2-D (per unit length in y)."""
        return self.hy if self.dims == 3 else 1.0

    @property
    def Nzp(self):
        """Number of particle cells along zeta."""
        return self.Nz + self.ext

    @property
    def ntiles(self):
        return (self.Nx // self.tile[0], self.Ny // self.tile[1],
                -(-self.Nzp // self.tile[2]))


def _pow2(v):
    return v >= 1 and (v & (v - 1)) == 0


def from_config(cfg):
    """Turn a workload dict (see workloads.py) into normalised parameters."""
    lu = float(cfg.get("length_unit", 1.0))
    dims = int(cfg["dims"])
    Nx, Ny, Nz = (int(v) for v in cfg["n"])
    if dims == 2:
        Ny = 1
    hx = cfg["d"][0] * lu
    hy = cfg["d"][1] * lu if dims == 3 else 1.0
    h = cfg["d"][2] * lu
    dtau = cfg.get("dtau", 0.0) * lu
    if dtau == 0.0:
        dtau = 0.5 * h
    n_e = float(cfg.get("n_e", 0.0))
    ppc = tuple(int(v) for v in cfg.get("ppc", (1, 1, 1)))
    if dims == 2:
        ppc = (ppc[0], 1, ppc[2])
    tile = tuple(int(v) for v in cfg.get("tile", (8, 8, 8)))
    if dims == 2:
        tile = (tile[0], 1, tile[2])

    for v in (Nx, Nz) + ((Ny,) if dims == 3 else ()):
        if not _pow2(v):
            raise ConfigError("grid sizes must be powers of two")
    if Nx % tile[0] or Ny % tile[1] or Nz % tile[2]:
        raise ConfigError("tile must divide the grid")
    if 2.0 * dtau > h * (1.0 + 1e-12):
        raise ConfigError("slow step too large: need 2 dtau <= h")
    if n_e > 0.0 and dtau * h > 4.0 / n_e:
        raise ConfigError("slow step violates Delta*h <= 4/omega_p^2")

    a0 = float(cfg.get("a0", 0.0))
    fwhm = float(cfg.get("fwhm", 0.0)) * lu
    # Reading: "FWHM duration" is the intensity FWHM of exp(-2 phi^2 / T^2),
    # the intensity of the paper's pulse exp(-phi^2 / T^2) (Sec. 6, E_laser).
    T = fwhm / math.sqrt(2.0 * math.log(2.0)) if fwhm > 0 else 0.0
    fp = int(cfg.get("filter_passes", 1))
    if not 0 <= fp <= 2:
        raise ConfigError("filter_passes must be 0, 1 or 2")
    ext = fp + 3
    L = (Nz - 1 + ext) * h
    zc = cfg.get("zeta_c", None)
    # Default pulse centre (reading; unstated for the 3-D workloads): two
    # pulse lengths behind the last field node.
    zeta_c = (Nz - 1) * h - 2.0 * T if zc is None else float(zc) * lu
    p = Params(dims=dims, Nx=Nx, Ny=Ny, Nz=Nz, hx=hx, hy=hy, h=h, dtau=dtau,
               n_e=n_e, ppc=ppc, load=int(cfg.get("load", 0)), a0=a0,
               waist=float(cfg.get("waist", 0.0)) * lu, T=T, zeta_c=zeta_c,
               pol=int(cfg.get("pol", 0)), seed=int(cfg.get("seed", 0)),
               tile=tile, filter_passes=fp, L=L, ext=ext, beam=cfg.get("beam"))
    # Beam/initialised macro-particle weight Q_b = q n h_x h_y h (Sec. 5.1),
    # shared among the ppc particles of a cell.
    p.w = n_e * hx * p.hy_eff * h / p.ppc_total
    b = cfg.get("beam") or {}
    if int(b.get("np", 0)) > 0:
        # Electron driver (reading for a PWFA workload; the paper simulates
        # none): Gaussian bunch n_b exp(-r^2/2 sr^2) exp(-(zeta - zc)^2/2 sz^2)
        # (rms sizes) of n_b (2 pi)^(3/2) sr^2 sz electrons shared equally by
        # np macro-particles; u_perp = 0, gamma ~ N(gamma, dgamma).
        if dims != 3 or n_e <= 0.0:
            raise ConfigError("a driver beam needs dims = 3 and a plasma")
        sr, sz = float(b["sr"]) * lu, float(b["sz"]) * lu
        zb = b.get("zc", None)
        beam = dict(n=float(b["n"]), sr=sr, sz=sz,
                    zc=(Nz - 1) * h - 6.0 * sz if zb is None else float(zb) * lu,
                    gamma=float(b["gamma"]), dgamma=float(b.get("dgamma", 0.0)), np=int(b["np"]))
        beam["w"] = beam["n"] * (2.0 * math.pi) ** 1.5 * sr * sr * sz / beam["np"]
        beam["rb"] = beam["w"] / p.w
        p.beam = beam
    else:
        p.beam = None
    return p
