"""Witness-bunch diagnostics in the style of Table 1 (Sec. 6) (oracle side,
test infrastructure only).

Over the macro-particles with gamma >= gamma_min, weighted by their number
of electrons w: the charge Q = q sum w, the mean Lorentz factor <gamma> (the
mean energy is <gamma> m c^2), the rms spread of gamma, the rms sizes
sigma_x, sigma_y, sigma_zeta, and the normalised rms emittances
eps_x = sqrt(<dx^2> <du_x^2> - <dx du_x>^2) (and y), d. = deviation from the
weighted mean, u = gamma v in units of c.  Positions are measured from the
axis node (Nx/2, Ny/2) transversally and from zeta = 0 along zeta.  The
paper defines none of these formulas; they are the textbook ones (e.g.
Reiser, Theory and Design of Charged Particle Beams, ch. 5)."""
import numpy as np


def moments(x, y, z, ux, uy, uz, w, gamma_min, q=-1.0):
    g = np.sqrt(1.0 + ux * ux + uy * uy + uz * uz)
    sel = g >= gamma_min
    out = dict(n_macro=int(np.count_nonzero(sel)))
    W = float(np.sum(w[sel]))
    out["charge"] = q * W
    if W <= 0.0:
        for k in ("gamma_mean", "gamma_rms", "sigma_x", "sigma_y", "sigma_z", "eps_x", "eps_y",
                  "mean_x", "mean_y", "mean_z"):
            out[k] = 0.0
        return out
    ws = w[sel] / W

    def mean(a):
        return float(np.sum(ws * a[sel]))

    def var(a, b=None):
        b = a if b is None else b
        return float(np.sum(ws * (a[sel] - mean(a)) * (b[sel] - mean(b))))

    out["gamma_mean"] = mean(g)
    out["gamma_rms"] = np.sqrt(max(var(g), 0.0))
    out["mean_x"], out["mean_y"], out["mean_z"] = mean(x), mean(y), mean(z)
    out["sigma_x"] = np.sqrt(max(var(x), 0.0))
    out["sigma_y"] = np.sqrt(max(var(y), 0.0))
    out["sigma_z"] = np.sqrt(max(var(z), 0.0))
    out["eps_x"] = np.sqrt(max(var(x) * var(ux) - var(x, ux) ** 2, 0.0))
    out["eps_y"] = np.sqrt(max(var(y) * var(uy) - var(y, uy) ** 2, 0.0))
    return out


def positions_tau(p, P):
    """Positions of tau-path particles (cell + offset) from the axis / zeta = 0."""
    x = (P.ix + P.dx) * p.hx - (p.Nx // 2) * p.hx
    y = ((P.iy + P.dy) * p.hy - (p.Ny // 2) * p.hy) if p.dims == 3 else np.zeros(len(P))
    z = (P.iz + P.dz) * p.h
    return x, y, z


def positions_march(m, P):
    """Positions of zeta-march particles (cell + offset in (0, 1] along zeta)."""
    p = m.p
    x = (P.ix + P.dx) * p.hx - (p.Nx // 2) * p.hx
    y = ((P.iy + P.dy) * p.hy - (p.Ny // 2) * p.hy) if p.dims == 3 else np.zeros(len(P))
    z = m.zn[P.iz] + P.dz * m.hz[P.iz]
    return x, y, z
