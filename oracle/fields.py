"""Galilean-frame Maxwell update: the FD-spectral scheme of Sec. 4.1 (oracle side).

Transverse directions are spectral (2-D Fourier transform, Sec. 3.1, eqs.
eq:2dBz/eq:2dEz); per transverse mode (k_x, k_y) the state is the universal
reduced system (eq:RxGu .. eq:EzGu) in the characteristic variables
    R_x = E_x + B_y, R_y = E_y - B_x, L_x = E_x - B_y, L_y = E_y + B_x
(eq:Rx .. eq:Ly), so that E_x = (R_x + L_x)/2, B_y = (R_x - L_x)/2,
E_y = (R_y + L_y)/2, B_x = (L_y - R_y)/2.

Node system (Sec. 4.1, eqs. RxN .. eqall).  Node "0" is zeta node n, node "1"
is n + 1, superscript 0/1 the old/new slow level; marching starts at the
right boundary and every node-1 quantity at the new level is already known.
Readings (each verified: the paper's closed form of App. B then equals the
direct solve of this system to roundoff, and fails to with the printed text):
  * the lower index is the zeta node (the text says "steps along s");
  * the L_y equation uses (B_z0^1 + B_z1^1)/2, symmetric with the L_x one;
  * the E_z equation carries +i k_y (B_x0 + B_x1)/2, as eq:EzGu does;
  * (App. B, used by the GPU path, not here: T_4 = -2 h Delta E_z0^0 K^2.)
Time level of the currents (reading): the paper needs j at both slow levels
and predicts j^1 by a predictor-corrector inside its own zeta march; with a
leap-frog step in tau the current J^{k+1/2} deposited by the step is used at
both levels (j^0 = j^1), which time-centres the Crank-Nicolson R update.

This module solves each node as a dense 6x6 complex system (the plain
definition of the scheme), batched over all transverse modes.

Current placement (reading): W_x sits at (i+1/2, j, n); the solver wants j_x
on the zeta half-node n+1/2 at node x_i, so j_x = shift(-h_x/2) of
(W_x(n) + W_x(n+1))/2, the shift done spectrally (factor exp(-i k_x h_x/2));
likewise j_y; J_z is already on the half-node.  Nyquist rows/columns are set
to zero in every solver input and output so that real fields stay real.
Boundaries: transverse periodic; the ghost node N_zeta carries zero fields at
every level; half-node currents from -1/2 to N_zeta - 1/2 are used.
"""
import numpy as np

from .deposit import G


def wavenumbers(p):
    kx = 2.0 * np.pi * np.fft.fftfreq(p.Nx, d=p.hx)
    ky = 2.0 * np.pi * np.fft.fftfreq(p.Ny, d=p.hy) if p.Ny > 1 else np.zeros(1)
    KX, KY = np.meshgrid(kx, ky, indexing="xy")   # shape (Ny, Nx)
    nyq = np.zeros((p.Ny, p.Nx), bool)
    nyq[:, p.Nx // 2] = True
    if p.Ny > 1:
        nyq[p.Ny // 2, :] = True
    return KX, KY, nyq


class SpectralState:
    """R_x, R_y, L_x, L_y, E_z, B_z per node n = 0 .. N_zeta - 1 and mode."""
    NAMES = ("Rx", "Ry", "Lx", "Ly", "Ez", "Bz")

    def __init__(self, p):
        shape = (p.Nz, p.Ny, p.Nx)
        for n in self.NAMES:
            setattr(self, n, np.zeros(shape, complex))

    def copy(self, p):
        s = SpectralState(p)
        for n in self.NAMES:
            setattr(s, n, getattr(self, n).copy())
        return s


def fft2(a):
    return np.fft.fft2(a, axes=(-2, -1))


def ifft2_real(a):
    r = np.fft.ifft2(a, axes=(-2, -1))
    return r.real


def node_matrix(kx, ky, h, D):
    """Left-hand side of the node system for unknowns (Rx, Ry, Lx, Ly, Ez, Bz)
    at node 0 / new level; rows RxN, RyN (times Delta), Lx, Ly (times h/2),
    Bz, Ez (times h).  kx, ky: arrays over modes.  Returns shape (M, 6, 6)."""
    i = 1j
    M = kx.size
    A = np.zeros((M, 6, 6), complex)
    ikx, iky = i * kx, i * ky
    # RxN: Rx - D/2 (i kx Ez + i ky Bz)
    A[:, 0, 0] = 1.0
    A[:, 0, 4] = -0.5 * D * ikx
    A[:, 0, 5] = -0.5 * D * iky
    # RyN: Ry - D/2 (i ky Ez - i kx Bz)
    A[:, 1, 1] = 1.0
    A[:, 1, 4] = -0.5 * D * iky
    A[:, 1, 5] = 0.5 * D * ikx
    # Lx: -Lx - h/4 i kx Ez + h/4 i ky Bz
    A[:, 2, 2] = -1.0
    A[:, 2, 4] = -0.25 * h * ikx
    A[:, 2, 5] = 0.25 * h * iky
    # Ly: -Ly - h/4 i ky Ez - h/4 i kx Bz
    A[:, 3, 3] = -1.0
    A[:, 3, 4] = -0.25 * h * iky
    A[:, 3, 5] = -0.25 * h * ikx
    # Bz: -Bz - h/2 (i kx (Ry + Ly)/2 - i ky (Rx + Lx)/2)
    A[:, 4, 5] = -1.0
    A[:, 4, 1] = -0.25 * h * ikx
    A[:, 4, 3] = -0.25 * h * ikx
    A[:, 4, 0] = 0.25 * h * iky
    A[:, 4, 2] = 0.25 * h * iky
    # Ez: -Ez - h/2 (-i kx (Rx - Lx)/2 + i ky (Ly - Ry)/2)
    A[:, 5, 4] = -1.0
    A[:, 5, 0] = 0.25 * h * ikx
    A[:, 5, 2] = -0.25 * h * ikx
    A[:, 5, 3] = -0.25 * h * iky
    A[:, 5, 1] = 0.25 * h * iky
    return A


def node_rhs(kx, ky, h, D, old, right, jm, jp):
    """Right-hand side.  old = (Rx0, Ry0, Ez0, Bz0) at node 0, old level;
    right = (Rx, Ry, Lx, Ly, Ez, Bz) at node 1, new level; jm / jp = (jx, jy, jz)
    on the half-nodes -1/2 and +1/2 (same at both levels)."""
    i = 1j
    ikx, iky = i * kx, i * ky
    Rx0, Ry0, Ez0, Bz0 = old
    Rx1, Ry1, Lx1, Ly1, Ez1, Bz1 = right
    Ex1 = 0.5 * (Rx1 + Lx1)
    Ey1 = 0.5 * (Ry1 + Ly1)
    By1 = 0.5 * (Rx1 - Lx1)
    Bx1 = 0.5 * (Ly1 - Ry1)
    b = np.zeros((kx.size, 6), complex)
    b[:, 0] = Rx0 + 0.5 * D * (ikx * Ez0 + iky * Bz0) - 0.25 * D * 2.0 * (jm[0] + jp[0])
    b[:, 1] = Ry0 + 0.5 * D * (iky * Ez0 - ikx * Bz0) - 0.25 * D * 2.0 * (jm[1] + jp[1])
    b[:, 2] = -Lx1 + 0.25 * h * (ikx * Ez1 - iky * Bz1) + 0.5 * h * jp[0]
    b[:, 3] = -Ly1 + 0.25 * h * (iky * Ez1 + ikx * Bz1) + 0.5 * h * jp[1]
    b[:, 4] = -Bz1 + 0.5 * h * (ikx * Ey1 - iky * Ex1)
    b[:, 5] = -Ez1 + 0.5 * h * (-ikx * By1 + iky * Bx1) + h * jp[2]
    return b


def march(p, old, jh, D):
    """One slow step of the field state.  ``old``: SpectralState at level k;
    ``jh``: (jx, jy, jz) spectral currents on half-nodes q = 0 .. N_zeta
    (half-node q - 1/2); ``D``: the slow step.  Returns the new SpectralState."""
    KX, KY, nyq = wavenumbers(p)
    kx, ky = KX.ravel(), KY.ravel()
    keep = ~nyq.ravel()
    A = node_matrix(kx[keep], ky[keep], p.h, D)
    new = SpectralState(p)
    right = [np.zeros(kx.size, complex) for _ in range(6)]
    for n in range(p.Nz - 1, -1, -1):
        oldn = [getattr(old, nm)[n].ravel() for nm in ("Rx", "Ry", "Ez", "Bz")]
        jm = [jh[c][n].ravel() for c in range(3)]
        jp = [jh[c][n + 1].ravel() for c in range(3)]
        rhs = node_rhs(kx[keep], ky[keep], p.h, D, [o[keep] for o in oldn],
                       [r[keep] for r in right], [v[keep] for v in jm],
                       [v[keep] for v in jp])
        sol = np.linalg.solve(A, rhs[..., None])[..., 0]
        vals = []
        for c in range(6):
            v = np.zeros(kx.size, complex)
            v[keep] = sol[:, c]
            vals.append(v)
            getattr(new, SpectralState.NAMES[c])[n] = v.reshape(p.Ny, p.Nx)
        right = vals
    return new


def binomial_filter(p, A):
    """One 1-2-1 pass along x and y (periodic) and zeta (zero beyond the
    stored planes)."""
    A = 0.25 * (np.roll(A, 1, axis=2) + 2.0 * A + np.roll(A, -1, axis=2))
    if p.dims == 3:
        A = 0.25 * (np.roll(A, 1, axis=1) + 2.0 * A + np.roll(A, -1, axis=1))
    Z = np.zeros_like(A)
    up = Z.copy()
    up[:-1] = A[1:]
    dn = Z.copy()
    dn[1:] = A[:-1]
    return 0.25 * (dn + 2.0 * A + up)


def half_node_currents(p, Jx, Jy, Jz):
    """Real-space node/half-node currents (plane = n + 2)
    -> spectral solver inputs on half-nodes q = 0 .. N_zeta (n + 1/2 with
    n = q - 1)."""
    KX, KY, nyq = wavenumbers(p)
    sx = np.exp(-0.5j * KX * p.hx)
    sy = np.exp(-0.5j * KY * p.hy) if p.dims == 3 else np.ones_like(KY, complex)
    FX, FY, FZ = fft2(Jx), fft2(Jy), fft2(Jz)
    q = np.arange(p.Nz + 1)
    jx = 0.5 * (FX[q + G - 1] + FX[q + G]) * sx
    jy = 0.5 * (FY[q + G - 1] + FY[q + G]) * sy
    jz = FZ[q + G - 1].copy()
    for a in (jx, jy, jz):
        a[:, nyq] = 0.0
    return jx, jy, jz


def real_fields(p, s):
    """Six real node fields (Ex, Ey, Ez, Bx, By, Bz), each of shape
    (N_zeta + ext + 1, Ny, Nx): nodes 0 .. N_zeta - 1 from the solver, zero at
    the ghost node N_zeta and on the nodes of the plasma ahead of the grid."""
    spec = [0.5 * (s.Rx + s.Lx), 0.5 * (s.Ry + s.Ly), s.Ez,
            0.5 * (s.Ly - s.Ry), 0.5 * (s.Rx - s.Lx), s.Bz]
    out = np.zeros((6, p.Nz + p.ext + 1, p.Ny, p.Nx))
    for c in range(6):
        out[c, :p.Nz] = ifft2_real(spec[c])
    return out


def beam_field(p, s, rho_b):
    """Add the field of a charge moving at c (driver beam) to the state:
    per zeta node the transverse Poisson problem div E_perp = rho with
    E_perp = -grad phi, so phi^ = rho^ / K^2, E_perp^ = -i k_perp phi^ (K = 0
    and Nyquist modes: 0), as a forward wave R_perp += 2 E_perp^ (B_perp = z x
    E_perp, so L = 0).  rho_b: node charge density, shape (N_zeta, Ny, Nx),
    filtered like the currents (binomial_filter, zero beyond the field nodes)
    so that the field matches the filtered current the solver receives."""
    KX, KY, nyq = wavenumbers(p)
    K2 = KX * KX + KY * KY
    for _ in range(p.filter_passes):
        rho_b = binomial_filter(p, rho_b)
    rh = fft2(rho_b)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(K2 > 0, rh / np.where(K2 > 0, K2, 1.0), 0.0)
    Rx = -2j * KX * phi
    Ry = -2j * KY * phi
    Rx[:, nyq] = 0.0
    Ry[:, nyq] = 0.0
    s.Rx = s.Rx + Rx
    s.Ry = s.Ry + Ry
    return s


def beam_current(p, rho_b):
    """Lab current of charge moving at c, J_z(n + 1/2) = (rho(n) + rho(n+1))/2
    (the time- and zeta-centred charge a step deposits for it), in the current
    plane layout, filtered like a step's current; solver inputs."""
    nplanes = p.Nz + p.ext + 4
    Jz = np.zeros((nplanes, p.Ny, p.Nx))
    r = np.zeros((p.Nz + 2, p.Ny, p.Nx))      # nodes -1 .. N_zeta
    r[1:p.Nz + 1] = rho_b
    Jz[G - 1:G + p.Nz] = 0.5 * (r[:-1] + r[1:])
    zero = np.zeros_like(Jz)
    J = [zero, zero.copy(), Jz]
    for _ in range(p.filter_passes):
        J = [binomial_filter(p, a) for a in J]
    return half_node_currents(p, *J)


def laser_state(p, rho_b=None):
    """Laser of Sec. 6 (eq. E_laser) as a pure forward wave in the Galilean
    frame: E_pol = a0 cos(phi) exp(-phi^2/T^2) exp(-r_perp^2/R^2), phi =
    zeta - zeta_c (k_0 = 1), on the field nodes n = 0 .. N_zeta - 1, axis at
    node (Nx/2, Ny/2); R_pol = 2 E_pol, L = 0; plus the field of a driver beam
    of node charge density rho_b (beam_field), if given.
    The zeta-constraint fields (L, E_z, B_z) are then made consistent by one
    march with Delta = 0, with the beam's current (beam_current) if there is a
    beam and no current otherwise."""
    s = SpectralState(p)
    zero = np.zeros((p.Nz + 1, p.Ny, p.Nx), complex)
    cur = (zero, zero, zero)
    if rho_b is not None:
        s = beam_field(p, s, rho_b)
        cur = beam_current(p, rho_b)
    if p.a0 == 0.0:
        return s if rho_b is None else march(p, s, cur, 0.0)
    zeta = np.arange(p.Nz) * p.h
    phi = zeta - p.zeta_c
    lon = p.a0 * np.cos(phi) * np.exp(-(phi * phi) / (p.T * p.T))
    x = np.arange(p.Nx) * p.hx - (p.Nx // 2) * p.hx
    if p.dims == 3:
        y = np.arange(p.Ny) * p.hy - (p.Ny // 2) * p.hy
    else:
        y = np.zeros(1)
    X, Y = np.meshgrid(x, y, indexing="xy")
    if p.waist > 0.0:
        tra = np.exp(-(X * X + Y * Y) / (p.waist * p.waist))
    else:
        tra = np.ones_like(X)
    E = lon[:, None, None] * tra[None]
    _, _, nyq = wavenumbers(p)
    R = fft2(2.0 * E)
    R[:, nyq] = 0.0
    if p.pol == 0:
        s.Rx = s.Rx + R
    else:
        s.Ry = s.Ry + R
    return march(p, s, cur, 0.0)
