"""Field gather and particle push (oracle side).

The transformed Vlasov equation (Sec. 5, eq:Vlasov1) has characteristics
    ds/d eta = 1,  d zeta/d eta = v_z - 1,  d r_perp/d eta = v_perp,
    dp/d eta = F,
and the paper integrates initialised ("beam") particles along s (Sec. 5.1).
Here every particle is advanced in tau = s with one explicit leap-frog step:
momenta live at half steps, positions at whole steps, the fields at level k
push u^{k-1/2} -> u^{k+1/2}, then r^{k} -> r^{k+1}.

Reading (the paper only states du/dt = F): the momentum update is the
Higuera-Cary scheme (Phys. Plasmas 24, 052104, 2017), exact for uniform
E x B drifts.  With eps = (q/m) dtau / 2:
    u-  = u + eps E,  beta = eps B,  sigma = 1 + |u-|^2 - |beta|^2,
    gamma+ = sqrt((sigma + sqrt(sigma^2 + 4 (|beta|^2 + (beta . u-)^2))) / 2),
    t = beta / gamma+ (as beta times 1/gamma+),  s = 1 / (1 + |t|^2),
    u+ = s (u- + (u- . t) t + u- x t),  u_new = u+ + eps E + u+ x t.
Position update in cell units:
    dx += (u_x / gamma) dtau / h_x,   dy += (u_y / gamma) dtau / h_y,
    dzeta += (v_z - 1) dtau / h,
with v = u (1/gamma) and v_z - 1 = -(1 + u_x^2 + u_y^2) (1/gamma) / (gamma + u_z)
when u_z >= 0 and u_z (1/gamma) - 1 otherwise (the same number, free of
cancellation for u_z >> 1).  Divisions are written as one reciprocal each
where several quotients share a denominator.

Field shape (reading; the paper states none): linear (cloud-in-cell) on the
nodes.  Fields sit at nodes at level k; the plane n = N_zeta is a ghost plane
of zero fields.
"""
import numpy as np


def cic_weights(d):
    return 1.0 - d, d


def gather(p, P, F):
    """Interpolate the six node fields F[c] (shape (Nz+1, Ny, Nx)) to every
    particle.  Returns an array (6, N).  Sum order: zeta node outermost, then
    y, then x; weight = (wx * wy) * wz.  The arithmetic runs in the precision
    of the inputs (FP64 normally; FP32 inputs reproduce an FP32 push)."""
    wx = cic_weights(P.dx)
    wz = cic_weights(P.dz)
    ix1 = (P.ix + 1) % p.Nx
    xs = (P.ix, ix1)
    out = np.zeros((6, len(P)), dtype=np.result_type(F.dtype, P.dx.dtype))
    if p.dims == 3:
        wy = cic_weights(P.dy)
        ys = (P.iy, (P.iy + 1) % p.Ny)
    else:
        wy = (None,)
        ys = (P.iy,)
    for c in (0, 1):
        zc = P.iz + c
        for b in range(len(ys)):
            for a in (0, 1):
                if p.dims == 3:
                    w = (wx[a] * wy[b]) * wz[c]
                else:
                    w = wx[a] * wz[c]
                for comp in range(6):
                    out[comp] = out[comp] + w * F[comp][zc, ys[b], xs[a]]
    return out


def higuera_cary(ux, uy, uz, E, B, eps):
    """One Higuera-Cary momentum step; E, B arrays of shape (3, N)."""
    Ex, Ey, Ez = E
    umx = ux + eps * Ex
    umy = uy + eps * Ey
    umz = uz + eps * Ez
    bx = eps * B[0]
    by = eps * B[1]
    bz = eps * B[2]
    um2 = umx * umx + umy * umy + umz * umz
    b2 = bx * bx + by * by + bz * bz
    sigma = 1.0 + um2 - b2
    bu = bx * umx + by * umy + bz * umz
    gp = np.sqrt((sigma + np.sqrt(sigma * sigma + 4.0 * (b2 + bu * bu))) * 0.5)
    rgp = 1.0 / gp
    tx = bx * rgp
    ty = by * rgp
    tz = bz * rgp
    s = 1.0 / (1.0 + (tx * tx + ty * ty + tz * tz))
    ut = umx * tx + umy * ty + umz * tz
    upx = s * ((umx + ut * tx) + (umy * tz - umz * ty))
    upy = s * ((umy + ut * ty) + (umz * tx - umx * tz))
    upz = s * ((umz + ut * tz) + (umx * ty - umy * tx))
    nx = (upx + eps * Ex) + (upy * tz - upz * ty)
    ny = (upy + eps * Ey) + (upz * tx - upx * tz)
    nz = (upz + eps * Ez) + (upx * ty - upy * tx)
    return nx, ny, nz


def velocities(ux, uy, uz):
    """Return (gamma, v_x, v_y, v_z - 1)."""
    uperp2 = ux * ux + uy * uy
    g = np.sqrt(1.0 + (uperp2 + uz * uz))
    rg = 1.0 / g
    vx = ux * rg
    vy = uy * rg
    vzm1 = np.where(uz >= 0.0, (-(1.0 + uperp2) * rg) / (g + uz), uz * rg - 1.0)
    return g, vx, vy, vzm1


def renormalise(d, shift):
    """Offset d plus displacement shift (cell units) -> (new offset, cell step k).
    k = floor(d + shift); d' = d + shift - k; a rounded d' == 1 becomes 0, k + 1."""
    t = d + shift
    k = np.floor(t)
    t = t - k
    up = t >= 1.0
    t = np.where(up, 0.0, t)
    k = k + up
    return t, k.astype(np.int64)


def push_and_move(p, P, F):
    """Gather, push and move every particle of P (modified in place).
    Returns the old cells/offsets, the per-axis cell steps and (v_y for the 2-D
    out-of-plane current)."""
    Fp = gather(p, P, F)
    eps = 0.5 * p.q * p.dtau
    P.ux, P.uy, P.uz = higuera_cary(P.ux, P.uy, P.uz, Fp[0:3], Fp[3:6], eps)
    g, vx, vy, vzm1 = velocities(P.ux, P.uy, P.uz)
    ax = p.dtau / p.hx
    az = p.dtau / p.h
    old = (P.ix.copy(), P.iy.copy(), P.iz.copy(), P.dx.copy(), P.dy.copy(), P.dz.copy())
    P.dx, kx = renormalise(P.dx, vx * ax)
    if p.dims == 3:
        ay = p.dtau / p.hy
        P.dy, ky = renormalise(P.dy, vy * ay)
    else:
        ky = np.zeros_like(kx)
    P.dz, kz = renormalise(P.dz, vzm1 * az)
    if np.any(np.abs(kx) > 1) or np.any(np.abs(ky) > 1) or np.any(np.abs(kz) > 1):
        raise FloatingPointError("a particle crossed more than one cell in a step")
    P.ix = (P.ix + kx) % p.Nx
    P.iy = (P.iy + ky) % p.Ny
    P.iz = P.iz + kz
    return old, (kx, ky, kz), vy
