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

Every product-plus-addend below is written madd(a, b, c) = a b + c.  In FP64 it
is a product rounded, then a sum rounded (the plain formula).  On FP32 inputs it
is one fused multiply-add, rounded once, which is what an FP32 push on hardware
with FMA computes; the grouping of every sum is the same in both precisions.
"""
import numpy as np


def fma32(a, b, c):
    """Fused multiply-add in FP32, rounded once to nearest-even.

    The product of two FP32 numbers is exact in FP64; the FP64 sum is made
    round-to-odd (sticky last bit from the exact TwoSum error), and rounding a
    round-to-odd value of at least p + 2 bits to p bits equals rounding the
    exact value (Boldo & Melquiond, IEEE Trans. Computers 57(4), 2008)."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    c = np.asarray(c, np.float32)
    p = a.astype(np.float64) * b.astype(np.float64)
    c64 = c.astype(np.float64)
    s = p + c64
    bb = s - p
    e = (p - (s - bb)) + (c64 - bb)
    even = (np.asarray(s).view(np.int64) & 1) == 0
    toward = np.where(e > 0, np.inf, -np.inf)
    s = np.where((e != 0) & even, np.nextafter(s, toward), s)
    return s.astype(np.float32)


def madd(a, b, c):
    """a * b + c: fused in FP32, product then sum in FP64."""
    if np.result_type(a, b, c) == np.float32:
        return fma32(a, b, c)
    return a * b + c


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
                    out[comp] = madd(w, F[comp][zc, ys[b], xs[a]], out[comp])
    return out


def higuera_cary(ux, uy, uz, E, B, eps):
    """One Higuera-Cary momentum step; E, B arrays of shape (3, N)."""
    Ex, Ey, Ez = E
    umx = madd(eps, Ex, ux)
    umy = madd(eps, Ey, uy)
    umz = madd(eps, Ez, uz)
    bx = eps * B[0]
    by = eps * B[1]
    bz = eps * B[2]
    um2 = madd(umz, umz, madd(umy, umy, umx * umx))
    b2 = madd(bz, bz, madd(by, by, bx * bx))
    sigma = (1.0 + um2) - b2
    bu = madd(bz, umz, madd(by, umy, bx * umx))
    gp = np.sqrt((sigma + np.sqrt(madd(sigma, sigma, 4.0 * madd(bu, bu, b2)))) * 0.5)
    rgp = 1.0 / gp
    tx = bx * rgp
    ty = by * rgp
    tz = bz * rgp
    s = 1.0 / (1.0 + madd(tz, tz, madd(ty, ty, tx * tx)))
    ut = madd(umz, tz, madd(umy, ty, umx * tx))
    upx = s * (madd(ut, tx, umx) + madd(umy, tz, -(umz * ty)))
    upy = s * (madd(ut, ty, umy) + madd(umz, tx, -(umx * tz)))
    upz = s * (madd(ut, tz, umz) + madd(umx, ty, -(umy * tx)))
    nx = madd(eps, Ex, upx) + madd(upy, tz, -(upz * ty))
    ny = madd(eps, Ey, upy) + madd(upz, tx, -(upx * tz))
    nz = madd(eps, Ez, upz) + madd(upx, ty, -(upy * tx))
    return nx, ny, nz


def velocities(ux, uy, uz):
    """Return (gamma, v_x, v_y, v_z - 1)."""
    uperp2 = madd(uy, uy, ux * ux)
    g = np.sqrt(1.0 + madd(uz, uz, uperp2))
    rg = 1.0 / g
    vx = ux * rg
    vy = uy * rg
    vzm1 = np.where(uz >= 0.0, (-(1.0 + uperp2) * rg) / (g + uz), madd(uz, rg, -1.0))
    return g, vx, vy, vzm1


def renormalise(d, shift, a=None):
    """Offset d plus displacement (cell units) -> (new offset, cell step k).
    The displacement is shift, or madd(shift, a, d) - d when a velocity shift
    and a factor a are given.  k = floor(t); d' = t - k; a rounded d' == 1
    becomes 0, k + 1."""
    t = d + shift if a is None else madd(shift, a, d)
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
    P.dx, kx = renormalise(P.dx, vx, ax)
    if p.dims == 3:
        ay = p.dtau / p.hy
        P.dy, ky = renormalise(P.dy, vy, ay)
    else:
        ky = np.zeros_like(kx)
    P.dz, kz = renormalise(P.dz, vzm1, az)
    if np.any(np.abs(kx) > 1) or np.any(np.abs(ky) > 1) or np.any(np.abs(kz) > 1):
        raise FloatingPointError("a particle crossed more than one cell in a step")
    P.ix = (P.ix + kx) % p.Nx
    P.iy = (P.iy + ky) % p.Ny
    P.iz = P.iz + kz
    return old, (kx, ky, kz), vy


def decode_abs(x, ih, n=None):
    """Cell and offset of absolute positions x along an axis: f = x * ih in the
    precision of x, cell = floor(f), offset = f - cell; with n (periodic axis)
    a cell equal to n wraps to 0."""
    f = x * ih
    c = np.floor(f)
    off = f - c
    c = c.astype(np.int64)
    if n is not None:
        c = np.where(c >= n, c - n, c)
    return c, off


def push_and_move_abs(p, X, Y, Z, ux, uy, uz, F):
    """Gather, push and move with absolute positions (x, y, zeta from the grid
    origin) instead of cell + offset, in the precision of the inputs (FP32 for
    the absolute-position precision mode).  Cells and offsets are decoded with
    the inverse steps rounded to that precision; the move adds v dtau to the
    position, wraps x and y into the periodic box and decodes again.
    Returns (X1, Y1, Z1, ux, uy, uz, old, new, steps) with old/new =
    (ix, iy, iz, dx, dy, dz)."""
    from .plasma import Particles
    dt = X.dtype.type
    ihx, ihy, ih = dt(1.0 / p.hx), dt(1.0 / p.hy), dt(1.0 / p.h)
    Lx, Ly = dt(p.Nx * p.hx), dt(p.Ny * p.hy)
    ix, dx = decode_abs(X, ihx, p.Nx)
    iy, dy = decode_abs(Y, ihy, p.Ny)
    iz, dz = decode_abs(Z, ih)
    top = iz >= p.Nzp
    iz = np.where(top, p.Nzp - 1, iz)
    dz = np.where(top, np.nextafter(dt(1), dt(0)), dz)
    P = Particles(ix=ix, iy=iy, iz=iz, dx=dx, dy=dy, dz=dz, ux=ux, uy=uy, uz=uz,
                  pid=np.zeros(len(ix), np.int64))
    Fp = gather(p, P, F)
    eps = 0.5 * p.q * p.dtau
    ux, uy, uz = higuera_cary(ux, uy, uz, Fp[0:3], Fp[3:6], eps)
    g, vx, vy, vzm1 = velocities(ux, uy, uz)
    dtau = dt(p.dtau)
    X1 = madd(vx, dtau, X)
    X1 = np.where(X1 >= Lx, X1 - Lx, np.where(X1 < 0, X1 + Lx, X1))
    Y1 = madd(vy, dtau, Y)
    Y1 = np.where(Y1 >= Ly, Y1 - Ly, np.where(Y1 < 0, Y1 + Ly, Y1))
    Z1 = madd(vzm1, dtau, Z)
    jx, ex = decode_abs(X1, ihx, p.Nx)
    jy, ey = decode_abs(Y1, ihy, p.Ny)
    jz, ez = decode_abs(Z1, ih)
    kx = jx - ix
    kx = np.where(kx > 1, kx - p.Nx, np.where(kx < -1, kx + p.Nx, kx))
    ky = jy - iy
    ky = np.where(ky > 1, ky - p.Ny, np.where(ky < -1, ky + p.Ny, ky))
    kz = jz - iz
    return (X1, Y1, Z1, ux, uy, uz, (ix, iy, iz, dx, dy, dz), (jx, jy, jz, ex, ey, ez),
            (kx, ky, kz))
