"""Oracle pins for the particle-field coupling: the 3-D gather, the transverse
half-cell shift of the solver currents, and the absolute-position (FP32-abs)
push and decoding.  Each pin is a closed form or a second, independent route
to the same number, chosen so that a plausible mistake (weights of two axes
swapped, the sign of the -h/2 shift flipped, the zeta average dropped, a
wrong inverse step or wrap) fails it.

* Gather: linear (cloud-in-cell) interpolation reproduces every trilinear
  function a + b x + c y + d z + e xy + f yz + g xz + k xyz exactly, so node
  fields sampled from one (different coefficients per axis and component)
  must gather to its value at the particle.
* Solver currents (Sec. 4.1, half-node currents of RxN .. eqall): W_x sits
  at x (i + 1/2), W_y at y (j + 1/2), both on zeta nodes; J_z on zeta
  half-nodes.  For a band-limited current cos(k.r + phi) the solver input on
  half-node n + 1/2 at the node (i, j) is, in closed form,
  cos(k_x x_i + k_y y_j + k_z (n + 1/2) h + phi) cos(k_z h / 2) for j_x and j_y
  (trigonometric identity of the zeta average, exact shift of a resolved
  mode) and the sampled value itself for j_z.
* Absolute positions: decoding against exact rational arithmetic; a uniform
  electric field against the closed-form first step; the FP64 absolute-
  position push against the cell + offset push (the same motion in two
  representations)."""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import params
from oracle.deposit import G
from oracle.fields import half_node_currents
from oracle.plasma import Particles
from oracle.push import gather, decode_abs, push_and_move_abs, push_and_move


def _p3(n=(8, 8, 16), dims=3):
    if dims == 3:
        cfg = workloads.small3d(precision="fp64", n=n, tile=(4, 4, 4), n_e=0.01)
        cfg["d"] = [0.4, 0.3, 0.05]       # h_x != h_y, so that swapped axes show
    else:
        cfg = workloads.lwfa2d_fp64()
        cfg["n"] = [n[0], 1, n[2]]
        cfg["tile"] = [4, 1, 4]
    return params.from_config(cfg)


def _particles(p, n, rng, interior=True):
    hi_x = p.Nx - 1 if interior else p.Nx
    hi_y = (p.Ny - 1 if interior else p.Ny) if p.dims == 3 else 1
    ix = rng.integers(0, hi_x, n)
    iy = rng.integers(0, hi_y, n)
    iz = rng.integers(0, p.Nz, n)
    z = np.zeros(n)
    return Particles(ix=ix, iy=iy, iz=iz, dx=rng.random(n), dy=rng.random(n) if p.dims == 3 else z,
                     dz=rng.random(n), ux=z.copy(), uy=z.copy(), uz=z.copy(), pid=np.zeros(n, np.int64))


@pytest.mark.parametrize("dims", [3, 2])
def test_gather_reproduces_trilinear_fields(dims):
    p = _p3(dims=dims)
    rng = np.random.default_rng(1)
    coef = rng.standard_normal((6, 8))
    if dims == 2:
        coef[:, [2, 4, 5, 7]] = 0.0        # no y dependence in 2-D
    z = np.arange(p.Nz + 1)[:, None, None].astype(float)
    y = np.arange(p.Ny)[None, :, None].astype(float)
    x = np.arange(p.Nx)[None, None, :].astype(float)

    def tri(c, X, Y, Z):
        return (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * Y + c[5] * Y * Z
                + c[6] * X * Z + c[7] * X * Y * Z)

    F = np.stack([np.broadcast_to(tri(coef[k], x, y, z), (p.Nz + 1, p.Ny, p.Nx)) for k in range(6)])
    P = _particles(p, 4000, rng)
    got = gather(p, P, F)
    X, Y, Z = P.ix + P.dx, P.iy + P.dy, P.iz + P.dz
    for k in range(6):
        want = tri(coef[k], X, Y, Z)
        assert np.max(np.abs(got[k] - want)) < 1e-12 * np.max(np.abs(want)), k


@pytest.mark.parametrize("dims", [3, 2])
def test_half_node_currents_of_a_resolved_mode(dims):
    p = _p3(n=(16, 8, 32), dims=dims)
    nplanes = p.Nz + p.ext + 4
    m1, m2, kz, phi = 3, (2 if dims == 3 else 0), 0.37, 0.41
    k1 = 2 * np.pi * m1 / (p.Nx * p.hx)
    k2 = 2 * np.pi * m2 / (p.Ny * p.hy) if dims == 3 else 0.0
    pl = np.arange(nplanes)[:, None, None]
    zeta = (pl - G) * p.h                                  # node n = plane - G
    yj = np.arange(p.Ny)[None, :, None] * (p.hy if dims == 3 else 0.0)
    xi = np.arange(p.Nx)[None, None, :] * p.hx
    Jx = np.cos(k1 * (xi + 0.5 * p.hx) + k2 * yj + kz * zeta + phi)
    Jy = np.cos(k1 * xi + k2 * (yj + (0.5 * p.hy if dims == 3 else 0.0)) + kz * zeta + phi) * 0.7
    Jz = np.cos(k1 * xi + k2 * yj + kz * (zeta + 0.5 * p.h) + phi) * 1.3   # half-node n + 1/2
    jx, jy, jz = half_node_currents(p, Jx, Jy, Jz)
    q = np.arange(p.Nz + 1)[:, None, None]
    zh = (q - 0.5) * p.h                                   # half-node q - 1/2
    base = np.cos(k1 * xi + k2 * yj + kz * zh + phi)
    avg = np.cos(0.5 * kz * p.h)
    back = lambda a: np.fft.ifft2(a, axes=(-2, -1))
    assert np.max(np.abs(back(jx) - base * avg)) < 1e-12
    assert np.max(np.abs(back(jy) - 0.7 * base * avg)) < 1e-12
    assert np.max(np.abs(back(jz) - 1.3 * base)) < 1e-12


def test_decode_abs_against_exact_rational_floor():
    rng = np.random.default_rng(2)
    for hval in (0.4 * 2 * np.pi, 0.05 * 2 * np.pi, 0.1):
        ih = np.float32(1.0 / hval)
        x = (rng.random(20000) * 512 * hval).astype(np.float32)
        c, off = decode_abs(x, ih)
        f32 = (x * ih).astype(np.float32)
        # the cell and offset partition the FP32 product exactly
        assert np.all((off >= 0) & (off < 1))
        assert np.array_equal(c.astype(np.float32) + off, f32)
        # and the cell is the exact floor of x / h in the rational sense
        # wherever the product is not within FP32 rounding of an integer
        for xv, cv in zip(x[:2000], c[:2000]):
            exact = Fraction(float(xv)) * Fraction(float(ih))
            fl = exact.numerator // exact.denominator
            if abs(float(exact - fl)) > 1e-6 and abs(float(exact - fl - 1)) > 1e-6:
                assert cv == fl
    # periodic wrap: a position that rounds up to the box length is cell 0
    n, hval = 64, 0.1
    ih = np.float32(1.0 / hval)
    x = np.float32(np.nextafter(np.float32(n / ih), np.float32(0)))
    c, _ = decode_abs(np.array([x]), ih, n)
    assert c[0] in (0, n - 1)
    c, _ = decode_abs(np.array([np.float32(n / ih)]), ih, n)
    assert c[0] == 0


def test_abs_push_in_uniform_electric_field_closed_form():
    # E = (Ex, Ey, Ez) uniform, B = 0: the Higuera-Cary step from rest gives
    # u = q dtau E exactly, and the move is v dtau with v = u / gamma
    p = _p3()
    rng = np.random.default_rng(3)
    n = 500
    E = np.array([0.3, -0.2, 0.1])
    F = np.zeros((6, p.Nz + p.ext + 1, p.Ny, p.Nx))
    for a in range(3):
        F[a] = E[a]
    for dt in (np.float64, np.float32):
        X = ((rng.integers(1, p.Nx - 1, n) + rng.random(n)) * p.hx).astype(dt)
        Y = ((rng.integers(1, p.Ny - 1, n) + rng.random(n)) * p.hy).astype(dt)
        Z = ((rng.integers(1, p.Nz - 1, n) + rng.random(n)) * p.h).astype(dt)
        z = np.zeros(n, dt)
        X1, Y1, Z1, ux, uy, uz, old, new, steps = push_and_move_abs(p, X, Y, Z, z, z.copy(), z.copy(),
                                                                    F.astype(dt))
        u = p.q * p.dtau * E
        gam = np.sqrt(1 + u @ u)
        tol = 1e-12 if dt is np.float64 else 2e-6
        for got, want in ((ux, u[0]), (uy, u[1]), (uz, u[2])):
            assert np.max(np.abs(got - want)) <= tol * abs(want)
        dx = u[0] / gam * p.dtau
        dy = u[1] / gam * p.dtau
        dz = (u[2] / gam - 1.0) * p.dtau
        ftol = 1e-12 if dt is np.float64 else 4e-6
        scale = max(p.Nx * p.hx, p.Nz * p.h)
        assert np.max(np.abs((X1 - X) - dx)) < ftol * scale
        assert np.max(np.abs((Y1 - Y) - dy)) < ftol * scale
        assert np.max(np.abs((Z1 - Z) - dz)) < ftol * scale


def test_abs_push_equals_cell_offset_push_in_fp64():
    # the same particles and fields moved in the two representations
    p = _p3()
    rng = np.random.default_rng(4)
    n = 3000
    F = np.zeros((6, p.Nz + p.ext + 1, p.Ny, p.Nx))
    F[:, :p.Nz] = 0.3 * rng.standard_normal((6, p.Nz, p.Ny, p.Nx))
    P = _particles(p, n, rng, interior=False)
    P.ux, P.uy, P.uz = (0.5 * rng.standard_normal(n) for _ in range(3))
    X = (P.ix + P.dx) * p.hx
    Y = (P.iy + P.dy) * p.hy
    Z = (P.iz + P.dz) * p.h
    X1, Y1, Z1, ux, uy, uz, old, new, steps = push_and_move_abs(p, X, Y, Z, P.ux.copy(), P.uy.copy(),
                                                                P.uz.copy(), F)
    push_and_move(p, P, F)
    assert np.max(np.abs(ux - P.ux)) < 1e-12 and np.max(np.abs(uz - P.uz)) < 1e-12
    xc = (P.ix + P.dx) * p.hx
    dxw = np.abs(X1 - xc)
    dxw = np.minimum(dxw, p.Nx * p.hx - dxw)           # periodic
    assert np.max(dxw) < 1e-12 * p.Nx * p.hx
    dyw = np.abs(Y1 - (P.iy + P.dy) * p.hy)
    dyw = np.minimum(dyw, p.Ny * p.hy - dyw)
    assert np.max(dyw) < 1e-12 * p.Ny * p.hy
    assert np.max(np.abs(Z1 - (P.iz + P.dz) * p.h)) < 1e-12 * p.Nz * p.h
    # cells agree wherever the position is not on a cell face
    jx, jy, jz = new[0], new[1], new[2]
    away = (np.abs(P.dx - 0.5) < 0.499) & (np.abs(P.dy - 0.5) < 0.499) & (np.abs(P.dz - 0.5) < 0.499)
    assert np.array_equal(jx[away], P.ix[away]) and np.array_equal(jz[away], P.iz[away])
    assert np.array_equal(jy[away], P.iy[away])
