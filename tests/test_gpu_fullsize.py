"""Parity at the benchmark size and launch configuration (3-D LWFA 256 x 256 x
512 cells, 2 particles per cell, FP32 cell+offset particles, 8 x 8 x 4
tiles: 67.6 million particles), on outputs the FP64 oracle computes one
sample at a time:

* the initial load and tile order of sampled tiles (bit-exact ids, cells,
  offsets);
* one step from the loaded state with uploaded fields: the FP32 push of
  every particle of sampled tiles (bit-exact against the oracle's push run
  in FP32 on the same inputs), the stable tile order after the step (the
  exact id sequence of sampled destination tiles, built from every source
  tile that can feed them), and the deposited current on a box of nodes
  (every particle that reaches it taken from the oracle);
* the initial laser field state (FFT and the zeta march with Delta = 0) on
  sampled transverse modes, from a direct DFT and a per-mode march.
"""
import numpy as np
import pytest

import workloads
from oracle import params as oparams
from oracle import plasma as oplasma
from oracle.deposit import deposit
from oracle.fields import node_matrix, node_rhs, wavenumbers
from oracle.push import push_and_move
from paper_2509_16793_amd.gempic import Sim

pytestmark = pytest.mark.gpu

CFG = workloads.lwfa3d_fp32()
F32_ONE_MINUS = np.nextafter(np.float32(1), np.float32(0))


def _tile_key(p, ix, iy, iz):
    tx, ty, tz = p.tile
    nTx, nTy = p.Nx // tx, p.Ny // ty
    return (iz // tz * nTy + iy // ty) * nTx + ix // tx


def _split_cells(p, cell):
    cell = cell.astype(np.int64)
    return cell % p.Nx, (cell // p.Nx) % p.Ny, cell // (p.Nx * p.Ny)


def _fields(p):
    """Smooth synthetic fields of laser strength on every node, all six
    components non-zero (FP32, [6][Nz][Ny][Nx]); strong enough to move
    particles across transverse cells within one step."""
    z = (np.arange(p.Nz) * p.h)[:, None, None]
    y = (np.arange(p.Ny) * p.hy)[None, :, None]
    x = (np.arange(p.Nx) * p.hx)[None, None, :]
    F = np.empty((6, p.Nz, p.Ny, p.Nx), np.float32)
    amp = (3.0, 2.0, 0.5, 1.5, 3.0, 0.4)
    for c in range(6):
        F[c] = (amp[c] * np.cos(0.9 * z + 0.05 * (c + 1) * x - 0.03 * c * y + c)
                * np.cos(0.04 * y + 0.02 * c * x)).astype(np.float32)
    return F


def _f32(P):
    for k in ("dx", "dy", "dz"):
        setattr(P, k, np.minimum(getattr(P, k).astype(np.float32), F32_ONE_MINUS))
    for k in ("ux", "uy", "uz"):
        setattr(P, k, getattr(P, k).astype(np.float32))
    return P


def _tile_cells(p, t):
    tx, ty, tz = p.tile
    nTx, nTy = p.Nx // tx, p.Ny // ty
    ix0, iy0, iz0 = (t % nTx) * tx, (t // nTx) % nTy * ty, t // (nTx * nTy) * tz
    return np.arange(ix0, ix0 + tx), np.arange(iy0, iy0 + ty), np.arange(iz0, iz0 + tz)


# sampled tiles (tx, ty, tz): corners, the axis, a laser-crossed region, the back
SAMPLES = [(0, 0, 0), (31, 31, 3), (15, 16, 60), (16, 15, 110), (7, 24, 126), (20, 3, 64)]


@pytest.fixture(scope="module")
def run():
    p = oparams.from_config(CFG)
    g = Sim(CFG, track_ids=True)
    spec0 = g.spectral()
    before = g.particles(ids=True)
    F = _fields(p)
    g.set_fields(F)
    g.step(1)
    after = g.particles(ids=True)
    J = g.fields(("Jx", "Jy", "Jz"))
    g.close()
    Fz = np.zeros((6, p.Nz + p.ext + 1, p.Ny, p.Nx), np.float32)
    Fz[:, :p.Nz] = F
    return dict(p=p, spec0=spec0, before=before, after=after, J=J, F=Fz)


def _gpu_tile(p, parts, t):
    """Index range of tile t in a tile-sorted GPU particle copy."""
    ix, iy, iz = _split_cells(p, parts["cell"])
    key = _tile_key(p, ix, iy, iz)
    assert np.all(np.diff(key) >= 0), "particles not sorted by tile"
    return np.searchsorted(key, t, "left"), np.searchsorted(key, t, "right")


def _tile_index(p, tx, ty, tz):
    return (tz * (p.Ny // p.tile[1]) + ty) * (p.Nx // p.tile[0]) + tx


def test_initial_load_and_order(run):
    p, before = run["p"], run["before"]
    # every full cell is loaded, plus the first window batch
    assert len(before["id"]) >= (p.Nzp - 1) * p.Ny * p.Nx * 2
    for tx, ty, tz in SAMPLES:
        t = _tile_index(p, tx, ty, tz)
        a, b = _gpu_tile(p, before, t)
        O = _f32(oplasma.load_box(p, *_tile_cells(p, t)))
        order = np.argsort(O.pid, kind="stable")
        assert b - a == len(O), (t, b - a, len(O))
        assert np.array_equal(before["id"][a:b], O.pid[order]), t
        ix, iy, iz = _split_cells(p, before["cell"][a:b])
        assert np.array_equal(ix, O.ix[order]) and np.array_equal(iy, O.iy[order])
        assert np.array_equal(iz, O.iz[order])
        for k, arr in enumerate((O.dx, O.dy, O.dz)):
            assert np.array_equal(before["off"][k][a:b], arr[order]), (t, k)


def _pushed(p, F, P):
    """Oracle FP32 push of an FP32 particle set; returns (old positions,
    steps, vy) of the deposit and updates P."""
    return push_and_move(p, P, F)


def test_push_bit_exact_on_sampled_tiles(run):
    p, after, F = run["p"], run["after"], run["F"]
    order = np.argsort(after["id"])
    ids_sorted = after["id"][order]
    crossed = 0
    for tx, ty, tz in SAMPLES:
        t = _tile_index(p, tx, ty, tz)
        O = _f32(oplasma.load_box(p, *_tile_cells(p, t)))
        ix0 = O.ix.copy()
        _pushed(p, F, O)
        keep = O.iz >= 0
        crossed += int(np.count_nonzero(O.ix != ix0))
        pos = order[np.searchsorted(ids_sorted, O.pid[keep])]
        assert np.array_equal(after["id"][pos], O.pid[keep])
        cell = (O.iz * p.Ny + O.iy) * p.Nx + O.ix
        assert np.array_equal(after["cell"][pos].astype(np.int64), cell[keep]), t
        for k, arr in enumerate((O.dx, O.dy, O.dz)):
            assert np.array_equal(after["off"][k][pos], arr[keep]), (t, "off", k)
        for k, arr in enumerate((O.ux, O.uy, O.uz)):
            assert np.array_equal(after["u"][k][pos], arr[keep]), (t, "u", k)
    assert crossed > 0, "no transverse crossing sampled"


def test_stable_tile_order_after_step(run):
    """New tile t holds, in their previous global order (tile-major, load
    order within a tile), the particles of the neighbouring tiles that moved
    into it."""
    p, after, F = run["p"], run["after"], run["F"]
    nTx, nTy = p.Nx // p.tile[0], p.Ny // p.tile[1]
    for tx, ty, tz in SAMPLES[:4]:
        t = _tile_index(p, tx, ty, tz)
        srcs = []
        for sz in (0, 1):
            for sy in (-1, 0, 1):
                for sx in (-1, 0, 1):
                    s = _tile_index(p, (tx + sx) % nTx, (ty + sy) % nTy, tz + sz)
                    O = _f32(oplasma.load_box(p, *_tile_cells(p, s)))
                    O = O.take(np.argsort(O.pid, kind="stable"))
                    _pushed(p, F, O)
                    srcs.append((s, O))
        srcs.sort(key=lambda so: so[0])          # previous order: tile-major
        want = []
        for s, O in srcs:
            inside = (O.iz >= 0) & (_tile_key(p, O.ix, O.iy, O.iz) == t)
            want.append(O.pid[inside])
        want = np.concatenate(want)
        a, b = _gpu_tile(p, after, t)
        assert np.array_equal(after["id"][a:b], want), t


def test_current_on_sampled_node_box(run):
    """FP32 current against the FP64 deposit of the oracle-pushed particles
    that reach the box.  Bar 1e-4: each contribution carries a few FP32
    roundings (~3e-7) and a truncation into the fixed-point tile, node sums of
    mixed-sign transverse contributions cancel (amplifying the relative error
    to ~1e-5 here), and two tiles' partial sums meet in FP32 atomics; a
    misplaced or missing contribution shows as an error of order 1e-1.  (The
    FP64 parity tests pin the deposit itself to 1e-10.)"""
    p, J, F = run["p"], run["J"], run["F"]
    for x0, y0, z0 in ((120, 124, 240), (8, 200, 40)):
        cells = (np.arange(x0 - 4, x0 + 12), np.arange(y0 - 4, y0 + 12), np.arange(z0 - 4, z0 + 10))
        O = _f32(oplasma.load_box(p, *cells))
        old, steps, vy = _pushed(p, F, O)
        new = (O.ix, O.iy, O.iz, O.dx, O.dy, O.dz)
        Jo = deposit(p, old, new, steps, vy)
        box = (slice(z0 + 2, z0 + 6), slice(y0, y0 + 8), slice(x0, x0 + 8))   # planes of nodes z0 .. z0+3
        for name, jo in zip(("Jx", "Jy", "Jz"), Jo):
            ref = jo[box]
            got = J[name][box].astype(np.float64)
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            print(f"{name} box ({x0}, {y0}, {z0}): rel. L2 {err:.2e}")
            assert err < 1e-4, (name, x0, y0, z0, err)


def test_initial_laser_state_on_sampled_modes(run):
    """Laser of Sec. 6 as a forward wave, then the march with Delta = 0 and no
    current, per transverse mode: rfft-free direct DFT of the separable laser
    and the node equations solved mode by mode."""
    p, spec = run["p"], run["spec0"]
    KX, KY, nyq = wavenumbers(p)
    modes = [(0, 0), (1, 0), (0, 1), (3, 2), (2, 255), (7, 9), (20, 230)]
    zeta = np.arange(p.Nz) * p.h
    phi = zeta - p.zeta_c
    lon = p.a0 * np.cos(phi) * np.exp(-(phi * phi) / (p.T * p.T))
    x = np.arange(p.Nx) * p.hx - (p.Nx // 2) * p.hx
    y = np.arange(p.Ny) * p.hy - (p.Ny // 2) * p.hy
    tra = np.exp(-(x[None, :] ** 2 + y[:, None] ** 2) / (p.waist * p.waist))
    ii = np.arange(p.Nx)
    jj = np.arange(p.Ny)
    scale = np.abs(spec[0]).max()
    for kxi, kyi in modes:
        ex = np.exp(-2j * np.pi * kxi * ii / p.Nx)
        ey = np.exp(-2j * np.pi * kyi * jj / p.Ny)
        that = ey @ tra @ ex
        kx, ky = KX[kyi, kxi], KY[kyi, kxi]
        A = node_matrix(np.array([kx]), np.array([ky]), p.h, 0.0)
        right = [np.zeros(1, complex) for _ in range(6)]
        out = np.zeros((6, p.Nz), complex)
        zero = [np.zeros(1, complex)] * 3
        for n in range(p.Nz - 1, -1, -1):
            old = [np.array([2.0 * lon[n] * that]), np.zeros(1, complex), np.zeros(1, complex),
                   np.zeros(1, complex)]
            rhs = node_rhs(np.array([kx]), np.array([ky]), p.h, 0.0, old, right, zero, zero)
            sol = np.linalg.solve(A, rhs[..., None])[..., 0]
            right = [sol[:, c] for c in range(6)]
            out[:, n] = sol[0]
        # unknowns in the library's order Rx, Ry, Lx, Ly, Ez, Bz
        got = spec[:, :, kyi, kxi]
        err = np.abs(got - out).max() / scale
        assert err < 2e-5, (kxi, kyi, err)
