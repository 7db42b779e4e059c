"""Every tile shape and the degenerate cases through the C ABI against the FP64
oracle: the 4x4x4 3-D tiles and the three 2-D tile shapes (8x1x8, 8x1x4,
4x1x4), a vacuum run (no particles: only the laser and the field solver), the
smallest grids the tiles allow, and a quiet-lattice plasma without a laser
(whose lab current cancels away from the exit boundary).

Bars as in test_gpu_parity: cells and ids exact, fields within relative L2
1e-10 in FP64 (2e-4 in FP32)."""
import numpy as np
import pytest

import workloads
from oracle.sim import Simulation
from paper_2509_16793_amd.gempic import Sim
from parity import oracle_particles, oracle_fields, rel_errors

pytestmark = pytest.mark.gpu


def _check(cfg, steps, bar=1e-10, particles=True):
    o = Simulation(cfg).run(steps)
    g = Sim(cfg, track_ids=True)
    g.step(steps)
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < bar, err
    if particles:
        cell, off, u, pid = oracle_particles(o)
        d = g.particles(ids=True)
        assert np.array_equal(d["id"], pid)
        assert np.array_equal(d["cell"].astype(np.int64), cell)
    return o, g


def test_small3d_tile444_fp64():
    _check(workloads.small3d(tile=(4, 4, 4)), 4)


def test_small3d_tile444_fp32():
    _check(workloads.small3d("fp32", tile=(4, 4, 4)), 4, bar=2e-4, particles=False)


@pytest.mark.parametrize("tile", [(8, 1, 4), (4, 1, 4)], ids=["t814", "t414"])
def test_lwfa2d_other_tiles(tile):
    cfg = workloads.lwfa2d_fp64()
    cfg["tile"] = list(tile)
    _check(cfg, 10)


def test_vacuum_laser_only():
    cfg = workloads.small3d(n_e=0.0)
    o, g = _check(cfg, 6)
    assert g._count() == 0
    # the laser is a forward wave and stays put: its field energy is conserved
    d = g.step(0, diag=True)
    assert d["n_particles"] == 0


def test_smallest_grid():
    # one tile per transverse direction, two along zeta (4x4x4 tiles)
    cfg = workloads.small3d(n=(4, 4, 8), tile=(4, 4, 4))
    cfg["waist"] = 0.5
    _check(cfg, 3)


def test_quiet_plasma_interior_current_vanishes():
    # a quiet lattice at rest in the lab streams through the window at -c: its
    # lab current W_zeta + rhobar cancels on every plane the field solver
    # uses away from the exit boundary (as the oracle pin states)
    cfg = dict(dims=3, n=[8, 8, 32], d=[0.25, 0.25, 0.05], n_e=0.01, ppc=[1, 2, 2], load=1,
               tile=[4, 4, 4], length_unit=2 * np.pi, precision="fp64")
    o, g = _check(cfg, 1)
    p = o.p
    scale = abs(p.q * p.w / (p.hx * p.hy * p.h))
    J = g.fields(("Jx", "Jy", "Jz"))
    used = slice(2 + 3, 2 + p.Nz + 1)
    for k, v in J.items():
        assert np.abs(v[used]).max() < 1e-12 * scale, k
    F = g.fields()
    assert max(np.abs(v[3:]).max() for v in F.values()) < 1e-14
    _check(cfg, 6)


# Ny = 256 takes the register-based four-step transform along y (16 x 16)
# forwards and backwards; FP64 fields against the oracle's numpy FFTs
def test_ny256_four_step_transform_fp64():
    _check(workloads.small3d(precision="fp64", n=(16, 256, 32), steps=2), 2)


def test_ny256_four_step_transform_fp32():
    _check(workloads.small3d(precision="fp32", n=(16, 256, 32), steps=2), 2, bar=2e-4, particles=False)


# Ny = 512: one radix-2 step over two 256-point four-step transforms
def test_ny512_transform_fp64():
    _check(workloads.small3d(precision="fp64", n=(16, 512, 32), steps=2), 2)


def test_ny512_transform_fp32():
    _check(workloads.small3d(precision="fp32", n=(16, 512, 32), steps=2), 2, bar=2e-4, particles=False)


# Nx = 256 rows: the x transforms at the benchmark's row length, FP64 and FP32
# fields against the oracle
def test_nx256_transforms_fp64():
    _check(workloads.small3d(precision="fp64", n=(256, 16, 32), steps=2), 2)


def test_nx256_transforms_fp32():
    _check(workloads.small3d(precision="fp32", n=(256, 16, 32), steps=2), 2, bar=2e-4, particles=False)


# Nx = 512 rows (the PWFA row length): the radix-2 step over two 256-point
# four-step x transforms
def test_nx512_transforms_fp64():
    _check(workloads.small3d(precision="fp64", n=(512, 8, 32), steps=2), 2)


def test_nx512_transforms_fp32():
    _check(workloads.small3d(precision="fp32", n=(512, 8, 32), steps=2), 2, bar=2e-4, particles=False)


# configurations the library rejects at creation, each with the reason it
# names: a grid size that is not a power of two, a tile shape it does not
# support, a slow step beyond h / 2, and a transverse grid wider than the LDS
# transforms hold (FP64 rows of 1024 nodes)
@pytest.mark.parametrize("n,change,why", [
    ((24, 32, 64), {}, "powers of two"),
    ((16, 16, 32), {"tile": [4, 4, 8]}, "tile must be"),
    ((16, 16, 32), {"dtau": 0.8 * 0.05}, "slow step too large"),
    ((1024, 8, 32), {}, "transverse grid too large"),
])
def test_invalid_configurations_are_rejected(n, change, why):
    from paper_2509_16793_amd.gempic import GempicError
    cfg = workloads.small3d(precision="fp64", n=n, steps=1)
    cfg.update(change)
    with pytest.raises(GempicError, match=why):
        Sim(cfg)
