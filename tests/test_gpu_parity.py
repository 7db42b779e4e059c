"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Bars: cell indices, ids (the stable sort permutation) and, from identical
inputs, the FP64 push bit for bit; fields within relative L2 1e-10 in FP64 and
2e-4 in FP32 (after 50 steps of the 2-D LWFA workload)."""
import numpy as np
import pytest

import workloads
from oracle.sim import Simulation
from paper_2509_16793_amd.gempic import Sim
from parity import (oracle_particles, upload, rel_errors, oracle_fields, oracle_currents,
                    gpu_particles_to_oracle)

pytestmark = pytest.mark.gpu


def _small3d(prec="fp64", **kw):
    return workloads.small3d(precision=prec, **kw)


def _compare_particles_exact(o, g):
    cell, off, u, pid = oracle_particles(o)
    d = g.particles(ids=True)
    assert len(d["cell"]) == len(cell)
    assert np.array_equal(d["id"], pid), "sort permutation differs"
    assert np.array_equal(d["cell"].astype(np.int64), cell), "cells differ"
    return d, off, u


@pytest.mark.parametrize("cfg", [workloads.lwfa2d_fp64(), _small3d()], ids=["lwfa2d", "small3d"])
def test_initial_state(cfg):
    o = Simulation(cfg)
    g = Sim(cfg, track_ids=True)
    d, off, u = _compare_particles_exact(o, g)
    dims = cfg["dims"]
    assert np.array_equal(d["off"][0], off[0]) and np.array_equal(d["off"][2], off[2])
    if dims == 3:
        assert np.array_equal(d["off"][1], off[1])
    assert not np.any(d["u"])
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-12, err


@pytest.mark.parametrize("cfg", [workloads.lwfa2d_fp64(), _small3d(), _small3d(tile=(8, 8, 4))],
                         ids=["lwfa2d", "small3d", "small3d_t884"])
def test_push_bit_exact_from_shared_state(cfg):
    o = Simulation(cfg).run(3)
    g = Sim(cfg, track_ids=True)
    upload(g, o, with_fields=True)
    o.step()
    g.step(1)
    d, off, u = _compare_particles_exact(o, g)
    dims = cfg["dims"]
    for a in (0, 2) + ((1,) if dims == 3 else ()):
        assert np.array_equal(d["off"][a], off[a]), f"offset axis {a}"
    for a in range(3):
        assert np.array_equal(d["u"][a], u[a]), f"momentum axis {a}"
    # currents of this step: the GPU sums them in 64-bit fixed point (absolute
    # resolution ~1e-15 of the largest single contribution); same bar as fields
    J = g.fields(("Jx", "Jy", "Jz"))
    err = rel_errors(oracle_currents(o, g.NPJ), J)
    assert max(err.values()) < 1e-10, err


def test_lwfa2d_fp64_100_steps():
    cfg = workloads.lwfa2d_fp64()
    o = Simulation(cfg)
    g = Sim(cfg, track_ids=True, deposit_rho=True)
    for chunk in (1, 9, 40, 50):
        o.run(chunk - 1)
        o.step(diag=True)
        dg = g.step(chunk, diag=True)
        err = rel_errors(oracle_fields(o), g.fields())
        assert max(err.values()) < 1e-10, (o.k, err)
        _compare_particles_exact(o, g)
        assert dg["n_particles"] == len(o.P)
        assert dg["continuity_rel"] < 1e-12
        assert abs(dg["charge_grid"] - o.diag["charge_grid"]) < 1e-12 * abs(o.diag["charge_grid"])
        assert abs(dg["field_energy"] - o.diag["field_energy"]) < 1e-10 * o.diag["field_energy"]
    J = g.fields(("Jx", "Jy", "Jz"))
    err = rel_errors(oracle_currents(o, g.NPJ), J)
    assert max(err.values()) < 1e-10, err


@pytest.mark.parametrize("tile", [(8, 8, 8), (8, 8, 4)], ids=["t888", "t884"])
def test_small3d_fp64_steps(tile):
    cfg = _small3d(tile=tile)
    o = Simulation(cfg)
    g = Sim(cfg, track_ids=True, deposit_rho=True)
    o.run(3)
    o.step(diag=True)
    dg = g.step(4, diag=True)
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-10, err
    _compare_particles_exact(o, g)
    assert dg["continuity_rel"] < 1e-12
    J = g.fields(("Jx", "Jy", "Jz"))
    err = rel_errors(oracle_currents(o, g.NPJ), J)
    assert max(err.values()) < 1e-10, err


def test_lwfa2d_fp32_50_steps():
    cfg = workloads.lwfa2d_fp64()
    cfg["precision"] = "fp32"
    o = Simulation(workloads.lwfa2d_fp64()).run(50)
    g = Sim(cfg)
    g.step(50)
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 2e-4, err


@pytest.mark.parametrize("tile", [(8, 8, 8), (8, 8, 4)], ids=["t888", "t884"])
def test_small3d_fp32_steps(tile):
    o = Simulation(_small3d(tile=tile)).run(4)
    g = Sim(_small3d("fp32", tile=tile))
    g.step(4)
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 2e-4, err


def test_fp32_push_bit_exact_from_shared_state():
    """FP32 kernel against the oracle's push run in FP32 on the same inputs:
    the integer cell decision is taken in the kernel's precision on both sides."""
    cfg64 = _small3d()
    o = Simulation(cfg64).run(3)
    g = Sim(_small3d("fp32"), track_ids=True)
    cell, off, u, pid = oracle_particles(o)
    g.set_state(o.k, cell, off.astype(np.float32), u.astype(np.float32), None, ids=pid)
    F32 = o.F[:, :o.p.Nz].astype(np.float32)
    g.set_fields(F32)
    before = gpu_particles_to_oracle(o.p, g.particles(ids=True), np.float32)
    g.step(1)
    after = g.particles(ids=True)
    from oracle.push import push_and_move
    Fz = np.zeros((6, o.p.Nz + o.p.ext + 1, o.p.Ny, o.p.Nx), np.float32)
    Fz[:, :o.p.Nz] = F32
    push_and_move(o.p, before, Fz)
    keep = before.iz >= 0
    order = np.argsort(after["id"])
    pos = order[np.searchsorted(after["id"][order], before.pid[keep])]
    assert np.array_equal(after["id"][pos], before.pid[keep])
    cellp = (before.iz * o.p.Ny + before.iy) * o.p.Nx + before.ix
    assert np.array_equal(after["cell"][pos].astype(np.int64), cellp[keep])
    for a, arr in enumerate((before.dx, before.dy, before.dz)):
        assert np.array_equal(after["off"][a][pos], arr[keep]), a
    for a, arr in enumerate((before.ux, before.uy, before.uz)):
        assert np.array_equal(after["u"][a][pos], arr[keep]), a
