"""Error paths, checkpoint/resume and dense tiles of the HIP library, through
its C ABI, against the FP64 oracle.

* A particle uploaded with a momentum that carries it over more than one cell
  in a step makes gempic_step return GEMPIC_ECFL; a non-finite momentum
  GEMPIC_ENUMERIC.  Both are flags the push kernel raises while it leaves the
  particle unchanged (every kernel exits normally); the handle then refuses
  further steps (GEMPIC_ESTATE) and still answers its getters.
* A run split into two handles (particles + spectral state read from the
  first, written into the second with gempic_set_state) continues like the
  uninterrupted run: ids exact, fields within 1e-12.
* Dense tiles (several 1024-particle chunks per tile: 8 and 16 ppc, and a
  driver bunch that puts more than ten chunks into one tile) keep the FP64
  bars: ids and cells exact, fields and J within 1e-10, continuity < 1e-12.
* FP32 cell + offset against the FP64 oracle on a 3-D case over 50 steps:
  fields within 2e-4 (independent evidence of the FP32 path)."""
import numpy as np
import pytest

import workloads
from oracle.sim import Simulation, tile_key
from paper_2509_16793_amd.gempic import GempicError, Sim
from parity import oracle_particles, rel_errors, oracle_fields, oracle_currents

pytestmark = pytest.mark.gpu

ECFL, ENUMERIC, ESTATE = -4, -5, -6


def _upload_modified(g, d, u):
    g.set_state(0, d["cell"], d["off"], u, g.spectral(), ids=d["id"])


def _thin_cells():
    # transverse cells narrower than the slow step: v_x dtau / h_x is up to
    # 0.025 / 0.005 = 5 cells, so a fast particle crosses several cells
    cfg = workloads.small3d(precision="fp64", n=(16, 16, 32), a0=0.0)
    cfg["d"] = [0.005, 0.4, 0.05]
    return cfg


def test_particle_crossing_more_than_one_cell_returns_ecfl():
    g = Sim(_thin_cells(), track_ids=True)
    d = g.particles(ids=True)
    u = d["u"].copy()
    u[0, 5] = 10.0
    _upload_modified(g, d, u)
    with pytest.raises(GempicError) as e:
        g.step(1)
    assert e.value.code == ECFL
    with pytest.raises(GempicError) as e:
        g.step(1)
    assert e.value.code == ESTATE
    # getters still answer; the offending particle was left as uploaded
    d2 = g.particles(ids=True)
    k = int(np.nonzero(d2["id"] == d["id"][5])[0][0])
    assert d2["u"][0, k] == 10.0 and d2["cell"][k] == d["cell"][5]


def test_non_finite_momentum_returns_enumeric():
    cfg = workloads.small3d(precision="fp64", n=(16, 16, 32))
    g = Sim(cfg, track_ids=True)
    d = g.particles(ids=True)
    u = d["u"].copy()
    u[2, 7] = np.nan
    _upload_modified(g, d, u)
    with pytest.raises(GempicError) as e:
        g.step(1)
    assert e.value.code == ENUMERIC
    with pytest.raises(GempicError) as e:
        g.step(1)
    assert e.value.code == ESTATE
    assert len(g.particles()["cell"]) > 0


def test_fp32_non_finite_momentum_returns_enumeric():
    cfg = workloads.small3d(precision="fp32", n=(16, 16, 32))
    g = Sim(cfg)
    d = g.particles()
    u = d["u"].copy()
    u[0, 3] = np.inf
    g.set_state(0, d["cell"], d["off"], u, g.spectral())
    with pytest.raises(GempicError) as e:
        g.step(1)
    assert e.value.code == ENUMERIC


def test_checkpoint_resume_reproduces_uninterrupted_run():
    # FP64: the global current flush sums in atomic order, so the two runs
    # differ by FP64 roundoff only (FP32 roundoff could move a particle that
    # sits on a cell face into the next cell and change the permutation)
    cfg = workloads.small3d(precision="fp64", n=(32, 32, 64))
    a = Sim(cfg, track_ids=True)
    a.step(5)
    d = a.particles(ids=True)
    sp = a.spectral()
    b = Sim(cfg, track_ids=True)
    b.set_state(5, d["cell"], d["off"], d["u"], sp, ids=d["id"])
    a.step(5)
    b.step(5)
    da, db = a.particles(ids=True), b.particles(ids=True)
    assert np.array_equal(da["id"], db["id"])
    assert np.array_equal(da["cell"], db["cell"])
    bar = 1e-12
    err = rel_errors(a.fields(), b.fields())
    assert max(err.values()) < bar, err
    assert np.max(np.abs(da["u"] - db["u"])) <= bar * max(1.0, np.abs(da["u"]).max())


def _fp64_parity(cfg, steps):
    o = Simulation(cfg)
    g = Sim(cfg, track_ids=True, deposit_rho=True)
    o.run(steps - 1)
    o.step(diag=True)
    dg = g.step(steps, diag=True)
    cell, off, u, pid = oracle_particles(o)
    d = g.particles(ids=True)
    assert np.array_equal(d["id"], pid), "sort permutation differs"
    assert np.array_equal(d["cell"].astype(np.int64), cell), "cells differ"
    assert np.max(np.abs(d["off"] - off)) < 1e-9
    assert np.max(np.abs(d["u"] - u)) < 1e-9 * max(1.0, np.abs(u).max())
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-10, err
    err = rel_errors(oracle_currents(o, g.NPJ), g.fields(("Jx", "Jy", "Jz")))
    assert max(err.values()) < 1e-10, err
    assert dg["continuity_rel"] < 1e-12
    return o


@pytest.mark.parametrize("ppc", [(2, 2, 2), (2, 2, 4)], ids=["8ppc", "16ppc"])
def test_dense_tiles_fp64(ppc):
    cfg = workloads.small3d(precision="fp64", n=(16, 16, 64), tile=(8, 8, 4), ppc=ppc)
    o = _fp64_parity(cfg, 3)
    counts = np.bincount(tile_key(o.p, o.P))
    assert counts.max() >= 2 * 1024     # several chunks per tile


def test_dense_driver_tile_fp64():
    cfg = workloads.pwfa_small(tile=(8, 8, 4), np_beam=160_000, n=(32, 32, 64))
    o = _fp64_parity(cfg, 2)
    counts = np.bincount(tile_key(o.p, o.P))
    assert counts.max() >= 10 * 1024    # more than ten chunks in one tile


def test_fp32_3d_fields_over_50_steps():
    cfg64 = workloads.small3d(precision="fp64", n=(16, 16, 64), steps=50)
    o = Simulation(cfg64).run(50)
    g = Sim(workloads.small3d(precision="fp32", n=(16, 16, 64), steps=50))
    g.step(50)
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 2e-4, err
