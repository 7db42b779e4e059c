"""The oracle's full step on the 2-D LWFA workload (64 x 256, 2 ppc): discrete
continuity of every step's deposit to roundoff, grid charge equal to particle
charge, and a deterministic particle order (stable tile sort)."""
import numpy as np

import workloads
from oracle.sim import Simulation, tile_key


def test_lwfa2d_steps_conserve_charge():
    s = Simulation(workloads.lwfa2d_fp64())
    for _ in range(6):
        s.step(diag=True)
        d = s.diag
        assert d["continuity_rel"] < 1e-12
        assert abs(d["charge_grid"] - d["charge_particles"]) < 1e-12 * abs(d["charge_particles"])
    key = tile_key(s.p, s.P)
    assert np.all(np.diff(key) >= 0)
    # laser is there and the wake starts
    assert 0.5 < np.abs(s.F[0]).max() < 1.5
    assert np.abs(s.diag["ez_axis"]).max() > 1e-3


def test_deterministic():
    a = Simulation(workloads.lwfa2d_fp64()).run(3)
    b = Simulation(workloads.lwfa2d_fp64()).run(3)
    assert np.array_equal(a.P.pid, b.P.pid)
    assert np.array_equal(a.F, b.F)
