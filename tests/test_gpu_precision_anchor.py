"""The precision study's reference (the library's FP64 mode at 8 ppc, the
physics of workloads.precision_study) anchored to the CPU oracle on a
16 x 16 x 512 transverse crop of the same physics (laser waist scaled to the
crop, 1,055,744 electrons), through the C ABI:

* FP64, 3 steps: cells and the sort permutation bit for bit, fields and
  currents within relative L2 1e-10, continuity below 1e-12;
* FP32 cell + offset, 3 steps: every field component within 2e-4 of its own
  norm or 30 units of 2^-24 of the largest component.

The oracle would need 62 GB and 129 s per step on a 64 x 64 crop, so the
crop is 16 x 16 cells across (8 ppc in all 512 planes)."""
import pytest

import workloads
from oracle.sim import Simulation
from paper_2509_16793_amd.gempic import Sim
from parity import check_fp32_fields, oracle_currents, oracle_fields, oracle_particles, rel_errors

pytestmark = pytest.mark.gpu


def _crop(precision):
    cfg = workloads.precision_study(precision)
    cfg["n"] = [16, 16, 512]
    cfg["waist"] = 2.0 * 16 / 32
    return cfg


def test_precision_study_reference_matches_oracle_on_a_crop():
    import numpy as np
    o = Simulation(_crop("fp64"))
    o.run(2)
    o.step(diag=True)
    g = Sim(_crop("fp64"), track_ids=True)
    dg = g.step(3, diag=True)
    err = rel_errors(oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-10, err
    cell, _, _, pid = oracle_particles(o)
    d = g.particles(ids=True)
    assert np.array_equal(d["id"], pid)
    assert np.array_equal(d["cell"].astype(np.int64), cell)
    assert dg["continuity_rel"] < 1e-12
    err = rel_errors(oracle_currents(o, g.NPJ), g.fields(("Jx", "Jy", "Jz")))
    assert max(err.values()) < 1e-10, err
    g.close()
    g32 = Sim(_crop("fp32"))
    g32.step(3)
    check_fp32_fields(oracle_fields(o), g32.fields())
    g32.close()
