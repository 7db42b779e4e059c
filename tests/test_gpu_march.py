"""Parity of the HIP zeta march (the paper's slow step: particles integrated
along zeta, interleaved with the right-to-left node march; Sec. 5 eq:trap1 /
eq:trap2, Sec. 5.1, Sec. 4.1) with the FP64 oracle (oracle/march.py),
through the C ABI.

Bars (FP64): fields and the cells' currents within relative L2 1e-10; every
particle (matched by id) in the same cell, offsets and momenta within 1e-9,
weights within 1e-14 relative and budgets within 1e-9 of Delta; the same
numbers of particles parked and gone.  The GPU sums a cell's currents with
FP64 atomics in arrival order, so both sides agree to roundoff, not bit for
bit.  FP32 (cell + offset) against the FP64 oracle: every field component
within 2e-4 of its own norm or 30 units of 2^-24 of the largest component.
Cases: GT1 with particles parked in the box (Delta < L) and streaming through
it (Delta > L), GT2, 2-D, Ny = 256 (the node solve between the four-step y
transforms; other Ny take the fused per-column kernel), a quiet plasma at
rest (exactly zero current), and vacuum."""
import numpy as np
import pytest

import workloads
from oracle.march import MarchSim
from paper_2509_16793_amd.gempic import Sim
from parity import check_fp32_fields, rel_errors

pytestmark = pytest.mark.gpu

FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def _cfg3(delta, scheme=1, n=(16, 16, 64), prec="fp64", **kw):
    cfg = workloads.small3d(precision=prec, n=n, tile=(8, 8, 4))
    cfg.update(delta=delta, scheme=scheme)
    cfg.update(kw)
    return cfg


def _cfg2(delta, scheme=1, prec="fp64"):
    cfg = workloads.lwfa2d_fp64()
    cfg.update(n=[32, 1, 128], precision=prec, delta=delta, scheme=scheme)
    return cfg


def _oracle_fields(o):
    return {nm: o.F0[c, :o.p.Nz] for c, nm in enumerate(FIELDS)}


def _compare(o, g, field_bar=1e-10):
    p = o.p
    err = rel_errors(_oracle_fields(o), g.fields())
    assert max(err.values()) < field_bar, err
    if field_bar > 1e-9:
        return
    # currents of the last step: plane n + 2 holds cell n
    J = g.fields(("Jx", "Jy", "Jz"))
    ref = {k: o.J[c] for c, k in enumerate(("Jx", "Jy", "Jz"))}
    got = {k: J[k][2:2 + p.Nz] for k in ref}
    err = rel_errors(ref, got)
    assert max(err.values()) < 1e-10, err
    d = g.particles(ids=True)
    extra = g.march_particles()
    order = np.argsort(d["id"], kind="stable")
    P = o.P
    assert len(order) == len(P)
    if len(P) == 0:          # every particle left the box in this step
        return
    assert np.array_equal(d["id"][order], P.pid)
    cell = d["cell"][order].astype(np.int64)
    ix, iy, iz = cell % p.Nx, (cell // p.Nx) % p.Ny, cell // (p.Nx * p.Ny)
    assert np.array_equal(ix, P.ix) and np.array_equal(iy, P.iy) and np.array_equal(iz, P.iz)
    off, u = d["off"][:, order], d["u"][:, order]
    assert np.max(np.abs(off[0] - P.dx)) < 1e-9 and np.max(np.abs(off[2] - P.dz)) < 1e-9
    if p.dims == 3:
        assert np.max(np.abs(off[1] - P.dy)) < 1e-9
    for a, ref_u in enumerate((P.ux, P.uy, P.uz)):
        assert np.max(np.abs(u[a] - ref_u)) < 1e-9 * max(1.0, np.abs(ref_u).max())
    w, b = extra["w"][order], extra["b"][order]
    assert np.max(np.abs(w - P.w)) <= 1e-14 * np.abs(P.w).max()
    assert np.max(np.abs(b - P.b)) < 1e-9 * o.m.Delta


@pytest.mark.parametrize("cfg", [_cfg3(0.5), _cfg3(50.0), _cfg3(0.5, scheme=2), _cfg2(0.7),
                                 _cfg3(0.5, n=(16, 256, 32))],
                         ids=["gt1_parked", "gt1_through", "gt2", "gt1_2d", "gt1_ny256"])
def test_march_fp64_matches_oracle(cfg):
    o = MarchSim(cfg)
    g = Sim(cfg, track_ids=True)
    err = rel_errors(_oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-12, err
    for k in range(3):
        o.step()
        dg = g.step(1, diag=True)
        _compare(o, g)
        assert dg["n_particles"] == len(o.P)
        assert abs(dg["tau"] - o.s) < 1e-12 * o.s
        wsum = float(np.sum(o.P.w))
        assert abs(dg["charge_particles"] + wsum) <= 1e-12 * wsum


def test_march_quiet_plasma_at_rest_deposits_nothing():
    cfg = _cfg3(0.5, a0=0.0, load=1)
    g = Sim(cfg, track_ids=True)
    g.step(2)
    J = g.fields(("Jx", "Jy", "Jz"))
    for k in J:
        assert not np.any(J[k]), k
    F = g.fields()
    for k in F:
        assert not np.any(F[k]), k


def test_march_vacuum_matches_oracle():
    cfg = _cfg3(3.0, n_e=0.0)
    o = MarchSim(cfg).run(2)
    g = Sim(cfg)
    g.step(2)
    err = rel_errors(_oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-12, err


@pytest.mark.parametrize("cfg", [_cfg3(0.5, prec="fp32"), _cfg3(50.0, scheme=2, prec="fp32")],
                         ids=["gt1", "gt2"])
def test_march_fp32_fields_against_fp64_oracle(cfg):
    c64 = dict(cfg)
    c64["precision"] = "fp64"
    o = MarchSim(c64).run(4)
    g = Sim(cfg)
    g.step(4)
    check_fp32_fields(_oracle_fields(o), g.fields())


def test_march_nonuniform_grid_and_changing_delta():
    """Sec. 7: h varying smoothly along zeta (a tanh ramp by 2.5 between the
    rear and the front) and Delta changed between steps; FP64 bars as above."""
    from test_oracle_march_grid import _smooth_nodes
    cfg = _cfg3(0.5, zeta_nodes=list(_smooth_nodes(64, 64 * 0.05, 2.5)))
    o = MarchSim(cfg)
    g = Sim(cfg, track_ids=True)
    err = rel_errors(_oracle_fields(o), g.fields())
    assert max(err.values()) < 1e-12, err
    for D in (0.5, 0.3, 0.8):
        o.step(Delta=D)
        g.set_slow_step(D)
        dg = g.step(1, diag=True)
        _compare(o, g)
        assert dg["n_particles"] == len(o.P)
        assert abs(dg["tau"] - o.s) < 1e-12 * o.s
