"""One Galilean PIC step in order, the stable tile sort and FP64 diagnostics
(oracle side).

Step k -> k+1 (tau^k = k dtau):
  1. gather the level-k node fields, Higuera-Cary push u^{k-1/2} -> u^{k+1/2},
     move r^k -> r^{k+1} along d zeta / d tau = v_z - 1      (push.py)
  2. deposit J^{k+1/2} (Esirkepov frame current + rhobar)    (deposit.py)
  3. drop particles that left at zeta < 0; append window batch k + 1
  4. stable sort by tile key
  5. binomial filter of J, transverse FFT, right-to-left march of the node
     system with slow step Delta = dtau, inverse FFT         (fields.py)

Tile key (reading; the paper keeps no particle order): tiles of
T_x x T_y x T_zeta cells, key = (t_zeta * nT_y + t_y) * nT_x + t_x, sorted
stably so particles of one tile keep their previous relative order; removed
particles are dropped, new ones enter after all existing ones.
"""
import numpy as np

from . import params as _params
from .plasma import Particles, load_beam, load_full_cells, inject_batch
from .push import push_and_move
from .deposit import G, deposit, deposit_rho, continuity_residual
from .fields import (laser_state, real_fields, march, half_node_currents,
                     binomial_filter)


def tile_key(p, P):
    nTx, nTy, _ = p.ntiles
    tx = P.ix // p.tile[0]
    ty = P.iy // p.tile[1]
    tz = P.iz // p.tile[2]
    return (tz * nTy + ty) * nTx + tx


def stable_sort(p, P):
    order = np.argsort(tile_key(p, P), kind="stable")
    return P.take(order)


class Simulation:
    def __init__(self, cfg):
        p = _params.from_config(cfg)
        self.p = p
        self.k = 0
        # initial order before the tile sort: plasma load, driver beam, window
        # batch 0
        B = load_beam(p)
        P = Particles.concat(Particles.concat(load_full_cells(p), B), inject_batch(p, 0))
        P.pid = np.arange(len(P), dtype=np.int64)
        self.next_pid = len(P)
        self.P = stable_sort(p, P)
        rho_b = None
        if len(B):
            r = deposit_rho(p, B.ix, B.iy, B.iz, B.dx, B.dy, B.dz, B.weight_ratio(p))
            rho_b = r[G:G + p.Nz]
        self.state = laser_state(p, rho_b)
        self.F = real_fields(p, self.state)
        self.J = None
        self.diag = None
        # optional replacement of the binomial filter: f(sim, (Jx, Jy, Jz)) ->
        # the three currents handed to the field solver
        self.current_filter = None

    @property
    def tau(self):
        return self.k * self.p.dtau

    def step(self, diag=False):
        p = self.p
        P = self.P
        wr = P.weight_ratio(p) if p.beam is not None else None
        if diag:
            rho0 = deposit_rho(p, P.ix, P.iy, P.iz, P.dx, P.dy, P.dz, wr)
        n_pushed = len(P) if wr is None else float(np.sum(wr))
        old, steps, vy = push_and_move(p, P, self.F)
        new = (P.ix, P.iy, P.iz, P.dx, P.dy, P.dz)
        Jx, Jy, Jz = deposit(p, old, new, steps, vy, wr)
        if diag:
            rho1 = deposit_rho(p, P.ix, P.iy, P.iz, P.dx, P.dy, P.dz, wr)
        P = P.take(P.iz >= 0)
        B = inject_batch(p, self.k + 1)
        B.pid = self.next_pid + np.arange(len(B), dtype=np.int64)
        self.next_pid += len(B)
        P = Particles.concat(P, B)
        self.P = stable_sort(p, P)
        self.J = (Jx, Jy, Jz)
        if self.current_filter is not None:
            fJ = list(self.current_filter(self, (Jx, Jy, Jz)))
        else:
            fJ = [Jx, Jy, Jz]
            for _ in range(p.filter_passes):
                fJ = [binomial_filter(p, a) for a in fJ]
        self.Jf = tuple(fJ)
        jh = half_node_currents(p, *fJ)
        self.state = march(p, self.state, jh, p.dtau)
        self.F = real_fields(p, self.state)
        self.k += 1
        if diag:
            self.diag = self.diagnostics(rho0, rho1, n_pushed)
        return self

    def run(self, n, diag=False):
        for _ in range(n):
            self.step(diag=diag)
        return self

    def diagnostics(self, rho0=None, rho1=None, n_pushed=None):
        """FP64 diagnostics of the last step: particle count after the step;
        charge of the pushed particles (q w N) and on the grid after the move
        (sum rho V, all particles before removal; beam particles count with
        their weight); field energy
        1/2 sum (E^2 + B^2) V over the field nodes; continuity residual of
        the raw deposit; on-axis E_z."""
        p = self.p
        V = p.hx * p.hy_eff * p.h
        P = self.P
        F = self.F[:, :p.Nz]
        d = dict(tau=self.tau, step=self.k, n_particles=len(P),
                 field_energy=float(0.5 * np.sum(F * F) * V),
                 ez_axis=self.F[2, :p.Nz, p.Ny // 2, p.Nx // 2].copy())
        if rho1 is not None:
            d["charge_particles"] = p.q * p.w * n_pushed
            d["charge_grid"] = float(np.sum(rho1) * V)
        if rho0 is not None:
            r = continuity_residual(p, rho0, rho1, *self.J)
            s = (rho1 - rho0) / p.dtau
            ns = float(np.sqrt(np.sum(s * s)))
            d["continuity_abs"] = float(np.sqrt(np.sum(r * r)))
            d["continuity_rel"] = d["continuity_abs"] / ns if ns > 0 else 0.0
        return d
