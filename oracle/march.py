"""The paper's own slow step (oracle side, test infrastructure only): the
particles are integrated along the fast coordinate zeta, interleaved with the
right-to-left march of the field solver, so that the slow step Delta may be
much larger than the fast step h.

Paper:
  * Sec. 5: characteristics of the transformed Vlasov equation parametrised
    by zeta, d s / d zeta = 1 / (v_z - 1), d r_perp / d zeta = v_perp /
    (v_z - 1), d p / d zeta = F / (v_z - 1); a particle is pushed until its
    slow coordinate reaches s^1 = s^0 + Delta (stop rule eq:trap1) or it
    leaves the box at the left; the zeta sub-step is the smaller of h and
    Delta (1 - v_z).  GT2 (eq:Vlasov2, eq:trap2): d s~ / d zeta =
    v_z / (v_z - 1), sub-step bound Delta (1 - v_z) / v_z.
  * Sec. 5.1: a fresh macro-particle, swept over by the domain in one slow
    step, carries Q_f = q n h_x h_y Delta; a macro-particle deposits
    j = (Q / (h_x h_y h)) v ds / Delta, ds the time it spends in the cell.
  * Sec. 4.1: node scheme RxN .. eqall, node n solved at the new level once
    node n + 1 is known; j^1 on the half-node below the node is predicted.
  * Sec. 7: Delta may change from step to step; h may vary (smoothly) along
    zeta.

Readings (where the paper is silent; the HIP path takes the same ones):
  M1  Integrator: the explicit midpoint rule.  A sub-step that reaches the
      node below the particle's cell is parametrised by zeta (it ends on the
      node exactly); a sub-step limited by the remaining slow budget, or by
      the transverse limit M4, is parametrised by lab time (= s in GT1).
  M2  Fields inside cell n (between nodes n and n + 1): linear in zeta
      between node n + 1 and node n at the new level, linear (cloud-in-cell)
      in x and y.  Node n at the new level depends on the currents of cell n,
      so each stage is a predictor-corrector pair (Sec. 4.1 names a
      predictor-corrector procedure): the predictor pushes the cell's
      particles with node n at the old level, deposits and solves node n;
      the corrector pushes them again, from their state at the start of the
      stage, with the predicted node n, deposits and solves node n again.
      Only the corrector's particles and currents are kept.
  M3  Predictor: j^1 on half-node n - 1/2 (needed by RxN, RyN at node n) is
      the previous step's j^0 there plus the change that half-node n + 1/2
      has just seen, j^1_{-1/2} = j^0_{-1/2} + (j^1_{+1/2} - j^0_{+1/2}).
      The four-term sum of the R rows is then 2 (j^1_{+1/2} + j^0_{-1/2}),
      centred on node n and on the middle of the slow step, and the R update
      keeps the amplitude of a mode whose current turns its phase (the
      laser in the plasma).  Taking j^0_{-1/2} alone would weigh the old
      level three to one, which multiplies the laser's amplitude by about
      1 + theta^2 / 4 per step, theta = Delta omega_p^2 / (2 omega): a few
      percent per step once Delta is several laser periods.
      j^0 of the level of creation.  In GT2 a particle at rest streams
      through the whole box at fixed s~, so the plasma's level-s0 current is
      its response to the initial fields: a startup march at creation pushes
      one fresh batch through them, with node solves of zero slow step (R
      unchanged, L, E_z and B_z taking the plasma's response), keeps its
      currents as j^0 and its fields as the initial ones, and discards the
      particles.  GT1 has no such level-s0 current (its plasma in the box
      is parked, and it takes up the laser's quiver within one laser
      period, not one slow step): its first step uses the current j^1 of
      half-node n + 1/2 for both levels and the predictor, which makes that
      step implicit in the current and damps the laser once by about
      1 / sqrt(1 + theta^2).
  M4  A sub-step moves at most half a transverse cell: its time is at most
      min(h_x, h_y) / 2.
  M5  Current of a sub-step inside cell n, charged to half-node n + 1/2:
      transverse components by Esirkepov's decomposition of the transverse
      move (cloud-in-cell in x, y), J_z = Q (d zeta + ds) / (V Delta) times the
      time-averaged transverse shape, i.e. Q v_z ds / (V Delta) (Sec. 5.1).
      Every current of cell n is complete before node n is solved, which the
      march needs; a 1-2-1 filter along zeta would need the half-node below,
      so only the transverse filter factor cos^2(k h / 2) per pass is used.
  M6  Fresh plasma: one batch per step, ppc_x x ppc_y particles per
      transverse cell at the right edge zeta = zeta_Nz (stratified offsets
      from SplitMix64, or cell centres), u = 0, budget Delta.  GT1 with
      Delta < L also loads, at creation, batches m = 1, 2, ... at
      zeta_Nz - m Delta (the plasma already in the box); GT2 needs none
      (a particle at rest streams through the whole box in one step).
  M7  Cells along zeta are half-open from below: cell n holds
      zeta_n < zeta <= zeta_{n+1}, offset (zeta - zeta_n) / h_n in (0, 1];
      a particle that reaches node 0 leaves.
  M8  A sub-step that is budget- or transverse-limited but would end below
      the node ends on the node.
  M9  Macro-particle weights are numbers of electrons, w = n(r_perp) h_x h_y
      Delta / (ppc_x ppc_y), with the Gaussian channel of Sec. 6
      (eq. n_plasma) n(r_perp) = n_e [1 + (ratio - 1) exp(-r_perp^2 / R^2)]
      sampled at the particle's transverse position when it is created.
"""
import math

import numpy as np

from . import params as _params
from . import rng
from .deposit import _window
from .fields import SpectralState, wavenumbers, node_matrix, fft2, ifft2_real

STREAM = 2       # SplitMix64 stream of the zeta-marching plasma
ROW0 = 1 << 20   # offset of the batch index in the generator's counter


class MarchParams:
    """Normalised parameters of a zeta-march run (units as params.py)."""

    def __init__(self, cfg):
        c = dict(cfg)
        c["dtau"] = 0.0
        self.p = p = _params.from_config(c)
        lu = float(cfg.get("length_unit", 1.0))
        self.scheme = int(cfg.get("scheme", 1))          # 1 = GT1, 2 = GT2
        if self.scheme not in (1, 2):
            raise _params.ConfigError("scheme must be 1 (GT1) or 2 (GT2)")
        zn = cfg.get("zeta_nodes")
        if zn is None:
            self.zn = np.arange(p.Nz + 1) * p.h
        else:
            self.zn = np.asarray(zn, float) * lu
            if self.zn.shape != (p.Nz + 1,) or self.zn[0] != 0.0 or np.any(np.diff(self.zn) <= 0):
                raise _params.ConfigError("zeta_nodes: Nz + 1 increasing values from 0")
        self.hz = np.diff(self.zn)
        self.Delta = float(cfg["delta"]) * lu
        self.ratio = float(cfg.get("ch_ratio", 1.0))
        self.R = float(cfg.get("ch_radius", 0.0)) * lu
        self.check_delta(self.Delta)

    def check_delta(self, D):
        if not D > 0:
            raise _params.ConfigError("Delta must be > 0")
        p = self.p
        # Sec. 4.2 stability estimate with the largest fast step
        if p.n_e > 0 and D * np.max(self.hz) > 4.0 / p.n_e:
            raise _params.ConfigError("slow step violates Delta*h <= 4/omega_p^2")

    @property
    def L(self):
        return self.zn[-1]

    def density(self, X, Y):
        """Electron density at transverse positions (normalised lengths from
        the grid origin), Gaussian channel about the axis (Nx/2, Ny/2)."""
        p = self.p
        if self.ratio == 1.0 or self.R <= 0.0:
            return np.full(np.shape(X), p.n_e)
        x = X - (p.Nx // 2) * p.hx
        y = (Y - (p.Ny // 2) * p.hy) if p.dims == 3 else 0.0 * X
        return p.n_e * (1.0 + (self.ratio - 1.0) * np.exp(-(x * x + y * y) / (self.R * self.R)))


class MP:
    """Zeta-march macro-particles: transverse cell + offset in [0, 1), zeta
    cell n + offset in (0, 1] (M7), momentum u, weight w (electrons), the
    remaining slow budget b of the current step, id."""
    FIELDS = ("ix", "iy", "dx", "dy", "iz", "dz", "ux", "uy", "uz", "w", "b", "pid")

    def __init__(self, **a):
        for k in self.FIELDS:
            setattr(self, k, np.asarray(a[k]))

    def __len__(self):
        return len(self.ix)

    def take(self, idx):
        return MP(**{k: getattr(self, k)[idx] for k in self.FIELDS})

    @staticmethod
    def concat(*parts):
        return MP(**{k: np.concatenate([getattr(a, k) for a in parts]) for k in MP.FIELDS})

    @staticmethod
    def empty():
        i, f = np.zeros(0, np.int64), np.zeros(0)
        return MP(ix=i, iy=i, dx=f, dy=f, iz=i, dz=f, ux=f, uy=f, uz=f, w=f, b=f, pid=i)


def batch(m, row, zeta, u0=(0.0, 0.0, 0.0)):
    """ppc_x x ppc_y particles per transverse cell at zeta, generator row
    `row` (fresh batch of step k: row k; initial batch m >= 1: row -m)."""
    p = m.p
    ppx, ppy = p.ppc[0], p.ppc[1]
    j, i, sy, sx = np.meshgrid(np.arange(p.Ny), np.arange(p.Nx), np.arange(ppy), np.arange(ppx),
                               indexing="ij")
    j, i, sy, sx = (a.ravel() for a in (j, i, sy, sx))
    if p.load == 1:
        xi_x = np.full(i.shape, 0.5)
        xi_y = np.full(i.shape, 0.5)
    else:
        key = rng.stream_key(p.seed, STREAM)
        c = ((((np.uint64(row + ROW0) * np.uint64(p.Ny) + j.astype(np.uint64)) * np.uint64(p.Nx)
               + i.astype(np.uint64)) * np.uint64(ppy) + sy.astype(np.uint64)) * np.uint64(ppx)
             + sx.astype(np.uint64)) * np.uint64(2)
        xi_x = rng.uniform(key, c)
        xi_y = rng.uniform(key, c + np.uint64(1)) if p.dims == 3 else np.zeros(i.shape)
    dx = (sx + xi_x) / ppx
    dy = (sy + xi_y) / ppy if p.dims == 3 else np.zeros(i.shape)
    n = len(i)
    iz, dz = zeta_cell(m, np.full(n, zeta))
    w = m.density((i + dx) * p.hx, (j + dy) * p.hy) * p.hx * p.hy_eff * m.Delta / (ppx * ppy)
    return MP(ix=i, iy=j if p.dims == 3 else np.zeros(n, np.int64), dx=dx, dy=dy, iz=iz, dz=dz,
              ux=np.full(n, float(u0[0])), uy=np.full(n, float(u0[1])), uz=np.full(n, float(u0[2])),
              w=w, b=np.full(n, m.Delta), pid=np.zeros(n, np.int64))


def zeta_cell(m, zeta):
    """Cell n with zn[n] < zeta <= zn[n + 1] and the offset in (0, 1] (M7)."""
    n = np.searchsorted(m.zn, zeta, side="left") - 1
    n = np.clip(n, 0, len(m.hz) - 1)
    return n, (zeta - m.zn[n]) / m.hz[n]


def velocity(ux, uy, uz):
    """gamma, v_x, v_y, v_z and 1 - v_z (cancellation-free for u_z >= 0)."""
    up2 = ux * ux + uy * uy
    g = np.sqrt(1.0 + up2 + uz * uz)
    omv = np.where(uz >= 0.0, (1.0 + up2) / (g * (g + uz)), 1.0 - uz / g)
    return g, ux / g, uy / g, uz / g, omv


def transverse_advance(i, d, shift, N):
    """Offset d plus a shift in cells -> (cell, offset in [0, 1)), periodic."""
    t = d + shift
    k = np.floor(t)
    t = t - k
    up = t >= 1.0
    t = np.where(up, 0.0, t)
    k = k + up
    return (i + k.astype(np.int64)) % N, t, k.astype(np.int64)


def gather(m, F0, F1, n, ix, iy, dx, dy, t):
    """E and B (each (3, N)) at transverse (ix + dx, iy + dy) and fraction t
    of cell n: linear between node n of F0 and node n + 1 of F1 (M2),
    cloud-in-cell across."""
    p = m.p
    out = np.zeros((6, len(ix)))
    xs = (ix, (ix + 1) % p.Nx)
    wx = (1.0 - dx, dx)
    if p.dims == 3:
        ys = (iy, (iy + 1) % p.Ny)
        wy = (1.0 - dy, dy)
    else:
        ys, wy = (iy,), (np.ones(len(ix)),)
    for b in range(len(ys)):
        for a in range(2):
            w = wx[a] * wy[b]
            for c in range(6):
                out[c] += w * ((1.0 - t) * F0[c, n][ys[b], xs[a]] + t * F1[c, n + 1][ys[b], xs[a]])
    return out[0:3], out[3:6]


def force(E, B, vx, vy, vz, q):
    return (q * (E[0] + vy * B[2] - vz * B[1]),
            q * (E[1] + vz * B[0] - vx * B[2]),
            q * (E[2] + vx * B[1] - vy * B[0]))


class Deposit:
    """Currents of one cell (half-node n + 1/2) and the node fluxes used by
    the continuity pin."""

    def __init__(self, m):
        p = m.p
        self.Jx = np.zeros((p.Ny, p.Nx))
        self.Jy = np.zeros((p.Ny, p.Nx))
        self.Jz = np.zeros((p.Ny, p.Nx))


def deposit(m, dep, n, Qw, ix0, iy0, dx0, dy0, kx, ky, dx1, dy1, dzeta, ds, dy_len):
    """Currents of sub-steps inside cell n (M5): Qw = q w per particle,
    (ix0, iy0, dx0, dy0) -> (dx1, dy1) with cell steps (kx, ky), zeta move
    dzeta, time ds; dy_len = y displacement (2-D out-of-plane current)."""
    p = m.p
    D = m.Delta
    hn = m.hz[n]
    V = p.hx * p.hy_eff * hn
    bx, S0x, S1x = _window(ix0, kx, dx0, dx1)
    DSx = S1x - S0x
    tz = Qw * (dzeta + ds) / (D * V)
    if p.dims == 3:
        by, S0y, S1y = _window(iy0, ky, dy0, dy1)
        DSy = S1y - S0y
        cx = -Qw / (D * p.hy * hn)
        cy = -Qw / (D * p.hx * hn)
        for b in range(3):
            acc = 0.0
            for a in range(2):
                acc = acc + DSx[a] * (S0y[b] + 0.5 * DSy[b])
                np.add.at(dep.Jx, ((by + b) % p.Ny, (bx + a) % p.Nx), cx * acc)
        for a in range(3):
            acc = 0.0
            for b in range(2):
                acc = acc + DSy[b] * (S0x[a] + 0.5 * DSx[a])
                np.add.at(dep.Jy, ((by + b) % p.Ny, (bx + a) % p.Nx), cy * acc)
        for a in range(3):
            for b in range(3):
                T = S0x[a] * S0y[b] + 0.5 * (DSx[a] * S0y[b] + S0x[a] * DSy[b]) + DSx[a] * DSy[b] / 3.0
                np.add.at(dep.Jz, ((by + b) % p.Ny, (bx + a) % p.Nx), tz * T)
    else:
        cx = -Qw / (D * hn)
        z0 = np.zeros_like(ix0)
        acc = 0.0
        for a in range(2):
            acc = acc + DSx[a]
            np.add.at(dep.Jx, (z0, (bx + a) % p.Nx), cx * acc)
        ty = Qw * dy_len / (D * V)
        for a in range(3):
            T = S0x[a] + 0.5 * DSx[a]
            np.add.at(dep.Jy, (z0, (bx + a) % p.Nx), ty * T)
            np.add.at(dep.Jz, (z0, (bx + a) % p.Nx), tz * T)


class MarchSim:
    """Zeta-march slow steps.  ``solver=False`` keeps the fields F0 fixed
    (prescribed fields for particle pins); ``record=True`` keeps, per step,
    the cell currents and the node fluxes of the continuity pin."""

    def __init__(self, cfg, solver=True, record=False):
        self.m = m = MarchParams(cfg)
        self.lu = float(cfg.get("length_unit", 1.0))
        p = m.p
        self.solver = solver
        self.record = record
        self.k = 0
        self.s = 0.0
        self.state = init_state(m)
        self.F0 = real_fields(m, self.state)
        self.j0 = None
        parts = []
        if p.n_e > 0 and m.scheme == 1:
            mm = 1
            while m.L - mm * m.Delta > 0.0:
                parts.append(batch(m, -mm, m.L - mm * m.Delta))
                mm += 1
        self.P = MP.concat(*parts) if parts else MP.empty()
        self.P.pid = np.arange(len(self.P), dtype=np.int64)
        self.P.b = np.zeros(len(self.P))     # every step adds its Delta to the budget
        self.next_pid = len(self.P)
        self.inject_u0 = (0.0, 0.0, 0.0)     # fresh-batch momentum (pins only)
        self.diag = None
        self.left = MP.empty()
        self.trace = None                    # list: (n, particles on node n) per stage (pins)
        if self.solver and p.n_e > 0 and m.scheme == 2:
            self.step(startup=True)

    # ---- particle sub-steps inside cell n --------------------------------
    def _stage_particles(self, n, A, F1, dep, flux, Flow=None):
        """Push the particles A of cell n (M1 .. M8); returns (those that
        reached node n with budget left, those that stopped or left)."""
        m, p = self.m, self.p
        Flow = self.F0 if Flow is None else Flow    # node n (M2)
        q = p.q
        hn = m.hz[n]
        ds_perp = 0.5 * (min(p.hx, p.hy) if p.dims == 3 else p.hx)
        done_active, done_stop, done_left = [], [], []
        W = A
        while len(W):
            g, vx, vy, vz, omv = velocity(W.ux, W.uy, W.uz)
            dist = W.dz * hn
            ds_node = dist / omv
            rate = vz if m.scheme == 2 else np.ones(len(W))   # budget used per unit time
            # time the remaining budget allows (GT2: only when moving forward)
            with np.errstate(divide="ignore", invalid="ignore"):
                t_budget = np.where(rate > 0.0, W.b / np.where(rate > 0.0, rate, 1.0), np.inf)
            zstep = ds_node <= np.minimum(t_budget, ds_perp)
            dt = np.where(zstep, 0.0, np.minimum(t_budget, ds_perp))
            # a sub-step limited by the budget ends the particle's step (its
            # small rest, GT2: of either sign, is carried to the next step)
            blim = ~zstep & (t_budget <= ds_perp)
            # midpoint
            E, B = gather(m, Flow, F1, n, W.ix, W.iy, W.dx, W.dy, W.dz)
            Fx, Fy, Fz = force(E, B, vx, vy, vz, q)
            h1 = np.where(zstep, 0.5 * dist / omv, 0.5 * dt)
            uxm, uym, uzm = W.ux + h1 * Fx, W.uy + h1 * Fy, W.uz + h1 * Fz
            ixm, dxm, _ = transverse_advance(W.ix, W.dx, h1 * vx / p.hx, p.Nx)
            if p.dims == 3:
                iym, dym, _ = transverse_advance(W.iy, W.dy, h1 * vy / p.hy, p.Ny)
            else:
                iym, dym = W.iy, W.dy
            tm = np.where(zstep, 0.5 * W.dz, np.clip(W.dz - h1 * omv / hn, 0.0, 1.0))
            gm, vxm, vym, vzm, omvm = velocity(uxm, uym, uzm)
            Em, Bm = gather(m, Flow, F1, n, ixm, iym, dxm, dym, tm)
            Fxm, Fym, Fzm = force(Em, Bm, vxm, vym, vzm, q)
            ds = np.where(zstep, dist / omvm, dt)
            ux1, uy1, uz1 = W.ux + ds * Fxm, W.uy + ds * Fym, W.uz + ds * Fzm
            ix1, dx1, kx = transverse_advance(W.ix, W.dx, ds * vxm / p.hx, p.Nx)
            if p.dims == 3:
                iy1, dy1, ky = transverse_advance(W.iy, W.dy, ds * vym / p.hy, p.Ny)
            else:
                iy1, dy1, ky = W.iy, W.dy, np.zeros(len(W), np.int64)
            dz1 = np.where(zstep, 0.0, W.dz - ds * omvm / hn)
            reached = dz1 <= 0.0                      # M8: end on the node
            dz1 = np.where(reached, 0.0, dz1)
            dzeta = (dz1 - W.dz) * hn
            if np.any(np.abs(kx) > 1) or np.any(np.abs(ky) > 1):
                raise FloatingPointError("a sub-step crossed more than one transverse cell")
            Qw = q * W.w
            deposit(m, dep, n, Qw, W.ix, W.iy, W.dx, W.dy, kx, ky, dx1, dy1, dzeta, ds, ds * vym)
            used = ds * (vzm if m.scheme == 2 else 1.0)
            b1 = W.b - used
            if flux is not None and np.any(reached):
                r = reached
                wxs = (1.0 - dx1[r], dx1[r])
                ci = ((Qw[r] / (m.Delta * p.hx * p.hy_eff)))
                if p.dims == 3:
                    wys = (1.0 - dy1[r], dy1[r])
                    for b in range(2):
                        for a in range(2):
                            np.add.at(flux[n], ((iy1[r] + b) % p.Ny, (ix1[r] + a) % p.Nx), ci * wxs[a] * wys[b])
                else:
                    for a in range(2):
                        np.add.at(flux[n], (np.zeros(int(r.sum()), np.int64), (ix1[r] + a) % p.Nx), ci * wxs[a])
            W = MP(ix=ix1, iy=iy1, dx=dx1, dy=dy1, iz=W.iz, dz=dz1, ux=ux1, uy=uy1, uz=uz1, w=W.w,
                   b=b1, pid=W.pid)
            out = (b1 <= 0.0) | blim
            # reached the node: next cell with offset 1, or leave at node 0
            r_left = reached & (n == 0)
            r_go = reached & (n > 0)
            if np.any(r_go):
                W.iz = np.where(r_go, n - 1, W.iz)
                W.dz = np.where(r_go, 1.0, W.dz)
            done_left.append(W.take(r_left))
            done_active.append(W.take(r_go & ~out))
            done_stop.append(W.take((r_go & out) | (~reached & out)))
            W = W.take(~reached & ~out)
        return (MP.concat(*done_active) if done_active else MP.empty(),
                MP.concat(*done_stop) if done_stop else MP.empty(),
                MP.concat(*done_left) if done_left else MP.empty())

    @property
    def p(self):
        return self.m.p

    # ---- one slow step --------------------------------------------------
    def step(self, Delta=None, diag=False, startup=False):
        """One slow step; ``startup``: the GT2 startup march of M3 (nothing
        advances but the fields of the level of creation and j^0)."""
        m, p = self.m, self.p
        if Delta is not None:
            D = float(Delta) * self.lu
            m.check_delta(D)
            m.Delta = D
        D = m.Delta
        Dn = 0.0 if startup else D           # slow step of the node solves
        pid0 = self.next_pid
        if startup:
            diag = False
            assert len(self.P) == 0 and m.scheme == 2
        # budgets of the particles in the box: the new step's Delta plus the
        # carried (non-positive) rest of the last one
        P = self.P
        P.b = P.b + D
        if p.n_e > 0:
            Fb = batch(m, self.k, m.L, self.inject_u0)
            Fb.pid = self.next_pid + np.arange(len(Fb), dtype=np.int64)
            self.next_pid += len(Fb)
            P = MP.concat(P, Fb)
        rho0 = cell_charge(m, P) if (diag or self.record) else None
        flux = np.zeros((p.Nz + 1, p.Ny, p.Nx)) if (diag or self.record) else None
        Jrec = np.zeros((3, p.Nz, p.Ny, p.Nx))
        KX, KY, nyq = wavenumbers(p)
        F1 = np.zeros_like(self.F0)
        new = SpectralState(p)
        jst = np.zeros((2, p.Nz + 1, p.Ny, p.Nx), complex)   # j^1 of this step (x, y)
        first = self.j0 is None
        active = MP.empty()
        stopped = []
        left = []
        right = [np.zeros((p.Ny, p.Nx), complex) for _ in range(6)]
        def node_currents(n, jp1):
            """(j0 of n - 1/2, predicted j1 of n - 1/2 (M3), j0 of n + 1/2)
            for the R rows of node n, given j1 of n + 1/2."""
            if first:
                return jp1[:2], jp1[:2], jp1[:2]
            jm0 = (self.j0[0][n], self.j0[1][n])
            jp0 = (self.j0[0][n + 1], self.j0[1][n + 1])
            jm1 = tuple(jm0[c] + (jp1[c] - jp0[c]) for c in range(2))
            return jm0, jm1, jp0

        for n in range(p.Nz - 1, -1, -1):
            A = MP.concat(active, P.take(P.iz == n))
            dep = Deposit(m)
            Flow = None
            if self.solver and len(A):
                # predictor (M2): node n at the old level, then node n solved
                # with the currents of that push
                dp = Deposit(m)
                self._stage_particles(n, A, F1, dp, None)
                jq = solver_currents(m, dp.Jx, dp.Jy, dp.Jz, KX, KY, nyq)
                qm0, qm1, qp0 = node_currents(n, jq)
                old = [getattr(self.state, nm)[n] for nm in ("Rx", "Ry", "Ez", "Bz")]
                pred = solve_node(m, n, Dn, old, right, qm0, qm1, qp0, jq, KX, KY, nyq)
                Flow = self.F0.copy()
                Flow[:, n] = node_real_fields(pred)
            if len(A):
                active, st, lf = self._stage_particles(n, A, F1, dep, flux, Flow)
                stopped.append(st)
                left.append(lf)
                if self.trace is not None:
                    self.trace.append((n, MP.concat(active, lf)))
            else:
                active = MP.empty()
            Jrec[0, n], Jrec[1, n], Jrec[2, n] = dep.Jx, dep.Jy, dep.Jz
            if not self.solver:
                F1[:, n] = self.F0[:, n]
                continue
            jp1 = solver_currents(m, dep.Jx, dep.Jy, dep.Jz, KX, KY, nyq)
            jm0, jm1, jp0 = node_currents(n, jp1)
            jst[0][n + 1], jst[1][n + 1] = jp1[0], jp1[1]
            old = [getattr(self.state, nm)[n] for nm in ("Rx", "Ry", "Ez", "Bz")]
            vals = solve_node(m, n, Dn, old, right, jm0, jm1, jp0, jp1, KX, KY, nyq)
            for c, nm in enumerate(SpectralState.NAMES):
                getattr(new, nm)[n] = vals[c]
            right = vals
            F1[:, n] = node_real_fields(vals)
        # currents of the half-node below node 0 are those of no particle
        if startup:
            self.state = new
            self.F0 = F1
            self.j0 = (jst[0], jst[1])
            self.next_pid = pid0
            return self
        self.J = Jrec
        self.flux = flux
        P = MP.concat(*(stopped + [active])) if (stopped or len(active)) else MP.empty()
        self.left = MP.concat(*left) if left else MP.empty()
        order = np.argsort(P.pid, kind="stable")
        self.P = P.take(order)
        if self.solver:
            self.state = new
            self.F0 = F1
            self.j0 = (jst[0], jst[1])
        self.s += D
        self.k += 1
        if diag or self.record:
            rho1 = cell_charge(m, self.P) + 0.0
            self.rho0, self.rho1 = rho0, rho1
            self.diag = dict(step=self.k, s=self.s, n_particles=len(self.P),
                             field_energy=field_energy(m, self.F0),
                             ez_axis=self.F0[2, :p.Nz, p.Ny // 2, p.Nx // 2].copy())
        return self

    def run(self, n, **kw):
        for _ in range(n):
            self.step(**kw)
        return self


def solver_currents(m, Jx, Jy, Jz, KX, KY, nyq):
    """Cell currents of half-node n + 1/2 -> solver inputs: transverse FFT,
    J_x (J_y in 3-D) shifted from the face x_{i+1/2} to the node by
    exp(-i k_x h_x / 2), the transverse binomial factor cos^2(k h / 2) per
    pass (M5), Nyquist rows and columns zero."""
    p = m.p
    f = (np.cos(0.5 * KX * p.hx) ** 2) * ((np.cos(0.5 * KY * p.hy) ** 2) if p.dims == 3 else 1.0)
    fil = f ** p.filter_passes
    jx = fft2(Jx) * np.exp(-0.5j * KX * p.hx) * fil
    jy = fft2(Jy) * (np.exp(-0.5j * KY * p.hy) if p.dims == 3 else 1.0) * fil
    jz = fft2(Jz) * fil
    for a in (jx, jy, jz):
        a[nyq] = 0.0
    return jx, jy, jz


def solve_node(m, n, D, old, right, jm0, jm1, jp0, jp1, KX, KY, nyq):
    """Node system RxN .. eqall at node n (readings of fields.py) with the
    currents of both levels on both half-nodes: the R rows carry the
    four-term average (j^1_{-1/2} + j^0_{-1/2} + j^1_{+1/2} + j^0_{+1/2}) / 4,
    the L and E_z rows j^1_{+1/2}; h = h_n.  Direct 6 x 6 solve per mode."""
    p = m.p
    h = m.hz[n]
    kx, ky = KX.ravel(), KY.ravel()
    keep = ~nyq.ravel()
    A = node_matrix(kx[keep], ky[keep], h, D)
    i = 1j
    ikx, iky = i * kx[keep], i * ky[keep]
    Rx0, Ry0, Ez0, Bz0 = (o.ravel()[keep] for o in old)
    Rx1, Ry1, Lx1, Ly1, Ez1, Bz1 = (r.ravel()[keep] for r in right)
    Ex1, Ey1 = 0.5 * (Rx1 + Lx1), 0.5 * (Ry1 + Ly1)
    By1, Bx1 = 0.5 * (Rx1 - Lx1), 0.5 * (Ly1 - Ry1)
    sx = (jm1[0] + jm0[0] + jp1[0] + jp0[0]).ravel()[keep]
    sy = (jm1[1] + jm0[1] + jp1[1] + jp0[1]).ravel()[keep]
    jx1, jy1, jz1 = (a.ravel()[keep] for a in jp1)
    b = np.zeros((keep.sum(), 6), complex)
    b[:, 0] = Rx0 + 0.5 * D * (ikx * Ez0 + iky * Bz0) - 0.25 * D * sx
    b[:, 1] = Ry0 + 0.5 * D * (iky * Ez0 - ikx * Bz0) - 0.25 * D * sy
    b[:, 2] = -Lx1 + 0.25 * h * (ikx * Ez1 - iky * Bz1) + 0.5 * h * jx1
    b[:, 3] = -Ly1 + 0.25 * h * (iky * Ez1 + ikx * Bz1) + 0.5 * h * jy1
    b[:, 4] = -Bz1 + 0.5 * h * (ikx * Ey1 - iky * Ex1)
    b[:, 5] = -Ez1 + 0.5 * h * (-ikx * By1 + iky * Bx1) + h * jz1
    sol = np.linalg.solve(A, b[..., None])[..., 0]
    out = []
    for c in range(6):
        v = np.zeros(kx.size, complex)
        v[keep] = sol[:, c]
        out.append(v.reshape(p.Ny, p.Nx))
    return out


def node_real_fields(vals):
    """(Rx, Ry, Lx, Ly, Ez, Bz) spectra of one node -> six real fields."""
    Rx, Ry, Lx, Ly, Ez, Bz = vals
    spec = [0.5 * (Rx + Lx), 0.5 * (Ry + Ly), Ez, 0.5 * (Ly - Ry), 0.5 * (Rx - Lx), Bz]
    return np.stack([ifft2_real(a) for a in spec])


def real_fields(m, s):
    p = m.p
    out = np.zeros((6, p.Nz + 1, p.Ny, p.Nx))
    for n in range(p.Nz):
        out[:, n] = node_real_fields([getattr(s, nm)[n] for nm in SpectralState.NAMES])
    return out


def init_state(m):
    """Laser of Sec. 6 (eq. E_laser) on the nodes zeta_n as a pure forward wave
    (R_pol = 2 E_pol, L = 0), made consistent by one march with Delta = 0 and
    no current (as fields.laser_state, with the node spacing h_n)."""
    p = m.p
    s = SpectralState(p)
    KX, KY, nyq = wavenumbers(p)
    if p.a0 != 0.0:
        phi = m.zn[:p.Nz] - p.zeta_c
        lon = p.a0 * np.cos(phi) * np.exp(-(phi * phi) / (p.T * p.T))
        x = np.arange(p.Nx) * p.hx - (p.Nx // 2) * p.hx
        y = (np.arange(p.Ny) * p.hy - (p.Ny // 2) * p.hy) if p.dims == 3 else np.zeros(1)
        X, Y = np.meshgrid(x, y, indexing="xy")
        tra = np.exp(-(X * X + Y * Y) / (p.waist * p.waist)) if p.waist > 0.0 else np.ones_like(X)
        R = fft2(2.0 * lon[:, None, None] * tra[None])
        R[:, nyq] = 0.0
        setattr(s, "Rx" if p.pol == 0 else "Ry", R)
    zero = np.zeros((p.Ny, p.Nx), complex)
    new = SpectralState(p)
    right = [zero] * 6
    z3 = (zero, zero, zero)
    for n in range(p.Nz - 1, -1, -1):
        old = [getattr(s, nm)[n] for nm in ("Rx", "Ry", "Ez", "Bz")]
        vals = solve_node(m, n, 0.0, old, right, z3, z3, z3, z3, KX, KY, nyq)
        for c, nm in enumerate(SpectralState.NAMES):
            getattr(new, nm)[n] = vals[c]
        right = vals
    return new


def cell_charge(m, P):
    """Charge density per zeta cell (nearest cell along zeta, cloud-in-cell
    across), shape (Nz, Ny, Nx): q w / V_n per particle."""
    p = m.p
    rho = np.zeros((p.Nz, p.Ny, p.Nx))
    V = p.hx * p.hy_eff * m.hz[P.iz]
    c = p.q * P.w / V
    wxs = (1.0 - P.dx, P.dx)
    if p.dims == 3:
        wys = (1.0 - P.dy, P.dy)
        for b in range(2):
            for a in range(2):
                np.add.at(rho, (P.iz, (P.iy + b) % p.Ny, (P.ix + a) % p.Nx), c * wxs[a] * wys[b])
    else:
        for a in range(2):
            np.add.at(rho, (P.iz, P.iy, (P.ix + a) % p.Nx), c * wxs[a])
    return rho


def continuity_residual(m, rho0, rho1, J, flux):
    """Per cell: (rho1 - rho0) / Delta + D_perp . J_perp - (F(n + 1) - F(n)) / h_n,
    with F(n) the charge per area per Delta that crossed node n downwards.
    Zero to roundoff for the scheme's currents (the transverse Esirkepov
    decomposition inside cells plus the node crossings)."""
    p = m.p
    Jx, Jy = J[0], J[1]
    r = (rho1 - rho0) / m.Delta + (Jx - np.roll(Jx, 1, axis=2)) / p.hx
    if p.dims == 3:
        r = r + (Jy - np.roll(Jy, 1, axis=1)) / p.hy
    r = r - (flux[1:] - flux[:-1]) / m.hz[:, None, None]
    return r


def field_energy(m, F):
    """1/2 sum (E^2 + B^2) V over the nodes, V = h_x h_y times the mean of
    the two cells at the node (h_0 at node 0)."""
    p = m.p
    hnode = 0.5 * (np.r_[m.hz[0], m.hz[:-1]] + m.hz)
    V = p.hx * p.hy_eff * hnode
    return float(0.5 * np.sum(np.sum(F[:, :p.Nz] ** 2, axis=(0, 2, 3)) * V))
