// Zeta-march slow step: the paper's own particle scheme.  Particles are
// integrated along the fast coordinate zeta, interleaved with the right-to-left
// march of the field solver, so that the slow step Delta can exceed the fast
// step h by far (Sec. 5: characteristics of eq:Vlasov1 parametrised by zeta,
// stop rule eq:trap1; GT2: eq:Vlasov2, eq:trap2.  Sec. 5.1: fresh weight
// Q_f = q n h_x h_y Delta, current j = (Q / (h_x h_y h)) v ds / Delta.
// Sec. 4.1: node n solved at the new level once node n + 1 is known, the
// current below the node predicted).
//
// Stage n (cell n: zeta_n < zeta <= zeta_{n+1}):
//   1. k_mz_stage pushes every particle of the cell (the ones that reached
//      node n + 1 in stage n + 1 and the ones parked in the cell) by midpoint
//      sub-steps until it reaches node n, runs out of slow budget (it is then
//      parked for the next step) or, at node 0, leaves; the cell's currents
//      go to a real-space plane;
//   2. the plane is transformed (x, y);
//   3. k_mz_node solves node n for every transverse mode (App. B closed form
//      with the currents of both slow levels);
//   4. the node's six field spectra are transformed back into node records.
// Fields inside cell n are linear in zeta between nodes n + 1 and n at the
// new level; cloud-in-cell across.  Node n at the new level depends on the
// cell's own currents, so a stage runs 1-4 twice: the predictor pushes the
// particles with node n at the old level and only deposits (no particle is
// written), and its node solve writes only the node's records; the
// corrector pushes them again, from the same start, with the predicted node
// n and is kept.  A sub-step that reaches the
// node is parametrised by zeta and ends on it; a sub-step limited by the
// budget or by the transverse limit (half a cell) is parametrised by lab
// time and ends on the node if it would pass it.  GT1 spends budget at rate
// 1 per unit time, GT2 at rate v_z.  Transverse currents come from Esirkepov's
// decomposition of the transverse move inside the cell, J_z from
// Q (d zeta + ds) / (V Delta) times the time-averaged transverse shape.
// All of this mirrors the oracle's reading of the paper operation by
// operation (FP64), so that decisions taken on floating point (which sub-step
// kind, node reached, cell crossed) coincide.
#pragma once

// zeta-march particle store (structure of arrays); cell = (iz * Ny + iy) * Nx
// + ix; offsets ox, oy in [0, 1), oz in (0, 1]; w = electrons per
// macro-particle; b = slow budget left in the current step
template <typename T>
struct MzParts {
  int32_t* cell;
  T *ox, *oy, *oz, *ux, *uy, *uz, *w, *b;
  int64_t* id;   // nullable
};

#define ERR_MARCH 32   // a particle exceeded the sub-step bound of a stage

template <typename T>
struct MzStageArgs {
  Geom g;
  int n;               // the stage's cell
  T hn;                // h_n = zeta_{n+1} - zeta_n
  T hx, hy;            // transverse steps (hy = 1 in 2-D)
  T D;                 // slow step Delta
  T ds_perp;           // transverse sub-step limit min(hx, hy) / 2
  int scheme;          // 1 = GT1, 2 = GT2
  int pred;            // predictor pass: deposit only, no particle written
  int cap;             // sub-steps per particle and stage (hang guard)
  int capacity;        // of each particle buffer
  const T* F0;         // records [Nz][Ny][Nx][6] giving node n: the old level
                       // (predictor) or the predicted new level (corrector)
  const T* F1;         // new-level node records (node n + 1 already written)
  T* dep;              // [3][Ny][Nx] currents of cell n
  MzParts<T> in;       // particles that reached node n + 1 in stage n + 1
  const int* in_count;
  MzParts<T> park;     // parked store (sorted by cell)
  const int* pstart;
  const int* pcount;
  MzParts<T> out;      // particles that reach node n with budget left
  int* out_count;
  MzParts<T> stop;     // particles whose budget ran out in this step
  int* stop_count;
  int* left_count;     // particles that left at node 0
  int* err;
};

template <typename T>
GP_DEV void mz_velocity(T ux, T uy, T uz, T* g, T* vx, T* vy, T* vz, T* omv) {
  T up2 = ux * ux + uy * uy;
  T gm = sqrt(((T)1 + up2) + uz * uz);
  *g = gm;
  *vx = ux / gm;
  *vy = uy / gm;
  *vz = uz / gm;
  *omv = uz >= (T)0 ? ((T)1 + up2) / (gm * (gm + uz)) : (T)1 - uz / gm;
}

// offset d plus a shift in cells -> new offset in [0, 1) and the cell step
template <typename T>
GP_DEV int mz_advance(T d, T shift, T* out) {
  T t = d + shift;
  T k = floor(t);
  t = t - k;
  int ki = (int)k;
  if (t >= (T)1) { t = (T)0; ki += 1; }
  *out = t;
  return ki;
}

// E, B at transverse (ix + dx, iy + dy), fraction t of cell n: linear between
// node n of F0 and node n + 1 of F1 (zero at the ghost node Nz)
template <typename T, int DIM>
GP_DEV void mz_gather(const MzStageArgs<T>& a, int ix, int iy, T dx, T dy, T t, T f[6]) {
  const Geom& g = a.g;
  const int n = a.n;
  const bool top = n + 1 >= g.Nz;
  const int xs[2] = {ix, ix + 1 == g.Nx ? 0 : ix + 1};
  const int ys[2] = {iy, DIM == 3 ? (iy + 1 == g.Ny ? 0 : iy + 1) : iy};
  const T wx[2] = {(T)1 - dx, dx};
  const T wy[2] = {(T)1 - dy, dy};
  constexpr int NB = DIM == 3 ? 2 : 1;
  // every record of both levels is loaded before any is used, so that the
  // loads are in flight together; at the top cell the new-level node is the
  // ghost node (zero fields): its loads read node n instead (in bounds) and
  // the values are replaced by zero
  const int64_t up = top ? 0 : (int64_t)g.Ny * g.Nx * 6;
  T v0[NB][2][6], v1[NB][2][6];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
      const int64_t r0 = (((int64_t)n * g.Ny + ys[b]) * g.Nx + xs[aa]) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        v0[b][aa][c] = a.F0[r0 + c];
        v1[b][aa][c] = a.F1[r0 + up + c];
      }
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) f[c] = (T)0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
      const T w = DIM == 3 ? wx[aa] * wy[b] : wx[aa];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const T u1 = top ? (T)0 : v1[b][aa][c];
        f[c] = f[c] + w * (((T)1 - t) * v0[b][aa][c] + t * u1);
      }
    }
  }
}

template <typename T>
GP_DEV void mz_force(const T f[6], T vx, T vy, T vz, T* Fx, T* Fy, T* Fz) {
  const T q = (T)-1;
  *Fx = q * ((f[0] + vy * f[5]) - vz * f[4]);
  *Fy = q * ((f[1] + vz * f[3]) - vx * f[5]);
  *Fz = q * ((f[2] + vx * f[4]) - vy * f[3]);
}

// 3-node window starting at min(c0, c0 + k) with the old and new linear weights
template <typename T>
GP_DEV void mz_window(int k, T d0, T d1, T S0[3], T S1[3]) {
  const int o0 = k < 0 ? 1 : 0, o1 = k > 0 ? 1 : 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    S0[i] = (i == o0 ? (T)1 - d0 : (T)0) + (i == o0 + 1 ? d0 : (T)0);
    S1[i] = (i == o1 ? (T)1 - d1 : (T)0) + (i == o1 + 1 ? d1 : (T)0);
  }
}

// a current contribution; exact zeros (the third window node of a sub-step
// that crosses no transverse cell face) issue no atomic
template <typename T>
GP_DEV void mz_add(T* p, T v) {
  if (v != (T)0) atomicAdd(p, v);
}

// currents of one sub-step inside cell n (Qw = q w)
template <typename T, int DIM>
GP_DEV void mz_deposit(const MzStageArgs<T>& a, T Qw, int ix0, int iy0, T dx0, T dy0, int kx, int ky, T dx1,
                       T dy1, T dzeta, T ds, T dy_len) {
  const Geom& g = a.g;
  const T D = a.D, hn = a.hn;
  const T V = (a.hx * a.hy) * hn;
  T S0x[3], S1x[3], DSx[3];
  mz_window(kx, dx0, dx1, S0x, S1x);
#pragma unroll
  for (int i = 0; i < 3; ++i) DSx[i] = S1x[i] - S0x[i];
  const int bx = ix0 + min(kx, 0);
  int xs[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int x = bx + i;
    xs[i] = x < 0 ? x + g.Nx : (x >= g.Nx ? x - g.Nx : x);
  }
  const int64_t P = (int64_t)g.Ny * g.Nx;
  T* Jx = a.dep;
  T* Jy = a.dep + P;
  T* Jz = a.dep + 2 * P;
  const T tz = Qw * (dzeta + ds) / (D * V);
  if constexpr (DIM == 3) {
    T S0y[3], S1y[3], DSy[3];
    mz_window(ky, dy0, dy1, S0y, S1y);
#pragma unroll
    for (int i = 0; i < 3; ++i) DSy[i] = S1y[i] - S0y[i];
    const int by = iy0 + min(ky, 0);
    int ys[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      int y = by + i;
      ys[i] = y < 0 ? y + g.Ny : (y >= g.Ny ? y - g.Ny : y);
    }
    const T cx = -Qw / ((D * a.hy) * hn);
    const T cy = -Qw / ((D * a.hx) * hn);
    // without a crossing in x (y) the second face's sum DS[0] + DS[1]
    // vanishes (the window's third node has no weight): it is left out
    // rather than deposited as a rounding residue
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T acc = (T)0;
#pragma unroll
      for (int aa = 0; aa < 2; ++aa) {
        acc = acc + DSx[aa] * (S0y[b] + (T)0.5 * DSy[b]);
        if (aa == 0 || kx != 0) mz_add(Jx + (int64_t)ys[b] * g.Nx + xs[aa], cx * acc);
      }
    }
#pragma unroll
    for (int aa = 0; aa < 3; ++aa) {
      T acc = (T)0;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc = acc + DSy[b] * (S0x[aa] + (T)0.5 * DSx[aa]);
        if (b == 0 || ky != 0) mz_add(Jy + (int64_t)ys[b] * g.Nx + xs[aa], cy * acc);
      }
    }
#pragma unroll
    for (int aa = 0; aa < 3; ++aa) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        T w = (S0x[aa] * S0y[b] + (T)0.5 * (DSx[aa] * S0y[b] + S0x[aa] * DSy[b])) + DSx[aa] * DSy[b] / (T)3;
        mz_add(Jz + (int64_t)ys[b] * g.Nx + xs[aa], tz * w);
      }
    }
  } else {
    const T cx = -Qw / (D * hn);
    T acc = (T)0;
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
      acc = acc + DSx[aa];
      if (aa == 0 || kx != 0) mz_add(Jx + xs[aa], cx * acc);
    }
    const T ty = Qw * dy_len / (D * V);
#pragma unroll
    for (int aa = 0; aa < 3; ++aa) {
      T w = S0x[aa] + (T)0.5 * DSx[aa];
      mz_add(Jy + xs[aa], ty * w);
      mz_add(Jz + xs[aa], tz * w);
    }
  }
}

// position of a predicate's lane among the wave's set lanes, with one atomic
// per wave on the counter; -1 if the predicate is false
GP_DEV int mz_append(int* counter, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return -1;
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
  base = __shfl(base, leader);
  return pred ? base + (int)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

template <typename T>
GP_DEV void mz_store(const MzParts<T>& P, int i, int cell, T ox, T oy, T oz, T ux, T uy, T uz, T w, T b,
                     int64_t id) {
  P.cell[i] = cell;
  P.ox[i] = ox;
  P.oy[i] = oy;
  P.oz[i] = oz;
  P.ux[i] = ux;
  P.uy[i] = uy;
  P.uz[i] = uz;
  P.w[i] = w;
  P.b[i] = b;
  if (P.id) P.id[i] = id;
}

// Stage n.  A wave takes 64 consecutive particles of the stage's list (the
// active ones first, then the cell's parked ones); the grid strides over the
// list, whose length only the device knows.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_mz_stage(MzStageArgs<T> a) {
  const Geom& g = a.g;
  const int n = a.n;
  // a counter may have run past the capacity (the appends beyond it were
  // dropped and flagged): never read past the buffer
  const int na = min(*a.in_count, a.capacity);
  const int p0 = a.pstart[n];
  const int total = na + a.pcount[n];
  const int lane = (int)(threadIdx.x & 63);
  const int stride = (int)(gridDim.x * blockDim.x);
  for (int t0 = (int)(blockIdx.x * blockDim.x + (threadIdx.x & ~63u)); t0 < total; t0 += stride) {
    const int t = t0 + lane;
    const bool valid = t < total;
    int cell = 0;
    T ox = 0, oy = 0, oz = 1, ux = 0, uy = 0, uz = 0, w = 0, b = 0;
    int64_t id = 0;
    if (valid) {
      const MzParts<T>& S = t < na ? a.in : a.park;
      const int i = t < na ? t : p0 + (t - na);
      cell = S.cell[i];
      ox = S.ox[i]; oy = S.oy[i]; oz = S.oz[i];
      ux = S.ux[i]; uy = S.uy[i]; uz = S.uz[i];
      w = S.w[i]; b = S.b[i];
      if (S.id) id = S.id[i];
    }
    int ix = cell % g.Nx;
    int iy = (cell / g.Nx) % g.Ny;
    // 0 working, 1 reached node n with budget (next stage), 2 stopped, 3 left
    int status = valid ? 0 : 4;
    int izc = n;   // the particle's cell after the stage
    int iter = 0;
    while (status == 0) {
      if (++iter > a.cap) { atomicOr(a.err, ERR_MARCH); status = 2; break; }
      if (!(ux == ux && uy == uy && uz == uz)) { atomicOr(a.err, ERR_NUMERIC); status = 2; break; }
      T gm, vx, vy, vz, omv;
      mz_velocity(ux, uy, uz, &gm, &vx, &vy, &vz, &omv);
      const T dist = oz * a.hn;
      const T ds_node = dist / omv;
      const T rate = a.scheme == 2 ? vz : (T)1;
      const T t_budget = rate > (T)0 ? b / rate : (T)INFINITY;
      const T lim = min(t_budget, a.ds_perp);
      const bool zstep = ds_node <= lim;
      const T dt = zstep ? (T)0 : lim;
      const bool blim = !zstep && t_budget <= a.ds_perp;
      T f[6];
      mz_gather<T, DIM>(a, ix, iy, ox, oy, oz, f);
      T Fx, Fy, Fz;
      mz_force(f, vx, vy, vz, &Fx, &Fy, &Fz);
      const T h1 = zstep ? (T)0.5 * dist / omv : (T)0.5 * dt;
      const T uxm = ux + h1 * Fx, uym = uy + h1 * Fy, uzm = uz + h1 * Fz;
      T oxm, oym = oy;
      int kxm = mz_advance(ox, h1 * vx / a.hx, &oxm);
      int ixm = ix + kxm;
      ixm = ixm < 0 ? ixm + g.Nx : (ixm >= g.Nx ? ixm - g.Nx : ixm);
      int iym = iy;
      if (DIM == 3) {
        int kym = mz_advance(oy, h1 * vy / a.hy, &oym);
        iym = iy + kym;
        iym = iym < 0 ? iym + g.Ny : (iym >= g.Ny ? iym - g.Ny : iym);
      }
      T tm;
      if (zstep) {
        tm = (T)0.5 * oz;
      } else {
        tm = oz - h1 * omv / a.hn;
        tm = tm < (T)0 ? (T)0 : (tm > (T)1 ? (T)1 : tm);
      }
      T gmm, vxm, vym, vzm, omvm;
      mz_velocity(uxm, uym, uzm, &gmm, &vxm, &vym, &vzm, &omvm);
      T fm[6];
      mz_gather<T, DIM>(a, ixm, iym, oxm, oym, tm, fm);
      T Fxm, Fym, Fzm;
      mz_force(fm, vxm, vym, vzm, &Fxm, &Fym, &Fzm);
      const T ds = zstep ? dist / omvm : dt;
      const T ux1 = ux + ds * Fxm, uy1 = uy + ds * Fym, uz1 = uz + ds * Fzm;
      T ox1, oy1 = oy;
      const int kx = mz_advance(ox, ds * vxm / a.hx, &ox1);
      int ky = 0;
      if (DIM == 3) ky = mz_advance(oy, ds * vym / a.hy, &oy1);
      T oz1 = zstep ? (T)0 : oz - ds * omvm / a.hn;
      const bool reached = oz1 <= (T)0;
      if (reached) oz1 = (T)0;
      const T dzeta = (oz1 - oz) * a.hn;
      if (kx < -1 || kx > 1 || ky < -1 || ky > 1) { atomicOr(a.err, ERR_CFL); status = 2; break; }
      mz_deposit<T, DIM>(a, (T)-1 * w, ix, iy, ox, oy, kx, ky, ox1, oy1, dzeta, ds, ds * vym);
      const T used = a.scheme == 2 ? ds * vzm : ds;
      b = b - used;
      const bool out = b <= (T)0 || blim;
      ux = ux1; uy = uy1; uz = uz1;
      ix = ix + kx;
      ix = ix < 0 ? ix + g.Nx : (ix >= g.Nx ? ix - g.Nx : ix);
      if (DIM == 3) {
        iy = iy + ky;
        iy = iy < 0 ? iy + g.Ny : (iy >= g.Ny ? iy - g.Ny : iy);
      }
      ox = ox1; oy = oy1; oz = oz1;
      if (reached) {
        if (n == 0) {
          status = 3;
        } else {
          izc = n - 1;
          oz = (T)1;
          status = out ? 2 : 1;
        }
      } else if (out) {
        status = 2;
      }
    }
    if (a.pred) continue;
    const int ncell = (izc * g.Ny + (DIM == 3 ? iy : 0)) * g.Nx + ix;
    const int po = mz_append(a.out_count, status == 1);
    if (po >= a.capacity) atomicOr(a.err, ERR_CAPACITY);
    else if (po >= 0) mz_store(a.out, po, ncell, ox, oy, oz, ux, uy, uz, w, b, id);
    const int ps = mz_append(a.stop_count, status == 2);
    if (ps >= a.capacity) atomicOr(a.err, ERR_CAPACITY);
    else if (ps >= 0) mz_store(a.stop, ps, ncell, ox, oy, oz, ux, uy, uz, w, b, id);
    const int pl = mz_append(a.left_count, status == 3);
    (void)pl;
  }
}

// ---------------------------------------------------------------------------
// Node n of the march for every transverse mode (one thread per (ky, kx)):
// App. B closed form (readings of the tau path's k_march) with the currents
// of both slow levels.  On half-node n + 1/2 the new-level currents are the
// transforms of cell n's deposit, shifted from the faces x_{i+1/2} (y_{j+1/2}
// in 3-D) to the nodes by exp(-i k h / 2) and filtered transversally by
// cos^2(k h / 2) per pass; j^0 is the previous step's (stored), and j^1 on
// half-node n - 1/2 is predicted as j^0 there plus the change half-node
// n + 1/2 has seen, j^0_{-1/2} + (j^1_{+1/2} - j^0_{+1/2}), so that the R
// rows' four-term sum is 2 (j^1_{+1/2} + j^0_{-1/2}), centred on the node
// and on the middle of the slow step: the R update then keeps the amplitude
// of a mode whose current only turns its phase.  In GT2 j^0 of the first
// step is the startup march's current; first = 1 (GT1's first step, no
// plasma, or the startup march itself, whose zero slow step takes no current
// into the R rows) uses j^1 of half-node n + 1/2.
// The kernel also stores j^1 for the next step, records the cell's raw
// currents (jrec), clears the deposit plane for the next stage and resets a
// particle counter.
template <typename T>
struct MzNodeArgs {
  Geom g;
  int n;
  T h;                  // h_n
  T D;                  // slow step (0: consistency march)
  int first;            // no j^0 yet
  const cplx<T>* jhat;  // [3][Ny][Nxh] transforms of the cell's deposit (nullable: no current)
  cplx<T>* j0[2];       // [Nz + 1][Ny][Nxh] solver currents x, y of the previous step
  cplx<T>* st[4];       // Rx, Ry, Ez, Bz [Nz][Ny][Nxh]: old level in, new level out
  cplx<T>* L[2];        // Lx, Ly [Nz][Ny][Nxh]
  cplx<T>* out[6];      // Ex, Ey, Ez, Bx, By, Bz spectra of node n
  T* dep;               // nullable: [3][Ny][Nx] deposit plane to clear
  T* jrec[3];           // nullable: raw current planes to record into
  int* zero_count;      // nullable
  int pred;             // predictor: only out[] is written (and dep cleared)
};

// the deposit plane recorded (corrector) and cleared for the next pass, and
// the stage's particle counter reset; thread t of nt strides over the plane
template <typename T>
GP_DEV void mz_node_clear(const MzNodeArgs<T>& a, int64_t t, int64_t nt) {
  const Geom& g = a.g;
  const int64_t P = (int64_t)g.Ny * g.Nx;
  if (a.dep) {
    for (int64_t i = t; i < 3 * P; i += nt) {
      const int c = (int)(i / P);
      const int64_t r = i - (int64_t)c * P;
      if (a.jrec[0]) a.jrec[c][r] = a.dep[i];
      a.dep[i] = (T)0;
    }
  }
  if (t == 0 && a.zero_count) *a.zero_count = 0;
}

// node n for transverse mode m = ky Nxh + kx, given the transforms of the
// cell's deposit at that mode (jh; zero without current): the new level's
// state (R, E_z, B_z, L and this step's solver currents) unless predicting,
// and the six field spectra in out[]
template <typename T>
GP_DEV void mz_node_mode(const MzNodeArgs<T>& a, int64_t m, const cplx<T> jh[3], cplx<T> out[6]) {
  const Geom& g = a.g;
  const int64_t M = (int64_t)g.Ny * g.Nxh;
  const int n = a.n;
  const int64_t o = (int64_t)n * M + m;
  const int kyi = (int)(m / g.Nxh), kxi = (int)(m % g.Nxh);
  const cplx<T> z = mk((T)0, (T)0);
  if (g.Ny > 1 && kyi == g.Ny / 2) {
    for (int q = 0; q < 6; ++q) out[q] = z;
    if (a.pred) return;
    for (int q = 0; q < 4; ++q) a.st[q][o] = z;
    a.L[0][o] = z;
    a.L[1][o] = z;
    a.j0[0][o + M] = z;
    a.j0[1][o + M] = z;
    if (n == 0) { a.j0[0][m] = z; a.j0[1][m] = z; }
    return;
  }
  const double PI = 3.14159265358979323846;
  const double kxd = 2.0 * PI * (double)kxi / ((double)g.Nx * g.hx);
  const int kys = kyi <= g.Ny / 2 ? kyi : kyi - g.Ny;
  const double kyd = g.Ny > 1 ? 2.0 * PI * (double)kys / ((double)g.Ny * g.hy) : 0.0;
  double fxy = cos(0.5 * kxd * g.hx);
  fxy *= fxy;
  if (g.dims == 3) { double fy = cos(0.5 * kyd * g.hy); fxy *= fy * fy; }
  double phi = 1.0;
  for (int p = 0; p < g.P; ++p) phi *= fxy;
  const cplx<T> sx = mk((T)(phi * cos(0.5 * kxd * g.hx)), (T)(-phi * sin(0.5 * kxd * g.hx)));
  const cplx<T> sy = g.dims == 3 ? mk((T)(phi * cos(0.5 * kyd * g.hy)), (T)(-phi * sin(0.5 * kyd * g.hy)))
                                 : mk((T)phi, (T)0);
  const T kx = (T)kxd, ky = (T)kyd;
  const cplx<T> jxp = sx * jh[0], jyp = sy * jh[1], jzp = (T)phi * jh[2];
  const cplx<T> jx0m = a.first ? jxp : a.j0[0][o];
  const cplx<T> jy0m = a.first ? jyp : a.j0[1][o];
  // four-term sums with the predicted j^1_{-1/2}: 2 (j^1_{+1/2} + j^0_{-1/2})
  const cplx<T> Jx = (T)2 * (jxp + jx0m);
  const cplx<T> Jy = (T)2 * (jyp + jy0m);
  const T h = a.h, D = a.D;
  const T K2 = kx * kx + ky * ky;
  const T Dd = (T)16 + h * ((T)2 * D + h) * K2;
  const T inv = (T)1 / Dd;
  const T c16 = (T)16 - h * h * K2;
  const cplx<T> Rx0 = a.st[0][o], Ry0 = a.st[1][o], Ez0 = a.st[2][o], Bz0 = a.st[3][o];
  cplx<T> Rx1 = z, Ry1 = z, Lx1 = z, Ly1 = z, Ez1 = z, Bz1 = z;
  if (n + 1 < g.Nz) {
    Rx1 = a.st[0][o + M]; Ry1 = a.st[1][o + M]; Ez1 = a.st[2][o + M]; Bz1 = a.st[3][o + M];
    Lx1 = a.L[0][o + M]; Ly1 = a.L[1][o + M];
  }
  const cplx<T> Wx = (Rx0 + Rx1) - (T)2 * Lx1;
  const cplx<T> Wy = (Ry0 + Ry1) - (T)2 * Ly1;
  const cplx<T> Ux = (Rx0 + Rx1) + (T)2 * Lx1;
  const cplx<T> Uy = (Ry0 + Ry1) + (T)2 * Ly1;
  cplx<T> Ez = c16 * Ez1 - ((T)16 * h) * jzp - mul_i((h * D) * (kx * Jx + ky * Jy)) -
               ((T)2 * h * D * K2) * Ez0 + mul_i(((T)2 * h * h) * (kx * jxp + ky * jyp)) +
               mul_i(((T)4 * h) * (kx * Wx + ky * Wy));
  Ez = inv * Ez;
  cplx<T> Bz = c16 * Bz1 + mul_i(((T)2 * h * h) * (kx * jyp - ky * jxp)) + mul_i((h * D) * (kx * Jy - ky * Jx)) -
               ((T)2 * h * D * K2) * Bz0 + mul_i(((T)4 * h) * (ky * Ux - kx * Uy));
  Bz = inv * Bz;
  const cplx<T> Ezs = Ez + Ez0, Bzs = Bz + Bz0;
  const cplx<T> Rx = Rx0 + mul_i(((T)0.5 * D) * (kx * Ezs + ky * Bzs)) - ((T)0.25 * D) * Jx;
  const cplx<T> Ry = Ry0 + mul_i(((T)0.5 * D) * (ky * Ezs - kx * Bzs)) - ((T)0.25 * D) * Jy;
  const cplx<T> Ezp = Ez1 + Ez, Bzp = Bz + Bz1;
  const cplx<T> Lx = Lx1 - ((T)0.5 * h) * (mul_i((T)0.5 * (kx * Ezp - ky * Bzp)) + jxp);
  const cplx<T> Ly = Ly1 - ((T)0.5 * h) * (mul_i((T)0.5 * (ky * Ezp + kx * Bzp)) + jyp);
  if (!a.pred) {
    a.st[0][o] = Rx;
    a.st[1][o] = Ry;
    a.st[2][o] = Ez;
    a.st[3][o] = Bz;
    a.L[0][o] = Lx;
    a.L[1][o] = Ly;
  }
  out[0] = (T)0.5 * (Rx + Lx);
  out[1] = (T)0.5 * (Ry + Ly);
  out[2] = Ez;
  out[3] = (T)0.5 * (Ly - Ry);
  out[4] = (T)0.5 * (Rx - Lx);
  out[5] = Bz;
  if (a.pred) return;
  a.j0[0][o + M] = jxp;
  a.j0[1][o + M] = jyp;
  if (n == 0) { a.j0[0][m] = z; a.j0[1][m] = z; }
}


// node n for every mode, one thread per mode (spectra already transformed
// along y, or Ny = 1)
template <typename T>
__global__ __launch_bounds__(256) void k_mz_node(MzNodeArgs<T> a) {
  const int64_t M = (int64_t)a.g.Ny * a.g.Nxh;
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  mz_node_clear(a, m, (int64_t)gridDim.x * blockDim.x);
  if (m >= M) return;
  cplx<T> jh[3] = {mk((T)0, (T)0), mk((T)0, (T)0), mk((T)0, (T)0)};
  if (a.jhat) {
    jh[0] = a.jhat[m];
    jh[1] = a.jhat[M + m];
    jh[2] = a.jhat[2 * M + m];
  }
  cplx<T> out[6];
  mz_node_mode(a, m, jh, out);
#pragma unroll
  for (int q = 0; q < 6; ++q) a.out[q][m] = out[q];
}

// One kx column per work-group: the cell's deposit, transformed along x
// (jhx, [3][Ny][Nxh]), is transformed along y in LDS, node n is solved for
// each of the column's modes, and the six field spectra are transformed back
// along y in LDS and written to out[] (still to be transformed along x).
// Fuses the forward y transform, k_mz_node and the inverse y transforms of a
// pass; dynamic LDS: 2 x 6 sequences of Ny + FFTY_PAD plus Ny twiddles.
template <typename T>
__global__ __launch_bounds__(256) void k_mz_colnode(MzNodeArgs<T> a, const cplx<T>* jhx, const cplx<T>* twy) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Geom& g = a.g;
  const int Ny = g.Ny, Nxh = g.Nxh;
  const int S = Ny + FFTY_PAD;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* B = A + 6 * S;
  cplx<T>* tl = B + 6 * S;
  const int kx = blockIdx.x;
  mz_node_clear(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
  const int64_t M = (int64_t)Ny * Nxh;
  for (int i = threadIdx.x; i < 3 * Ny; i += blockDim.x) {
    const int c = i / Ny, ky = i - c * Ny;
    A[c * S + ky] = a.jhat ? jhx[c * M + (int64_t)ky * Nxh + kx] : mk((T)0, (T)0);
  }
  __syncthreads();
  cplx<T>* Z = lds_fft(A, B, tl, Ny, 3, twy, false, S);
  cplx<T>* W = Z == A ? B : A;
  for (int ky = threadIdx.x; ky < Ny; ky += blockDim.x) {
    const cplx<T> jh[3] = {Z[ky], Z[S + ky], Z[2 * S + ky]};
    cplx<T> out[6];
    mz_node_mode(a, (int64_t)ky * Nxh + kx, jh, out);
#pragma unroll
    for (int q = 0; q < 6; ++q) W[q * S + ky] = out[q];
  }
  __syncthreads();
  cplx<T>* R = lds_fft(W, Z, tl, Ny, 6, twy, true, S);
  const T sc = (T)1 / (T)Ny;
  for (int i = threadIdx.x; i < 6 * Ny; i += blockDim.x) {
    const int q = i / Ny, ky = i - q * Ny;
    a.out[q][(int64_t)ky * Nxh + kx] = sc * R[q * S + ky];
  }
}

// ---------------------------------------------------------------------------
// A batch of ppc_x x ppc_y fresh particles per transverse cell at one zeta
// (cell iz, offset oz), in (j, i, sy, sx) order: offsets from SplitMix64 on
// the counter ((((row + 2^20) Ny + j) Nx + i) ppc_y + sy) ppc_x + sx) * 2
// (+1 for y), or cell centres (quiet); weight n(r_perp) h_x h_y Delta /
// (ppc_x ppc_y) with the Gaussian channel n_e [1 + (ratio - 1) exp(-r^2/R^2)]
// about the axis (Nx/2, Ny/2); u = 0; budget b0; ids id0 + index.
struct MzBatchArgs {
  Geom g;
  int ppcx, ppcy, quiet;
  uint64_t key;
  int64_t row;
  int iz;
  double oz;
  double n_e, ratio, R, Delta, b0;
  int base;            // first slot in the destination
  int64_t id0;
  int capacity;
  int* err;
};

template <typename T>
__global__ __launch_bounds__(256) void k_mz_batch(MzBatchArgs a, MzParts<T> P) {
  const Geom& g = a.g;
  const int64_t nb = (int64_t)g.Ny * g.Nx * a.ppcy * a.ppcx;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb) return;
  const int sx = (int)(idx % a.ppcx);
  int64_t r = idx / a.ppcx;
  const int sy = (int)(r % a.ppcy);
  r /= a.ppcy;
  const int i = (int)(r % g.Nx);
  const int j = (int)(r / g.Nx);
  double xi_x = 0.5, xi_y = 0.5;
  if (!a.quiet) {
    uint64_t c = (((((uint64_t)(a.row + (1ll << 20)) * (uint64_t)g.Ny + (uint64_t)j) * (uint64_t)g.Nx +
                    (uint64_t)i) * (uint64_t)a.ppcy + (uint64_t)sy) * (uint64_t)a.ppcx + (uint64_t)sx) * 2ull;
    xi_x = sm_uniform(a.key, c);
    xi_y = g.dims == 3 ? sm_uniform(a.key, c + 1ull) : 0.0;
  }
  const double dx = ((double)sx + xi_x) / (double)a.ppcx;
  const double dy = g.dims == 3 ? ((double)sy + xi_y) / (double)a.ppcy : 0.0;
  double dens = a.n_e;
  if (!(a.ratio == 1.0 || a.R <= 0.0)) {
    const double X = ((double)i + dx) * g.hx, Y = ((double)j + dy) * g.hy;
    const double x = X - (double)(g.Nx / 2) * g.hx;
    const double y = g.dims == 3 ? Y - (double)(g.Ny / 2) * g.hy : 0.0;
    dens = a.n_e * (1.0 + (a.ratio - 1.0) * exp(-(x * x + y * y) / (a.R * a.R)));
  }
  const double hy_eff = g.dims == 3 ? g.hy : 1.0;
  const double w = dens * g.hx * hy_eff * a.Delta / (double)(a.ppcx * a.ppcy);
  const int64_t s = (int64_t)a.base + idx;
  if (s >= a.capacity) { atomicOr(a.err, ERR_CAPACITY); return; }
  const int cell = (a.iz * g.Ny + (g.dims == 3 ? j : 0)) * g.Nx + i;
  mz_store<T>(P, (int)s, cell, (T)dx, (T)dy, (T)a.oz, (T)0, (T)0, (T)0, (T)w, (T)a.b0, a.id0 + idx);
}

// step start: the parked particles' budgets gain Delta; counters of the
// first stage and of the step are set
template <typename T>
__global__ void k_mz_begin(MzParts<T> park, const int* park_total, int capacity, T Delta, int* act_first,
                           int first_count, int* act_next, int* stop_count, int* left_count) {
  const int n = min(*park_total, capacity);
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x))
    park.b[i] = park.b[i] + Delta;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *act_first = first_count;
    *act_next = 0;
    *stop_count = 0;
    *left_count = 0;
  }
}

// stopped particles -> parked store sorted by cell along zeta: counts, scan,
// scatter (order within a cell is that of the atomics)
__global__ void k_mz_count(const int32_t* cell, const int* count, int capacity, int nxy, int* pcount) {
  const int n = min(*count, capacity);
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x))
    atomicAdd(&pcount[cell[i] / nxy], 1);
}

__global__ __launch_bounds__(1024) void k_mz_scan(const int* pcount, int Nz, int* pstart, int* cursor,
                                                  int* park_total) {
  __shared__ int part[1024];
  const int per = (Nz + 1023) / 1024;
  const int t = threadIdx.x;
  int s = 0;
  for (int k = 0; k < per; ++k) {
    const int c = t * per + k;
    if (c < Nz) s += pcount[c];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int k = 0; k < per; ++k) {
    const int c = t * per + k;
    if (c < Nz) {
      pstart[c] = run;
      cursor[c] = run;
      run += pcount[c];
    }
  }
  if (t == 1023) *park_total = part[1023];
}

template <typename T>
__global__ void k_mz_scatter(MzParts<T> src, const int* count, int capacity, int nxy, int* cursor,
                             MzParts<T> dst) {
  const int n = min(*count, capacity);
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x)) {
    const int c = src.cell[i];
    const int pos = atomicAdd(&cursor[c / nxy], 1);
    mz_store<T>(dst, pos, c, src.ox[i], src.oy[i], src.oz[i], src.ux[i], src.uy[i], src.uz[i], src.w[i],
                src.b[i], src.id ? src.id[i] : 0);
  }
}

// FP64 sum of the weights of the parked particles (diagnostics)
template <typename T>
__global__ __launch_bounds__(256) void k_mz_wsum(const T* w, const int* count, double* out) {
  __shared__ double sh[256];
  const int n = *count;
  double s = 0.0;
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x))
    s += (double)w[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// field energy partial sums: sum over the nodes n < Nz of hnode[n] times the
// squares of the six components (block b takes a contiguous slice of nodes)
template <typename T>
__global__ __launch_bounds__(256) void k_mz_energy(const T* F6, const double* hnode, int Nz, int64_t nxy,
                                                   double* partial) {
  __shared__ double sh[4];
  const int64_t n_rec = (int64_t)Nz * nxy;
  const int64_t per = (n_rec + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n_rec, i0 + per);
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double r = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = (double)F6[i * 6 + c];
      r += v * v;
    }
    s += hnode[i / nxy] * r;
  }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Witness-bunch sums (Table 1 style): over the particles with gamma >=
// gamma_min, weighted by their electrons w, the 16 sums
//   W, W g, W g^2, W x, W x^2, W y, W y^2, W z, W z^2,
//   W ux, W ux^2, W x ux, W uy, W uy^2, W y uy, count
// with x, y measured from the axis node (Nx/2, Ny/2) and z = zeta.  The
// positions come from cell + offset: along zeta (iz + oz) h in the tau
// scheme, zn[iz] + oz (zn[iz + 1] - zn[iz]) in the zeta march.  Weights: the
// march's per-particle w, else w_plasma or (GEMPIC_BEAM_BIT) w_beam.
#define BUNCH_NS 16
template <typename T>
struct BunchArgs {
  Geom g;
  const int* count32;       // march: parked count (nullable)
  const int64_t* count64;   // tau: particles in the buffer (nullable)
  int capacity;
  const int32_t* cell;
  const T *ox, *oy, *oz, *ux, *uy, *uz;
  const T* w;               // nullable (tau scheme)
  double w_plasma, w_beam;
  const double* zn;         // nullable (tau scheme)
  double gamma_min;
  double* partial;          // [gridDim][BUNCH_NS]
};

template <typename T>
__global__ __launch_bounds__(256) void k_bunch(BunchArgs<T> a) {
  __shared__ double sh[4];
  const Geom& g = a.g;
  int64_t n = a.count32 ? (int64_t)*a.count32 : *a.count64;
  n = min(n, (int64_t)a.capacity);
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  double s[BUNCH_NS];
#pragma unroll
  for (int k = 0; k < BUNCH_NS; ++k) s[k] = 0.0;
  const double xa = (double)(g.Nx / 2) * g.hx, ya = (double)(g.Ny / 2) * g.hy;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double ux = (double)a.ux[i], uy = (double)a.uy[i], uz = (double)a.uz[i];
    const double gm = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    if (!(gm >= a.gamma_min)) continue;
    int c = a.cell[i];
    double w;
    if (a.w) {
      w = (double)a.w[i];
    } else {
      w = (c & GEMPIC_BEAM_BIT) ? a.w_beam : a.w_plasma;
      c &= ~GEMPIC_BEAM_BIT;
    }
    const int ix = c % g.Nx, iy = (c / g.Nx) % g.Ny, iz = c / (g.Nx * g.Ny);
    const double x = ((double)ix + (double)a.ox[i]) * g.hx - xa;
    const double y = g.dims == 3 ? ((double)iy + (double)a.oy[i]) * g.hy - ya : 0.0;
    const double z = a.zn ? a.zn[iz] + (double)a.oz[i] * (a.zn[iz + 1] - a.zn[iz])
                          : ((double)iz + (double)a.oz[i]) * g.h;
    const double v[BUNCH_NS] = {w,          w * gm,      w * gm * gm, w * x,      w * x * x,  w * y,
                                w * y * y,  w * z,       w * z * z,   w * ux,     w * ux * ux, w * x * ux,
                                w * uy,     w * uy * uy, w * y * uy,  1.0};
#pragma unroll
    for (int k = 0; k < BUNCH_NS; ++k) s[k] += v[k];
  }
  for (int k = 0; k < BUNCH_NS; ++k) {
    double t = block_sum(s[k], sh);
    if (threadIdx.x == 0) a.partial[blockIdx.x * BUNCH_NS + k] = t;
    __syncthreads();
  }
}
