// Particle kernels: loading, window injection, fused gather + push + deposit,
// and the stable tile sort.
//
// Particles are a structure of arrays: int32 linear cell (iz * Ny + iy) * Nx
// + ix, offsets ox, oy, oz in [0,1) and momenta ux, uy, uz (u = gamma v) in
// the precision T, optionally an int64 id.  They are kept sorted by tile
// (tiles of Tx x Ty x Tz cells, tile index (tz * nTy + ty) * nTx + tx), stable
// within a tile; each tile's range is cut into chunks of at most GP_CHUNK
// particles, one work-group per chunk.
#pragma once
#include "common.h"

template <typename T>
struct PartPtrs {
  int32_t* cell;
  T* ox;
  T* oy;
  T* oz;
  T* ux;
  T* uy;
  T* uz;
  int64_t* id;   // nullable
};

struct ChunkTab {
  int32_t* tile;    // [max_chunks] tile of each chunk
  int32_t* start;   // [max_chunks]
  int32_t* end;     // [max_chunks]
  int32_t* first;   // [NT] first chunk of each tile
  int32_t* count;   // [NT] chunks of each tile
  int32_t* n;       // [1] number of chunks
};

template <typename T> GP_DEV T one_minus();
template <> GP_DEV float one_minus<float>() { return 0x1.fffffep-1f; }
template <> GP_DEV double one_minus<double>() { return 0x1.fffffffffffffp-1; }

// Offset computed in FP64, stored in T; a value that rounds to 1 stays below.
template <typename T> GP_DEV T store_offset(double d) {
  T t = (T)d;
  return t < (T)1 ? t : one_minus<T>();
}

// An FP64 position in cell c rounded to FP32, then moved by single ulps until
// it decodes (abs_cell, unwrapped) to c: rounding never moves a new particle
// into another cell, and so never into another tile.
GP_DEV float place_abs(double pos, int c, float ih) {
  float x = (float)pos, off;
  while (abs_cell(x, ih, &off) > c) x = nextafterf(x, 0.0f);
  while (abs_cell(x, ih, &off) < c) x = nextafterf(x, 3.0e38f);
  return x;
}

// A new particle of cell (i, j, iz) at FP64 offsets (dx, dy, dz): cell word
// and offsets in T, or (g.abs_pos, FP32 only) the absolute position (place_abs);
// a staging buffer also keeps the cell.
template <typename T>
GP_DEV void put_particle(const PartPtrs<T>& P, int64_t o, const Geom& g, int i, int j, int iz,
                         double dx, double dy, double dz) {
  if (P.cell) P.cell[o] = (iz * g.Ny + j) * g.Nx + i;
  if (g.abs_pos) {
    P.ox[o] = (T)place_abs(((double)i + dx) * g.hx, i, g.ihx);
    if (g.dims == 3) P.oy[o] = (T)place_abs(((double)j + dy) * g.hy, j, g.ihy);
    P.oz[o] = (T)place_abs(((double)iz + dz) * g.h, iz, g.ih);
  } else {
    P.ox[o] = store_offset<T>(dx);
    if (g.dims == 3) P.oy[o] = store_offset<T>(dy);
    P.oz[o] = store_offset<T>(dz);
  }
  P.ux[o] = (T)0;
  P.uy[o] = (T)0;
  P.uz[o] = (T)0;
}

// ---------------------------------------------------------------------------
// Loading: every lattice particle of the full cells 0 .. Nzp - 2 of one tile,
// written at tile_base[t] in (m, j, i, sy, sx) order.  Sub-row m of lab z has
// particles at z offset (m % ppc_z + xi_z) / ppc_z in cell m / ppc_z.
struct LoadArgs {
  Geom g;
  int ppcx, ppcy, ppcz;
  int quiet;
  uint64_t key;
  const int64_t* tile_base;
};

template <typename T>
__global__ void k_load_full(LoadArgs a, PartPtrs<T> P) {
  const Geom& g = a.g;
  int t = blockIdx.x;
  int tx = t % g.nTx, ty = (t / g.nTx) % g.nTy, tz = t / (g.nTx * g.nTy);
  int x0 = tx * g.Tx, y0 = ty * g.Ty, z0 = tz * g.Tz;
  int zend = min(z0 + g.Tz, g.Nzp - 1);
  if (zend <= z0) return;
  int ppxy = a.ppcx * a.ppcy;
  int64_t m_first = (int64_t)z0 * a.ppcz;
  int64_t n_local = (int64_t)(zend - z0) * a.ppcz * g.Ty * g.Tx * ppxy;
  int64_t base = a.tile_base[t];
  for (int64_t l = threadIdx.x; l < n_local; l += blockDim.x) {
    int s = (int)(l % ppxy);
    int64_t r = l / ppxy;
    int il = (int)(r % g.Tx); r /= g.Tx;
    int jl = (int)(r % g.Ty); r /= g.Ty;
    int64_t m = m_first + r;
    int sx = s % a.ppcx, sy = s / a.ppcx;
    int i = x0 + il, j = y0 + jl;
    uint64_t gidx = ((((uint64_t)m * g.Ny + j) * g.Nx + i) * a.ppcy + sy) * a.ppcx + sx;
    double xix = a.quiet ? 0.5 : sm_uniform(a.key, gidx * 3 + 0);
    double xiz = a.quiet ? 0.5 : sm_uniform(a.key, gidx * 3 + 2);
    double dx = fmin(((double)sx + xix) / (double)a.ppcx, 0x1.fffffffffffffp-1);
    double dz = fmin(((double)(m % a.ppcz) + xiz) / (double)a.ppcz, 0x1.fffffffffffffp-1);
    double dy = 0.0;
    if (g.dims == 3) {
      double xiy = a.quiet ? 0.5 : sm_uniform(a.key, gidx * 3 + 1);
      dy = fmin(((double)sy + xiy) / (double)a.ppcy, 0x1.fffffffffffffp-1);
    }
    int iz = (int)(m / a.ppcz);
    int64_t o = base + l;
    put_particle<T>(P, o, g, i, j, iz, dx, dy, dz);
    if (P.id) P.id[o] = (int64_t)gidx;
  }
}

// ---------------------------------------------------------------------------
// Driver beam (sampled on the host in FP64, already in tile order): particle
// i goes to slot dst[i]; its cell word carries GEMPIC_BEAM_BIT.
struct BeamArgs {
  int64_t n;
  const int32_t* cell;
  const double* off;     // [3][n]
  const double* uz;
  const int64_t* dst;
  int64_t id0;           // id of beam particle 0
};

template <typename T>
__global__ void k_place_beam(BeamArgs a, PartPtrs<T> P, int dims) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int64_t o = a.dst[i];
  P.cell[o] = a.cell[i] | GEMPIC_BEAM_BIT;
  P.ox[o] = store_offset<T>(a.off[i]);
  if (dims == 3) P.oy[o] = store_offset<T>(a.off[a.n + i]);
  P.oz[o] = store_offset<T>(a.off[2 * a.n + i]);
  P.ux[o] = (T)0;
  P.uy[o] = (T)0;
  P.uz[o] = (T)a.uz[i];
  if (P.id) P.id[o] = a.id0 + i;
}

// Charge density q w_b / V of the beam on the field nodes n < Nz (linear
// weights from the FP64 offsets); rho is [Nz][Ny][Nx].
template <typename T>
__global__ void k_beam_rho(BeamArgs a, Geom g, double qv, T* rho) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int c = a.cell[i];
  int ix = c & (g.Nx - 1), iy = (c >> g.lnx) & (g.Ny - 1), iz = c >> (g.lnx + g.lny);
  double dx = a.off[i], dy = a.off[a.n + i], dz = a.off[2 * a.n + i];
  const double wx[2] = {1.0 - dx, dx}, wy[2] = {1.0 - dy, dy}, wz[2] = {1.0 - dz, dz};
  for (int cc = 0; cc < 2; ++cc) {
    int z = iz + cc;
    if (z >= g.Nz) continue;
    for (int b = 0; b < 2; ++b)
      for (int aa = 0; aa < 2; ++aa) {
        int x = (ix + aa) & (g.Nx - 1), y = (iy + b) & (g.Ny - 1);
        atomicAdd(rho + ((int64_t)z * g.Ny + y) * g.Nx + x, (T)(qv * ((wx[aa] * wy[b]) * wz[cc])));
      }
  }
}

// Cells of n particles with absolute FP32 positions (decoded as in the push).
__global__ void k_abs_cells(Geom g, const float* px, const float* py, const float* pz, int64_t n,
                            int32_t* cell) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float o;
  int ix = abs_cell(px[i], g.ihx, &o);
  if (ix >= g.Nx) ix -= g.Nx;
  int iy = g.dims == 3 ? abs_cell(py[i], g.ihy, &o) : 0;
  if (iy >= g.Ny) iy -= g.Ny;
  int iz = min(abs_cell(pz[i], g.ih, &o), g.Nzp - 1);
  cell[i] = iz < 0 ? -1 : (iz * g.Ny + iy) * g.Nx + ix;
}

// Driver-beam particles (cell words with GEMPIC_BEAM_BIT) among the first n.
__global__ __launch_bounds__(256) void k_count_beam(const int32_t* cell, const int64_t* n, unsigned long long* out) {
  __shared__ unsigned long long s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const int64_t N = *n;
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    int w = cell[i];
    c += (w >= 0 && (w & GEMPIC_BEAM_BIT)) ? 1ull : 0ull;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, s);
}

// ---------------------------------------------------------------------------
// Window batch b: lattice particles with lo <= z_m < hi (no lower bound for
// b = 0) among sub-rows m_lo .. m_hi, placed at zeta = z_m - b dtau in the
// entry cell.  One work-group per transverse tile; candidates in
// (m, j, i, sy, sx) order restricted to the tile, compacted with a block scan
// into the staging area of the tile.
struct InjArgs {
  Geom g;
  int ppcx, ppcy, ppcz;
  int quiet;
  uint64_t key;
  int b;              // batch index
  int64_t m_lo, m_hi;
  double lo, hi, hz, shift;   // thresholds, sub-row length, b * dtau
  int64_t stage_per_tile;
  int32_t* inj_count;   // [NT], written for the entry-row tiles
  int32_t* stage_g;     // [nTx * nTy * stage_per_tile] generation index
  int32_t* gflag;       // nullable: [Ny * Nx * ppc * nm] selection flags (ids)
};

template <typename T>
__global__ __launch_bounds__(256) void k_inject(InjArgs a, PartPtrs<T> S) {
  const Geom& g = a.g;
  __shared__ int wsum[8];
  __shared__ int running;
  int tt = blockIdx.x;                         // transverse tile index ty * nTx + tx
  int tx = tt % g.nTx, ty = tt / g.nTx;
  int x0 = tx * g.Tx, y0 = ty * g.Ty;
  int ppxy = a.ppcx * a.ppcy;
  int64_t nm = a.m_hi - a.m_lo + 1;
  int64_t ncand = nm * g.Ty * g.Tx * ppxy;
  int64_t sbase = (int64_t)tt * a.stage_per_tile;
  if (threadIdx.x == 0) running = 0;
  __syncthreads();
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t row = 0; row < ncand; row += blockDim.x) {
    int64_t l = row + threadIdx.x;
    bool sel = false;
    double dx = 0, dy = 0, dz = 0;
    int iz = 0, i = 0, j = 0;
    int64_t gidx = 0;
    if (l < ncand) {
      int s = (int)(l % ppxy);
      int64_t r = l / ppxy;
      int il = (int)(r % g.Tx); r /= g.Tx;
      int jl = (int)(r % g.Ty); r /= g.Ty;
      int64_t m = a.m_lo + r;
      int sx = s % a.ppcx, sy = s / a.ppcx;
      i = x0 + il;
      j = y0 + jl;
      uint64_t lat = ((((uint64_t)m * g.Ny + j) * g.Nx + i) * a.ppcy + sy) * a.ppcx + sx;
      double xiz = a.quiet ? 0.5 : sm_uniform(a.key, lat * 3 + 2);
      double z = ((double)m + xiz) * a.hz;
      sel = z < a.hi && (a.b == 0 || z >= a.lo);
      gidx = ((r * g.Ny + j) * g.Nx + i) * ppxy + s;
      if (a.gflag) a.gflag[gidx] = sel ? 1 : 0;
      if (sel) {
        double xix = a.quiet ? 0.5 : sm_uniform(a.key, lat * 3 + 0);
        dx = fmin(((double)sx + xix) / (double)a.ppcx, 0x1.fffffffffffffp-1);
        if (g.dims == 3) {
          double xiy = a.quiet ? 0.5 : sm_uniform(a.key, lat * 3 + 1);
          dy = fmin(((double)sy + xiy) / (double)a.ppcy, 0x1.fffffffffffffp-1);
        }
        double zeta = z - a.shift;
        double sz = zeta / g.h;
        double fz = floor(sz);
        dz = sz - fz;
        iz = (int)fz;
        if (iz < g.Nzp - 1) { iz = g.Nzp - 1; dz = 0.0; }
      }
    }
    // block-wide exclusive scan of sel, in candidate order
    uint64_t bal = __ballot(sel);
    int wrank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int off = running;
    for (int w = 0; w < wid; ++w) off += wsum[w];
    if (sel) {
      int64_t o = sbase + off + wrank;
      put_particle<T>(S, o, g, i, j, iz, dx, dy, dz);
      a.stage_g[o] = (int32_t)gidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wsum[w];
      running += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int t = ((g.nTz - 1) * g.nTy + ty) * g.nTx + tx;
    a.inj_count[t] = running;
  }
}

#include "push.h"

// ---------------------------------------------------------------------------
// Stable sort by tile, step 1: destination code and rank of every particle of
// a chunk among the chunk's particles with the same code (array order).
GP_DEV int tile_step(int src, int dst, int n) {
  // step from source to destination tile index along a periodic axis of n tiles
  int d = dst - src;
  if (d < 0) d += n;
  if (d == 0) return 0;
  if (d == 1) return 1;
  if (d == n - 1) return -1;
  return 99;
}

struct SortArgs {
  Geom g;
  ChunkTab ct;
  const int32_t* cell;     // null with absolute positions: cells from px, py, pz
  const float* px;
  const float* py;
  const float* pz;
  int32_t* code;        // [N] code << 24 | rank
  int32_t* counts;      // [max_chunks * NCODE]
  int* err;
};

// One wavefront per chunk, no barriers: the codes of all rows of 64
// particles first (their loads in flight together), then the rows in order.
// Lane k < NCODE keeps the number of earlier particles with code k, so a
// particle's rank is that count plus the same-code lanes below it.
__global__ __launch_bounds__(64) void k_sort_rank(SortArgs a) {
  const Geom& g = a.g;
  int c = blockIdx.x;
  if (c >= *a.ct.n) return;
  int t = a.ct.tile[c];
  int p0 = a.ct.start[c], p1 = a.ct.end[c];
  int tx = t % g.nTx, ty = (t / g.nTx) % g.nTy, tz = t / (g.nTx * g.nTy);
  const int lane = threadIdx.x;
  constexpr int NR = GP_CHUNK / 64;
  static_assert(GP_CHUNK % 64 == 0, "chunks are whole rows of 64");
  if (p1 - p0 > GP_CHUNK) {                 // the chunk table never builds these
    if (lane == 0) atomicOr(a.err, ERR_TILE);
    return;
  }
  if (p1 <= p0) {
    if (lane < NCODE) a.counts[c * NCODE + lane] = 0;
    return;
  }
  // cells of every row first: unconditional loads (lanes past the chunk
  // read its first particle), so that all of them are in flight together
  int cellv[NR];
  if (a.cell) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int p = p0 + r * 64 + lane;
      cellv[r] = a.cell[p < p1 ? p : p0];
    }
  } else {
    float xs[NR], ys[NR], zs[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int p = p0 + r * 64 + lane, q = p < p1 ? p : p0;
      xs[r] = a.px[q];
      ys[r] = g.dims == 3 ? a.py[q] : 0.0f;
      zs[r] = a.pz[q];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      float o;
      int ix = abs_cell(xs[r], g.ihx, &o);
      if (ix >= g.Nx) ix -= g.Nx;
      int iy = g.dims == 3 ? abs_cell(ys[r], g.ihy, &o) : 0;
      if (iy >= g.Ny) iy -= g.Ny;
      int iz = min(abs_cell(zs[r], g.ih, &o), g.Nzp - 1);
      cellv[r] = iz < 0 ? -1 : (iz * g.Ny + iy) * g.Nx + ix;
    }
  }
  int code[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int p = p0 + r * 64 + lane;
    code[r] = -1;
    if (p < p1) {
      int cell = cellv[r];
      if (cell < 0) {
        code[r] = CODE_REMOVED;
      } else {
        cell &= ~GEMPIC_BEAM_BIT;
        // power-of-two grid and tile sizes: shifts and masks
        int ix = cell & (g.Nx - 1);
        int iy = (cell >> g.lnx) & (g.Ny - 1);
        int iz = cell >> (g.lnx + g.lny);
        int sx = tile_step(tx, ix >> (__ffs(g.Tx) - 1), g.nTx);
        int sy = tile_step(ty, iy >> (__ffs(g.Ty) - 1), g.nTy);
        int sz = (iz >> (__ffs(g.Tz) - 1)) - tz;
        if (sx == 99 || sy == 99 || sz < -1 || sz > 0) {
          atomicOr(a.err, ERR_TILE);
          code[r] = CODE_REMOVED;
        } else {
          code[r] = (sz + 1) * 9 + (sy + 1) * 3 + (sx + 1);
        }
      }
    }
  }
  const uint64_t lt = (1ull << lane) - 1ull;
  int run = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (p0 + r * 64 >= p1) break;
    const int cd = code[r];
    int myrank = 0, add = 0;
    uint64_t active = __ballot(cd >= 0);
    while (active) {
      int leader = __ffsll((unsigned long long)active) - 1;
      int lc = __shfl(cd, leader);
      uint64_t m = __ballot(cd == lc);
      if (cd == lc) myrank = __popcll(m & lt);
      if (lane == lc) add = __popcll(m);
      active &= ~m;
    }
    const int base = __shfl(run, cd < 0 ? 0 : cd);
    if (cd >= 0) a.code[p0 + r * 64 + lane] = (cd << 24) | (base + myrank);
    run += add;
  }
  if (lane < NCODE) a.counts[c * NCODE + lane] = run;
}

// Step 2: per destination tile, offsets of every (source chunk, code) group in
// array order (source tiles ascending, chunks ascending), then the injected
// particles; writes the new tile counts.
struct OffArgs {
  Geom g;
  ChunkTab ct;              // old chunk table
  const int32_t* counts;    // [chunks * NCODE]
  int32_t* offs;            // [chunks * NCODE]
  const int32_t* inj_count; // [NT]
  int32_t* inj_off;         // [NT]
  int64_t* tile_count;      // [NT]
};

// Three destination tiles per wavefront, 18 lanes each (lanes 54 .. 63
// idle): lane i of tile t's group takes the step (sz, sy, sx) =
// (-(i / 9), (i % 9) / 3 - 1, i % 3 - 1) from source tile t - step; a step is
// kept only if it is the canonical step between the two tiles (small
// periodic grids reach one source by several steps).  The sources'
// particles follow each other in increasing source index.
constexpr int OFF_TPW = 3;                    // tiles per wavefront

__global__ __launch_bounds__(256) void k_tile_offsets(OffArgs a) {
  const Geom& g = a.g;
  const int lane = threadIdx.x & 63;
  const int grp = lane / 18, i = lane - grp * 18, g0 = grp * 18;
  const int t = (blockIdx.x * 4 + (threadIdx.x >> 6)) * OFF_TPW + grp;
  const bool own = grp < OFF_TPW && t < g.NT;
  const int tx = t % g.nTx, ty = (t / g.nTx) % g.nTy, tz = t / (g.nTx * g.nTy);
  int valid = 0, src = 0, cod = 0;
  if (own) {
    const int sz = -(i / 9), sy = (i % 9) / 3 - 1, sx = i % 3 - 1;
    const int szr = tz - sz;
    if (szr < g.nTz) {
      int sxt = tx - sx; sxt = ((sxt % g.nTx) + g.nTx) % g.nTx;
      int syt = ty - sy; syt = ((syt % g.nTy) + g.nTy) % g.nTy;
      if (tile_step(sxt, tx, g.nTx) == sx && tile_step(syt, ty, g.nTy) == sy) {
        valid = 1;
        src = (szr * g.nTy + syt) * g.nTx + sxt;
        cod = (sz + 1) * 9 + (sy + 1) * 3 + (sx + 1);
      }
    }
  }
  int f = 0, n = 0;
  if (valid) {
    f = a.ct.first[src];
    n = a.ct.count[src];
  }
  long long tot = 0;                          // this source's particles for t
  for (int k = 0; k < n; ++k) tot += a.counts[(f + k) * NCODE + cod];
  long long pre = 0, all = 0;                 // sources below this one; all sources
  for (int j = 0; j < 18; ++j) {
    const int vj = __shfl(valid, g0 + j);
    const int sj = __shfl(src, g0 + j);
    const long long tj = __shfl(tot, g0 + j);
    if (vj) {
      all += tj;
      if (sj < src) pre += tj;
    }
  }
  if (valid) {
    long long run = pre;
    for (int k = 0; k < n; ++k) {
      const int ci = (f + k) * NCODE + cod;
      a.offs[ci] = (int32_t)run;
      run += a.counts[ci];
    }
  }
  if (own && i == 0) {
    a.inj_off[t] = (int32_t)all;
    a.tile_count[t] = all + a.inj_count[t];
  }
}

// Step 3: exclusive scans of the tile counts (-> tile_base, total) and of the chunk
// counts per tile (-> ch_first, ch_count, nchunks) in three kernels: sums of
// SCAN_PER tiles per block, a single-block scan of those sums (with the
// capacity check), and the per-block scans offset by it.
#define SCAN_PER 4096
#define SCAN_MAXB 1024

// in-place inclusive scan of two 1024-entry LDS arrays (all 1024 threads)
GP_DEV void block_scan2(int64_t* sa, int64_t* sb) {
  int tid = threadIdx.x;
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t va = tid >= o ? sa[tid - o] : 0;
    int64_t vb = tid >= o ? sb[tid - o] : 0;
    __syncthreads();
    sa[tid] += va;
    sb[tid] += vb;
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void k_scan_tiles_sum(int NT, const int64_t* tile_count, int64_t* part) {
  __shared__ int64_t sa[1024];
  __shared__ int64_t sb[1024];
  int tid = threadIdx.x;
  int i0 = blockIdx.x * SCAN_PER, i1 = min(NT, i0 + SCAN_PER);
  int64_t s1 = 0, s2 = 0;
  for (int i = i0 + tid; i < i1; i += 1024) {
    int64_t n = tile_count[i];
    s1 += n;
    s2 += (n + GP_CHUNK - 1) / GP_CHUNK;
  }
  sa[tid] = s1;
  sb[tid] = s2;
  __syncthreads();
  block_scan2(sa, sb);
  if (tid == 1023) {
    part[2 * blockIdx.x] = sa[1023];
    part[2 * blockIdx.x + 1] = sb[1023];
  }
}

__global__ __launch_bounds__(1024) void k_scan_tiles_top(int nb, int64_t* part, int64_t* total, int32_t* nchunks,
                                                         int64_t capacity, int* err) {
  __shared__ int64_t sa[1024];
  __shared__ int64_t sb[1024];
  int tid = threadIdx.x;
  int64_t a = tid < nb ? part[2 * tid] : 0, b = tid < nb ? part[2 * tid + 1] : 0;
  sa[tid] = a;
  sb[tid] = b;
  __syncthreads();
  block_scan2(sa, sb);
  if (tid < nb) {
    part[2 * tid] = sa[tid] - a;          // exclusive offsets
    part[2 * tid + 1] = sb[tid] - b;
  }
  if (tid == 1023) {
    *total = sa[1023];
    *nchunks = (int32_t)sb[1023];
    // over capacity: no chunk is processed any more (the error is reported)
    if (sa[1023] > capacity) { atomicOr(err, ERR_CAPACITY); *nchunks = 0; *total = 0; }
  }
}

__global__ __launch_bounds__(1024) void k_scan_tiles_apply(int NT, const int64_t* tile_count, const int64_t* part,
                                                           int64_t* tile_base, int32_t* ch_first,
                                                           int32_t* ch_count) {
  __shared__ int64_t sa[1024];
  __shared__ int64_t sb[1024];
  constexpr int PER = SCAN_PER / 1024;
  int tid = threadIdx.x;
  int i0 = blockIdx.x * SCAN_PER + tid * PER;
  int64_t n[PER];
  int64_t s1 = 0, s2 = 0;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    n[r] = i0 + r < NT ? tile_count[i0 + r] : 0;
    s1 += n[r];
    s2 += (n[r] + GP_CHUNK - 1) / GP_CHUNK;
  }
  sa[tid] = s1;
  sb[tid] = s2;
  __syncthreads();
  block_scan2(sa, sb);
  int64_t r1 = part[2 * blockIdx.x] + sa[tid] - s1;
  int64_t r2 = part[2 * blockIdx.x + 1] + sb[tid] - s2;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (i0 + r >= NT) break;
    int nc = (int)((n[r] + GP_CHUNK - 1) / GP_CHUNK);
    tile_base[i0 + r] = r1;
    ch_first[i0 + r] = (int32_t)r2;
    ch_count[i0 + r] = nc;
    r1 += n[r];
    r2 += nc;
  }
}

// Step 4: chunk table of the sorted array.
__global__ void k_build_chunks(int NT, const int64_t* tile_base, const int64_t* tile_count,
                               ChunkTab ct, int max_chunks) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NT) return;
  int f = ct.first[t], n = ct.count[t];
  int64_t b = tile_base[t], e = b + tile_count[t];
  for (int k = 0; k < n; ++k) {
    int c = f + k;
    if (c >= max_chunks) return;
    ct.tile[c] = t;
    ct.start[c] = (int32_t)(b + (int64_t)k * GP_CHUNK);
    ct.end[c] = (int32_t)min(e, b + (int64_t)(k + 1) * GP_CHUNK);
  }
}

// Step 5: scatter the chunk's particles to their sorted positions.
template <typename T>
struct ScatArgs {
  Geom g;
  ChunkTab ct;              // old chunk table
  const int32_t* code;
  const int32_t* offs;
  const int64_t* tile_base; // new
  int64_t capacity;
  int* err;
};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_scatter(ScatArgs<T> a, PartPtrs<T> A, PartPtrs<T> B) {
  const Geom& g = a.g;
  int c = blockIdx.x;
  if (c >= *a.ct.n) return;
  int t = a.ct.tile[c];
  int p0 = a.ct.start[c], p1 = a.ct.end[c];
  int tx = t % g.nTx, ty = (t / g.nTx) % g.nTy, tz = t / (g.nTx * g.nTy);
  // the chunk's rows of 256 in phases (codes, destinations, loads, stores),
  // so that each phase's memory operations are in flight together
  constexpr int R = GP_CHUNK / 256;
  static_assert(GP_CHUNK % 256 == 0, "chunks are whole rows of 256");
  int64_t o[R];
  if (p1 <= p0) return;
  // rows that hold particles (uniform): no loads for the empty ones
  const int nrow = (p1 - p0 + 255) / 256;
  int crv[R];                               // codes of every row, loads in flight together
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = p0 + r * 256 + (int)threadIdx.x;
    crv[r] = r < nrow ? a.code[p < p1 ? p : p0] : (CODE_REMOVED << 24);
  }
  // destinations: the tile base and chunk offset loads of every row in flight
  // together (rows without a destination read those of the staying code)
  int64_t tbv[R];
  int ofv[R], rkv[R];
  bool okv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = p0 + r * 256 + (int)threadIdx.x;
    const int cr = crv[r];
    const int code0 = cr >> 24;
    okv[r] = p < p1 && code0 != CODE_REMOVED;
    const int code = okv[r] ? code0 : 13;   // 13: the staying code
    rkv[r] = cr & 0xFFFFFF;
    int sz = code / 9 - 1, sy = (code / 3) % 3 - 1, sx = code % 3 - 1;
    int dx = tx + sx; if (dx < 0) dx += g.nTx; if (dx >= g.nTx) dx -= g.nTx;
    int dy = ty + sy; if (dy < 0) dy += g.nTy; if (dy >= g.nTy) dy -= g.nTy;
    int dz = tz + sz;
    int dt = (dz * g.nTy + dy) * g.nTx + dx;
    tbv[r] = r < nrow ? a.tile_base[dt] : 0;
    ofv[r] = r < nrow ? a.offs[c * NCODE + code] : 0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) o[r] = okv[r] ? tbv[r] + ofv[r] + rkv[r] : -1;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (o[r] >= a.capacity) {
      atomicOr(a.err, ERR_CAPACITY);
      o[r] = -1;
    }
  // particle rows: unconditional loads (rows without a destination read the
  // chunk's first particle), stores only where there is a destination
  int32_t cell[R];
  T ox[R], oy[R], oz[R], ux[R], uy[R], uz[R];
  int64_t id[R];
  const bool hasc = B.cell != nullptr, hasid = B.id != nullptr;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r >= nrow) break;
    const int p = o[r] >= 0 ? p0 + r * 256 + (int)threadIdx.x : p0;
    cell[r] = hasc ? A.cell[p] : 0;
    ox[r] = A.ox[p];
    oy[r] = DIM == 3 ? A.oy[p] : (T)0;
    oz[r] = A.oz[p];
    ux[r] = A.ux[p];
    uy[r] = A.uy[p];
    uz[r] = A.uz[p];
    id[r] = hasid ? A.id[p] : 0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (o[r] < 0) continue;
    const int64_t q = o[r];
    if (B.cell) B.cell[q] = cell[r];
    B.ox[q] = ox[r];
    if (DIM == 3) B.oy[q] = oy[r];
    B.oz[q] = oz[r];
    B.ux[q] = ux[r];
    B.uy[q] = uy[r];
    B.uz[q] = uz[r];
    if (B.id) B.id[q] = id[r];
  }
}

// Step 6: staged window particles after every particle already in their tile.
struct InjCopyArgs {
  Geom g;
  const int32_t* inj_count;  // [NT]
  const int32_t* inj_off;    // [NT]
  const int64_t* tile_base;
  int64_t stage_per_tile;
  const int32_t* stage_g;
  const int32_t* grank;      // nullable: exclusive scan of the generation flags
  const int64_t* next_id;    // nullable
  int64_t capacity;
  int* err;
};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_inject_copy(InjCopyArgs a, PartPtrs<T> S, PartPtrs<T> B) {
  const Geom& g = a.g;
  int tt = blockIdx.x;
  int tx = tt % g.nTx, ty = tt / g.nTx;
  int t = ((g.nTz - 1) * g.nTy + ty) * g.nTx + tx;
  int n = a.inj_count[t];
  int64_t sb = (int64_t)tt * a.stage_per_tile;
  int64_t db = a.tile_base[t] + a.inj_off[t];
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    int64_t s = sb + k, o = db + k;
    if (o >= a.capacity) { atomicOr(a.err, ERR_CAPACITY); continue; }
    if (B.cell) B.cell[o] = S.cell[s];
    B.ox[o] = S.ox[s];
    if (DIM == 3) B.oy[o] = S.oy[s];
    B.oz[o] = S.oz[s];
    B.ux[o] = S.ux[s];
    B.uy[o] = S.uy[s];
    B.uz[o] = S.uz[s];
    if (B.id) B.id[o] = *a.next_id + a.grank[a.stage_g[s]];
  }
}

// Exclusive scan of int32 flags (single work-group), total added to *acc.
__global__ __launch_bounds__(1024) void k_scan_flags(int64_t n, const int32_t* in, int32_t* out,
                                                     int64_t* acc_total) {
  __shared__ int64_t sa[1024];
  int tid = threadIdx.x;
  int64_t per = (n + 1023) / 1024;
  int64_t i0 = tid * per, i1 = min(n, i0 + per);
  int64_t s = 0;
  for (int64_t i = i0; i < i1; ++i) s += in[i];
  sa[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t v = tid >= o ? sa[tid - o] : 0;
    __syncthreads();
    sa[tid] += v;
    __syncthreads();
  }
  int64_t r = tid ? sa[tid - 1] : 0;
  for (int64_t i = i0; i < i1; ++i) {
    int32_t v = in[i];
    out[i] = (int32_t)r;
    r += v;
  }
  __syncthreads();
  if (tid == 1023 && acc_total) *acc_total += sa[1023];
}
