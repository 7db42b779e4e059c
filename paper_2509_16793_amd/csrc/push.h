// Fused gather + push + move + deposit.  A work-group walks a segment of a
// column of tiles (fixed transverse tile, increasing zeta tile) and takes
// every particle of each tile in one pass.  Particles only move towards -zeta
// (at most one cell), so the current planes a tile shares with the next tile
// of the column stay in LDS and only the planes no later tile touches are
// flushed; the last node plane of the field tile is likewise carried over.
//
// Gather: linear (CIC) weights on the 8 (3-D) / 4 (2-D) nodes around the
// particle, from an LDS copy of the tile's (T+1)^3 node records (E, B
// interleaved); zeta nodes >= Nz carry zero.
// Push: Higuera-Cary with eps = (q/m) dtau / 2.  Move: offsets advance by
// v dtau / h_axis, zeta by (v_z - 1) dtau / h with the cancellation-free
// v_z - 1; a cell step beyond one raises ERR_CFL, a non-finite momentum
// ERR_NUMERIC, and the particle is left unchanged.  Gather, push and move follow a fixed operation order without
// contraction beyond the fused multiply-adds written out (FP32 only), so FP64
// and FP32 results reproduce a reference bit for bit.
// Deposit: Esirkepov frame current W on the staggered grid plus the time- and
// zeta-centred charge for the lab J_z, accumulated in an LDS tile of
// (TX+3) x (TY+3) x (TZ+4) nodes per component (origin x0-1, y0-1, node z0-2),
// then added to the global arrays with one atomic per non-zero node.  The LDS
// tile holds 64-bit fixed-point integers: integer LDS atomics run tens of
// times faster than floating-point ones on gfx950, and the tile sums become
// exact and independent of the order of the atomics.  The scale is a power of
// two chosen on the host: a single contribution (bounded by the largest
// coefficient) truncates to an int32 at 2^-30 of that bound, so the 64-bit
// sums cannot overflow below 2^33 particles.  The FP64 mode (parity, not
// throughput) accumulates in FP64 LDS atomics instead, at full precision and
// without a range limit.
// A wave in which no particle crosses a transverse cell boundary takes a
// reduced stencil (2 x 2 transverse nodes, 28 instead of 72 contributions);
// the omitted terms are exactly zero.
#pragma once

template <typename T>
struct PushArgs {
  Geom g;
  const T* F6;         // node records [Nz][Ny][Nx][6]: Ex Ey Ez Bx By Bz
  T* J[3];             // [NPJ][Ny][Nx]
  T* rho0;             // nullable: charge before the move
  T* rho1;             // nullable: charge after the move
  T eps;               // (q/m) dtau / 2
  T ax, ay, az;        // dtau / hx, dtau / hy, dtau / h
  T cx, cy, cz;        // -q w / (dtau hy h), -q w / (dtau hx h), -q w / (dtau hx hy) (2-D: hy = 1)
  T cjy;               // 2-D out-of-plane: q w / (hx h)
  T crho;              // q w / V
  T rb;                // weight of a driver-beam particle over the plasma weight
  T dtau;              // slow step (absolute-position move)
  T fscale, finv;      // fixed-point scale of the LDS tile (power of two) and its inverse
  const int64_t* tile_base;   // [NT] first particle of each tile
  const int64_t* tile_count;  // [NT] particles of each tile
  const int64_t* total;       // particles in the buffer (0 after a capacity overflow)
  unsigned long long* Jfix[3]; // deterministic FP32 flush: 64-bit fixed-point current sums
  int seg_len;                // zeta tiles per work-group segment
  int nseg;                   // segments per column
  int* err;
};

template <typename T> struct Vec2;
template <> struct Vec2<float> { using t = float2; };
template <> struct Vec2<double> { using t = double2; };

// a * b + c: one fused multiply-add in FP32 (rounded once); product, then sum,
// in FP64.  The grouping of every sum of the push is the same in both.
template <typename T> GP_DEV T madd(T a, T b, T c);
template <> GP_DEV float madd<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> GP_DEV double madd<double>(double a, double b, double c) { return a * b + c; }

// accumulator of the LDS deposit tile
template <typename T> struct Fix;
template <> struct Fix<float> {
  // fixed point: a single contribution fits in int32 at the FP32 scale, the
  // sums in 64-bit two's complement (no overflow below 2^33 contributions)
  using t = unsigned long long;
  // truncation: the bias is below 2^-30 of the largest single contribution
  static GP_DEV unsigned long long to(float v) { return (unsigned long long)(long long)(int)v; }
  // sum -> value, within two ulp
  static GP_DEV float value(unsigned long long v) {
    float hi = (float)(int)(unsigned)(v >> 32);
    float lo = (float)(unsigned)(v & 0xFFFFFFFFull);
    return hi * 4294967296.0f + lo;
  }
};
// deterministic deposit: the 64-bit fixed-point node sums of one current
// component to FP32, converted as the ordinary flush converts a tile's sums
__global__ void k_fix_to_float(const unsigned long long* fix, float* J, int64_t n, float finv) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    J[i] = Fix<float>::value(fix[i]) * finv;
}

template <> struct Fix<double> {
  // FP64 (the parity mode): native FP64 LDS atomics, no range limit
  using t = double;
  static GP_DEV double to(double v) { return v; }
  static GP_DEV double value(double v) { return v; }
};

// value of lane - 1 (row_shr:1) / lane + 1 (row_shl:1) within a 16-lane DPP
// row; 0 at the row's edge
GP_DEV int dpp_from_left(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true); }
GP_DEV int dpp_from_right(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x101, 0xf, 0xf, true); }

// 3-node window starting at min(c0, c0 + k): old and new linear weights.
template <typename T>
GP_DEV void window3(int k, T d0, T d1, T* S0, T* S1) {
  int off0 = k < 0 ? 1 : 0;
  int off1 = k > 0 ? 1 : 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S0[a] = (a == off0 ? (T)1 - d0 : (T)0) + (a == off0 + 1 ? d0 : (T)0);
    S1[a] = (a == off1 ? (T)1 - d1 : (T)0) + (a == off1 + 1 ? d1 : (T)0);
  }
}

// particle state of one lane, loaded one row ahead of its use
template <typename T>
struct PLoad {
  int cell;
  T ox, oy, oz, ux, uy, uz;
};

// Particle rows go through buffer resources: a scalar base (the row's first
// particle) and a range of the row's particles, with the lane's byte offset
// as the only per-lane address part.  Lanes past the range read zero and
// their stores are dropped by the hardware range check.
template <int B> struct RowIO;
template <> struct RowIO<4> {
  template <typename Q> static GP_DEV Q ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(Q, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  }
  template <typename Q> static GP_DEV void st(Q v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
  }
};
template <> struct RowIO<8> {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  template <typename Q> static GP_DEV Q ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(Q, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  }
  template <typename Q> static GP_DEV void st(Q v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, 0, 0);
  }
};

template <typename Q>
GP_DEV __amdgpu_buffer_rsrc_t row_rsrc(Q* p, int base, int n) {
  // raw buffer (no stride), n elements; dword 3 = 32-bit data format on gfx9
  return __builtin_amdgcn_make_buffer_rsrc((void*)(p + base), (short)0, max(n, 0) * (int)sizeof(Q),
                                           0x00020000);
}
template <typename Q>
GP_DEV Q row_ld(Q* p, int base, int n, unsigned lane) {
  return RowIO<sizeof(Q)>::template ld<Q>(row_rsrc(p, base, n), lane * (unsigned)sizeof(Q));
}
template <typename Q>
GP_DEV void row_st(Q v, Q* p, int base, int n, unsigned lane) {
  RowIO<sizeof(Q)>::template st<Q>(v, row_rsrc(p, base, n), lane * (unsigned)sizeof(Q));
}

// the n particles base .. base + n - 1, one per lane (lanes >= n get zeros)
template <typename T, int DIM, bool ABS>
GP_DEV PLoad<T> load_row(const PartPtrs<T>& P, int base, int n, unsigned lane) {
  PLoad<T> s;
  // absolute positions: the offsets hold x, y, zeta and there is no cell word
  s.cell = ABS ? 0 : row_ld(P.cell, base, n, lane);
  s.ox = row_ld(P.ox, base, n, lane);
  s.oy = DIM == 3 ? row_ld(P.oy, base, n, lane) : (T)0;
  s.oz = row_ld(P.oz, base, n, lane);
  s.ux = row_ld(P.ux, base, n, lane);
  s.uy = row_ld(P.uy, base, n, lane);
  s.uz = row_ld(P.uz, base, n, lane);
  return s;
}

// SPEC: cell words may carry GEMPIC_BEAM_BIT (driver-beam particles, weight rb
// times the plasma weight); the bit is kept through the move.
// ABS: particles hold absolute FP32 positions; cells and offsets are decoded
// from them (abs_cell), the move adds v dtau to the position in FP32 (periodic
// wrap transversally) and the new cell and offset are decoded again.
// DET (FP32 only): the flush adds the tile's exact fixed-point sums to the
// 64-bit integer arrays Jfix with integer atomics instead of adding their
// FP32 values to J, so that no summation order reaches the current; a later
// pass converts Jfix to J.
template <typename T, int DIM, bool RHO, int TX, int TY, int TZ, int NTHR, bool SPEC, bool ABS, bool DET = false>
__global__ __launch_bounds__(NTHR) void k_push_deposit(PushArgs<T> a, PartPtrs<T> P) {
  static_assert(!DET || std::is_same<T, float>::value, "the deterministic flush needs the fixed-point tile");
  constexpr int FX = TX + 1, FY = DIM == 3 ? TY + 1 : 1, FZ = TZ + 1;
  constexpr int FN = FX * FY * FZ;
  // current tile: J_x and J_y on planes 1 .. JZ-1, J_z on planes 0 .. JZ-1
  // (plane jz = node z0 + jz - 2); slab q starts at JOFF(q) and holds plane
  // JFIRST(q) first
  constexpr int JX = TX + 3, JY = DIM == 3 ? TY + 3 : 1, JZ = TZ + 4;
  constexpr int JP = JX * JY;                     // entries per plane
  constexpr int JN = JP * (3 * JZ - 2);           // all three slabs
  constexpr int RX = TX + 3, RY = DIM == 3 ? TY + 3 : 1, RZ = TZ + 2;
  constexpr int RN = RX * RY * RZ;
  constexpr int SJ = JN + (RHO ? 2 * RN : 0);
  using A = typename Fix<T>::t;
  // one LDS block, field tile first: the gather's node offsets stay small
  // enough for immediate LDS offsets
  constexpr int NF8 = (6 * FN * (int)sizeof(T) + 15) / 16 * 2;
  __shared__ __align__(16) A smem[NF8 + SJ];
  T* const sF = reinterpret_cast<T*>(smem);
  A* const sJ = smem + NF8;
  using V2 = typename Vec2<T>::t;

  const Geom& g = a.g;
  // work item: XCD-major so that the blocks one XCD runs are neighbouring columns
  const int ncol = g.nTx * g.nTy;
  const int nitem = ncol * a.nseg;
  const int per_xcd = (nitem + 7) / 8;
  const int item = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (item >= nitem) return;
  // segments from the front of the box backwards: the laser or a driver,
  // whose tiles hold the most work, sit near the front and start first
  const int segi = item / ncol, colm = item - segi * ncol;
  const int seg = a.nseg - 1 - segi;
  const int tx = colm % g.nTx, ty = colm / g.nTx;
  const int tz0 = seg * a.seg_len, tz1 = min(g.nTz, tz0 + a.seg_len);
  if (tz0 >= tz1) return;
  const int x0 = tx * TX, y0 = ty * TY;
  const int64_t ntot = *a.total;
  const int mx = g.Nx - 1, my = g.Ny - 1;
  const int64_t plane_stride = (int64_t)g.Ny * g.Nx;

  for (int idx = threadIdx.x; idx < SJ; idx += NTHR) sJ[idx] = (A)0;

  // particle range of a tile of this column
  auto range = [&](int tzz, int* q0, int* q1) {
    const int tt = (tzz * g.nTy + ty) * g.nTx + tx;
    const int64_t pb = a.tile_base[tt];
    // uniform values: kept in scalar registers, so that row addresses are
    // scalar bases plus the lane offset
    *q0 = __builtin_amdgcn_readfirstlane((int)min(pb, ntot));
    *q1 = __builtin_amdgcn_readfirstlane((int)min(pb + a.tile_count[tt], ntot));
  };
  int p0, p1;
  range(tz0, &p0, &p1);
  // the next row's particles are loaded while the current row is processed
  const unsigned lane = threadIdx.x;
  PLoad<T> nxt = load_row<T, DIM, ABS>(P, p0, p1 - p0, lane);

  for (int tz = tz0; tz < tz1; ++tz) {
  const int z0 = tz * TZ;
  int np0 = 0, np1 = 0;
  if (tz + 1 < tz1) range(tz + 1, &np0, &np1);
  // field node records: all planes for the first tile, planes 1 .. TZ after
  // the carried plane 0 (3 pairs per node, one thread per (y, x, pair)); a
  // plane's address is a uniform base plus the thread's 32-bit byte offset
  {
    for (int it = threadIdx.x; it < 3 * FX * FY; it += NTHR) {
      int part = it % 3, r = it / 3;
      int lx = r % FX, ly = r / FX;
      int gx = x0 + lx; if (gx >= g.Nx) gx -= g.Nx;
      int gy = y0 + ly; if (gy >= g.Ny) gy -= g.Ny;
      const unsigned boff = ((unsigned)(gy * g.Nx + gx) * 3u + (unsigned)part) * (unsigned)sizeof(V2);
      V2* dst = reinterpret_cast<V2*>(sF + 6 * (ly * FX + lx)) + part;
      auto fetch = [&](int lz) {
        const int gz = z0 + lz;
        V2 v;
        if (gz < g.Nz) {
          const char* plane = reinterpret_cast<const char*>(a.F6 + 6 * (int64_t)gz * plane_stride);
          v = *reinterpret_cast<const V2*>(plane + boff);
        } else {
          v.x = (T)0; v.y = (T)0;
        }
        return v;
      };
      V2 v[FZ];
#pragma unroll
      for (int lz = 1; lz < FZ; ++lz) v[lz] = fetch(lz);
      if (tz == tz0) dst[0] = fetch(0);
#pragma unroll
      for (int lz = 1; lz < FZ; ++lz) dst[3 * lz * FX * FY] = v[lz];
    }
  }
  __syncthreads();

  for (int row = p0; row < p1; row += NTHR) {
    const bool inrow = row + (int)lane < p1;
    const PLoad<T> cur = nxt;
    // prefetch: the next row of this tile, else the first row of the next tile
    {
      const bool same = row + NTHR < p1;
      const int nb = same ? row + NTHR : np0;
      nxt = load_row<T, DIM, ABS>(P, nb, (same ? p1 : np1) - nb, lane);
    }
    // Every lane runs the gather, push and move; lanes past the row (which
    // loaded zeros) and lanes whose particle is not in this tile (an error)
    // work on a stand-in at the tile's first node with zero offsets and
    // momenta, and only valid lanes store, report errors or deposit.
    const int spec = SPEC ? (cur.cell & GEMPIC_BEAM_BIT) : 0;
    int ix, iy, iz;
    T ax0 = (T)0, ay0 = (T)0, az0 = (T)0;   // decoded offsets (absolute positions)
    if constexpr (ABS) {
      float o;
      ix = abs_cell(cur.ox, g.ihx, &o);
      if (ix >= g.Nx) ix -= g.Nx;
      ax0 = o;
      iy = 0;
      if (DIM == 3) {
        iy = abs_cell(cur.oy, g.ihy, &o);
        if (iy >= g.Ny) iy -= g.Ny;
        ay0 = o;
      }
      iz = abs_cell(cur.oz, g.ih, &o);
      az0 = o;
      if (iz >= g.Nzp) { iz = g.Nzp - 1; az0 = (T)0x1.fffffep-1f; }
    } else {
      const int cell = cur.cell ^ spec;
      ix = cell & mx;
      iy = (cell >> g.lnx) & my;
      iz = cell >> (g.lnx + g.lny);
    }
    int lx = ix - x0, ly = iy - y0, lz = iz - z0;
    const bool intile = lx >= 0 && lx < TX && ly >= 0 && ly < (DIM == 3 ? TY : 1) && lz >= 0 && lz < TZ;
    if (inrow && !intile) atomicOr(a.err, ERR_TILE);
    bool valid = inrow && intile;
    if (!valid) lx = ly = lz = 0;
    T dx0 = valid ? (ABS ? ax0 : cur.ox) : (T)0;
    T dz0 = valid ? (ABS ? az0 : cur.oz) : (T)0;
    T dy0 = DIM == 3 && valid ? (ABS ? ay0 : cur.oy) : (T)0;
    T ux = valid ? cur.ux : (T)0, uy = valid ? cur.uy : (T)0, uz = valid ? cur.uz : (T)0;
    int kx = 0, ky = 0, kz = 0;
    T dx1 = (T)0, dy1 = (T)0, dz1 = (T)0, vy = (T)0;
    T X1 = (T)0, Y1 = (T)0, Z1 = (T)0;   // new absolute position (ABS)
    {
        // gather
        T wx[2] = {(T)1 - dx0, dx0};
        T wz[2] = {(T)1 - dz0, dz0};
        T wy[2] = {(T)1 - dy0, dy0};
        // sums start from the first node's products (0 + x differs from x
        // only in the sign of a zero)
        T f[6];
        int nb = (lz * FY + ly) * FX + lx;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
#pragma unroll
          for (int b = 0; b < (DIM == 3 ? 2 : 1); ++b) {
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) {
              T w = DIM == 3 ? (wx[aa] * wy[b]) * wz[cc] : wx[aa] * wz[cc];
              const V2* rec = reinterpret_cast<const V2*>(sF + 6 * (nb + (cc * FY + b) * FX + aa));
              V2 r0 = rec[0], r1 = rec[1], r2 = rec[2];
              const T v[6] = {r0.x, r0.y, r1.x, r1.y, r2.x, r2.y};
              const bool first = cc == 0 && b == 0 && aa == 0;
#pragma unroll
              for (int k = 0; k < 6; ++k) f[k] = first ? w * v[k] : madd(w, v[k], f[k]);
            }
          }
        }

        // Higuera-Cary push
        T eps = a.eps;
        T umx = madd(eps, f[0], ux);
        T umy = madd(eps, f[1], uy);
        T umz = madd(eps, f[2], uz);
        T bx = eps * f[3], by = eps * f[4], bz = eps * f[5];
        T um2 = madd(umz, umz, madd(umy, umy, umx * umx));
        T b2 = madd(bz, bz, madd(by, by, bx * bx));
        T sigma = ((T)1 + um2) - b2;
        T bu = madd(bz, umz, madd(by, umy, bx * umx));
        T gp = sqrt((sigma + sqrt(madd(sigma, sigma, (T)4 * madd(bu, bu, b2)))) * (T)0.5);
        T rgp = (T)1 / gp;
        T tx_ = bx * rgp, ty_ = by * rgp, tz_ = bz * rgp;
        T s = (T)1 / ((T)1 + madd(tz_, tz_, madd(ty_, ty_, tx_ * tx_)));
        T ut = madd(umz, tz_, madd(umy, ty_, umx * tx_));
        T upx = s * (madd(ut, tx_, umx) + madd(umy, tz_, -(umz * ty_)));
        T upy = s * (madd(ut, ty_, umy) + madd(umz, tx_, -(umx * tz_)));
        T upz = s * (madd(ut, tz_, umz) + madd(umx, ty_, -(umy * tx_)));
        ux = madd(eps, f[0], upx) + madd(upy, tz_, -(upz * ty_));
        uy = madd(eps, f[1], upy) + madd(upz, tx_, -(upx * tz_));
        uz = madd(eps, f[2], upz) + madd(upx, ty_, -(upy * tx_));

        // move
        T uperp2 = madd(uy, uy, ux * ux);
        T gam = sqrt((T)1 + madd(uz, uz, uperp2));
        T rg = (T)1 / gam;
        T vx = ux * rg;
        vy = uy * rg;
        T vzm1 = uz >= (T)0 ? (-((T)1 + uperp2) * rg) / (gam + uz) : madd(uz, rg, (T)-1);
        if constexpr (ABS) {
          float o;
          X1 = madd(vx, a.dtau, cur.ox);
          if (X1 >= g.Lx) X1 -= g.Lx; else if (X1 < (T)0) X1 += g.Lx;
          int ix1 = abs_cell(X1, g.ihx, &o);
          if (ix1 >= g.Nx) ix1 -= g.Nx;
          dx1 = o;
          kx = ix1 - ix;
          if (kx > 1) kx -= g.Nx; else if (kx < -1) kx += g.Nx;
          if (DIM == 3) {
            Y1 = madd(vy, a.dtau, cur.oy);
            if (Y1 >= g.Ly) Y1 -= g.Ly; else if (Y1 < (T)0) Y1 += g.Ly;
            int iy1 = abs_cell(Y1, g.ihy, &o);
            if (iy1 >= g.Ny) iy1 -= g.Ny;
            dy1 = o;
            ky = iy1 - iy;
            if (ky > 1) ky -= g.Ny; else if (ky < -1) ky += g.Ny;
          }
          Z1 = madd(vzm1, a.dtau, cur.oz);
          int iz1 = abs_cell(Z1, g.ih, &o);
          dz1 = o;
          kz = iz1 - iz;
        } else {
          T tnx = madd(vx, a.ax, dx0);
          T kxf = floor(tnx);
          dx1 = tnx - kxf;
          kx = (int)kxf;
          if (dx1 >= (T)1) { dx1 = (T)0; kx += 1; }
          if (DIM == 3) {
            T tny = madd(vy, a.ay, dy0);
            T kyf = floor(tny);
            dy1 = tny - kyf;
            ky = (int)kyf;
            if (dy1 >= (T)1) { dy1 = (T)0; ky += 1; }
          }
          T tnz = madd(vzm1, a.az, dz0);
          T kzf = floor(tnz);
          dz1 = tnz - kzf;
          kz = (int)kzf;
          if (dz1 >= (T)1) { dz1 = (T)0; kz += 1; }
        }
    }
    // a non-finite momentum (ERR_NUMERIC) or a step beyond one cell (ERR_CFL)
    // leaves the particle unchanged; the cell steps of a non-finite move are
    // never read
    const bool nanu = !(ux == ux && uy == uy && uz == uz);
    if (valid && nanu) atomicOr(a.err, ERR_NUMERIC);
    const bool cfl_bad = !nanu && (kx < -1 || kx > 1 || ky < -1 || ky > 1 || kz < -1 || kz > 0);
    if (valid && cfl_bad) atomicOr(a.err, ERR_CFL);
    valid = valid && !cfl_bad && !nanu;
    if (!valid) kx = ky = kz = 0;
    if (valid) {
      int nix = (ix + kx) & mx;
      int niy = (iy + ky) & my;
      int niz = iz + kz;
      const int nr = p1 - row;
      if constexpr (ABS) {
        row_st(X1, P.ox, row, nr, lane);
        if (DIM == 3) row_st(Y1, P.oy, row, nr, lane);
        row_st(Z1, P.oz, row, nr, lane);
      } else {
        row_st(((niz * g.Ny + niy) * g.Nx + nix) | spec, P.cell, row, nr, lane);
        row_st(dx1, P.ox, row, nr, lane);
        if (DIM == 3) row_st(dy1, P.oy, row, nr, lane);
        row_st(dz1, P.oz, row, nr, lane);
      }
      row_st(ux, P.ux, row, nr, lane);
      row_st(uy, P.uy, row, nr, lane);
      row_st(uz, P.uz, row, nr, lane);
    }

    // ---- deposit (sums: FMA contraction allowed) ----
    if (__any(valid)) {
#pragma clang fp contract(fast)
      auto add = [](A* p, T v) { atomicAdd(p, Fix<T>::to(v)); };
      const T fs = a.fscale;
      // invalid lanes deposit zeros at a valid LDS address
      T S0x[3], S1x[3], S0z[3], S1z[3], S0y[3], S1y[3];
      window3<T>(kx, dx0, dx1, S0x, S1x);
      window3<T>(kz, dz0, dz1, S0z, S1z);
      if (DIM == 3) window3<T>(ky, dy0, dy1, S0y, S1y);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        S0x[i] = valid ? S0x[i] : (T)0;
        S1x[i] = valid ? S1x[i] : (T)0;
      }
      T DSx[3], DSy[3], DSz[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        DSx[i] = S1x[i] - S0x[i];
        DSz[i] = S1z[i] - S0z[i];
        DSy[i] = DIM == 3 ? S1y[i] - S0y[i] : (T)0;
      }
      const T third = (T)(1.0 / 3.0);
      // A, B along zeta: W factors S0*(A) + DS*(B)
      T Az[3], Bz[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) { Az[i] = S0z[i] + (T)0.5 * DSz[i]; Bz[i] = (T)0.5 * S0z[i] + third * DSz[i]; }
      int jx0 = lx + min(kx, 0) + 1;
      int jy0 = DIM == 3 ? ly + min(ky, 0) + 1 : 0;
      int jz0 = lz + kz + 2;            // node base_z (kz <= 0)
      A* sJx = sJ + ((jz0 - 1) * JY + jy0) * JX + jx0;
      A* sJy = sJx + (JZ - 1) * JP;
      A* sJz = sJx + 2 * (JZ - 1) * JP;  // half-node plane base_z - 1
      const T wr = SPEC && spec ? a.rb : (T)1;
      T qr = (T)0.25 * a.crho * fs * wr;
      T cx = a.cx * fs * wr, cy = a.cy * fs * wr, cz = a.cz * fs * wr;
      if (DIM == 3) {
        // Transverse window: 3 x 3 nodes when a particle of the wave crosses a
        // transverse cell boundary, taken one node at a time (weights
        // recomputed, J_x and J_y from running prefixes of DS_x, DS_y) to keep
        // few values live; else 2 x 2, unrolled (the third window node, the
        // second J_x half-node and the second J_y half-node carry exactly zero).
        const bool general = __any(kx != 0 || ky != 0);
        T s0e[4], s1e[4];
        s0e[0] = S0z[0]; s0e[1] = S0z[0] + S0z[1]; s0e[2] = S0z[1] + S0z[2]; s0e[3] = S0z[2];
        s1e[0] = S1z[0]; s1e[1] = S1z[0] + S1z[1]; s1e[2] = S1z[1] + S1z[2]; s1e[3] = S1z[2];
        T pz0 = cz * DSz[0], pz1 = cz * (DSz[0] + DSz[1]);
        if (general) {
          const int ox0 = kx < 0 ? 1 : 0, ox1 = kx > 0 ? 1 : 0;
          const int oy0 = ky < 0 ? 1 : 0, oy1 = ky > 0 ? 1 : 0;
          T prex = (T)0;
#pragma unroll 1
          for (int aa = 0; aa < 3; ++aa) {
            T s0x = valid ? (aa == ox0 ? (T)1 - dx0 : (T)0) + (aa == ox0 + 1 ? dx0 : (T)0) : (T)0;
            T s1x = valid ? (aa == ox1 ? (T)1 - dx1 : (T)0) + (aa == ox1 + 1 ? dx1 : (T)0) : (T)0;
            T dsx = s1x - s0x;
            prex += dsx;
            T px = cx * prex;
            T Fx[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) Fx[cc] = s0x * Az[cc] + dsx * Bz[cc];
            T prey = (T)0;
#pragma unroll 1
            for (int b = 0; b < 3; ++b) {
              T s0y = (b == oy0 ? (T)1 - dy0 : (T)0) + (b == oy0 + 1 ? dy0 : (T)0);
              T s1y = (b == oy1 ? (T)1 - dy1 : (T)0) + (b == oy1 + 1 ? dy1 : (T)0);
              T dsy = s1y - s0y;
              prey += dsy;
              if (aa < 2) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                  add(&sJx[(cc * JY + b) * JX + aa], px * (s0y * Az[cc] + dsy * Bz[cc]));
              }
              if (b < 2) {
                T py = cy * prey;
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) add(&sJy[(cc * JY + b) * JX + aa], py * Fx[cc]);
              }
              T Fz = s0x * (s0y + (T)0.5 * dsy) + dsx * ((T)0.5 * s0y + third * dsy);
              T t0 = qr * (s0x * s0y), t1 = qr * (s1x * s1y);
              A* pz = &sJz[b * JX + aa];
              add(pz + 0 * JY * JX, t0 * s0e[0] + t1 * s1e[0]);
              add(pz + 1 * JY * JX, t0 * s0e[1] + t1 * s1e[1] + pz0 * Fz);
              add(pz + 2 * JY * JX, t0 * s0e[2] + t1 * s1e[2] + pz1 * Fz);
              add(pz + 3 * JY * JX, t0 * s0e[3] + t1 * s1e[3]);
            }
          }
        } else {
          // no transverse crossing in this wave: x and y windows start at the
          // cell, the third window node and the second half-node carry zero
          T Cy[2], Dy[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) { Cy[i] = S0y[i] + (T)0.5 * DSy[i]; Dy[i] = (T)0.5 * S0y[i] + third * DSy[i]; }
          T px0 = cx * DSx[0], py0 = cy * DSy[0];
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              add(&sJx[(cc * JY + b) * JX + 0], px0 * (S0y[b] * Az[cc] + DSy[b] * Bz[cc]));
          if constexpr (std::is_same<T, float>::value) {
            // A wave is usually one zeta sub-row of the tile's columns, so the
            // window of lane l starts one node right of lane l - 1's: the node
            // they share gets lane l - 1's second value added to lane l's
            // first (as integers: exact), moved by a DPP shift, and one atomic
            // instead of two.  Both lanes test the same address relation, so
            // each value is added exactly once whatever the layout.
            const int key = (jz0 * JY + jy0) * JX + jx0 + 2;   // never 0 or 1
            const bool take = dpp_from_left(key) + 1 == key;
            const bool give = key + 1 == dpp_from_right(key);
            auto add2 = [&](A* p0, T v0, T v1) {
              const int i1 = (int)v1;             // Fix<float>::to without the widening
              const int r = dpp_from_left(i1);
              long long i0 = (int)v0;
              if (take) i0 += r;                  // two int32 terms: no overflow in 64 bits
              atomicAdd(p0, (A)i0);
              if (!give) atomicAdd(p0 + 1, (A)(long long)i1);
            };
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              add2(&sJy[(cc * JY + 0) * JX + 0], py0 * (S0x[0] * Az[cc] + DSx[0] * Bz[cc]),
                   py0 * (S0x[1] * Az[cc] + DSx[1] * Bz[cc]));
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              T Fz0 = S0x[0] * Cy[b] + DSx[0] * Dy[b], Fz1 = S0x[1] * Cy[b] + DSx[1] * Dy[b];
              T t00 = qr * (S0x[0] * S0y[b]), t10 = qr * (S1x[0] * S1y[b]);
              T t01 = qr * (S0x[1] * S0y[b]), t11 = qr * (S1x[1] * S1y[b]);
              A* pz = &sJz[b * JX + 0];
              add2(pz + 0 * JY * JX, t00 * s0e[0] + t10 * s1e[0], t01 * s0e[0] + t11 * s1e[0]);
              add2(pz + 1 * JY * JX, t00 * s0e[1] + t10 * s1e[1] + pz0 * Fz0, t01 * s0e[1] + t11 * s1e[1] + pz0 * Fz1);
              add2(pz + 2 * JY * JX, t00 * s0e[2] + t10 * s1e[2] + pz1 * Fz0, t01 * s0e[2] + t11 * s1e[2] + pz1 * Fz1);
              add2(pz + 3 * JY * JX, t00 * s0e[3] + t10 * s1e[3], t01 * s0e[3] + t11 * s1e[3]);
            }
          } else {
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
#pragma unroll
              for (int cc = 0; cc < 3; ++cc)
                add(&sJy[(cc * JY + 0) * JX + aa], py0 * (S0x[aa] * Az[cc] + DSx[aa] * Bz[cc]));
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
#pragma unroll
              for (int b = 0; b < 2; ++b) {
                T Fz = S0x[aa] * Cy[b] + DSx[aa] * Dy[b];
                T t0 = qr * (S0x[aa] * S0y[b]), t1 = qr * (S1x[aa] * S1y[b]);
                A* pz = &sJz[b * JX + aa];
                add(pz + 0 * JY * JX, t0 * s0e[0] + t1 * s1e[0]);
                add(pz + 1 * JY * JX, t0 * s0e[1] + t1 * s1e[1] + pz0 * Fz);
                add(pz + 2 * JY * JX, t0 * s0e[2] + t1 * s1e[2] + pz1 * Fz);
                add(pz + 3 * JY * JX, t0 * s0e[3] + t1 * s1e[3]);
              }
          }
        }
      } else {
        // 2-D (x, zeta): W_x, out-of-plane J_y = q w v_y x time-averaged shape, J_z
        T px[2] = {cx * DSx[0], cx * (DSx[0] + DSx[1])};
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          add(&sJx[cc * JX + 0], px[0] * Az[cc]);
          add(&sJx[cc * JX + 1], px[1] * Az[cc]);
        }
        T cyv = a.cjy * fs * wr * vy;
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            T wt = S0x[aa] * Az[cc] + DSx[aa] * Bz[cc];
            add(&sJy[cc * JX + aa], cyv * wt);
          }
        T pz0 = cz * DSz[0], pz1 = cz * (DSz[0] + DSz[1]);
        T s0e[4] = {S0z[0], S0z[0] + S0z[1], S0z[1] + S0z[2], S0z[2]};
        T s1e[4] = {S1z[0], S1z[0] + S1z[1], S1z[1] + S1z[2], S1z[2]};
#pragma unroll
        for (int aa = 0; aa < 3; ++aa) {
          T Fz = S0x[aa] + (T)0.5 * DSx[aa];
          T t0 = qr * S0x[aa], t1 = qr * S1x[aa];
          A* pz = &sJz[aa];
          add(pz + 0 * JX, t0 * s0e[0] + t1 * s1e[0]);
          add(pz + 1 * JX, t0 * s0e[1] + t1 * s1e[1] + pz0 * Fz);
          add(pz + 2 * JX, t0 * s0e[2] + t1 * s1e[2] + pz1 * Fz);
          add(pz + 3 * JX, t0 * s0e[3] + t1 * s1e[3]);
        }
      }
      if (RHO && valid) {
        // charge before and after the move; rho tile origin (x0-1, y0-1, node z0-1)
        A* sR0 = sJ + JN;
        A* sR1 = sR0 + RN;
        T cr = a.crho * fs * wr;
        constexpr int oy = DIM == 3 ? 1 : 0;
        T w0x[2] = {(T)1 - dx0, dx0}, w0y[2] = {(T)1 - dy0, dy0}, w0z[2] = {(T)1 - dz0, dz0};
        T w1x[2] = {(T)1 - dx1, dx1}, w1y[2] = {(T)1 - dy1, dy1}, w1z[2] = {(T)1 - dz1, dz1};
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
          for (int b = 0; b < (DIM == 3 ? 2 : 1); ++b)
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) {
              T v0 = DIM == 3 ? w0x[aa] * w0y[b] * w0z[cc] : w0x[aa] * w0z[cc];
              T v1 = DIM == 3 ? w1x[aa] * w1y[b] * w1z[cc] : w1x[aa] * w1z[cc];
              add(&sR0[((lz + 1 + cc) * RY + (ly + oy + b)) * RX + (lx + 1 + aa)], cr * v0);
              add(&sR1[((lz + kz + 1 + cc) * RY + (ly + ky + oy + b)) * RX + (lx + kx + 1 + aa)], cr * v1);
            }
      }
    }
  }
  __syncthreads();

  // flush the planes no later tile of the segment touches (all of them after
  // the last tile), carry the rest down by TZ planes.  One thread per column
  // (x, y) of a slab; slab q is handled by waves 2q, 2q+1 of a 128-lane block
  // (one column per lane, JP <= 128), so that q is uniform in a wave and the
  // destination plane is a uniform base plus the lane's 32-bit byte offset.
  // Global x = x0 - 1 + jx, y = y0 - 1 + jy, plane = z0 + jz.
  {
    const bool last = tz + 1 == tz1;
    static_assert(JP <= 128, "one column per lane of a 128-lane block");
    for (int col = threadIdx.x; col < 3 * 128; col += NTHR) {
      const int q = __builtin_amdgcn_readfirstlane(col >> 7);
      const int l = col & 127;
      if (l < JP) {
        int jx = l % JX, jy = l / JX;
        int gx = (x0 - 1 + jx) & mx;
        int gy = DIM == 3 ? (y0 - 1 + jy) & my : 0;
        const unsigned boff = (unsigned)(gy * g.Nx + gx) * (unsigned)sizeof(T);
        T* const dq = a.J[q];
        auto put = [&](A iv, int jz) {
          const int plane = z0 + jz;
          if (iv != (A)0 && plane < g.NPJ) {
            if constexpr (DET) {
              atomicAdd(a.Jfix[q] + (int64_t)plane * plane_stride + boff / (unsigned)sizeof(T), iv);
            } else {
              char* base = reinterpret_cast<char*>(dq + (int64_t)plane * plane_stride);
              atomicAdd(reinterpret_cast<T*>(base + boff), Fix<T>::value(iv) * a.finv);
            }
          }
        };
        // a slab's planes below TZ + first are final: the next tile's deposits
        // of that component start at plane TZ + first
        auto slab = [&](auto first_c) {
          constexpr int first = decltype(first_c)::value;
          A* sc = sJ + q * (JZ - 1) * JP + l - first * JP;   // sc[jz * JP]: plane jz
          A iv[JZ];
#pragma unroll
          for (int jz = first; jz < JZ; ++jz) iv[jz] = sc[jz * JP];
#pragma unroll
          for (int jz = first; jz < TZ + first; ++jz) put(iv[jz], jz);
          if (last) {
#pragma unroll
            for (int jz = TZ + first; jz < JZ; ++jz) put(iv[jz], jz);
          } else {
#pragma unroll
            for (int jz = first; jz < JZ; ++jz) {
              const int src = jz + TZ;
              sc[jz * JP] = src < JZ ? iv[src] : (A)0;
            }
          }
        };
        if (q < 2) slab(std::integral_constant<int, 1>());
        else slab(std::integral_constant<int, 0>());
      }
    }
    if (RHO) {
      // rho tiles: origin node z0 - 1 (plane z0 + 1), RZ planes
      const int rflush = last ? RZ : TZ;
      for (int col = threadIdx.x; col < 2 * RY * RX; col += NTHR) {
        int q = col / (RY * RX), l = col - q * (RY * RX);
        int rx = l % RX, ry = l / RX;
        int gx = (x0 - 1 + rx) & mx;
        int gy = DIM == 3 ? (y0 - 1 + ry) & my : 0;
        T* dst = (q == 0 ? a.rho0 : a.rho1) + (int64_t)gy * g.Nx + gx;
        A* sc = sJ + JN + q * RN + ry * RX + rx;
        for (int rz = 0; rz < rflush; ++rz) {
          A iv = sc[rz * RY * RX];
          int plane = z0 + 1 + rz;
          if (iv != (A)0 && plane < g.NPJ) atomicAdd(dst + plane * plane_stride, Fix<T>::value(iv) * a.finv);
        }
        if (!last) {
          for (int rz = TZ; rz < RZ; ++rz) {
            sc[(rz - TZ) * RY * RX] = sc[rz * RY * RX];
            sc[rz * RY * RX] = (A)0;
          }
          for (int rz = RZ - TZ; rz < TZ; ++rz) sc[rz * RY * RX] = (A)0;
        }
      }
    }
    // the last field plane becomes the first one of the next tile
    if (!last) {
      for (int it = threadIdx.x; it < 3 * FX * FY; it += NTHR) {
        V2* f = reinterpret_cast<V2*>(sF);
        f[it] = f[3 * TZ * FX * FY + it];
      }
    }
  }
  __syncthreads();
  // an empty tile consumed no prefetch: load the next tile's first row now
  if (p0 >= p1) nxt = load_row<T, DIM, ABS>(P, np0, np1 - np0, lane);
  p0 = np0;
  p1 = np1;
  }  // zeta tiles of the segment
}
