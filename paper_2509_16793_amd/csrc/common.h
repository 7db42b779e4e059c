// Shared device/host definitions of the gfx950 Galilean PIC library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GP_DEV __device__ __forceinline__
#define GP_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// complex arithmetic (interleaved re, im)
template <typename T>
struct cplx {
  T x, y;
};

template <typename T> GP_HD cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }
template <typename T> GP_HD cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> GP_HD cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> GP_HD cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> GP_HD cplx<T> operator*(T s, cplx<T> a) { return mk(s * a.x, s * a.y); }
template <typename T> GP_HD cplx<T> conj(cplx<T> a) { return mk(a.x, -a.y); }
// i * a
template <typename T> GP_HD cplx<T> mul_i(cplx<T> a) { return mk(-a.y, a.x); }

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) used as a counter generator:
// output(key, c) = mix(key + (c + 1) * GAMMA), uniform = (output >> 11) * 2^-53.
#define SM_GAMMA 0x9E3779B97F4A7C15ull
GP_HD uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
GP_HD double sm_uniform(uint64_t key, uint64_t counter) {
  uint64_t x = sm_mix(key + (counter + 1ull) * SM_GAMMA) >> 11;
  return (double)x * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Geometry shared by the kernels (all lengths already normalised).
struct Geom {
  int dims;
  int Nx, Ny, Nz;        // field grid; Ny = 1 in 2-D
  int lnx, lny;          // log2 Nx, log2 Ny
  int Nzp;               // particle cells along zeta (Nz + ext)
  int ext;               // plasma cells beyond the last field node
  int P;                 // binomial filter passes
  int NPJ;               // current/charge planes: node n = -2 .. Nz + ext + 1 -> plane n + 2
  int NPF;               // current planes the field solver reads: Nz + 3 + P
  int Tx, Ty, Tz;        // tile in cells
  int nTx, nTy, nTz, NT; // tile grid
  int Nxh;               // stored transverse x modes: Nx / 2 (Nyquist dropped)
  double hx, hy, h, dtau;
  double qw;             // charge q * w of a macro-particle
  double V;              // cell volume hx * hy_eff * h
  int abs_pos;           // particles store absolute FP32 positions (no cell array)
  float ihx, ihy, ih;    // FP32 inverse steps that decode an absolute position
  float Lx, Ly;          // FP32 periodic lengths Nx hx, Ny hy
};

// Cell and offset of an absolute FP32 position along an axis of n cells:
// f = x * (1/h) in FP32, cell = floor(f), offset = f - cell; a cell equal to n
// (x rounded up to the periodic length) wraps to 0 when periodic.
GP_DEV int abs_cell(float x, float ih, float* off) {
  float f = x * ih;
  float c = floorf(f);
  *off = f - c;
  return (int)c;
}

// Sort codes: destination tile relative to the source tile, steps
// sz in {-1, 0}, sy, sx in {-1, 0, 1}: code = (sz + 1) * 9 + (sy + 1) * 3 + sx + 1.
#define NCODE 19
#define CODE_REMOVED 18

// Error flags raised on the device (bit mask).
#define ERR_CFL 1
#define ERR_TILE 2
#define ERR_CAPACITY 4
#define ERR_NUMERIC 8

#define GP_CHUNK 1024      // max particles per work-group chunk
