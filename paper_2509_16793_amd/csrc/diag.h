// FP64 diagnostics: deterministic two-pass reductions (fixed partition into
// work-group partial sums, then one work-group summing the partials).
#pragma once
#include "common.h"

#define DIAG_BLOCKS 1024

GP_DEV double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// partial[b] = sum over the b-th slice of sum_k (s_k * a_k[i])^2 or of a_k[i]
template <typename T>
__global__ __launch_bounds__(256) void k_partial(const T* a0, const T* a1, const T* a2, const T* a3,
                                                 const T* a4, const T* a5, int narr, int64_t n,
                                                 int square, double* partial) {
  __shared__ double sh[4];
  const T* arr[6] = {a0, a1, a2, a3, a4, a5};
  int64_t per = (n + gridDim.x - 1) / gridDim.x;
  int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  double s = 0.0;
  for (int q = 0; q < narr; ++q)
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      double v = (double)arr[q][i];
      s += square ? v * v : v;
    }
  double r = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// Continuity residual of the raw deposit at every stored node:
//   r = (rho1 - rho0)/dtau - (rb(n+1/2) - rb(n-1/2))/h + D.J,
//   rb(n+1/2) = (rho0_n + rho0_{n+1} + rho1_n + rho1_{n+1}) / 4;
// partial sums of r^2 and of ((rho1 - rho0)/dtau)^2.
template <typename T>
__global__ __launch_bounds__(256) void k_continuity(Geom g, const T* rho0, const T* rho1, const T* Jx,
                                                    const T* Jy, const T* Jz, double* partial) {
  __shared__ double sh[4];
  int64_t nxy = (int64_t)g.Ny * g.Nx;
  int64_t n = (int64_t)g.NPJ * nxy;
  int64_t per = (n + gridDim.x - 1) / gridDim.x;
  int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
  double s = 0.0, t = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    int64_t p = i / nxy, r = i - p * nxy;
    int y = (int)(r / g.Nx), x = (int)(r % g.Nx);
    auto rb = [&](int64_t pl) -> double {
      if (pl < 0) return 0.0;
      int64_t o = pl * nxy + r;
      double v = (double)rho0[o] + (double)rho1[o];
      if (pl + 1 < g.NPJ) v += (double)rho0[o + nxy] + (double)rho1[o + nxy];
      return 0.25 * v;
    };
    double dr = ((double)rho1[i] - (double)rho0[i]) / g.dtau;
    double res = dr - (rb(p) - rb(p - 1)) / g.h;
    int xm = x == 0 ? g.Nx - 1 : x - 1;
    res += ((double)Jx[i] - (double)Jx[p * nxy + (int64_t)y * g.Nx + xm]) / g.hx;
    if (g.dims == 3) {
      int ym = y == 0 ? g.Ny - 1 : y - 1;
      res += ((double)Jy[i] - (double)Jy[p * nxy + (int64_t)ym * g.Nx + x]) / g.hy;
    }
    double jzm = p > 0 ? (double)Jz[i - nxy] : 0.0;
    res += ((double)Jz[i] - jzm) / g.h;
    s += res * res;
    t += dr * dr;
  }
  double a = block_sum(s, sh);
  double b = block_sum(t, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = a;
    partial[2 * blockIdx.x + 1] = b;
  }
}

__global__ __launch_bounds__(256) void k_final(const double* partial, int nb, int stride, double* out) {
  __shared__ double sh[4];
  for (int c = 0; c < stride; ++c) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i * stride + c];
    double r = block_sum(s, sh);
    if (threadIdx.x == 0) out[c] = r;
  }
}
