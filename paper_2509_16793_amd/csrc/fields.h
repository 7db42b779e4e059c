// Field kernels: batched transverse 2-D FFT of real planes, the right-to-left
// march of the node scheme (Sec. 4.1) with the analytic node solution (App. B),
// and small helpers.
//
// Spectral layout: [plane][ky][kx] complex with kx = 0 .. Nx/2 - 1 (the kx
// Nyquist column is dropped: the solver zeroes it), ky in FFT order; the
// ky Nyquist row is stored and held at zero.  Forward transform
// sum f exp(-i k.r), inverse with 1/(Nx Ny).
#pragma once
#include "common.h"

// ---------------------------------------------------------------------------
// Stockham FFT of nseq sequences of length N (a power of two) held in LDS:
// radix-4 passes, then one radix-2 pass when log2 N is odd.  x holds the
// input, y is the ping-pong buffer; the pointer to the result is returned.
// tl (LDS, N entries) receives the full circle of twiddles exp(-2 pi i t / N)
// from tw (global, t < N/2); the inverse uses their conjugates (no scaling).
// Sequence sq starts at element sq * S of x and y (S >= N; a padded stride
// spreads column-wise accesses over the LDS banks).
// Every thread of the block must call it (it synchronises).
template <typename T>
GP_DEV cplx<T>* lds_fft(cplx<T>* x, cplx<T>* y, cplx<T>* tl, int N, int nseq, const cplx<T>* tw,
                        bool inverse, int S = 0) {
  if (S < N) S = N;
  const int half = N >> 1;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    cplx<T> w = tw[t < half ? t : t - half];
    if (t >= half) w = mk(-w.x, -w.y);
    if (inverse) w.y = -w.y;
    tl[t] = w;
  }
  __syncthreads();
  int Ns = 1;
  const int q4 = N >> 2;
  for (; Ns * 4 <= N; Ns <<= 2) {
    const int step = N / (4 * Ns);
    for (int idx = threadIdx.x; idx < nseq * q4; idx += blockDim.x) {
      int sq = idx / q4, j = idx - sq * q4;
      int k = j & (Ns - 1);
      const cplx<T>* xs = x + sq * S;
      int ts = k * step;
      cplx<T> a0 = xs[j];
      cplx<T> a1 = tl[ts] * xs[j + q4];
      cplx<T> a2 = tl[2 * ts] * xs[j + 2 * q4];
      cplx<T> a3 = tl[3 * ts] * xs[j + 3 * q4];
      cplx<T> b0 = a0 + a2, b1 = a0 - a2, b2 = a1 + a3, b3 = a1 - a3;
      cplx<T> ib3 = mul_i(b3);
      cplx<T>* ys = y + sq * S;
      int d = ((j - k) << 2) + k;
      ys[d] = b0 + b2;
      ys[d + Ns] = inverse ? b1 + ib3 : b1 - ib3;
      ys[d + 2 * Ns] = b0 - b2;
      ys[d + 3 * Ns] = inverse ? b1 - ib3 : b1 + ib3;
    }
    __syncthreads();
    cplx<T>* t = x; x = y; y = t;
  }
  if (Ns < N) {
    // radix-2 pass, Ns = N / 2
    for (int idx = threadIdx.x; idx < nseq * half; idx += blockDim.x) {
      int sq = idx / half, j = idx - sq * half;
      int k = j & (Ns - 1);
      const cplx<T>* xs = x + sq * S;
      cplx<T> a = xs[j];
      cplx<T> b = tl[k * (half / Ns)] * xs[j + half];
      cplx<T>* ys = y + sq * S;
      int d = ((j - k) << 1) + k;
      ys[d] = a + b;
      ys[d + Ns] = a - b;
    }
    __syncthreads();
    cplx<T>* t = x; x = y; y = t;
  }
  return x;
}

// exp(-+2 pi i e / 256), 0 <= e < 256, from a table tw[t] = exp(-2 pi i t / N)
// (t < N / 2) of N = 256 S
template <typename T>
GP_DEV cplx<T> twid256(const cplx<T>* tw, int e, bool inverse, int S = 1) {
  cplx<T> w = e < 128 ? tw[e * S] : mk(-tw[(e - 128) * S].x, -tw[(e - 128) * S].y);
  if (inverse) w.y = -w.y;
  return w;
}
// 4-point DFT in place
template <typename T>
GP_DEV void dft4(cplx<T>& a0, cplx<T>& a1, cplx<T>& a2, cplx<T>& a3, bool inverse) {
  const cplx<T> b0 = a0 + a2, b1 = a0 - a2, b2 = a1 + a3, b3 = a1 - a3;
  const cplx<T> ib3 = mul_i(b3);
  a0 = b0 + b2;
  a2 = b0 - b2;
  a1 = inverse ? b1 + ib3 : b1 - ib3;
  a3 = inverse ? b1 - ib3 : b1 + ib3;
}
// 16-point DFT of v[n] as 4 x 4 (n = 4 m1 + m2, k = l1 + 4 l2); the result
// for k = l1 + 4 l2 is left in v[4 l1 + l2]
template <typename T>
GP_DEV void dft16(cplx<T> v[16], const cplx<T>* tw, bool inverse, int S = 1) {
#pragma unroll
  for (int m2 = 0; m2 < 4; ++m2) dft4(v[m2], v[4 + m2], v[8 + m2], v[12 + m2], inverse);
#pragma unroll
  for (int l1 = 1; l1 < 4; ++l1)
#pragma unroll
    for (int m2 = 1; m2 < 4; ++m2) v[4 * l1 + m2] = v[4 * l1 + m2] * twid256(tw, 16 * m2 * l1, inverse, S);
#pragma unroll
  for (int l1 = 0; l1 < 4; ++l1) dft4(v[4 * l1], v[4 * l1 + 1], v[4 * l1 + 2], v[4 * l1 + 3], inverse);
}

// Forward x transform of row pairs for Nx = 256 (two-for-one, as
// k_fft_x_r2c), as the four-step 16 x 16 DFT: 16 threads per row pair read
// the pair's rows 16 n1 + l straight into registers, the inner DFT, twiddles
// and one LDS transpose precede the outer DFT, and the spectra of both rows
// are split from the pair's transform in LDS, which reuses the transpose
// buffer (17 KB in FP32: up to 9 work-groups fit in a CU's LDS).  8 pairs per
// 128-thread work-group; rows past the end read row 0 and are not written.
constexpr int R2C256_P = 8;
template <typename T>
__global__ __launch_bounds__(128) void k_fft_x_r2c_256(const T* in, cplx<T>* out, int64_t rows, const cplx<T>* tw) {
  constexpr int P = R2C256_P;
  __shared__ cplx<T> sT[P * 272];
  cplx<T>* const sZ = sT;                    // the pair's transform, after the transpose
  const int q = threadIdx.x >> 4, l = threadIdx.x & 15;
  const int64_t r0 = 2 * ((int64_t)blockIdx.x * P + q), r1 = r0 + 1;
  const int64_t a0 = r0 < rows ? r0 : 0, a1 = r1 < rows ? r1 : 0;
  cplx<T> v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const T x0 = in[a0 * 256 + 16 * n1 + l], x1 = in[a1 * 256 + 16 * n1 + l];
    v[n1] = mk(r0 < rows ? x0 : (T)0, r1 < rows ? x1 : (T)0);
  }
  dft16(v, tw, false);
  cplx<T>* st = sT + q * 272;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = (p >> 2) + 4 * (p & 3);
    st[k1 * 17 + l] = k1 == 0 || l == 0 ? v[p] : v[p] * twid256(tw, l * k1, false);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = st[l * 17 + m];
  dft16(v, tw, false);
  __syncthreads();
  cplx<T>* sz = sZ + q * 256;
#pragma unroll
  for (int p = 0; p < 16; ++p) sz[l + 16 * ((p >> 2) + 4 * (p & 3))] = v[p];
  __syncthreads();
  for (int idx = threadIdx.x; idx < P * 128; idx += 128) {
    const int qq = idx >> 7, k = idx & 127;
    const int64_t b0 = 2 * ((int64_t)blockIdx.x * P + qq), b1 = b0 + 1;
    const cplx<T> zk = sZ[qq * 256 + k];
    const cplx<T> zc = conj(sZ[qq * 256 + ((256 - k) & 255)]);
    const cplx<T> A = (T)0.5 * (zk + zc);
    const cplx<T> D = zk - zc;
    const cplx<T> B = mk((T)0.5 * D.y, (T)-0.5 * D.x);
    if (b0 < rows) out[b0 * 128 + k] = A;
    if (b1 < rows) out[b1 * 128 + k] = B;
  }
}

// Forward x transform of row pairs for Nx = 512 (two-for-one, as
// k_fft_x_r2c): the even and the odd nodes of a pair's rows each take the
// 256-point four-step transform of k_fft_x_r2c_256 (16 threads each), then
// Z[k] = E[k] + W512^k O[k] and Z[k + 256] = E[k] - W512^k O[k] give the
// pair's transform, and the spectra of both rows are split from it; E and O
// reuse the transpose buffer.  4 pairs per 128-thread work-group; rows past
// the end read row 0 and are not written.  tw holds exp(-2 pi i t / 512) for
// t < 256.
constexpr int R2C512_P = 4;
template <typename T>
__global__ __launch_bounds__(128) void k_fft_x_r2c_512(const T* in, cplx<T>* out, int64_t rows, const cplx<T>* tw) {
  constexpr int P = R2C512_P;
  __shared__ cplx<T> sT[P * 2 * 272];
  cplx<T>* const sH = sT;                    // per pair: E[0..255], O[0..255], after the transpose
  const int q = threadIdx.x >> 5, h = (threadIdx.x >> 4) & 1, l = threadIdx.x & 15;
  const int64_t r0 = 2 * ((int64_t)blockIdx.x * P + q), r1 = r0 + 1;
  const int64_t a0 = r0 < rows ? r0 : 0, a1 = r1 < rows ? r1 : 0;
  cplx<T> v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int n = 2 * (16 * n1 + l) + h;
    const T x0 = in[a0 * 512 + n], x1 = in[a1 * 512 + n];
    v[n1] = mk(r0 < rows ? x0 : (T)0, r1 < rows ? x1 : (T)0);
  }
  dft16(v, tw, false, 2);
  cplx<T>* st = sT + (2 * q + h) * 272;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = (p >> 2) + 4 * (p & 3);
    st[k1 * 17 + l] = k1 == 0 || l == 0 ? v[p] : v[p] * twid256(tw, l * k1, false, 2);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = st[l * 17 + m];
  dft16(v, tw, false, 2);
  __syncthreads();
  cplx<T>* sh = sH + q * 512 + h * 256;
#pragma unroll
  for (int p = 0; p < 16; ++p) sh[l + 16 * ((p >> 2) + 4 * (p & 3))] = v[p];
  __syncthreads();
  for (int idx = threadIdx.x; idx < P * 256; idx += 128) {
    const int qq = idx >> 8, k = idx & 255;
    const cplx<T>* E = sH + qq * 512;
    const cplx<T>* O = E + 256;
    const cplx<T> zk = E[k] + tw[k] * O[k];
    // Z[512 - k] = E[256 - k] - W512^(256 - k) O[256 - k] for k > 0; Z[0] for k = 0
    const int j = (256 - k) & 255;
    const cplx<T> zm = k == 0 ? zk : E[j] - tw[j] * O[j];
    const cplx<T> zc = conj(zm);
    const int64_t b0 = 2 * ((int64_t)blockIdx.x * P + qq), b1 = b0 + 1;
    const cplx<T> A = (T)0.5 * (zk + zc);
    const cplx<T> D = zk - zc;
    const cplx<T> B = mk((T)0.5 * D.y, (T)-0.5 * D.x);
    if (b0 < rows) out[b0 * 256 + k] = A;
    if (b1 < rows) out[b1 * 256 + k] = B;
  }
}

// Forward transform along x of pairs of real rows (two-for-one): rows 2r and
// 2r+1 of in[rows][Nx] -> out[rows][Nxh].  nseq pairs per work-group.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_r2c(const T* in, cplx<T>* out, int64_t rows, int Nx,
                                                   int nseq, const cplx<T>* tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* x = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* y = x + nseq * Nx;
  cplx<T>* tl = y + nseq * Nx;
  int64_t pair0 = (int64_t)blockIdx.x * nseq;
  for (int idx = threadIdx.x; idx < nseq * Nx; idx += blockDim.x) {
    int sq = idx / Nx, n = idx - sq * Nx;
    int64_t r0 = 2 * (pair0 + sq), r1 = r0 + 1;
    T a = r0 < rows ? in[r0 * Nx + n] : (T)0;
    T b = r1 < rows ? in[r1 * Nx + n] : (T)0;
    x[idx] = mk(a, b);
  }
  __syncthreads();
  cplx<T>* Z = lds_fft(x, y, tl, Nx, nseq, tw, false);
  int Nxh = Nx >> 1;
  for (int idx = threadIdx.x; idx < nseq * Nxh; idx += blockDim.x) {
    int sq = idx / Nxh, k = idx - sq * Nxh;
    int64_t r0 = 2 * (pair0 + sq), r1 = r0 + 1;
    cplx<T> zk = Z[sq * Nx + k];
    cplx<T> zc = conj(Z[sq * Nx + ((Nx - k) & (Nx - 1))]);
    cplx<T> A = (T)0.5 * (zk + zc);
    cplx<T> D = zk - zc;                  // B = D / (2 i) = -i D / 2
    cplx<T> B = mk((T)0.5 * D.y, (T)-0.5 * D.x);
    if (r0 < rows) out[r0 * Nxh + k] = A;
    if (r1 < rows) out[r1 * Nxh + k] = B;
  }
}

// Inverse x transform of the six field components for Nx = 256, four-step:
// 16 threads per (row pair, component) assemble the pair's Hermitian
// sequence x[j] = A[j] + i B[j] (x[256 - j] = conj(A[j]) + i conj(B[j]),
// x[128] = 0) straight into registers, run the inverse 16 x 16 DFT with one
// LDS transpose, and leave z[n] in the same LDS buffer; the node records of
// both rows are then written as in k_fft_x_c2r6.  2 row pairs per 192-thread
// work-group; rows past the end read row 0 and are not written.
constexpr int C2R256_P = 2;
template <typename T>
__global__ __launch_bounds__(192) void k_fft_x_c2r6_256(const cplx<T>* i0, const cplx<T>* i1, const cplx<T>* i2,
                                                        const cplx<T>* i3, const cplx<T>* i4, const cplx<T>* i5,
                                                        T* out, int64_t rows, const cplx<T>* tw) {
  constexpr int P = C2R256_P;
  __shared__ cplx<T> sT[P * 6 * 272];
  const int pr = threadIdx.x / 96, rest = threadIdx.x - 96 * pr;
  const int q = rest >> 4, l = rest & 15;
  const cplx<T>* in = q == 0 ? i0 : q == 1 ? i1 : q == 2 ? i2 : q == 3 ? i3 : q == 4 ? i4 : i5;
  const int64_t r0 = 2 * ((int64_t)blockIdx.x * P + pr), r1 = r0 + 1;
  const int64_t a0 = r0 < rows ? r0 : 0, a1 = r1 < rows ? r1 : 0;
  cplx<T> v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int j = 16 * n1 + l;
    const int jj = n1 < 8 ? j : (256 - j) & 127;
    const cplx<T> A = in[a0 * 128 + jj], B = in[a1 * 128 + jj];
    if (n1 < 8) v[n1] = A + mul_i(B);
    else v[n1] = j == 128 ? mk((T)0, (T)0) : conj(A) + mul_i(conj(B));
  }
  dft16(v, tw, true);
  cplx<T>* st = sT + (pr * 6 + q) * 272;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = (p >> 2) + 4 * (p & 3);
    st[k1 * 17 + l] = k1 == 0 || l == 0 ? v[p] : v[p] * twid256(tw, l * k1, true);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = st[l * 17 + m];
  dft16(v, tw, true);
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 16; ++p) st[l + 16 * ((p >> 2) + 4 * (p & 3))] = v[p];
  __syncthreads();
  const T sc = (T)1 / (T)256;
  for (int idx = threadIdx.x; idx < P * 256; idx += 192) {
    const int pp = idx >> 8, n = idx & 255;
    const int64_t b0 = 2 * ((int64_t)blockIdx.x * P + pp), b1 = b0 + 1;
    T a[6], b[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cplx<T> z = sT[(pp * 6 + c) * 272 + n];
      a[c] = sc * z.x;
      b[c] = sc * z.y;
    }
    if (b0 < rows) {
      T* o = out + (b0 * 256 + n) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = a[c];
    }
    if (b1 < rows) {
      T* o = out + (b1 * 256 + n) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = b[c];
    }
  }
}

// Inverse x transform of the six field components for Nx = 512: per
// (row pair, component) the even and the odd nodes of the Hermitian sequence
// each take the inverse 256-point four-step transform of k_fft_x_c2r6_256
// (16 threads each), and z[m] = E[m] + W512^-m O[m], z[m + 256] = E[m] -
// W512^-m O[m] are formed as the node records are written.  One row pair per
// 192-thread work-group; E and O reuse the transpose buffer.  tw holds
// exp(-2 pi i t / 512) for t < 256.
template <typename T>
__global__ __launch_bounds__(192) void k_fft_x_c2r6_512(const cplx<T>* i0, const cplx<T>* i1, const cplx<T>* i2,
                                                        const cplx<T>* i3, const cplx<T>* i4, const cplx<T>* i5,
                                                        T* out, int64_t rows, const cplx<T>* tw) {
  __shared__ cplx<T> sT[12 * 272];           // per (component, half); then E, O per component
  const int q = threadIdx.x >> 5, h = (threadIdx.x >> 4) & 1, l = threadIdx.x & 15;
  const cplx<T>* in = q == 0 ? i0 : q == 1 ? i1 : q == 2 ? i2 : q == 3 ? i3 : q == 4 ? i4 : i5;
  const int64_t r0 = 2 * (int64_t)blockIdx.x, r1 = r0 + 1;
  const int64_t a0 = r0 < rows ? r0 : 0, a1 = r1 < rows ? r1 : 0;
  cplx<T> v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int j = 2 * (16 * n1 + l) + h;
    const int jj = n1 < 8 ? j : (512 - j) & 255;
    const cplx<T> A = in[a0 * 256 + jj], B = in[a1 * 256 + jj];
    if (n1 < 8) v[n1] = A + mul_i(B);
    else v[n1] = j == 256 ? mk((T)0, (T)0) : conj(A) + mul_i(conj(B));
  }
  dft16(v, tw, true, 2);
  cplx<T>* st = sT + (2 * q + h) * 272;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = (p >> 2) + 4 * (p & 3);
    st[k1 * 17 + l] = k1 == 0 || l == 0 ? v[p] : v[p] * twid256(tw, l * k1, true, 2);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = st[l * 17 + m];
  dft16(v, tw, true, 2);
  __syncthreads();
  cplx<T>* sh = sT + q * 512 + h * 256;
#pragma unroll
  for (int p = 0; p < 16; ++p) sh[l + 16 * ((p >> 2) + 4 * (p & 3))] = v[p];
  __syncthreads();
  const T sc = (T)1 / (T)512;
  for (int n = threadIdx.x; n < 512; n += 192) {
    const int m = n & 255;
    cplx<T> w = tw[m];
    w.y = -w.y;
    T a[6], b[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cplx<T> wO = w * sT[c * 512 + 256 + m];
      const cplx<T> E = sT[c * 512 + m];
      const cplx<T> z = n < 256 ? E + wO : E - wO;
      a[c] = sc * z.x;
      b[c] = sc * z.y;
    }
    if (r0 < rows) {
      T* o = out + (r0 * 512 + n) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = a[c];
    }
    if (r1 < rows) {
      T* o = out + (r1 * 512 + n) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = b[c];
    }
  }
}

// Inverse of the x transform for the six field components at once, written
// as interleaved node records out[row][Nx][6] (scaled by 1/Nx).
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_c2r6(const cplx<T>* i0, const cplx<T>* i1, const cplx<T>* i2,
                                                    const cplx<T>* i3, const cplx<T>* i4, const cplx<T>* i5,
                                                    T* out, int64_t rows, int Nx, int nseq, const cplx<T>* tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const cplx<T>* in[6] = {i0, i1, i2, i3, i4, i5};
  cplx<T>* x = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* y = x + 6 * nseq * Nx;
  cplx<T>* tl = y + 6 * nseq * Nx;
  int64_t pair0 = (int64_t)blockIdx.x * nseq;
  int Nxh = Nx >> 1;
  // spectrum k of both rows gives the Hermitian pair n = k and n = Nx - k
  // (each input read once); the Nyquist entry n = Nxh is zero
  for (int idx = threadIdx.x; idx < 6 * nseq * Nxh; idx += blockDim.x) {
    int sq6 = idx / Nxh, k = idx - sq6 * Nxh;
    int q = sq6 / nseq, sq = sq6 - q * nseq;
    int64_t r0 = 2 * (pair0 + sq), r1 = r0 + 1;
    cplx<T> A = r0 < rows ? in[q][r0 * Nxh + k] : mk((T)0, (T)0);
    cplx<T> B = r1 < rows ? in[q][r1 * Nxh + k] : mk((T)0, (T)0);
    cplx<T>* xs = x + sq6 * Nx;
    xs[k] = A + mul_i(B);
    if (k > 0) xs[Nx - k] = conj(A) + mul_i(conj(B));
    else xs[Nxh] = mk((T)0, (T)0);
  }
  __syncthreads();
  cplx<T>* Z = lds_fft(x, y, tl, Nx, 6 * nseq, tw, true);
  T sc = (T)1 / (T)Nx;
  // one node per thread: its six components are consecutive in the record
  for (int r = threadIdx.x; r < nseq * Nx; r += blockDim.x) {
    int sq = r / Nx, n = r - sq * Nx;
    int64_t r0 = 2 * (pair0 + sq), r1 = r0 + 1;
    T a[6], b[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      cplx<T> z = Z[(q * nseq + sq) * Nx + n];
      a[q] = sc * z.x;
      b[q] = sc * z.y;
    }
    if (r0 < rows) {
      T* o = out + (r0 * Nx + n) * 6;
#pragma unroll
      for (int q = 0; q < 6; ++q) o[q] = a[q];
    }
    if (r1 < rows) {
      T* o = out + (r1 * Nx + n) * 6;
#pragma unroll
      for (int q = 0; q < 6; ++q) o[q] = b[q];
    }
  }
}

// Component q of interleaved node records <-> a plain array.
template <typename T>
__global__ void k_deinterleave(const T* rec, T* out, int q, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = rec[6 * i + q];
}
// Component q of the node records along the column (iy, ix), every zeta
// plane, in FP64.
template <typename T>
__global__ void k_axis(const T* rec, double* out, int q, int Nz, int64_t plane, int64_t col) {
  int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < Nz) out[z] = (double)rec[6 * (z * plane + col) + q];
}
template <typename T>
__global__ void k_interleave(T* rec, const T* in, int q, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rec[6 * i + q] = in[i];
}

// padding of the column stride of k_fft_y in LDS (complex elements)
constexpr int FFTY_PAD = 2;

// Transform along y (columns), in place: data[planes][Ny][Nxh]; a work-group
// takes ncol consecutive kx columns of one plane.  Inverse scales by 1/Ny.
template <typename T>
__global__ __launch_bounds__(512) void k_fft_y(cplx<T>* data, int Ny, int Nxh, int ncol,
                                               const cplx<T>* tw, int inverse) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int S = Ny + FFTY_PAD;                // column stride in LDS
  cplx<T>* x = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* y = x + ncol * S;
  cplx<T>* tl = y + ncol * S;
  int cpp = Nxh / ncol;                       // column groups per plane
  int64_t plane = blockIdx.x / cpp;
  int c0 = (blockIdx.x % cpp) * ncol;
  cplx<T>* base = data + plane * Ny * Nxh + c0;
  for (int idx = threadIdx.x; idx < ncol * Ny; idx += blockDim.x) {
    int row = idx / ncol, c = idx - row * ncol;
    x[c * S + row] = base[(int64_t)row * Nxh + c];
  }
  __syncthreads();
  cplx<T>* Z = lds_fft(x, y, tl, Ny, ncol, tw, inverse != 0, S);
  T sc = inverse ? (T)1 / (T)Ny : (T)1;
  for (int idx = threadIdx.x; idx < ncol * Ny; idx += blockDim.x) {
    int row = idx / ncol, c = idx - row * ncol;
    base[(int64_t)row * Nxh + c] = sc * Z[c * S + row];
  }
}

// Transform along y for Ny = 256 as 16 x 16 (four-step): with row
// n = 16 n1 + n2 and mode k = k1 + 16 k2,
//   X[k1 + 16 k2] = sum_n2 W16^(n2 k2) W256^(n2 k1) sum_n1 W16^(n1 k1) x[16 n1 + n2].
// Thread (column c, n2) takes the 16 rows n2 + 16 n1 into registers, does the
// inner 16-point DFT there and applies W256^(n2 k1); after one LDS transpose
// thread (c, k1) does the outer DFT and writes the rows k1 + 16 k2.  A
// work-group takes the columns of one 128-byte segment of every row (16 FP32
// or 8 FP64 complex values), 16 threads per column; the inverse conjugates
// the twiddles and scales by 1/256.  tw holds exp(-2 pi i t / 256) for
// t < 128.
// columns per work-group (one 128-byte row segment)
template <typename T> constexpr int fy_nc() { return 128 / (int)sizeof(cplx<T>); }
template <typename T>
__global__ __launch_bounds__(256) void k_fft_y256(cplx<T>* data, int Nxh, const cplx<T>* tw, int inverse) {
  constexpr int NC = fy_nc<T>(), KS = 16 * NC + 4;
  __shared__ cplx<T> sY[16 * KS];      // [k1][n2][c]
  const int cpp = Nxh / NC;
  const int64_t plane = blockIdx.x / cpp;
  const int c0 = (int)(blockIdx.x % cpp) * NC;
  const int c = threadIdx.x % NC, q = threadIdx.x / NC;   // q: n2, then k1
  cplx<T>* col = data + plane * 256 * Nxh + c0 + c;
  const bool inv = inverse != 0;
  cplx<T> v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = col[(int64_t)(16 * n1 + q) * Nxh];
  dft16(v, tw, inv);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = (p >> 2) + 4 * (p & 3);
    sY[k1 * KS + q * NC + c] = k1 == 0 || q == 0 ? v[p] : v[p] * twid256(tw, q * k1, inv);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = sY[q * KS + m * NC + c];
  dft16(v, tw, inv);
  const T sc = inv ? (T)1 / (T)256 : (T)1;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k2 = (p >> 2) + 4 * (p & 3);
    col[(int64_t)(q + 16 * k2) * Nxh] = sc * v[p];
  }
}

// Transform along y for Ny = 512: with NC columns per work-group, the even
// rows (the first 16 NC threads) and the odd rows (the other 16 NC) each take
// the 256-point four-step transform above, then X[k] = E[k] + W512^k O[k] and
// X[k + 256] = E[k] - W512^k O[k].  tw holds exp(-2 pi i t / 512) for t < 256.
template <typename T>
__global__ __launch_bounds__(512) void k_fft_y512(cplx<T>* data, int Nxh, const cplx<T>* tw, int inverse) {
  constexpr int NC = fy_nc<T>(), KS = 16 * NC + 4, TH = 16 * NC;
  __shared__ cplx<T> sY[2 * 16 * KS];  // per half [k1][n2][c]; then the halves' results [h][k][c]
  const int cpp = Nxh / NC;
  const int64_t plane = blockIdx.x / cpp;
  const int c0 = (int)(blockIdx.x % cpp) * NC;
  const int h = threadIdx.x / TH, t = threadIdx.x % TH;
  const int c = t % NC, q = t / NC;   // q: n2, then k1
  cplx<T>* const base = data + plane * 512 * Nxh + c0;
  cplx<T>* col = base + c;
  cplx<T>* sh = sY + h * 16 * KS;
  const bool inv = inverse != 0;
  cplx<T> v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = col[(int64_t)(2 * (16 * n1 + q) + h) * Nxh];
  dft16(v, tw, inv, 2);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k1 = (p >> 2) + 4 * (p & 3);
    sh[k1 * KS + q * NC + c] = k1 == 0 || q == 0 ? v[p] : v[p] * twid256(tw, q * k1, inv, 2);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = sh[q * KS + m * NC + c];
  dft16(v, tw, inv, 2);
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k = q + 16 * ((p >> 2) + 4 * (p & 3));
    sY[(h * 256 + k) * NC + c] = v[p];
  }
  __syncthreads();
  const T sc = inv ? (T)1 / (T)512 : (T)1;
  for (int idx = threadIdx.x; idx < 256 * NC; idx += 2 * TH) {
    const int cc = idx % NC, k = idx / NC;
    const cplx<T> E = sY[k * NC + cc], O = sY[(256 + k) * NC + cc];
    cplx<T> w = tw[k];
    if (inv) w.y = -w.y;
    const cplx<T> wO = w * O;
    base[(int64_t)k * Nxh + cc] = sc * (E + wO);
    base[(int64_t)(k + 256) * Nxh + cc] = sc * (E - wO);
  }
}

// ---------------------------------------------------------------------------
// The march.  One thread per transverse mode (ky, kx); zeta nodes n = Nz-1 .. 0.
// Node "1" (n + 1, new level) is known; node 0 (n) is solved with App. B:
//   K^2 = kx^2 + ky^2,  D = 16 + h (2 Delta + h) K^2,
//   Jx = sum of the four j_x (both levels, both half-nodes), likewise Jy,
//   Wx = -2 Lx1 + Rx0^0 + Rx1,  Ux = 2 Lx1 + Rx0^0 + Rx1 (and y),
//   Ez0^1 = [Ez1 (16 - h^2 K^2) - 16 h jz+ - i h Delta (kx Jx + ky Jy)
//            - 2 h Delta Ez0^0 K^2 + 2 i h^2 (kx jx+ + ky jy+)
//            + 4 i h (kx Wx + ky Wy)] / D,
//   Bz0^1 = [Bz1 (16 - h^2 K^2) + 2 i h^2 (kx jy+ - ky jx+)
//            + i h Delta (kx Jy - ky Jx) - 2 h Delta Bz0^0 K^2
//            + 4 i h (ky Ux - kx Uy)] / D,
// then Rx, Ry from RxN/RyN and Lx, Ly from the L equations, with the readings
// (Ly equation with (Bz0^1 + Bz1^1)/2; Ez equation with + i ky (Bx0 + Bx1)/2;
// T4 with a minus sign) under which this closed form solves the node system.
// Currents j^0 = j^1 = the step's deposit.  Solver current on half-node
// n + 1/2 (plane n + 2 of the raw deposit):
//   jx = filt[(Jx(n) + Jx(n+1)) / 2] exp(-i kx hx / 2), jy likewise with ky hy
//   (3-D), jz = filt[Jz(n + 1/2)],
// where filt is the binomial filter: (1,2,1)/4 per pass along zeta (zero
// beyond the stored planes) and cos^2(k h / 2) per pass and transverse axis.
template <typename T>
struct MarchArgs {
  Geom g;
  const cplx<T>* J[3];     // raw current spectra [NPF][Ny][Nxh]; null = no current
  cplx<T>* st[4];          // Rx, Ry, Ez, Bz [Nz][Ny][Nxh] (old level in, new level out)
  cplx<T>* out[6];         // Ex, Ey, Ez, Bx, By, Bz spectra [Nz][Ny][Nxh]
  cplx<T>* L[2];           // nullable: Lx, Ly of the new level
  T Delta;
};

// Raw current planes of one component around the plane being filtered:
// r[k] = plane c - P + k for the centre plane c, plus the next lower plane.
template <typename T, int P>
struct PlaneWin {
  cplx<T> r[2 * P + 1];
  cplx<T> nxt;
};

template <typename T>
GP_DEV cplx<T> load_plane(const cplx<T>* A, int q, int NPF, int64_t stride, int64_t m) {
  return (q >= 0 && q < NPF) ? A[(int64_t)q * stride + m] : mk((T)0, (T)0);
}

// binomial filter along the plane index (P passes), in the order of the
// plane offsets -P .. P; out-of-range planes hold zero
template <typename T, int P>
GP_DEV cplx<T> win_filter(const PlaneWin<T, P>& w) {
  if (P == 0) return w.r[0];
  const T w1[3] = {(T)0.25, (T)0.5, (T)0.25};
  const T w2[5] = {(T)0.0625, (T)0.25, (T)0.375, (T)0.25, (T)0.0625};
  cplx<T> r = mk((T)0, (T)0);
#pragma unroll
  for (int k = 0; k < 2 * P + 1; ++k) r = r + (P == 1 ? w1[k] : w2[k]) * w.r[k];
  return r;
}

// move the window centre one plane down (the prefetched plane enters)
template <typename T, int P>
GP_DEV void win_slide(PlaneWin<T, P>& w) {
#pragma unroll
  for (int k = 2 * P; k > 0; --k) w.r[k] = w.r[k - 1];
  w.r[0] = w.nxt;
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_march(MarchArgs<T> a) {
  const Geom& g = a.g;
  int64_t M = (int64_t)g.Ny * g.Nxh;
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  int kyi = (int)(m / g.Nxh), kxi = (int)(m % g.Nxh);
  const double PI = 3.14159265358979323846;
  double kxd = 2.0 * PI * (double)kxi / ((double)g.Nx * g.hx);
  int kys = kyi <= g.Ny / 2 ? kyi : kyi - g.Ny;
  double kyd = g.Ny > 1 ? 2.0 * PI * (double)kys / ((double)g.Ny * g.hy) : 0.0;
  bool nyq = g.Ny > 1 && kyi == g.Ny / 2;
  int64_t stride = M;
  if (nyq) {
    cplx<T> z = mk((T)0, (T)0);
    for (int n = 0; n < g.Nz; ++n) {
      int64_t o = (int64_t)n * stride + m;
      for (int q = 0; q < 4; ++q) a.st[q][o] = z;
      for (int q = 0; q < 6; ++q) a.out[q][o] = z;
      if (a.L[0]) { a.L[0][o] = z; a.L[1][o] = z; }
    }
    return;
  }
  T kx = (T)kxd, ky = (T)kyd;
  T h = (T)g.h, D = a.Delta;
  T K2 = kx * kx + ky * ky;
  T Dd = (T)16 + h * ((T)2 * D + h) * K2;
  T inv = (T)1 / Dd;
  T c16 = (T)16 - h * h * K2;
  // transverse filter and half-cell shifts
  double fx = cos(0.5 * kxd * g.hx), fxy = fx * fx;
  if (g.dims == 3) { double fy = cos(0.5 * kyd * g.hy); fxy *= fy * fy; }
  double phi = P == 0 ? 1.0 : (P == 1 ? fxy : fxy * fxy);
  cplx<T> sx = mk((T)(0.5 * phi * cos(0.5 * kxd * g.hx)), (T)(-0.5 * phi * sin(0.5 * kxd * g.hx)));
  cplx<T> sy = g.dims == 3 ? mk((T)(0.5 * phi * cos(0.5 * kyd * g.hy)), (T)(-0.5 * phi * sin(0.5 * kyd * g.hy)))
                           : mk((T)(0.5 * phi), (T)0);
  T phz = (T)phi;
  const bool hasJ = a.J[0] != nullptr;
  const int NPF = g.NPF;
  // filtered planes of Jx, Jy (nodal) carried between iterations
  cplx<T> fxp = mk((T)0, (T)0), fyp = fxp;   // filtered plane n + 2 (node n + 1 of half-node n + 1/2)
  cplx<T> jxp = fxp, jyp = fxp, jzp = fxp;   // solver currents on half-node n + 1/2
  PlaneWin<T, P> W[3];
  if (hasJ) {
    // windows centred on plane Nz + 2, then slid to Nz + 1
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * P + 1; ++k) W[c].r[k] = load_plane(a.J[c], g.Nz + 2 - P + k, NPF, stride, m);
    }
    cplx<T> f2 = win_filter(W[0]), e2 = win_filter(W[1]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      W[c].nxt = load_plane(a.J[c], g.Nz + 1 - P, NPF, stride, m);
      win_slide(W[c]);
    }
    // half-node q = Nz: planes Nz + 1, Nz + 2
    cplx<T> f1 = win_filter(W[0]), e1 = win_filter(W[1]);
    jxp = sx * (f1 + f2);
    fxp = f1;
    jyp = sy * (e1 + e2);
    fyp = e1;
    jzp = phz * win_filter(W[2]);
  }
  // Node n uses its old state and the raw current plane n + 1 - P, both
  // loaded PD nodes ahead into ring slot (Nz - 1 - n) mod PD (the loop is
  // unrolled by PD so that every slot index is static).
  constexpr int PD = sizeof(T) == 4 ? 8 : 4;
  cplx<T> S[PD][4], Pl[PD][3];
#pragma unroll
  for (int i = 0; i < PD; ++i) {
    int n = g.Nz - 1 - i;
    if (n >= 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) S[i][q] = a.st[q][(int64_t)n * stride + m];
      if (hasJ) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Pl[i][c] = load_plane(a.J[c], n + 1 - P, NPF, stride, m);
      }
    }
  }
  cplx<T> Rx1 = mk((T)0, (T)0), Ry1 = Rx1, Lx1 = Rx1, Ly1 = Rx1, Ez1 = Rx1, Bz1 = Rx1;
  for (int n0 = g.Nz - 1; n0 >= 0; n0 -= PD) {
#pragma unroll
  for (int i = 0; i < PD; ++i) {
    const int n = n0 - i;
    if (n < 0) break;
    int64_t o = (int64_t)n * stride + m;
    const cplx<T> Rx0 = S[i][0], Ry0 = S[i][1], Ez0 = S[i][2], Bz0 = S[i][3];
    cplx<T> jxm = mk((T)0, (T)0), jym = jxm, jzm = jxm;
    if (hasJ) {
      // half-node n - 1/2: planes n + 1 (new) and n + 2 (carried)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        W[c].nxt = Pl[i][c];
        win_slide(W[c]);
      }
      cplx<T> f1 = win_filter(W[0]);
      jxm = sx * (f1 + fxp);
      fxp = f1;
      cplx<T> e1 = win_filter(W[1]);
      jym = sy * (e1 + fyp);
      fyp = e1;
      jzm = phz * win_filter(W[2]);
    }
    // refill the slot with node n - PD
    if (n - PD >= 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) S[i][q] = a.st[q][o - PD * stride];
      if (hasJ) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Pl[i][c] = load_plane(a.J[c], n - PD + 1 - P, NPF, stride, m);
      }
    }
    cplx<T> Jx = (T)2 * (jxm + jxp);
    cplx<T> Jy = (T)2 * (jym + jyp);
    cplx<T> Wx = (Rx0 + Rx1) - (T)2 * Lx1;
    cplx<T> Wy = (Ry0 + Ry1) - (T)2 * Ly1;
    cplx<T> Ux = (Rx0 + Rx1) + (T)2 * Lx1;
    cplx<T> Uy = (Ry0 + Ry1) + (T)2 * Ly1;
    cplx<T> Ez = c16 * Ez1 - ((T)16 * h) * jzp
                 - mul_i((h * D) * (kx * Jx + ky * Jy))
                 - ((T)2 * h * D * K2) * Ez0
                 + mul_i(((T)2 * h * h) * (kx * jxp + ky * jyp))
                 + mul_i(((T)4 * h) * (kx * Wx + ky * Wy));
    Ez = inv * Ez;
    cplx<T> Bz = c16 * Bz1 + mul_i(((T)2 * h * h) * (kx * jyp - ky * jxp))
                 + mul_i((h * D) * (kx * Jy - ky * Jx))
                 - ((T)2 * h * D * K2) * Bz0
                 + mul_i(((T)4 * h) * (ky * Ux - kx * Uy));
    Bz = inv * Bz;
    cplx<T> Ezs = Ez + Ez0, Bzs = Bz + Bz0;
    cplx<T> Rx = Rx0 + mul_i(((T)0.5 * D) * (kx * Ezs + ky * Bzs)) - ((T)0.25 * D) * Jx;
    cplx<T> Ry = Ry0 + mul_i(((T)0.5 * D) * (ky * Ezs - kx * Bzs)) - ((T)0.25 * D) * Jy;
    cplx<T> Ezp = Ez1 + Ez, Bzp = Bz + Bz1;
    cplx<T> Lx = Lx1 - ((T)0.5 * h) * (mul_i((T)0.5 * (kx * Ezp - ky * Bzp)) + jxp);
    cplx<T> Ly = Ly1 - ((T)0.5 * h) * (mul_i((T)0.5 * (ky * Ezp + kx * Bzp)) + jyp);
    a.st[0][o] = Rx;
    a.st[1][o] = Ry;
    a.st[2][o] = Ez;
    a.st[3][o] = Bz;
    a.out[0][o] = (T)0.5 * (Rx + Lx);
    a.out[1][o] = (T)0.5 * (Ry + Ly);
    a.out[2][o] = Ez;
    a.out[3][o] = (T)0.5 * (Ly - Ry);
    a.out[4][o] = (T)0.5 * (Rx - Lx);
    a.out[5][o] = Bz;
    if (a.L[0]) { a.L[0][o] = Lx; a.L[1][o] = Ly; }
    Rx1 = Rx; Ry1 = Ry; Lx1 = Lx; Ly1 = Ly; Ez1 = Ez; Bz1 = Bz;
    jxp = jxm; jyp = jym; jzp = jzm;
  }
  }
}

// E/B spectra from a given (R, L, Ez, Bz) state (state upload).
template <typename T>
__global__ void k_state_to_fields(const cplx<T>* Rx, const cplx<T>* Ry, const cplx<T>* Lx,
                                  const cplx<T>* Ly, const cplx<T>* Ez, const cplx<T>* Bz,
                                  cplx<T>* o0, cplx<T>* o1, cplx<T>* o2, cplx<T>* o3, cplx<T>* o4,
                                  cplx<T>* o5, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  o0[i] = (T)0.5 * (Rx[i] + Lx[i]);
  o1[i] = (T)0.5 * (Ry[i] + Ly[i]);
  o2[i] = Ez[i];
  o3[i] = (T)0.5 * (Ly[i] - Ry[i]);
  o4[i] = (T)0.5 * (Rx[i] - Lx[i]);
  o5[i] = Bz[i];
}

// Laser field E_pol(x, y, zeta) = lon[n] * tra[j][i] on the field nodes,
// times 2 (R = 2 E for a pure forward wave).
template <typename T>
__global__ void k_laser(T* out, const double* lon, const double* tra, int Nz, int64_t nxy) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Nz * nxy) return;
  int64_t n = i / nxy, r = i - n * nxy;
  out[i] = (T)(2.0 * (lon[n] * tra[r]));
}

// zero a buffer of T
// Field of the driver beam as a forward wave: per zeta node, phi^ = rho_f^ /
// K^2, E_perp^ = -i k_perp phi^, R_perp += 2 E_perp^ (Nyquist rows and K = 0
// give 0).  rho_f is the node charge after the current filter: P passes of
// 1-2-1 along zeta (zero beyond the nodes 0 .. Nz-1, each pass) and the
// transverse factor (cos^2(k_x h_x/2) cos^2(k_y h_y/2))^P.  rho_hat and R in
// the [Nz][Ny][Nx/2] half-spectrum layout.
template <typename T>
__global__ void k_beam_R(const cplx<T>* rho_hat, cplx<T>* Rx, cplx<T>* Ry, int Nz, int Ny, int Nxh,
                         double hx, double hy, int P) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nsp = (int64_t)Nz * Ny * Nxh;
  if (idx >= nsp) return;
  const int64_t pl = (int64_t)Ny * Nxh;
  int i = (int)(idx % Nxh);
  int j = (int)((idx / Nxh) % Ny);
  int n = (int)(idx / pl);
  if (Ny > 1 && j == Ny / 2) return;
  double kx = 2.0 * M_PI * (double)i / ((double)(2 * Nxh) * hx);
  int jj = j < (Ny + 1) / 2 ? j : j - Ny;
  double ky = Ny > 1 ? 2.0 * M_PI * (double)jj / ((double)Ny * hy) : 0.0;
  double K2 = kx * kx + ky * ky;
  if (K2 == 0.0) return;
  const int64_t m0 = idx - (int64_t)n * pl;   // this mode in plane 0
  auto raw = [&](int m, double* re, double* im) {
    if (m < 0 || m >= Nz) { *re = 0.0; *im = 0.0; return; }
    cplx<T> v = rho_hat[(int64_t)m * pl + m0];
    *re = (double)v.x; *im = (double)v.y;
  };
  auto pass1 = [&](int m, double* re, double* im) {
    if (m < 0 || m >= Nz) { *re = 0.0; *im = 0.0; return; }
    double a, b, c, d, e, f;
    raw(m - 1, &a, &b); raw(m, &c, &d); raw(m + 1, &e, &f);
    *re = 0.25 * (a + 2.0 * c + e);
    *im = 0.25 * (b + 2.0 * d + f);
  };
  double pr, pi;
  if (P == 0) {
    raw(n, &pr, &pi);
  } else if (P == 1) {
    pass1(n, &pr, &pi);
  } else {
    double a, b, c, d, e, f;
    pass1(n - 1, &a, &b); pass1(n, &c, &d); pass1(n + 1, &e, &f);
    pr = 0.25 * (a + 2.0 * c + e);
    pi = 0.25 * (b + 2.0 * d + f);
  }
  double cx = std::cos(0.5 * kx * hx), cy = Ny > 1 ? std::cos(0.5 * ky * hy) : 1.0;
  double tr = 1.0;
  for (int q = 0; q < P; ++q) tr *= (cx * cx) * (cy * cy);
  pr *= tr / K2;
  pi *= tr / K2;
  // -2 i k (pr + i pi) = 2 k pi - 2 i k pr
  Rx[idx].x += (T)(2.0 * kx * pi);
  Rx[idx].y += (T)(-2.0 * kx * pr);
  Ry[idx].x += (T)(2.0 * ky * pi);
  Ry[idx].y += (T)(-2.0 * ky * pr);
}

// Lab current of charge moving at c from its node density: J_z(n + 1/2) =
// (rho(n) + rho(n + 1)) / 2 on planes n + 2, n = -1 .. Nz - 1 (rho zero
// outside the nodes 0 .. Nz - 1); Jz holds NPJ planes.
template <typename T>
__global__ void k_beam_jz(const T* rho, T* Jz, int Nz, int64_t nxy) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)(Nz + 1) * nxy) return;
  int n = (int)(idx / nxy) - 1;
  int64_t r = idx % nxy;
  T a = n >= 0 ? rho[(int64_t)n * nxy + r] : (T)0;
  T b = n + 1 < Nz ? rho[(int64_t)(n + 1) * nxy + r] : (T)0;
  Jz[(int64_t)(n + 2) * nxy + r] = (T)0.5 * (a + b);
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// The same fill with one 16-byte store per thread over a 16-byte aligned p;
// threads past the nv = n / W vectors write the n % W tail elements.
template <typename T>
__global__ void k_fill16(T* p, int64_t n, T v) {
  constexpr int W = 16 / (int)sizeof(T);
  struct alignas(16) V { T e[W]; };
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = n / W;
  if (i < nv) {
    V x;
#pragma unroll
    for (int k = 0; k < W; ++k) x.e[k] = v;
    reinterpret_cast<V*>(p)[i] = x;
  } else if (i - nv < n - nv * W) {
    p[nv * W + (i - nv)] = v;
  }
}
