// Learned current denoiser on gfx950: BF16 MFMA 3x3x3 convolutions
// (3 -> 16 -> 32 -> 16 -> 3, ReLU, FP32 accumulation), the staggered curl
// correction of the binomially filtered current, the continuity test that
// selects between them, and the training step (loss, backward, Adam).
//
// Layouts
//   boxes are (Z, Y, X) voxels, x and y periodic, zero beyond the Z planes;
//   currents, A and their gradients: FP32 planar [3][Z][Y][X];
//   hidden activations and their gradients: bf16 channels-last [Z][Y][X][C],
//   32 channels as two halves [2][Z][Y][X][16];
//   parameters: FP32, layer by layer W[Cout][Cin][kz][ky][kx] then b[Cout].
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 with the
// output channels as the MFMA rows (operand A = weights, kept in VGPRs for
// the whole work-group) and 16 consecutive x voxels as the columns (operand
// B = activations, one 16-byte LDS read per lane from a halo tile).  The
// reduction index k = (tap, input channel) is split in steps of 32; a lane
// group g (lanes 16g .. 16g+15) supplies the 8 values k = 32 s + 8 g + e of
// both operands, so operands A and B agree element by element.  The k-steps
// are ordered by (group of (dz, dx) taps, dy), so that one LDS read serves
// three output rows; 32-channel inputs are reduced in two 16-channel phases,
// each with its half of the halo in its own LDS buffer.  The 16 -> 3 output
// layer instead folds its y taps into the MFMA rows (row 4 c + dy) and sums
// the three partial rows in-lane.  The data gradient is
// the same kernel with flipped taps and transposed channels; weight
// gradients are MFMAs with the voxels as the reduction index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gempic.h"
#include "../../include/gempic_denoise.h"
#include "common.h"
#include "dn_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int NLAYER = 4;
constexpr int L_CIN[NLAYER] = {3, 16, 32, 16};
constexpr int L_COUT[NLAYER] = {16, 32, 16, 3};
constexpr int pad_in(int c) { return c <= 8 ? 8 : c; }          // MFMA k-chunks of 8
constexpr int pad_out(int c) { return c <= 16 ? 16 : 32; }      // MFMA rows of 16

int64_t layer_woff(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += (int64_t)L_COUT[i] * L_CIN[i] * 27 + L_COUT[i];
  return o;
}
int64_t n_params() { return layer_woff(NLAYER); }
// 32-channel inputs are convolved in two phases of 16 channels (halves of
// the halo tile in LDS, double-buffered); a phase reduces over 16 or fewer
// channels
GP_HD constexpr int conv_split(int cinp) { return cinp == 32 ? 2 : 1; }
// the output layer (16 -> 3) folds its y taps into the MFMA rows: row
// 4 c + dy of operand A holds output channel c at tap row dy, and the
// reduction index is (dz, dx, input channel) only: five k-steps of 32
constexpr int FOLD_NKS = 5;
int64_t fold_units() { return (int64_t)FOLD_NKS * 64; }
int64_t packed_units(int cinp, int coutp) {
  int ce = cinp / conv_split(cinp);
  int tpk = 32 / ce;
  int nks = 3 * ((9 + tpk - 1) / tpk);
  return (int64_t)conv_split(cinp) * nks * (coutp / 16) * 64;
}

constexpr int TZ = 4, TY = 8, TX = 16;        // output tile of one work-group
// halo rows whose LDS fragments are read ahead of their MFMAs: all of them,
// or half with 32 output channels (twice the accumulators in registers)
constexpr int pf_rows(int nct) { return nct == 2 ? 5 : TY + 2; }
constexpr int HZ = TZ + 2, HY = TY + 2, HX = TX + 2;
constexpr int HALO = HZ * HY * HX;            // 1080 voxels
constexpr int TILE = TZ * TY * TX;            // 512 voxels

GP_DEV unsigned f2bf(float f) {               // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
// two floats -> packed bf16 (round to nearest even, v_cvt_pk_bf16_f32)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
GP_DEV unsigned pack_bf16(float lo, float hi) {
  f32x2 v = {lo, hi};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

GP_DEV float bf2f(unsigned b) { return __uint_as_float(b << 16); }

// Hidden activations (and their gradients) are bf16 channels-last; a
// 32-channel tensor is stored as two 16-channel halves one after the other,
// [half][voxel][16], so that either half of a voxel's channels (the part one
// phase of the next convolution reduces over) is 32 contiguous bytes.
// 16-byte unit u (channels 8u .. 8u + 7) of voxel v of a tensor with U units
// per voxel and V voxels:
template <int U>
GP_DEV int64_t unit_at(int64_t v, int u, int64_t V) {
  if constexpr (U == 4) return ((int64_t)(u >> 1) * V + v) * 2 + (u & 1);
  else return v * U + u;
}
// element (channel c) of voxel v, for a tensor with C channels
template <int C>
GP_DEV int64_t chan_at(int64_t v, int c, int64_t V) {
  if constexpr (C == 32) return ((int64_t)(c >> 4) * V + v) * 16 + (c & 15);
  else return v * C + c;
}
GP_DEV int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// weight packing: MFMA operand A for every (k-step s, row tile j, lane)
struct PackArgs {
  const float* W;     // layer weights [cout][cin][27]
  int cin, cout;      // layer channels
  int cinp, coutp;    // padded channels of the packed convolution
  int transpose;      // 1: data-gradient convolution (cout -> cin, flipped taps)
  int fold;           // 1: output layer with its y taps folded into the rows (cinp = 16, cout <= 4)
  u32x4* out;
  int64_t units;
};

__global__ void k_pack(PackArgs a) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= a.units) return;
  int lane = (int)(u % 64);
  int64_t r = u / 64;
  int nct = a.coutp / 16;
  int j = (int)(r % nct);
  r /= nct;
  int g = lane >> 4, n = lane & 15;
  if (a.fold) {
    // k-step s: lane-group slot g / 2 takes the (dz, dx) combination
    // q = 2 s + g / 2 (q = 9: zero padding), input channels 8 (g % 2) .. + 7;
    // row n is output channel n / 4 at tap row dy = n % 4 (dy = 3: zero)
    int s = (int)r;
    int q = 2 * s + g / 2;
    int co = n / 4, dy = n % 4;
    unsigned w[8];
    for (int e = 0; e < 8; ++e) {
      int ci = 8 * (g % 2) + e;
      float v = 0.0f;
      if (q < 9 && dy < 3 && co < a.cout && ci < a.cin) v = a.W[((int64_t)co * a.cin + ci) * 27 + (q / 3) * 9 + dy * 3 + q % 3];
      w[e] = f2bf(v);
    }
    u32x4 o;
    o[0] = w[0] | (w[1] << 16);
    o[1] = w[2] | (w[3] << 16);
    o[2] = w[4] | (w[5] << 16);
    o[3] = w[6] | (w[7] << 16);
    a.out[u] = o;
    return;
  }
  // phase p reduces over the packed input channels p ce .. p ce + ce - 1;
  // its k-step s = 3 cg + (dy + 1) takes, in lane-group slot i, the (dz, dx)
  // combination q = cg tpk + i (q > 8: zero padding) at that dy
  int ce = a.cinp / conv_split(a.cinp);
  int tpk = 32 / ce;
  int nks = 3 * ((9 + tpk - 1) / tpk);
  int s = (int)(r % nks), p = (int)(r / nks);
  int q = (s / 3) * tpk + (g * 8) / ce;
  int tp = q < 9 ? (q / 3) * 9 + (s % 3) * 3 + q % 3 : 27;   // tap of the packed convolution
  int c0 = p * ce + (g * 8) % ce;
  int orow = 16 * j + n;                    // packed output channel
  unsigned w[8];
  for (int e = 0; e < 8; ++e) {
    int cin_p = c0 + e;                     // packed input channel
    int co, ci, t;
    if (a.transpose) { co = cin_p; ci = orow; t = 26 - tp; }
    else { co = orow; ci = cin_p; t = tp; }
    float v = 0.0f;
    if (tp <= 26 && co < a.cout && ci < a.cin) v = a.W[((int64_t)co * a.cin + ci) * 27 + t];
    w[e] = f2bf(v);
  }
  u32x4 o;
  o[0] = w[0] | (w[1] << 16);
  o[1] = w[2] | (w[3] << 16);
  o[2] = w[4] | (w[5] << 16);
  o[3] = w[6] | (w[7] << 16);
  a.out[u] = o;
}

// ---------------------------------------------------------------------------
// convolution (forward, or data gradient with packed transposed weights)
//   INMODE 0: bf16 channels-last input with CINP channels
//   INMODE 1: FP32 planar 3-component input times in_scale (CINP = 8)
//   OUTMODE 0: bf16 channels-last, + bias, ReLU
//   OUTMODE 1: FP32 planar, first 3 channels, + bias
//   OUTMODE 2: bf16 channels-last, zero where mask <= 0 (ReLU derivative)
struct ConvArgs {
  int Z, Y, X;
  const u32x4* in;
  const float* inf[3];
  float in_scale;
  const u32x4* wp;
  const float* bias;
  unsigned short* out;
  float* outf[3];
  const unsigned short* mask;
};

// 16 zero bytes: the source of halo voxels outside the box for direct
// global-to-LDS loads
__device__ u32x4 g_zero16;

template <int CINP, int COUTP, int INMODE, int OUTMODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv(ConvArgs a) {
  constexpr int U = CINP / 8;               // 16-byte units per voxel
  constexpr int KS = conv_split(CINP);      // phases per tile
  constexpr int CE = CINP / KS;             // channels of a phase
  constexpr int UE = CE / 8;                // units of a phase (in LDS)
  constexpr int TPK = 32 / CE;              // taps per k-step
  constexpr int NCG = (9 + TPK - 1) / TPK;  // column groups of (dz, dx) combinations
  constexpr int NKS = 3 * NCG;              // k-steps of a phase: (column group, dy)
  constexpr int NCT = COUTP / 16;
  static_assert(TZ == 4, "one output plane per wave");
  // FOLD (the 16 -> 3 output layer): operand A row 4 c + dy is output channel
  // c at tap row dy, the k-steps run over (dz, dx, input channel) only, and
  // each halo row h has its own accumulator; output row r of channel c (lane
  // group c) is then the in-lane sum of rows dy of the accumulators of halo
  // rows r + dy: 5 (TY + 2) MFMAs per wave and tile instead of 3 NCG TY
  constexpr bool FOLD = INMODE == 0 && OUTMODE == 1 && CINP == 16 && COUTP == 16;
  constexpr int NKSW = FOLD ? FOLD_NKS : NKS;   // packed k-steps per phase
  constexpr int NACC = FOLD ? TY + 2 : TY;      // accumulators per row tile
  constexpr int PF = pf_rows(NCT);          // halo rows read ahead
  // DIRECT (two-unit phases: 16-channel inputs with 32 output channels, and
  // both halves of 32-channel inputs): two halo buffers; the next phase's
  // halo is read straight from global memory into the other buffer
  // (global_load_lds) while the current one is used.  Its tile is
  // voxel-major, sX[voxel * 2 + unit]: a wave instruction then loads both
  // units of 32 voxels, 32 contiguous bytes each (one unit of 64 voxels
  // would take 16 bytes out of every 32 or 64 and touch twice or four times
  // the cache lines).  (16 -> 16 channels: the second buffer would cost a
  // wave per SIMD; there the registers take the halo instead.)
  // Otherwise the tile is unit-major, sX[unit * HALO_P + voxel], the unit
  // stride padded so that the units start on different banks.
  // Either way the 16 lanes of a lane group read one unit of 16 consecutive
  // voxels.
  constexpr bool DIRECT = INMODE == 0 && UE == 2 && (COUTP == 32 || KS == 2);
  static_assert(KS == 1 || DIRECT, "split phases are double-buffered");
  constexpr int NCH2 = (HALO + 31) / 32;    // DIRECT: 32-voxel chunks of the tile
  constexpr int HALO_P = HALO + 2;
  constexpr int BUFU = DIRECT ? NCH2 * 64 : HALO_P * UE;   // 16-byte units per halo buffer
  constexpr int VS = DIRECT ? UE : 1;       // stride of one voxel in units
  __shared__ u32x4 sXbuf[(DIRECT ? 2 : 1) * BUFU];
  u32x4* sX = sXbuf;

  // Persistent work-groups walk the output tiles t0, t0 + gridDim.x, ... (t0
  // below).  The weights are loaded once per work-group.  The next tile's halo is
  // fetched while the current tile is computed: directly into the other LDS
  // buffer (DIRECT), else its first PU channel units (INMODE 0) or its FP32
  // input planes (INMODE 1) into registers, the rest after the tile.
  const int nbx = a.X / TX, nby = a.Y / TY;
  const int ntile = nbx * nby * ((a.Z + TZ - 1) / TZ);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
  bf16x8 wr[KS][NKSW][NCT];
#pragma unroll
  for (int p = 0; p < KS; ++p)
#pragma unroll
    for (int s = 0; s < NKSW; ++s)
#pragma unroll
      for (int j = 0; j < NCT; ++j)
        wr[p][s][j] = __builtin_bit_cast(bf16x8, a.wp[((p * NKSW + s) * NCT + j) * 64 + lane]);

  // biases in registers: loaded from global memory in the epilogue, they
  // would be reloaded after every output store (the pointers may alias) and
  // each reload would wait for all outstanding stores and loads
  float bias_r[NCT][4];
#pragma unroll
  for (int j = 0; j < NCT; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = 16 * j + 4 * g + i;
      if (FOLD) bias_r[j][i] = i == 0 && g < 3 ? a.bias[g] : 0.0f;
      else bias_r[j][i] = OUTMODE == 0 ? a.bias[co] : OUTMODE == 1 && j == 0 && i < 3 ? a.bias[i] : 0.0f;
    }

  // units prefetched into registers (register budget); the folded output
  // layer has the registers to take its whole halo, so no part of it is
  // loaded between the barriers
  constexpr int PU = FOLD ? U : U >= 4 ? 2 : 1;
  // staging of channel units [U0, U0 + UW): one halo row (HX voxels x UW
  // units, contiguous in global memory apart from the periodic wrap) per
  // group of HX * UW threads; row k of this thread is first + k * PER
  auto halo_rows = [&](int t, auto u0c, auto uwc, auto&& put) {
    constexpr int U0 = decltype(u0c)::value, UW = decltype(uwc)::value;
    constexpr int RW = HX * UW, PER = 256 / RW, NR = (HZ * HY + PER - 1) / PER;
    int b = t;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby, bz = b / nby;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int iw = tid % RW;
    const int hx = iw / UW, part = U0 + iw - hx * UW;
    const int gx = wrapi(x0 + hx - 1, a.X);
    const int first = tid < PER * RW ? tid / RW : HZ * HY;   // spare threads idle
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int row = first + k * PER;
      if (row < HZ * HY) {
        const int hz = row / HY, hy = row - hz * HY;
        const int gz = z0 + hz - 1;
        const int gy = wrapi(y0 + hy - 1, a.Y);
        const bool inz = gz >= 0 && gz < a.Z;
        put(k, part * HALO_P + row * HX + hx, inz,
            unit_at<U>(((int64_t)gz * a.Y + gy) * a.X + gx, part, (int64_t)a.Z * a.Y * a.X));
      }
    }
  };
  constexpr int NPR = (HZ * HY + 256 / (HX * PU) - 1) / (256 / (HX * PU));
  u32x4 pre[INMODE == 0 && !DIRECT ? NPR : 1];
  using IC0 = std::integral_constant<int, 0>;
  using ICPU = std::integral_constant<int, PU>;
  using ICU = std::integral_constant<int, U>;
  using ICR = std::integral_constant<int, (U > PU ? U - PU : 1)>;
  auto ld = [&](bool inz, int64_t gi) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (inz) v = a.in[gi];
    return v;
  };
  auto stage_direct_all = [&](int t) {
    halo_rows(t, IC0{}, ICU{}, [&](int, int idx, bool inz, int64_t gi) { sX[idx] = ld(inz, gi); });
  };
  auto stage_rest = [&](int t) {      // units PU .. U - 1 (when U > PU)
    halo_rows(t, ICPU{}, ICR{}, [&](int, int idx, bool inz, int64_t gi) { sX[idx] = ld(inz, gi); });
  };
  auto prefetch = [&](int t) {
    halo_rows(t, IC0{}, ICPU{}, [&](int k, int, bool inz, int64_t gi) { pre[k] = ld(inz, gi); });
  };
  auto place = [&](int t) {
    halo_rows(t, IC0{}, ICPU{}, [&](int k, int idx, bool, int64_t) { sX[idx] = pre[k]; });
  };
  // INMODE 1: FP32 planar input (3 components), scaled and packed to bf16;
  // halo voxel hv = tid + k * 256
  constexpr int NV = (HALO + 255) / 256;
  float pin[INMODE == 1 ? 3 * NV : 1];
  auto input_vox = [&](int t, auto&& put) {
    int b = t;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby, bz = b / nby;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int hv = tid + k * 256;
      if (hv < HALO) {
        int hz = hv / (HY * HX), r = hv - hz * (HY * HX), hy = r / HX, hx = r - hy * HX;
        int gz = z0 + hz - 1;
        int gy = wrapi(y0 + hy - 1, a.Y), gx = wrapi(x0 + hx - 1, a.X);
        put(k, hv, gz >= 0 && gz < a.Z, ((int64_t)gz * a.Y + gy) * a.X + gx);
      }
    }
  };
  auto pack_in = [&](float c0, float c1, float c2) {
    u32x4 v = {pack_bf16(c0 * a.in_scale, c1 * a.in_scale), pack_bf16(c2 * a.in_scale, 0.0f), 0u, 0u};
    return v;
  };
  auto stage_input = [&](int t) {
    input_vox(t, [&](int, int hv, bool inz, int64_t o) {
      sX[hv] = inz ? pack_in(a.inf[0][o], a.inf[1][o], a.inf[2][o]) : pack_in(0.0f, 0.0f, 0.0f);
    });
  };
  auto prefetch_input = [&](int t) {
    input_vox(t, [&](int k, int, bool inz, int64_t o) {
      pin[3 * k] = inz ? a.inf[0][o] : 0.0f;
      pin[3 * k + 1] = inz ? a.inf[1][o] : 0.0f;
      pin[3 * k + 2] = inz ? a.inf[2][o] : 0.0f;
    });
  };
  auto place_input = [&](int t) {
    input_vox(t, [&](int k, int hv, bool, int64_t) { sX[hv] = pack_in(pin[3 * k], pin[3 * k + 1], pin[3 * k + 2]); });
  };

  // units p UE .. p UE + UE - 1 of tile t's halo into dst: chunk c of 32
  // voxels per wave instruction, lane l loading unit l % 2 of voxel
  // 32 c + l / 2 into dst[64 c + l]
  auto direct_load = [&](int t, int p, u32x4* dst) {
    int b = t;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby, bz = b / nby;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    for (int c = wave; c < NCH2; c += 4) {
      const int u = lane & 1;
      const int hv = c * 32 + (lane >> 1);
      const u32x4* src = &g_zero16;
      if (hv < HALO) {
        const int hz = hv / (HY * HX), r = hv - hz * (HY * HX), hy = r / HX, hx = r - hy * HX;
        const int gz = z0 + hz - 1;
        if (gz >= 0 && gz < a.Z) {
          const int gy = wrapi(y0 + hy - 1, a.Y), gx = wrapi(x0 + hx - 1, a.X);
          src = a.in + unit_at<U>(((int64_t)gz * a.Y + gy) * a.X + gx, p * UE + u, (int64_t)a.Z * a.Y * a.X);
        }
      }
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(dst + c * 64),
                                       16, 0, 0);
    }
  };

  // XCD-aware walk: work-groups are dispatched round-robin over the 8 XCDs,
  // so work-group b runs on XCD b % 8.  The G tiles of one round of the walk
  // (a contiguous range of the x-fastest tile order) are split into 8 runs of
  // G / 8 consecutive tiles, run r going to the work-groups of XCD r: the
  // tiles one XCD computes together are neighbours in x and y and share their
  // halos in that XCD's L2 (with the round-robin order they were 8 columns
  // apart).  When G / 8 tiles make whole slabs of TZ planes, a work-group's
  // next tile is the one behind it in z, on the same XCD.  Any other grid
  // keeps the plain order.
  const int G = (int)gridDim.x;
  int t = (G & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
  if (t >= ntile) return;
  int buf = 0;
  if (DIRECT) {
    direct_load(t, 0, sXbuf);
    __builtin_amdgcn_s_waitcnt(0);
  } else if (INMODE == 0) {
    stage_direct_all(t);
  } else {
    stage_input(t);
  }
  __syncthreads();

  for (; t < ntile; t += gridDim.x) {
  int b = t;
  const int bx = b % nbx;
  b /= nbx;
  const int by = b % nby, bz = b / nby;
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
  f32x4 acc[NACC][NCT];
#pragma unroll
  for (int r = 0; r < NACC; ++r)
#pragma unroll
    for (int j = 0; j < NCT; ++j) acc[r][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int p = 0; p < KS; ++p) {
  // the phase after this one: the next half of this tile, or the next tile
  const bool last = p == KS - 1;
  const int tn = last ? t + (int)gridDim.x : t;
  sX = sXbuf + buf * BUFU;
  if (tn < ntile) {
    if (DIRECT) direct_load(tn, last ? 0 : p + 1, sXbuf + (buf ^ 1) * BUFU);
    else if (INMODE == 0) prefetch(tn);
    else prefetch_input(tn);
  }

  if constexpr (FOLD) {
    // k-step s: lane group g reads the (dz, dx) combination q = 2 s + g / 2
    // (q = 9 is padding with zero weights; its read is clamped to q = 8),
    // channel unit g % 2, of every halo row h
    const int q0 = g >> 1, c0u = g & 1;
    const int lb = c0u * HALO_P + (wave + 1) * HY * HX + n + 1;
#pragma unroll
    for (int s = 0; s < FOLD_NKS; ++s) {
      int q = 2 * s + q0;
      q = q > 8 ? 8 : q;
      const int off = lb + (q / 3 - 1) * HY * HX + (q % 3 - 1);
#pragma unroll
      for (int h = 0; h < TY + 2; ++h) {
        const bf16x8 f = __builtin_bit_cast(bf16x8, sX[off + h * HX]);
        acc[h][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[p][s][0], f, acc[h][0], 0, 0, 0);
      }
    }
  } else
  // Each wave computes the TY rows (16 x voxels each) of output plane
  // z0 + wave.  The k-steps are ordered (column group cg, dy): column group
  // cg holds the (dz, dx) combinations cg * TPK .. cg * TPK + TPK - 1, one per
  // lane-group slot, so that the activation fragment read at halo row h serves
  // the output rows h - 1 - dy for the three dy: NCG * (TY + 2) LDS reads per
  // wave instead of one per k-step and row.
  {
    const int slot = (g * 8) / CE;          // this lane group's slot within a k-step
    const int c0u = ((g * 8) % CE) / 8;     // and its 16-byte channel unit
    const int lb = (DIRECT ? c0u : c0u * HALO_P) + ((wave + 1) * HY * HX + n + 1) * VS;
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      int q;
      if (TPK == 1) q = cg;
      else if (TPK == 2) q = slot ? 2 * cg + 1 : 2 * cg;
      else q = slot == 0 ? 4 * cg : slot == 1 ? 4 * cg + 1 : slot == 2 ? 4 * cg + 2 : 4 * cg + 3;
      q = q > 8 ? 8 : q;                    // padding slots (zero weights)
      const int off = lb + ((q / 3 - 1) * HY * HX + (q % 3 - 1)) * VS;
      // the fragments of PF halo rows are read before the first of their
      // MFMAs, so that the reads of later rows are in flight while the MFMAs
      // of earlier ones run (a read waited for right before its three MFMAs
      // leaves the matrix pipe idle for the LDS latency)
#pragma unroll
      for (int h0 = 0; h0 < TY + 2; h0 += PF) {
      bf16x8 fr[PF];
#pragma unroll
      for (int i = 0; i < PF; ++i)
        if (h0 + i < TY + 2) fr[i] = __builtin_bit_cast(bf16x8, sX[off + (h0 + i) * HX * VS]);
      // keep the instruction scheduler from sinking the reads back to their
      // uses
      if (PF > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = h0; h < h0 + PF && h < TY + 2; ++h) {
        const bf16x8 f = fr[h - h0];
#pragma unroll
        for (int dyi = 0; dyi < 3; ++dyi) {
          const int r = h - dyi;
          if (r >= 0 && r < TY) {
#pragma unroll
            for (int j = 0; j < NCT; ++j)
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[p][3 * cg + dyi][j], f, acc[r][j], 0, 0, 0);
          }
        }
      }
      }
    }
  }
  if (tn < ntile) {
    if (DIRECT) {
      // own loads done, then every wave's loads and every read of this buffer
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      buf ^= 1;
    } else {
      __syncthreads();
      if (INMODE == 0) {
        place(tn);
        if (PU < U) stage_rest(tn);
      } else {
        place_input(tn);
      }
      __syncthreads();
    }
  }
  // epilogue after the barrier: the output stores drain while the next tile
  // is computed instead of holding up the wait above
  if (last) {
    const int z = z0 + wave;
#pragma unroll
    for (int r = 0; r < TY; ++r) {
      if (z >= a.Z) break;
      int64_t vox = ((int64_t)z * a.Y + (y0 + r)) * a.X + (x0 + n);
      if (FOLD) {
        // lane group g < 3 holds output channel g: rows dy = 0, 1, 2 of the
        // accumulators of halo rows r, r + 1, r + 2
        if (g < 3)
          a.outf[g][vox] = ((acc[r][0][0] + acc[r + 1][0][1]) + acc[r + 2][0][2]) + bias_r[0][0];
      } else if (OUTMODE == 1) {
        if (g == 0) {
          a.outf[0][vox] = acc[r][0][0] + bias_r[0][0];
          a.outf[1][vox] = acc[r][0][1] + bias_r[0][1];
          a.outf[2][vox] = acc[r][0][2] + bias_r[0][2];
        }
      } else {
#pragma unroll
        for (int j = 0; j < NCT; ++j) {
          int co0 = 16 * j + 4 * g;
          float v[4];
          if (OUTMODE == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[r][j][i] + bias_r[j][i], 0.0f);
          } else {
            u32x2 m = *(const u32x2*)(a.mask + chan_at<COUTP>(vox, co0, (int64_t)a.Z * a.Y * a.X));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              unsigned mb = (i & 1) ? (m[i >> 1] >> 16) : (m[i >> 1] & 0xFFFFu);
              v[i] = bf2f(mb) > 0.0f ? acc[r][j][i] : 0.0f;
            }
          }
          u32x2 o;
          o[0] = pack_bf16(v[0], v[1]);
          o[1] = pack_bf16(v[2], v[3]);
          *(u32x2*)(a.out + chan_at<COUTP>(vox, co0, (int64_t)a.Z * a.Y * a.X)) = o;
        }
      }
    }
  }
  }  // phases
  }  // tiles of this work-group
}

// ---------------------------------------------------------------------------
// weight and bias gradients of one layer:
//   gW[co][ci][t] += sum_v gy[v][co] x[v + off(t)][ci],  gb[co] += sum_v gy[v][co]
//   XMODE 0: x bf16 channels-last with XS channels; 1: FP32 planar x in_scale (XS = 4)
//   GMODE 0: gy bf16 channels-last with GS channels; 1: FP32 planar (GS = 4)
struct WgradArgs {
  int Z, Y, X;
  const u32x4* x;
  const float* xf[3];
  float x_scale;
  const u32x4* gy;
  const float* gyf[3];
  float* gW;
  float* gb;
};

template <int CIN, int COUT, int XS, int GS, int XMODE, int GMODE>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  constexpr int MT = (COUT + 15) / 16, NT = (CIN + 15) / 16;
  constexpr int NTILE = 27 * MT * NT;
  constexpr int PERW = (NTILE + 3) / 4;
  __shared__ u32x4 sXv[HALO * XS / 8 + 1];
  __shared__ u32x4 sGv[TILE * GS / 8 + 1];
  unsigned short* sX = (unsigned short*)sXv;
  unsigned short* sG = (unsigned short*)sGv;

  const int nbx = a.X / TX, nby = a.Y / TY;
  int b = blockIdx.x;
  const int bx = b % nbx;
  b /= nbx;
  const int by = b % nby, bz = b / nby;
  const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
  const int tid = threadIdx.x;

  if (XMODE == 0) {
    constexpr int U = XS / 8;
    for (int u = tid; u < HALO * U; u += 256) {
      int hv = u / U, part = u - hv * U;
      int hz = hv / (HY * HX), r = hv - hz * (HY * HX), hy = r / HX, hx = r - hy * HX;
      int gz = z0 + hz - 1;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (gz >= 0 && gz < a.Z) {
        int gy = wrapi(y0 + hy - 1, a.Y), gx = wrapi(x0 + hx - 1, a.X);
        v = a.x[unit_at<U>(((int64_t)gz * a.Y + gy) * a.X + gx, part, (int64_t)a.Z * a.Y * a.X)];
      }
      sXv[u] = v;
    }
  } else {
    for (int hv = tid; hv < HALO; hv += 256) {
      int hz = hv / (HY * HX), r = hv - hz * (HY * HX), hy = r / HX, hx = r - hy * HX;
      int gz = z0 + hz - 1;
      float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
      if (gz >= 0 && gz < a.Z) {
        int gy = wrapi(y0 + hy - 1, a.Y), gx = wrapi(x0 + hx - 1, a.X);
        int64_t o = ((int64_t)gz * a.Y + gy) * a.X + gx;
        c0 = a.xf[0][o] * a.x_scale;
        c1 = a.xf[1][o] * a.x_scale;
        c2 = a.xf[2][o] * a.x_scale;
      }
      u32x2 v = {f2bf(c0) | (f2bf(c1) << 16), f2bf(c2)};
      ((u32x2*)sX)[hv] = v;
    }
  }
  if (GMODE == 0) {
    constexpr int U = GS / 8;
    for (int u = tid; u < TILE * U; u += 256) {
      int tv = u / U, part = u - tv * U;
      int zz = tv / (TY * TX), r = tv - zz * (TY * TX), yy = r / TX, xx = r - yy * TX;
      int gz = z0 + zz;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (gz < a.Z) v = a.gy[unit_at<U>(((int64_t)gz * a.Y + (y0 + yy)) * a.X + (x0 + xx), part, (int64_t)a.Z * a.Y * a.X)];
      sGv[u] = v;
    }
  } else {
    for (int tv = tid; tv < TILE; tv += 256) {
      int zz = tv / (TY * TX), r = tv - zz * (TY * TX), yy = r / TX, xx = r - yy * TX;
      int gz = z0 + zz;
      float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
      if (gz < a.Z) {
        int64_t o = ((int64_t)gz * a.Y + (y0 + yy)) * a.X + (x0 + xx);
        c0 = a.gyf[0][o];
        c1 = a.gyf[1][o];
        c2 = a.gyf[2][o];
      }
      u32x2 v = {f2bf(c0) | (f2bf(c1) << 16), f2bf(c2)};
      ((u32x2*)sG)[tv] = v;
    }
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
  f32x4 acc[PERW];
#pragma unroll
  for (int i = 0; i < PERW; ++i) acc[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  for (int q = 0; q < TILE / 32; ++q) {
    // lane group g: 8 consecutive x voxels of tile row 2q + g/2
    int row = 2 * q + (g >> 1);
    int zz = row / TY, yy = row - zz * TY, xx0 = 8 * (g & 1);
    int tv0 = (zz * TY + yy) * TX + xx0;
    bf16x8 af[MT];
#pragma unroll
    for (int jc = 0; jc < MT; ++jc) {
      int co = 16 * jc + n;
      unsigned w[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) w[e] = co < COUT ? sG[(tv0 + e) * GS + co] : 0u;
      u32x4 p = {w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16), w[6] | (w[7] << 16)};
      af[jc] = __builtin_bit_cast(bf16x8, p);
    }
#pragma unroll
    for (int i = 0; i < PERW; ++i) {
      int idx = wave + 4 * i;
      if (idx < NTILE) {
        int t = idx / (MT * NT), rem = idx - t * (MT * NT), jc = rem / NT, ji = rem - jc * NT;
        int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        int ci = 16 * ji + n;
        int hb = ((zz + 1 + dz) * HY + (yy + 1 + dy)) * HX + (xx0 + 1 + dx);
        unsigned w[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = ci < CIN ? sX[(hb + e) * XS + ci] : 0u;
        u32x4 p = {w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16), w[6] | (w[7] << 16)};
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[jc], __builtin_bit_cast(bf16x8, p), acc[i], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < PERW; ++i) {
    int idx = wave + 4 * i;
    if (idx < NTILE) {
      int t = idx / (MT * NT), rem = idx - t * (MT * NT), jc = rem / NT, ji = rem - jc * NT;
      int ci = 16 * ji + n;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        int co = 16 * jc + 4 * g + k;
        if (co < COUT && ci < CIN) atomicAdd(&a.gW[((int64_t)co * CIN + ci) * 27 + t], acc[i][k]);
      }
    }
  }
  for (int co = tid; co < COUT; co += 256) {
    float s = 0.0f;
    for (int tv = 0; tv < TILE; ++tv) s += bf2f(sG[tv * GS + co]);
    atomicAdd(&a.gb[co], s);
  }
}

// ---------------------------------------------------------------------------
// elementwise stencils on FP32 planar boxes
struct Box {
  int Z, Y, X;
  GP_DEV int64_t at(int z, int y, int x) const { return ((int64_t)z * Y + y) * X + x; }
};

struct P3 { const float* p[3]; };
struct W3 { float* p[3]; };

// one 1-2-1 pass along x, y (periodic) and zeta (zero beyond the planes).
// A thread takes an FY-row y strip of one x column of one component
// (blockIdx.z) through FZ planes: the x- then y-filtered rows of the planes
// z - 1 and z stay in registers, so that every input row is read once per
// plane (plus the two halo rows).  skip (device, nullable): when it points at
// a non-zero flag every work-group returns at once (the fallback filter that
// runs only when the network's current is rejected).
constexpr int FY = 4, FZ = 8;

__global__ __launch_bounds__(256) void k_filter(Box B, P3 in, W3 out, const int* skip) {
  if (skip && *skip) return;
  const int ncol = B.X * (B.Y / FY);
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= ncol) return;
  const int x = w % B.X, y0 = (w / B.X) * FY;
  const int z0 = blockIdx.y * FZ;
  const int c = blockIdx.z;
  const int xl = wrapi(x - 1, B.X), xr = wrapi(x + 1, B.X);
  const int64_t plane = (int64_t)B.Y * B.X;
  {
    float a[FY], b[FY];
#pragma unroll
    for (int j = 0; j < FY; ++j) a[j] = b[j] = 0.0f;
#pragma unroll
    for (int k = -1; k <= FZ; ++k) {
      const int z = z0 + k;
      float s[FY];
      if (z >= 0 && z < B.Z) {
        const float* p = in.p[c] + z * plane;
        float r[FY + 2];
#pragma unroll
        for (int j = 0; j < FY + 2; ++j) {
          const float* row = p + wrapi(y0 + j - 1, B.Y) * B.X;
          r[j] = 0.25f * row[xl] + 0.5f * row[x] + 0.25f * row[xr];
        }
#pragma unroll
        for (int j = 0; j < FY; ++j) s[j] = 0.25f * r[j] + 0.5f * r[j + 1] + 0.25f * r[j + 2];
      } else {
#pragma unroll
        for (int j = 0; j < FY; ++j) s[j] = 0.0f;
      }
      if (k >= 1 && z - 1 < B.Z) {
        float* q = out.p[c] + (z - 1) * plane + (int64_t)y0 * B.X + x;
#pragma unroll
        for (int j = 0; j < FY; ++j) q[j * B.X] = 0.25f * a[j] + 0.5f * b[j] + 0.25f * s[j];
      }
#pragma unroll
      for (int j = 0; j < FY; ++j) {
        a[j] = b[j];
        b[j] = s[j];
      }
    }
  }
}

struct CurlArgs {
  Box B;
  float s, ihx, ihy, ih;
};

// s * curl(A) at (z, y, x), zero for planes outside the box
GP_DEV void curl_at(const CurlArgs& a, P3 A, int z, int y, int x, float c[3]) {
  if (z < 0 || z >= a.B.Z) { c[0] = c[1] = c[2] = 0.0f; return; }
  const Box& B = a.B;
  int64_t v = B.at(z, y, x);
  int64_t vy = B.at(z, wrapi(y - 1, B.Y), x);
  int64_t vx = B.at(z, y, wrapi(x - 1, B.X));
  float axz = z > 0 ? A.p[0][B.at(z - 1, y, x)] : 0.0f;
  float ayz = z > 0 ? A.p[1][B.at(z - 1, y, x)] : 0.0f;
  float ax = A.p[0][v], ay = A.p[1][v], az = A.p[2][v];
  c[0] = a.s * ((az - A.p[2][vy]) * a.ihy - (ay - ayz) * a.ih);
  c[1] = a.s * ((ax - axz) * a.ih - (az - A.p[2][vx]) * a.ihx);
  c[2] = a.s * ((ay - A.p[1][vx]) * a.ihx - (ax - A.p[0][vy]) * a.ihy);
}

GP_DEV double block_sum_d(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// Jd = Jf + s curl(A); per-block partial sums of |D.(s curl A)|^2, |D.Jf|^2,
// |s curl A|^2 and |Jf|^2 into part[4 * block + {0, 1, 2, 3}] (a fixed grid
// of COMB_BLOCKS blocks strides over the work, so that the sums need no
// global atomics).
// A work item is one (x, y) column through CZ planes: the values of plane
// z - 1 that the curl and the divergences need are carried in registers.
// (With one filter pass, k_combine_f1 below forms Jf itself.)
constexpr int COMB_BLOCKS = 2048;
constexpr int CZ = 8;

__global__ __launch_bounds__(256) void k_combine(CurlArgs a, P3 Jf, P3 A, W3 Jd, double* part) {
  __shared__ double sh[4];
  const Box& B = a.B;
  const int ncol = B.X * B.Y;
  const int nwork = ncol * ((B.Z + CZ - 1) / CZ);
  const int64_t plane = ncol;
  double num = 0.0, den = 0.0, cc = 0.0, jj = 0.0;
  for (int w = blockIdx.x * 256 + threadIdx.x; w < nwork; w += gridDim.x * 256) {
    const int col = w % ncol, z0 = (w / ncol) * CZ;
    const int x = col % B.X, y = col / B.X;
    const int xm = wrapi(x - 1, B.X), ym = wrapi(y - 1, B.Y);
    const int cx = y * B.X + xm, cy = ym * B.X + x, cxy = ym * B.X + xm;
    // plane z0 - 1 (zero below the box): A_x at (y, x) and (y - 1, x),
    // A_y at (y, x) and (y, x - 1), z-component of the curl and Jf_z
    float pax = 0.0f, paxy = 0.0f, pay = 0.0f, payx = 0.0f, pc2 = 0.0f, pj2 = 0.0f;
    if (z0 > 0) {
      const int64_t o = (z0 - 1) * plane;
      pax = A.p[0][o + col];
      paxy = A.p[0][o + cy];
      pay = A.p[1][o + col];
      payx = A.p[1][o + cx];
      pc2 = a.s * ((pay - payx) * a.ihx - (pax - paxy) * a.ihy);
      pj2 = Jf.p[2][o + col];
    }
    const int zend = min(z0 + CZ, B.Z);
    for (int z = z0; z < zend; ++z) {
      const int64_t o = z * plane;
      const float ax = A.p[0][o + col], ay = A.p[1][o + col], az = A.p[2][o + col];
      const float axy = A.p[0][o + cy], ayx = A.p[1][o + cx];
      const float azx = A.p[2][o + cx], azy = A.p[2][o + cy], azxy = A.p[2][o + cxy];
      const float c0 = a.s * ((az - azy) * a.ihy - (ay - pay) * a.ih);
      const float c1 = a.s * ((ax - pax) * a.ih - (az - azx) * a.ihx);
      const float c2 = a.s * ((ay - ayx) * a.ihx - (ax - axy) * a.ihy);
      const float c0x = a.s * ((azx - azxy) * a.ihy - (ayx - payx) * a.ih);   // c0 at x - 1
      const float c1y = a.s * ((axy - paxy) * a.ih - (azy - azxy) * a.ihx);   // c1 at y - 1
      const float j0 = Jf.p[0][o + col], j1 = Jf.p[1][o + col], j2 = Jf.p[2][o + col];
      Jd.p[0][o + col] = j0 + c0;
      Jd.p[1][o + col] = j1 + c1;
      Jd.p[2][o + col] = j2 + c2;
      const double dc = (double)(c0 - c0x) * a.ihx + (double)(c1 - c1y) * a.ihy + (double)(c2 - pc2) * a.ih;
      const double df = (double)(j0 - Jf.p[0][o + cx]) * a.ihx + (double)(j1 - Jf.p[1][o + cy]) * a.ihy +
                        (double)(j2 - pj2) * a.ih;
      num += dc * dc;
      den += df * df;
      cc += (double)c0 * c0 + (double)c1 * c1 + (double)c2 * c2;
      jj += (double)j0 * j0 + (double)j1 * j1 + (double)j2 * j2;
      pax = ax;
      paxy = axy;
      pay = ay;
      payx = ayx;
      pc2 = c2;
      pj2 = j2;
    }
  }
  double tn = block_sum_d(num, sh);
  __syncthreads();
  double td = block_sum_d(den, sh);
  __syncthreads();
  double tc = block_sum_d(cc, sh);
  __syncthreads();
  double tj = block_sum_d(jj, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = tn;
    part[4 * blockIdx.x + 1] = td;
    part[4 * blockIdx.x + 2] = tc;
    part[4 * blockIdx.x + 3] = tj;
  }
}

// k_combine with one binomial pass formed inside: the filtered current is
// computed from the raw one in k_filter's operation order (the same values
// bit for bit) and never stored.  A work item is a strip of FYS rows
// (y0 .. y0 + FYS - 1) of one x column through FCZ planes.  Per plane it
// filters, along x then y, five streams (J_x at x and x - 1, J_y at the rows
// and the row above, J_z), carried over three planes for the zeta pass; the
// x-filtered rows of the raw current and A's values at y - 1 are shared by
// the rows of the strip.  The partial sums are those of k_combine, added in
// another order.
constexpr int FCZ = 32;
template <int FYS>
__global__ __launch_bounds__(256) void k_combine_f1(CurlArgs a, P3 J, P3 A, W3 Jd, double* part) {
  __shared__ double sh[4];
  const Box& B = a.B;
  const int nstrip = B.X * (B.Y / FYS);
  const int nwork = nstrip * ((B.Z + FCZ - 1) / FCZ);
  const int64_t plane = (int64_t)B.Y * B.X;
  double num = 0.0, den = 0.0, cc = 0.0, jj = 0.0;
  auto rx = [](const float* row, int l, int c, int r) { return 0.25f * row[l] + 0.5f * row[c] + 0.25f * row[r]; };
  auto ry = [](float m, float c, float p) { return 0.25f * m + 0.5f * c + 0.25f * p; };
  // x-then-y filtered plane z: J_x at (y, x) and (y, x - 1), J_y at y - 1 ..
  // y0 + FYS - 1 (s1[i] at row y0 + i - 1), J_z; zero outside the box
  struct S {
    float s0[FYS], s0x[FYS], s1[FYS + 1], s2[FYS];
  };
  for (int w = blockIdx.x * 256 + threadIdx.x; w < nwork; w += gridDim.x * 256) {
    const int st = w % nstrip, z0 = (w / nstrip) * FCZ;
    const int x = st % B.X, y0 = (st / B.X) * FYS;
    const int xm = wrapi(x - 1, B.X), xm2 = wrapi(x - 2, B.X), xp = wrapi(x + 1, B.X);
    int rows[FYS + 3];                      // row offsets of y0 - 2 .. y0 + FYS
#pragma unroll
    for (int r = 0; r < FYS + 3; ++r) rows[r] = wrapi(y0 - 2 + r, B.Y) * B.X;
    auto splane = [&](int z, bool only2) {
      S o;
#pragma unroll
      for (int i = 0; i < FYS; ++i) o.s0[i] = o.s0x[i] = o.s2[i] = 0.0f;
#pragma unroll
      for (int i = 0; i <= FYS; ++i) o.s1[i] = 0.0f;
      if (z < 0 || z >= B.Z) return o;
      const int64_t zo = (int64_t)z * plane;
      float r2[FYS + 2];
#pragma unroll
      for (int r = 0; r < FYS + 2; ++r) r2[r] = rx(J.p[2] + zo + rows[r + 1], xm, x, xp);
#pragma unroll
      for (int i = 0; i < FYS; ++i) o.s2[i] = ry(r2[i], r2[i + 1], r2[i + 2]);
      if (only2) return o;
      float r0[FYS + 2], r0x[FYS + 2], r1[FYS + 3];
#pragma unroll
      for (int r = 0; r < FYS + 2; ++r) {
        const float* row = J.p[0] + zo + rows[r + 1];
        r0[r] = rx(row, xm, x, xp);
        r0x[r] = rx(row, xm2, xm, x);
      }
#pragma unroll
      for (int r = 0; r < FYS + 3; ++r) r1[r] = rx(J.p[1] + zo + rows[r], xm, x, xp);
#pragma unroll
      for (int i = 0; i < FYS; ++i) {
        o.s0[i] = ry(r0[i], r0[i + 1], r0[i + 2]);
        o.s0x[i] = ry(r0x[i], r0x[i + 1], r0x[i + 2]);
      }
#pragma unroll
      for (int i = 0; i <= FYS; ++i) o.s1[i] = ry(r1[i], r1[i + 1], r1[i + 2]);
      return o;
    };
    S sm = splane(z0 - 1, false), sc = splane(z0, false);
    // plane z0 - 1 (zero below the box), per row: A_x at y and y - 1, A_y at
    // x and x - 1, the z-component of the curl and the filtered J_z
    float pax[FYS], paxy[FYS], pay[FYS], payx[FYS], pc2[FYS], pj2[FYS];
#pragma unroll
    for (int i = 0; i < FYS; ++i) pax[i] = paxy[i] = pay[i] = payx[i] = pc2[i] = pj2[i] = 0.0f;
    if (z0 > 0) {
      const int64_t o = (int64_t)(z0 - 1) * plane;
      const S smm = splane(z0 - 2, true);
#pragma unroll
      for (int i = 0; i < FYS; ++i) {
        const int64_t c = o + rows[i + 2] + x;
        pax[i] = A.p[0][c];
        paxy[i] = i ? pax[i - 1] : A.p[0][o + rows[1] + x];
        pay[i] = A.p[1][c];
        payx[i] = A.p[1][o + rows[i + 2] + xm];
        pc2[i] = a.s * ((pay[i] - payx[i]) * a.ihx - (pax[i] - paxy[i]) * a.ihy);
        pj2[i] = ry(smm.s2[i], sm.s2[i], sc.s2[i]);
      }
    }
    const int zend = min(z0 + FCZ, B.Z);
    for (int z = z0; z < zend; ++z) {
      const int64_t o = (int64_t)z * plane;
      const S sp = splane(z + 1, false);
      // A at row y0 - 1 (x and x - 1), then row by row
      float axy = A.p[0][o + rows[1] + x], azy = A.p[2][o + rows[1] + x], azxy = A.p[2][o + rows[1] + xm];
      float j1y = ry(sm.s1[0], sc.s1[0], sp.s1[0]);
      float c1y_prev = 0.0f;
#pragma unroll
      for (int i = 0; i < FYS; ++i) {
        const int64_t c = o + rows[i + 2] + x;
        const float ax = A.p[0][c], ay = A.p[1][c], az = A.p[2][c];
        const float ayx = A.p[1][c - x + xm], azx = A.p[2][c - x + xm];
        const float j0 = ry(sm.s0[i], sc.s0[i], sp.s0[i]);
        const float j1 = ry(sm.s1[i + 1], sc.s1[i + 1], sp.s1[i + 1]);
        const float j2 = ry(sm.s2[i], sc.s2[i], sp.s2[i]);
        const float j0x = ry(sm.s0x[i], sc.s0x[i], sp.s0x[i]);
        const float c0 = a.s * ((az - azy) * a.ihy - (ay - pay[i]) * a.ih);
        const float c1 = a.s * ((ax - pax[i]) * a.ih - (az - azx) * a.ihx);
        const float c2 = a.s * ((ay - ayx) * a.ihx - (ax - axy) * a.ihy);
        const float c0x = a.s * ((azx - azxy) * a.ihy - (ayx - payx[i]) * a.ih);   // c0 at x - 1
        // c1 at y - 1: the row above's c1, or (first row) from row y0 - 1
        const float c1y = i ? c1y_prev : a.s * ((axy - paxy[i]) * a.ih - (azy - azxy) * a.ihx);
        Jd.p[0][c] = j0 + c0;
        Jd.p[1][c] = j1 + c1;
        Jd.p[2][c] = j2 + c2;
        const double dc = (double)(c0 - c0x) * a.ihx + (double)(c1 - c1y) * a.ihy + (double)(c2 - pc2[i]) * a.ih;
        const double df = (double)(j0 - j0x) * a.ihx + (double)(j1 - j1y) * a.ihy + (double)(j2 - pj2[i]) * a.ih;
        num += dc * dc;
        den += df * df;
        cc += (double)c0 * c0 + (double)c1 * c1 + (double)c2 * c2;
        jj += (double)j0 * j0 + (double)j1 * j1 + (double)j2 * j2;
        // carried to the next plane (z; axy still holds A_x of the row
        // above) and to the next row (y)
        paxy[i] = axy;
        pax[i] = ax;
        pay[i] = ay;
        payx[i] = ayx;
        pc2[i] = c2;
        pj2[i] = j2;
        axy = ax;
        azy = az;
        azxy = azx;
        j1y = j1;
        c1y_prev = c1;
      }
      sm = sc;
      sc = sp;
    }
  }
  double tn = block_sum_d(num, sh);
  __syncthreads();
  double td = block_sum_d(den, sh);
  __syncthreads();
  double tc = block_sum_d(cc, sh);
  __syncthreads();
  double tj = block_sum_d(jj, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = tn;
    part[4 * blockIdx.x + 1] = td;
    part[4 * blockIdx.x + 2] = tc;
    part[4 * blockIdx.x + 3] = tj;
  }
}

// sum the partials and decide between the corrected and the filtered current.
// Two criteria, both needed to keep the network's current:
//  - continuity: ||D.(s curl A)|| / ||D.Jf|| <= thr.  D.curl vanishes
//    identically, so for a finite A this ratio is FP32 rounding; it rejects a
//    non-finite output (a finiteness guard), not a wrong one;
//  - size: ||s curl A|| <= DN_CORR_MAX ||Jf||.  The filtered current is the
//    yardstick: a correction larger than the current it corrects is taken
//    as the network's failure (a finite but wrong output).
constexpr double DN_CORR_MAX = 1.0;
__global__ __launch_bounds__(256) void k_decide(const double* part, int nparts, double thr, int* use_net,
                                                double* rel, int64_t* fallbacks) {
  __shared__ double sh[4];
  double num = 0.0, den = 0.0, cc = 0.0, jj = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    num += part[4 * i];
    den += part[4 * i + 1];
    cc += part[4 * i + 2];
    jj += part[4 * i + 3];
  }
  num = block_sum_d(num, sh);
  __syncthreads();
  den = block_sum_d(den, sh);
  __syncthreads();
  cc = block_sum_d(cc, sh);
  __syncthreads();
  jj = block_sum_d(jj, sh);
  if (threadIdx.x != 0) return;
  double q = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
  double m = jj > 0.0 ? sqrt(cc / jj) : (cc > 0.0 ? INFINITY : 0.0);
  int ok = q <= thr && m <= DN_CORR_MAX;     // false for NaN
  *use_net = ok;
  if (rel) *rel = q;
  if (!ok && fallbacks) *fallbacks += 1;
}

// a fixed grid strides over the box: when the network's current is kept
// (the usual case) every work-group returns at once
constexpr int SEL_BLOCKS = 1024;
__global__ __launch_bounds__(256) void k_select(Box B, const int* use_net, P3 Jf, W3 Jd) {
  if (*use_net) return;
  const int64_t nv = (int64_t)B.Z * B.Y * B.X;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x)
    for (int q = 0; q < 3; ++q) Jd.p[q][v] = Jf.p[q][v];
}

// training loss on planes [lo, hi): r = (Jf + s curl A - Jt) / n_e,
// loss += lscale sum r^2, gJ = gscale r (zero outside the planes)
struct LossArgs {
  CurlArgs c;
  int lo, hi;
  float inv_ne, gscale;
  double lscale;
};

__global__ __launch_bounds__(256) void k_loss(LossArgs a, P3 Jf, P3 A, P3 Jt, W3 gJ, double* loss) {
  __shared__ double sh[4];
  const Box& B = a.c.B;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nv = (int64_t)B.Z * B.Y * B.X;
  double l = 0.0;
  if (v < nv) {
    int x = (int)(v % B.X);
    int64_t r = v / B.X;
    int y = (int)(r % B.Y), z = (int)(r / B.Y);
    bool in = z >= a.lo && z < a.hi;
    float c[3];
    curl_at(a.c, A, z, y, x, c);
    for (int q = 0; q < 3; ++q) {
      float rr = in ? (Jf.p[q][v] + c[q] - Jt.p[q][v]) * a.inv_ne : 0.0f;
      l += (double)rr * rr;
      gJ.p[q][v] = a.gscale * rr;
    }
  }
  double t = block_sum_d(l, sh);
  if (threadIdx.x == 0) atomicAdd(loss, t * a.lscale);
}

// gA = s curl^T(gJ)
__global__ void k_curl_adj(CurlArgs a, P3 G, W3 gA) {
  const Box& B = a.B;
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nv = (int64_t)B.Z * B.Y * B.X;
  if (v >= nv) return;
  int x = (int)(v % B.X);
  int64_t r = v / B.X;
  int y = (int)(r % B.Y), z = (int)(r / B.Y);
  int64_t vy = B.at(z, wrapi(y + 1, B.Y), x), vx = B.at(z, y, wrapi(x + 1, B.X));
  bool up = z + 1 < B.Z;
  int64_t vz = up ? B.at(z + 1, y, x) : 0;
  float gx = G.p[0][v], gy = G.p[1][v], gz = G.p[2][v];
  float gxz = up ? G.p[0][vz] : 0.0f, gyz = up ? G.p[1][vz] : 0.0f;
  gA.p[0][v] = a.s * ((gy - gyz) * a.ih - (gz - G.p[2][vy]) * a.ihy);
  gA.p[1][v] = a.s * (-(gx - gxz) * a.ih + (gz - G.p[2][vx]) * a.ihx);
  gA.p[2][v] = a.s * ((gx - G.p[0][vy]) * a.ihy - (gy - G.p[1][vx]) * a.ihx);
}

// Adam with bias correction (c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t))
__global__ void k_adam(float* th, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

template <typename T>
__global__ void k_zero(T* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
struct gempic_dn {
  hipStream_t s = nullptr;
  std::string err;
  std::vector<void*> ptrs;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  u32x4* fw[NLAYER] = {};
  u32x4* bw[NLAYER] = {};    // data-gradient packs of layers 1 .. 3
  int64_t cap = 0;           // voxels the inference buffers hold
  int64_t cap_train = 0;     // voxels the training buffers hold
  unsigned short *act[3] = {}, *gact[3] = {};
  float* A = nullptr;        // [3][cap]
  float *tJf = nullptr, *tJt = nullptr, *tgJ = nullptr, *tgA = nullptr, *tA = nullptr;
  unsigned short* tact[3] = {};
  double* red = nullptr;     // loss
  double* part = nullptr;    // partial sums of the continuity test
  int* use_net = nullptr;
  double* rel = nullptr;
  int64_t* fallbacks = nullptr;
  int64_t t = 0;             // Adam steps taken
  bool packed = false;

  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) ptrs.erase(it);
    (void)hipFree(p);
  }
};

static int dn_fail(gempic_dn* d, int code, const std::string& m) {
  if (d) d->err = m;
  return code;
}

#define DNCHK(d, expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return dn_fail(d, GEMPIC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static int check_box(gempic_dn* d, int Z, int Y, int X) {
  if (Z < 1 || Y < TY || X < TX || Y % TY || X % TX)
    return dn_fail(d, GEMPIC_EINVAL, "box must have Z >= 1, Y a multiple of 8 and X a multiple of 16");
  if ((int64_t)X * Y * ((Z + CZ - 1) / CZ) >= (int64_t(1) << 31) - (int64_t(COMB_BLOCKS) << 8))
    return dn_fail(d, GEMPIC_EINVAL, "box too large for the denoiser: X * Y * ceil(Z / 8) must stay below 2^31");
  return GEMPIC_OK;
}

// k_conv runs persistent work-groups: as many as can be resident at once
// (occupancy x compute units), each walking its share of the output tiles
template <typename K>
static unsigned conv_grid(K kernel, unsigned ntile) {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0);
  unsigned n = (unsigned)(std::max(1, per) * std::max(1, cus));
  return std::min(ntile, n);
}

static unsigned conv_blocks(int Z, int Y, int X) {
  return (unsigned)((X / TX) * (Y / TY) * ((Z + TZ - 1) / TZ));
}

static int repack(gempic_dn* d, hipStream_t s) {
  for (int l = 0; l < NLAYER; ++l) {
    PackArgs p;
    p.W = d->theta + layer_woff(l);
    p.cin = L_CIN[l];
    p.cout = L_COUT[l];
    p.cinp = pad_in(L_CIN[l]);
    p.coutp = pad_out(L_COUT[l]);
    p.transpose = 0;
    p.fold = l == NLAYER - 1;
    p.out = d->fw[l];
    p.units = p.fold ? fold_units() : packed_units(p.cinp, p.coutp);
    k_pack<<<nblk(p.units, 256), 256, 0, s>>>(p);
    if (l > 0) {
      p.cinp = pad_in(L_COUT[l]);
      p.coutp = pad_out(L_CIN[l]);
      p.transpose = 1;
      p.fold = 0;
      p.out = d->bw[l];
      p.units = packed_units(p.cinp, p.coutp);
      k_pack<<<nblk(p.units, 256), 256, 0, s>>>(p);
    }
  }
  d->packed = true;
  return GEMPIC_OK;
}

static const float* bias_of(gempic_dn* d, int l) {
  return d->theta + layer_woff(l) + (int64_t)L_COUT[l] * L_CIN[l] * 27;
}

// forward through the four layers: acts[0..2] (bf16), A (FP32 planar)
static void net_forward(gempic_dn* d, hipStream_t s, int Z, int Y, int X, const float* const J[3],
                        float in_scale, unsigned short* const acts[3], float* const Aout[3]) {
  unsigned nb = conv_blocks(Z, Y, X);
  ConvArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Z = Z; a.Y = Y; a.X = X;
  for (int q = 0; q < 3; ++q) a.inf[q] = J[q];
  a.in_scale = in_scale;
  a.wp = d->fw[0]; a.bias = bias_of(d, 0); a.out = acts[0];
  k_conv<8, 16, 1, 0><<<conv_grid(k_conv<8, 16, 1, 0>, nb), 256, 0, s>>>(a);
  a.in = (const u32x4*)acts[0]; a.wp = d->fw[1]; a.bias = bias_of(d, 1); a.out = acts[1];
  k_conv<16, 32, 0, 0><<<conv_grid(k_conv<16, 32, 0, 0>, nb), 256, 0, s>>>(a);
  a.in = (const u32x4*)acts[1]; a.wp = d->fw[2]; a.bias = bias_of(d, 2); a.out = acts[2];
  k_conv<32, 16, 0, 0><<<conv_grid(k_conv<32, 16, 0, 0>, nb), 256, 0, s>>>(a);
  a.in = (const u32x4*)acts[2]; a.wp = d->fw[3]; a.bias = bias_of(d, 3); a.out = nullptr;
  for (int q = 0; q < 3; ++q) a.outf[q] = Aout[q];
  k_conv<16, 16, 0, 1><<<conv_grid(k_conv<16, 16, 0, 1>, nb), 256, 0, s>>>(a);
}

static void filter(hipStream_t s, int Z, int Y, int X, const float* const in[3], float* const out[3],
                   float* const tmp[3], int passes) {
  Box B{Z, Y, X};
  int64_t nv = (int64_t)Z * Y * X;
  P3 pi{{in[0], in[1], in[2]}};
  if (passes <= 0) {
    for (int q = 0; q < 3; ++q) (void)hipMemcpyAsync(out[q], in[q], nv * 4, hipMemcpyDeviceToDevice, s);
    return;
  }
  dim3 grid(nblk((int64_t)X * (Y / FY), 256), (unsigned)((Z + FZ - 1) / FZ), 3);
  if (passes == 1) {
    k_filter<<<grid, 256, 0, s>>>(B, pi, W3{{out[0], out[1], out[2]}}, nullptr);
    return;
  }
  k_filter<<<grid, 256, 0, s>>>(B, pi, W3{{tmp[0], tmp[1], tmp[2]}}, nullptr);
  k_filter<<<grid, 256, 0, s>>>(B, P3{{tmp[0], tmp[1], tmp[2]}}, W3{{out[0], out[1], out[2]}}, nullptr);
}

int dn_reserve(gempic_dn* d, int64_t nv) {
  if (nv <= d->cap) return GEMPIC_OK;
  for (int q = 0; q < 3; ++q) { d->release(d->act[q]); d->act[q] = nullptr; }
  d->release(d->A);
  d->A = nullptr;
  d->cap = 0;
  d->act[0] = (unsigned short*)d->alloc(nv * 16 * 2);
  d->act[1] = (unsigned short*)d->alloc(nv * 32 * 2);
  d->act[2] = (unsigned short*)d->alloc(nv * 16 * 2);
  d->A = (float*)d->alloc(nv * 3 * 4);
  if (!d->act[0] || !d->act[1] || !d->act[2] || !d->A)
    return dn_fail(d, GEMPIC_ENOMEM, "denoiser activation buffers");
  d->cap = nv;
  return GEMPIC_OK;
}

static int reserve_train(gempic_dn* d, int64_t nv) {
  if (nv <= d->cap_train) return GEMPIC_OK;
  for (int q = 0; q < 3; ++q) {
    d->release(d->tact[q]); d->tact[q] = nullptr;
    d->release(d->gact[q]); d->gact[q] = nullptr;
  }
  for (float** p : {&d->tJf, &d->tJt, &d->tgJ, &d->tgA, &d->tA}) { d->release(*p); *p = nullptr; }
  d->cap_train = 0;
  const int ch[3] = {16, 32, 16};
  bool ok = true;
  for (int q = 0; q < 3; ++q) {
    d->tact[q] = (unsigned short*)d->alloc(nv * ch[q] * 2);
    d->gact[q] = (unsigned short*)d->alloc(nv * ch[q] * 2);
    ok = ok && d->tact[q] && d->gact[q];
  }
  for (float** p : {&d->tJf, &d->tJt, &d->tgJ, &d->tgA, &d->tA}) {
    *p = (float*)d->alloc(nv * 3 * 4);
    ok = ok && *p;
  }
  if (!ok) return dn_fail(d, GEMPIC_ENOMEM, "denoiser training buffers");
  d->cap_train = nv;
  return GEMPIC_OK;
}

static CurlArgs curl_args(int Z, int Y, int X, double n_e, const double hs[3]) {
  CurlArgs c;
  c.B = Box{Z, Y, X};
  c.s = (float)(n_e * hs[2]);
  c.ihx = (float)(1.0 / hs[0]);
  c.ihy = (float)(1.0 / hs[1]);
  c.ih = (float)(1.0 / hs[2]);
  return c;
}

// device workspace of one denoised box: activations, network output A
// ([3][nv] planar), the continuity test's partial sums and its decision
struct DnWork {
  unsigned short* act[3];
  float* A;
  double* part;      // 4 * COMB_BLOCKS
  int* use_net;
  double* rel;
};

static int dn_step_ws(gempic_dn* d, hipStream_t s, int Z, int Y, int X, const float* const J[3],
                      float* const Jf[3], float* const Jd[3], float* const tmp[3], double n_e, const double hs[3],
                      int passes, double thr, int64_t* fallbacks, double* rel, const DnWork& w) {
  int64_t nv = (int64_t)Z * Y * X;
  if (!d->packed) repack(d, s);
  // one binomial pass is formed inside the combine (the filtered current is
  // never stored); the fallback then filters the raw current into Jd
  const bool f1 = passes == 1;
  if (!f1) filter(s, Z, Y, X, J, Jf, tmp, passes);
  float* Ap[3] = {w.A, w.A + nv, w.A + 2 * nv};
  net_forward(d, s, Z, Y, X, J, (float)(1.0 / n_e), w.act, Ap);
  CurlArgs c = curl_args(Z, Y, X, n_e, hs);
  if (f1)
    k_combine_f1<2><<<COMB_BLOCKS, 256, 0, s>>>(c, P3{{J[0], J[1], J[2]}}, P3{{Ap[0], Ap[1], Ap[2]}},
                                                W3{{Jd[0], Jd[1], Jd[2]}}, w.part);
  else
    k_combine<<<COMB_BLOCKS, 256, 0, s>>>(c, P3{{Jf[0], Jf[1], Jf[2]}}, P3{{Ap[0], Ap[1], Ap[2]}},
                                          W3{{Jd[0], Jd[1], Jd[2]}}, w.part);
  k_decide<<<1, 256, 0, s>>>(w.part, COMB_BLOCKS, thr, w.use_net, rel ? rel : w.rel,
                             fallbacks ? fallbacks : d->fallbacks);
  if (f1) {
    dim3 grid(nblk((int64_t)X * (Y / FY), 256), (unsigned)((Z + FZ - 1) / FZ), 3);
    k_filter<<<grid, 256, 0, s>>>(c.B, P3{{J[0], J[1], J[2]}}, W3{{Jd[0], Jd[1], Jd[2]}}, w.use_net);
  } else {
    k_select<<<SEL_BLOCKS, 256, 0, s>>>(c.B, w.use_net, P3{{Jf[0], Jf[1], Jf[2]}}, W3{{Jd[0], Jd[1], Jd[2]}});
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dn_fail(d, GEMPIC_EDEVICE, std::string("denoiser launch: ") + hipGetErrorString(e));
  return GEMPIC_OK;
}

int dn_step(gempic_dn* d, hipStream_t s, int Z, int Y, int X, const float* const J[3], float* const Jf[3],
            float* const Jd[3], float* const tmp[3], double n_e, const double hs[3], int passes, double thr,
            int64_t* fallbacks, double* rel) {
  int64_t nv = (int64_t)Z * Y * X;
  int rc = check_box(d, Z, Y, X);
  if (rc) return rc;
  if (!(n_e > 0)) return dn_fail(d, GEMPIC_EINVAL, "denoiser needs n_e > 0");
  if ((rc = dn_reserve(d, nv))) return rc;
  DnWork w{{d->act[0], d->act[1], d->act[2]}, d->A, d->part, d->use_net, d->rel};
  return dn_step_ws(d, s, Z, Y, X, J, Jf, Jd, tmp, n_e, hs, passes, thr, fallbacks, rel, w);
}

const char* dn_error(const gempic_dn* d) { return d ? d->err.c_str() : ""; }

// one crop of a training batch: accumulate gradients into d->grad
static void train_crop(gempic_dn* d, hipStream_t s, int Z, int Y, int X, const float* const Jr[3],
                       const float* const Jt[3], double n_e, const double hs[3], int passes, int lo, int hi,
                       int nbatch) {
  int64_t nv = (int64_t)Z * Y * X;
  unsigned nb = conv_blocks(Z, Y, X);
  float* Jf[3] = {d->tJf, d->tJf + nv, d->tJf + 2 * nv};
  float* Jtf[3] = {d->tJt, d->tJt + nv, d->tJt + 2 * nv};
  float* gJ[3] = {d->tgJ, d->tgJ + nv, d->tgJ + 2 * nv};
  float* gA[3] = {d->tgA, d->tgA + nv, d->tgA + 2 * nv};
  float* Ap[3] = {d->tA, d->tA + nv, d->tA + 2 * nv};
  // gJ doubles as the scratch of a second filter pass (it is written later)
  filter(s, Z, Y, X, Jr, Jf, gJ, passes);
  filter(s, Z, Y, X, Jt, Jtf, gJ, passes);
  float in_scale = (float)(1.0 / n_e);
  net_forward(d, s, Z, Y, X, Jr, in_scale, d->tact, Ap);
  LossArgs la;
  la.c = curl_args(Z, Y, X, n_e, hs);
  la.lo = lo;
  la.hi = hi;
  double N = 3.0 * (double)(hi - lo) * Y * X;
  la.inv_ne = (float)(1.0 / n_e);
  la.gscale = (float)(2.0 / (n_e * N * nbatch));
  la.lscale = 1.0 / (N * nbatch);
  k_loss<<<nblk(nv, 256), 256, 0, s>>>(la, P3{{Jf[0], Jf[1], Jf[2]}}, P3{{Ap[0], Ap[1], Ap[2]}},
                                       P3{{Jtf[0], Jtf[1], Jtf[2]}}, W3{{gJ[0], gJ[1], gJ[2]}}, d->red + 2);
  k_curl_adj<<<nblk(nv, 256), 256, 0, s>>>(la.c, P3{{gJ[0], gJ[1], gJ[2]}}, W3{{gA[0], gA[1], gA[2]}});

  float* gW[NLAYER];
  float* gb[NLAYER];
  for (int l = 0; l < NLAYER; ++l) {
    gW[l] = d->grad + layer_woff(l);
    gb[l] = gW[l] + (int64_t)L_COUT[l] * L_CIN[l] * 27;
  }
  WgradArgs w;
  std::memset(&w, 0, sizeof(w));
  w.Z = Z; w.Y = Y; w.X = X;
  ConvArgs c;
  std::memset(&c, 0, sizeof(c));
  c.Z = Z; c.Y = Y; c.X = X;
  // layer 4: gy = gA (planar), x = act3
  w.x = (const u32x4*)d->tact[2];
  for (int q = 0; q < 3; ++q) w.gyf[q] = gA[q];
  w.gW = gW[3]; w.gb = gb[3];
  k_wgrad<16, 3, 16, 4, 0, 1><<<nb, 256, 0, s>>>(w);
  for (int q = 0; q < 3; ++q) c.inf[q] = gA[q];
  c.in_scale = 1.0f;
  c.wp = d->bw[3]; c.mask = d->tact[2]; c.out = d->gact[2];
  k_conv<8, 16, 1, 2><<<conv_grid(k_conv<8, 16, 1, 2>, nb), 256, 0, s>>>(c);
  // layer 3: gy = g3 (16 ch), x = act2 (32 ch)
  w.x = (const u32x4*)d->tact[1];
  w.gy = (const u32x4*)d->gact[2];
  w.gW = gW[2]; w.gb = gb[2];
  k_wgrad<32, 16, 32, 16, 0, 0><<<nb, 256, 0, s>>>(w);
  c.in = (const u32x4*)d->gact[2]; c.wp = d->bw[2]; c.mask = d->tact[1]; c.out = d->gact[1];
  k_conv<16, 32, 0, 2><<<conv_grid(k_conv<16, 32, 0, 2>, nb), 256, 0, s>>>(c);
  // layer 2: gy = g2 (32 ch), x = act1 (16 ch)
  w.x = (const u32x4*)d->tact[0];
  w.gy = (const u32x4*)d->gact[1];
  w.gW = gW[1]; w.gb = gb[1];
  k_wgrad<16, 32, 16, 32, 0, 0><<<nb, 256, 0, s>>>(w);
  c.in = (const u32x4*)d->gact[1]; c.wp = d->bw[1]; c.mask = d->tact[0]; c.out = d->gact[0];
  k_conv<32, 16, 0, 2><<<conv_grid(k_conv<32, 16, 0, 2>, nb), 256, 0, s>>>(c);
  // layer 1: gy = g1 (16 ch), x = J / n_e (planar)
  w.x = nullptr;
  for (int q = 0; q < 3; ++q) w.xf[q] = Jr[q];
  w.x_scale = in_scale;
  w.gy = (const u32x4*)d->gact[0];
  w.gW = gW[0]; w.gb = gb[0];
  k_wgrad<3, 16, 4, 16, 1, 0><<<nb, 256, 0, s>>>(w);
}

// ---------------------------------------------------------------------------
extern "C" {

size_t gempic_dn_nparams(void) { return (size_t)n_params(); }

int gempic_dn_create(const float* theta, size_t n, void* stream, gempic_dn_t** out) {
  if (!out) return GEMPIC_EINVAL;
  *out = nullptr;
  if (!theta || n != (size_t)n_params()) return GEMPIC_EINVAL;
  gempic_dn* d = new gempic_dn();
  d->s = (hipStream_t)stream;
  size_t pb = (size_t)n_params() * 4;
  d->theta = (float*)d->alloc(pb);
  d->m = (float*)d->alloc(pb);
  d->v = (float*)d->alloc(pb);
  d->grad = (float*)d->alloc(pb);
  bool ok = d->theta && d->m && d->v && d->grad;
  for (int l = 0; l < NLAYER; ++l) {
    d->fw[l] = (u32x4*)d->alloc(packed_units(pad_in(L_CIN[l]), pad_out(L_COUT[l])) * 16);
    ok = ok && d->fw[l];
    if (l > 0) {
      d->bw[l] = (u32x4*)d->alloc(packed_units(pad_in(L_COUT[l]), pad_out(L_CIN[l])) * 16);
      ok = ok && d->bw[l];
    }
  }
  d->red = (double*)d->alloc(4 * 8);
  d->part = (double*)d->alloc(4 * COMB_BLOCKS * 8);
  d->use_net = (int*)d->alloc(sizeof(int));
  d->rel = (double*)d->alloc(8);
  d->fallbacks = (int64_t*)d->alloc(8);
  ok = ok && d->red && d->part && d->use_net && d->rel && d->fallbacks;
  if (!ok) { gempic_dn_destroy(d); return GEMPIC_ENOMEM; }
  hipStream_t s = d->s;
  bool cp = hipMemcpyAsync(d->theta, theta, pb, hipMemcpyHostToDevice, s) == hipSuccess;
  k_zero<float><<<nblk(n_params(), 256), 256, 0, s>>>(d->m, n_params());
  k_zero<float><<<nblk(n_params(), 256), 256, 0, s>>>(d->v, n_params());
  k_zero<float><<<nblk(n_params(), 256), 256, 0, s>>>(d->grad, n_params());
  k_zero<double><<<1, 64, 0, s>>>(d->red, 4);
  k_zero<double><<<1, 64, 0, s>>>(d->rel, 1);
  k_zero<int64_t><<<1, 64, 0, s>>>(d->fallbacks, 1);
  repack(d, s);
  if (!cp || hipStreamSynchronize(s) != hipSuccess) { gempic_dn_destroy(d); return GEMPIC_EDEVICE; }
  *out = d;
  return GEMPIC_OK;
}

void gempic_dn_destroy(gempic_dn_t* d) {
  if (!d) return;
  (void)hipStreamSynchronize(d->s);
  for (void* p : d->ptrs) (void)hipFree(p);
  delete d;
}

const char* gempic_dn_last_error(const gempic_dn_t* d) { return dn_error(d); }

int gempic_dn_params(gempic_dn_t* d, float* theta, size_t n) {
  if (!d || !theta || n < (size_t)n_params()) return dn_fail(d, GEMPIC_EINVAL, "bad arguments");
  DNCHK(d, hipMemcpyAsync(theta, d->theta, n_params() * 4, hipMemcpyDeviceToHost, d->s));
  DNCHK(d, hipStreamSynchronize(d->s));
  return GEMPIC_OK;
}

int gempic_dn_grad(gempic_dn_t* d, float* grad, size_t n) {
  if (!d || !grad || n < (size_t)n_params()) return dn_fail(d, GEMPIC_EINVAL, "bad arguments");
  DNCHK(d, hipMemcpyAsync(grad, d->grad, n_params() * 4, hipMemcpyDeviceToHost, d->s));
  DNCHK(d, hipStreamSynchronize(d->s));
  return GEMPIC_OK;
}

int gempic_dn_apply(gempic_dn_t* d, const int32_t box[3], const float* jraw, double n_e, const double h[3],
                    int32_t passes, double threshold, float* jout, float* aout, int32_t* used, double* rel) {
  if (!d || !box || !jraw || !h || !jout) return dn_fail(d, GEMPIC_EINVAL, "null argument");
  if (passes < 0 || passes > 2) return dn_fail(d, GEMPIC_EINVAL, "passes must be 0, 1 or 2");
  int Z = box[0], Y = box[1], X = box[2];
  int rc = check_box(d, Z, Y, X);
  if (rc) return rc;
  int64_t nv = (int64_t)Z * Y * X;
  if ((rc = reserve_train(d, nv))) return rc;   // filtered current and scratch
  const float* J[3] = {jraw, jraw + nv, jraw + 2 * nv};
  float* Jf[3] = {d->tJf, d->tJf + nv, d->tJf + 2 * nv};
  float* tmp[3] = {d->tgJ, d->tgJ + nv, d->tgJ + 2 * nv};
  float* Jd[3] = {jout, jout + nv, jout + 2 * nv};
  rc = dn_step(d, d->s, Z, Y, X, J, Jf, Jd, tmp, n_e, h, passes, threshold, nullptr, nullptr);
  if (rc) return rc;
  if (aout) DNCHK(d, hipMemcpyAsync(aout, d->A, nv * 3 * 4, hipMemcpyDeviceToDevice, d->s));
  int un = 0;
  double rv = 0.0;
  DNCHK(d, hipMemcpyAsync(&un, d->use_net, sizeof(int), hipMemcpyDeviceToHost, d->s));
  DNCHK(d, hipMemcpyAsync(&rv, d->rel, 8, hipMemcpyDeviceToHost, d->s));
  DNCHK(d, hipStreamSynchronize(d->s));
  if (used) *used = un;
  if (rel) *rel = rv;
  return GEMPIC_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free variant of gempic_dn_apply.  Every per-box buffer lives in
// one file-scope device array: bf16 activations (16, 32, 16 channels), A,
// the filtered current, the second filter pass and the continuity test's
// partial sums and decision, each at a fixed offset sized for
// DN_NOALLOC_MAX_VOXELS voxels.  Each device holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (kept in g_scratch_ptr).  Every buffer is fully written
// before it is read, so nothing needs clearing between calls.
}  // extern "C"

constexpr int64_t DN_NOALLOC_MAX_VOXELS = int64_t(1) << 18;
constexpr size_t dn_round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t SCR_ACT0 = 0;
constexpr size_t SCR_ACT1 = SCR_ACT0 + dn_round256((size_t)DN_NOALLOC_MAX_VOXELS * 16 * 2);
constexpr size_t SCR_ACT2 = SCR_ACT1 + dn_round256((size_t)DN_NOALLOC_MAX_VOXELS * 32 * 2);
constexpr size_t SCR_A = SCR_ACT2 + dn_round256((size_t)DN_NOALLOC_MAX_VOXELS * 16 * 2);
constexpr size_t SCR_JF = SCR_A + dn_round256((size_t)DN_NOALLOC_MAX_VOXELS * 3 * 4);
constexpr size_t SCR_TMP = SCR_JF + dn_round256((size_t)DN_NOALLOC_MAX_VOXELS * 3 * 4);
constexpr size_t SCR_PART = SCR_TMP + dn_round256((size_t)DN_NOALLOC_MAX_VOXELS * 3 * 4);
constexpr size_t SCR_USE = SCR_PART + dn_round256((size_t)4 * COMB_BLOCKS * 8);
constexpr size_t SCR_REL = SCR_USE + 256;
constexpr size_t DN_SCRATCH_BYTES = SCR_REL + 256;   // 43,057,664 bytes (41.1 MiB)

static __device__ __align__(256) unsigned char scratch[DN_SCRATCH_BYTES];

constexpr int DN_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[DN_MAX_DEVICES];

// device address of the current device's scratch array (looked up once per
// device, with that device current)
static int scratch_address(gempic_dn* d, unsigned char** out) {
  int dev = 0;
  DNCHK(d, hipGetDevice(&dev));
  if (dev < 0 || dev >= DN_MAX_DEVICES) return dn_fail(d, GEMPIC_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return dn_fail(d, GEMPIC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return GEMPIC_OK;
}

extern "C" {

int gempic_dn_apply_noalloc(gempic_dn_t* d, const int32_t box[3], const float* jraw, double n_e,
                            const double h[3], int32_t passes, double threshold, float* jout, float* aout,
                            int32_t* used, double* rel) {
  if (!d || !box || !jraw || !h || !jout) return dn_fail(d, GEMPIC_EINVAL, "null argument");
  if (passes < 0 || passes > 2) return dn_fail(d, GEMPIC_EINVAL, "passes must be 0, 1 or 2");
  if (!(n_e > 0)) return dn_fail(d, GEMPIC_EINVAL, "denoiser needs n_e > 0");
  int Z = box[0], Y = box[1], X = box[2];
  int rc = check_box(d, Z, Y, X);
  if (rc) return rc;
  int64_t nv = (int64_t)Z * Y * X;
  if (nv > DN_NOALLOC_MAX_VOXELS)
    return dn_fail(d, GEMPIC_EINVAL, "box larger than the allocation-free limit of 2^18 voxels");
  unsigned char* base = nullptr;
  if ((rc = scratch_address(d, &base))) return rc;
  DnWork w;
  w.act[0] = (unsigned short*)(base + SCR_ACT0);
  w.act[1] = (unsigned short*)(base + SCR_ACT1);
  w.act[2] = (unsigned short*)(base + SCR_ACT2);
  w.A = (float*)(base + SCR_A);
  w.part = (double*)(base + SCR_PART);
  w.use_net = (int*)(base + SCR_USE);
  w.rel = (double*)(base + SCR_REL);
  float* jf = (float*)(base + SCR_JF);
  float* tp = (float*)(base + SCR_TMP);
  const float* J[3] = {jraw, jraw + nv, jraw + 2 * nv};
  float* Jf[3] = {jf, jf + nv, jf + 2 * nv};
  float* tmp[3] = {tp, tp + nv, tp + 2 * nv};
  float* Jd[3] = {jout, jout + nv, jout + 2 * nv};
  // fallbacks are counted in the handle's counter, as gempic_dn_apply does
  rc = dn_step_ws(d, d->s, Z, Y, X, J, Jf, Jd, tmp, n_e, h, passes, threshold, nullptr, nullptr, w);
  if (rc) return rc;
  if (aout) DNCHK(d, hipMemcpyAsync(aout, w.A, nv * 3 * 4, hipMemcpyDeviceToDevice, d->s));
  int un = 0;
  double rv = 0.0;
  DNCHK(d, hipMemcpyAsync(&un, w.use_net, sizeof(int), hipMemcpyDeviceToHost, d->s));
  DNCHK(d, hipMemcpyAsync(&rv, w.rel, 8, hipMemcpyDeviceToHost, d->s));
  DNCHK(d, hipStreamSynchronize(d->s));
  if (used) *used = un;
  if (rel) *rel = rv;
  return GEMPIC_OK;
}

int gempic_dn_train(gempic_dn_t* d, const int32_t box[3], int32_t nbatch, const float* jraw,
                    const float* jtarget, double n_e, const double h[3], int32_t passes, const int32_t region[2],
                    double lr, double* loss) {
  if (!d || !box || !jraw || !jtarget || !h || !region) return dn_fail(d, GEMPIC_EINVAL, "null argument");
  if (nbatch < 1) return dn_fail(d, GEMPIC_EINVAL, "nbatch must be >= 1");
  if (passes < 0 || passes > 2) return dn_fail(d, GEMPIC_EINVAL, "passes must be 0, 1 or 2");
  if (!(n_e > 0)) return dn_fail(d, GEMPIC_EINVAL, "n_e must be > 0");
  int Z = box[0], Y = box[1], X = box[2];
  int rc = check_box(d, Z, Y, X);
  if (rc) return rc;
  if (region[0] < 0 || region[1] > Z || region[0] >= region[1])
    return dn_fail(d, GEMPIC_EINVAL, "region must satisfy 0 <= lo < hi <= Z");
  int64_t nv = (int64_t)Z * Y * X;
  if ((rc = reserve_train(d, nv))) return rc;
  hipStream_t s = d->s;
  k_zero<float><<<nblk(n_params(), 256), 256, 0, s>>>(d->grad, n_params());
  k_zero<double><<<1, 64, 0, s>>>(d->red + 2, 1);
  for (int b = 0; b < nbatch; ++b) {
    const float* jr = jraw + (int64_t)b * 3 * nv;
    const float* jt = jtarget + (int64_t)b * 3 * nv;
    const float* Jr[3] = {jr, jr + nv, jr + 2 * nv};
    const float* Jt[3] = {jt, jt + nv, jt + 2 * nv};
    train_crop(d, s, Z, Y, X, Jr, Jt, n_e, h, passes, region[0], region[1], nbatch);
  }
  if (lr > 0) {
    d->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)d->t)));
    float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)d->t)));
    k_adam<<<nblk(n_params(), 256), 256, 0, s>>>(d->theta, d->m, d->v, d->grad, n_params(), (float)lr,
                                                 (float)b1, (float)b2, 1e-8f, c1, c2);
    repack(d, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dn_fail(d, GEMPIC_EDEVICE, std::string("training launch: ") + hipGetErrorString(e));
  if (loss) {
    DNCHK(d, hipMemcpyAsync(loss, d->red + 2, 8, hipMemcpyDeviceToHost, s));
    DNCHK(d, hipStreamSynchronize(s));
  }
  return GEMPIC_OK;
}

}  // extern "C"
