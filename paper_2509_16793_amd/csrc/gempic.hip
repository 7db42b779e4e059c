// Host driver and C ABI of the gfx950 Galilean PIC library (see include/gempic.h).
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gempic.h"
#include "../../include/gempic_denoise.h"
#include "common.h"
#include "diag.h"
#include "dn_internal.h"
#include "fields.h"
#include "particles.h"
#include "march.h"

namespace {

thread_local std::string g_create_error;

// roctx ranges around the phases of a step, so that rocprofv3 (--marker-trace,
// or --kernel-rename to name each kernel after its phase) attributes the
// kernels.  The roctx library is opened at run time; without it a range does
// nothing.  Ranges are host-side: they bracket the enqueueing of a phase.
struct RoctxLib {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
  RoctxLib() {
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr;
  }
};
const RoctxLib& roctx() {
  static const RoctxLib lib;
  return lib;
}
struct Range {
  const bool on;
  explicit Range(const char* name) : on(roctx().push != nullptr) {
    if (on) roctx().push(name);
  }
  void next(const char* name) {
    if (!on) return;
    roctx().pop();
    roctx().push(name);
  }
  ~Range() {
    if (on) roctx().pop();
  }
};

struct Dev {
  std::vector<void*> ptrs;
  hipError_t last = hipSuccess;
  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) { last = e; return nullptr; }
    ptrs.push_back(p);
    return p;
  }
  void free(void* p) {
    for (size_t i = 0; i < ptrs.size(); ++i)
      if (ptrs[i] == p) {
        (void)hipFree(p);
        ptrs.erase(ptrs.begin() + (long)i);
        return;
      }
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct gempic {
  gempic_config cfg;
  Geom g;
  int prec;          // 0 fp64, 1 fp32
  size_t esz;        // sizeof(T)
  hipStream_t s;
  int ppcx, ppcy, ppcz, quiet;
  uint64_t key;
  double L, hz, w, Tlas, zeta_c, waist;
  int64_t nbeam;     // driver-beam particles created (0: no beam)
  double wb;         // weight of a driver-beam particle
  unsigned long long* bcount;   // diagnostics: beam particles in the buffer
  int64_t step;
  bool failed;
  std::string err;
  Dev dev;

  // particles: two buffers of 7 arrays (cell, ox, oy, oz, ux, uy, uz) + ids
  void* part[2][7];
  int64_t* ids[2];
  int cur;
  void* stage[7];
  int32_t* stage_g;
  int64_t capacity, stage_per_tile, max_nm;
  int max_chunks;
  ChunkTab ct[2];
  int ctc;
  int32_t *code, *counts, *offs, *inj_count, *inj_off, *gflag, *grank;
  int64_t *tile_count, *tile_base, *total, *next_id, *inj_total, *pushed;
  int64_t* scan_part;   // per-block partial sums of the tile scan
  int* err_dev;
  // grids
  void* F6;          // gather fields: node records [Nz][Ny][Nx][6]
  void* J[3];
  void* rho[2];
  void* Jhat[3];
  void* st[4];
  void* outs[6];
  void* Lsp[2];
  void* twx;
  void* twy;
  double* partial;
  double* dres;
  // learned current denoiser (not owned): filtered and denoised currents
  gempic_dn* dn;
  double dn_thr;
  void* Jf[3];
  void* Jd[3];
  void* Jt[3];
  int64_t* dn_fallbacks;
  double* dn_rel;
  // deterministic deposit (FP32, tau scheme): 64-bit fixed-point current sums
  bool det;
  void* Jfix[3];
  // zeta march (scheme 1 = GT1, 2 = GT2)
  int scheme;
  double Delta;                 // slow step of the next step (normalised)
  std::vector<double> zn;       // node positions zeta_0 .. zeta_Nz (normalised)
  int64_t nperp;                // fresh particles per batch
  int64_t mz_batches;           // batches loaded at creation
  int mz_cap;                   // capacity of each march particle buffer
  int mz_first;                 // no previous-step current yet
  int mz_stage_blocks;
  int mz_subcap;                // sub-step bound per particle and stage
  void* mz_part[4][10];         // park, stop, active 0, active 1: cell ox oy oz ux uy uz w b id
  int* mz_cnt;                  // active[2], stop, left, parked total
  int *mz_pstart, *mz_pcount, *mz_cursor;
  void *mz_dep, *mz_jhat, *mz_out6, *mz_zj;
  void* mz_j0[2];
  void* F6b;                    // new-level node records
  double* mz_hnode;             // node volumes / (h_x h_y): (h_{n-1} + h_n) / 2
  double* mz_zn;                // node positions on the device
  double s_total;               // slow coordinate reached (sum of the steps' Delta)
  // timing: five events per step while enabled
  bool timing;
  std::vector<hipEvent_t> ev;
  int64_t tsteps;
};

static int fail(gempic* g, int code, const std::string& msg) {
  if (g) {
    g->err = msg;
    if (code == GEMPIC_EDEVICE || code == GEMPIC_ECFL || code == GEMPIC_ENUMERIC ||
        code == GEMPIC_ECAPACITY)
      g->failed = true;
  } else {
    g_create_error = msg;
  }
  return code;
}

#define HIPCHK(g, expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(g, GEMPIC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

static bool pow2(int v) { return v >= 1 && (v & (v - 1)) == 0; }

// a kernel launch that failed (bad configuration, too much LDS) leaves a
// sticky error that hipGetLastError reports; map it to GEMPIC_EDEVICE
static int launch_check(gempic* g, const char* phase) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(g, GEMPIC_EDEVICE, std::string(phase) + ": " + hipGetErrorString(e));
  return GEMPIC_OK;
}

// tile_base / total and the chunk table heads of t from g->tile_count
static void scan_tiles(gempic* g, ChunkTab& t) {
  const Geom& G = g->g;
  int nb = (G.NT + SCAN_PER - 1) / SCAN_PER;
  k_scan_tiles_sum<<<nb, 1024, 0, g->s>>>(G.NT, g->tile_count, g->scan_part);
  k_scan_tiles_top<<<1, 1024, 0, g->s>>>(nb, g->scan_part, g->total, t.n, g->capacity, g->err_dev);
  k_scan_tiles_apply<<<nb, 1024, 0, g->s>>>(G.NT, g->tile_count, g->scan_part, g->tile_base, t.first, t.count);
}
static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Driver beam sampled on the host in FP64.  Particle i draws four SplitMix64
// uniforms u_k = uniform(key, 4 i + k); the Box-Muller transform of
// (1 - u_0, u_1) gives the transverse pair, of (1 - u_2, u_3) the zeta and
// gamma deviates.  Positions wrap transversally; particles outside the field
// box in zeta, 0 <= zeta < (Nz - 1) h, are not created.
struct HostBeam {
  int64_t n = 0;
  std::vector<int32_t> cell, tile;
  std::vector<double> off;   // [3][n]
  std::vector<double> uz;
  std::vector<int64_t> dst;
};

static void sample_beam(const gempic* g, HostBeam* hb) {
  const Geom& G = g->g;
  const gempic_config* c = &g->cfg;
  double lu = c->length_unit;
  uint64_t key = sm_mix(c->seed ^ (1ull << 56));
  double sr = c->beam_sr * lu, sz = c->beam_sz * lu;
  double zc = std::isnan(c->beam_zc) ? (double)(G.Nz - 1) * G.h - 6.0 * sz : c->beam_zc * lu;
  double Lx = (double)G.Nx * G.hx, Ly = (double)G.Ny * G.hy, zmax = (double)(G.Nz - 1) * G.h;
  double xc = (double)(G.Nx / 2) * G.hx, yc = (double)(G.Ny / 2) * G.hy;
  const double below1 = 0x1.fffffffffffffp-1;
  std::vector<double> ox, oy, oz;
  for (int64_t i = 0; i < c->beam_np; ++i) {
    uint64_t k = 4ull * (uint64_t)i;
    double u0 = 1.0 - sm_uniform(key, k), u1 = sm_uniform(key, k + 1);
    double u2 = 1.0 - sm_uniform(key, k + 2), u3 = sm_uniform(key, k + 3);
    double r1 = std::sqrt(-2.0 * std::log(u0)), r2 = std::sqrt(-2.0 * std::log(u2));
    double a1 = 2.0 * M_PI * u1, a2 = 2.0 * M_PI * u3;
    double x = xc + sr * r1 * std::cos(a1);
    double y = yc + sr * r1 * std::sin(a1);
    double zeta = zc + sz * r2 * std::cos(a2);
    double gam = c->beam_gamma + c->beam_dgamma * r2 * std::sin(a2);
    if (!(zeta >= 0.0 && zeta < zmax)) continue;
    x = std::fmod(x, Lx);
    if (x < 0.0) x += Lx;
    y = std::fmod(y, Ly);
    if (y < 0.0) y += Ly;
    double fx = x / G.hx, fy = y / G.hy, fz = zeta / G.h;
    int ix = std::min((int)std::floor(fx), G.Nx - 1);
    int iy = std::min((int)std::floor(fy), G.Ny - 1);
    int iz = (int)std::floor(fz);
    hb->cell.push_back((iz * G.Ny + iy) * G.Nx + ix);
    hb->tile.push_back(((iz / G.Tz) * G.nTy + iy / G.Ty) * G.nTx + ix / G.Tx);
    ox.push_back(std::min(fx - (double)ix, below1));
    oy.push_back(std::min(fy - (double)iy, below1));
    oz.push_back(std::min(fz - (double)iz, below1));
    hb->uz.push_back(gam > 1.0 ? std::sqrt(gam * gam - 1.0) : 0.0);
  }
  hb->n = (int64_t)hb->cell.size();
  hb->off.reserve(3 * hb->n);
  hb->off.insert(hb->off.end(), ox.begin(), ox.end());
  hb->off.insert(hb->off.end(), oy.begin(), oy.end());
  hb->off.insert(hb->off.end(), oz.begin(), oz.end());
}

template <typename T>
struct Impl {
  using C = cplx<T>;

  static PartPtrs<T> parts(gempic* g, int b) {
    PartPtrs<T> P;
    P.cell = (int32_t*)g->part[b][0];
    P.ox = (T*)g->part[b][1];
    P.oy = (T*)g->part[b][2];
    P.oz = (T*)g->part[b][3];
    P.ux = (T*)g->part[b][4];
    P.uy = (T*)g->part[b][5];
    P.uz = (T*)g->part[b][6];
    P.id = g->ids[b];
    return P;
  }
  static PartPtrs<T> staging(gempic* g) {
    PartPtrs<T> P;
    P.cell = (int32_t*)g->stage[0];
    P.ox = (T*)g->stage[1];
    P.oy = (T*)g->stage[2];
    P.oz = (T*)g->stage[3];
    P.ux = (T*)g->stage[4];
    P.uy = (T*)g->stage[5];
    P.uz = (T*)g->stage[6];
    P.id = nullptr;
    return P;
  }

  static void fill(gempic* g, void* p, int64_t n) {
    if (n <= 0) return;
    if (((uintptr_t)p & 15) == 0) {
      const int64_t w = 16 / (int64_t)sizeof(T);
      k_fill16<T><<<nblk(n / w + n % w, 256), 256, 0, g->s>>>((T*)p, n, (T)0);
    } else {
      k_fill<T><<<nblk(n, 256), 256, 0, g->s>>>((T*)p, n, (T)0);
    }
  }

  // ---- FFT helpers --------------------------------------------------------
  // transform along y of data[planes][Ny][Nxh] in place
  static void fft_y(gempic* g, C* data, int64_t planes, int inverse) {
    const Geom& G = g->g;
    if (G.Ny == 256 && G.Nxh % fy_nc<T>() == 0) {
      k_fft_y256<T><<<(unsigned)(planes * (G.Nxh / fy_nc<T>())), 16 * fy_nc<T>(), 0, g->s>>>(
          data, G.Nxh, (const C*)g->twy, inverse);
      return;
    }
    if (G.Ny == 512 && G.Nxh % fy_nc<T>() == 0) {
      k_fft_y512<T><<<(unsigned)(planes * (G.Nxh / fy_nc<T>())), 32 * fy_nc<T>(), 0, g->s>>>(
          data, G.Nxh, (const C*)g->twy, inverse);
      return;
    }
    int ncol = std::min(G.Nxh, std::max(1, 2048 / G.Ny));
    size_t sh = (2 * (size_t)ncol * (G.Ny + FFTY_PAD) + G.Ny) * sizeof(C);
    k_fft_y<T><<<(unsigned)(planes * (G.Nxh / ncol)), 512, sh, g->s>>>(data, G.Ny, G.Nxh, ncol, (const C*)g->twy,
                                                                      inverse);
  }
  static void fft_fwd(gempic* g, const T* in, C* out, int64_t planes) {
    fft_xfwd(g, in, out, planes);
    if (g->g.Ny > 1) fft_y(g, out, planes, 0);
  }
  // the x part of fft_fwd: real rows -> half spectra along x
  static void fft_xfwd(gempic* g, const T* in, C* out, int64_t planes) {
    const Geom& G = g->g;
    int64_t rows = planes * G.Ny;
    int64_t pairs = (rows + 1) / 2;
    int nseq = std::max(1, std::min<int>((int)std::min<int64_t>(pairs, 1 << 20), 1024 / G.Nx));
    size_t sh = (2 * (size_t)nseq + 1) * G.Nx * sizeof(C);
    if (G.Nx == 256)
      k_fft_x_r2c_256<T><<<(unsigned)((pairs + R2C256_P - 1) / R2C256_P), 128, 0, g->s>>>(in, out, rows, (const C*)g->twx);
    else if (G.Nx == 512)
      k_fft_x_r2c_512<T><<<(unsigned)((pairs + R2C512_P - 1) / R2C512_P), 128, 0, g->s>>>(in, out, rows, (const C*)g->twx);
    else
      k_fft_x_r2c<T><<<nblk(pairs, nseq), 256, sh, g->s>>>(in, out, rows, G.Nx, nseq, (const C*)g->twx);
  }
  // inverse x transforms of `rows` rows of six field spectra (in[q] + row
  // Nxh) -> interleaved real node records
  static void c2r6(gempic* g, const C* const in[6], T* dst, int64_t rows) {
    const Geom& G = g->g;
    int64_t pairs = (rows + 1) / 2;
    int nseq = std::max(1, std::min<int>((int)std::min<int64_t>(pairs, 1 << 20), 2048 / (6 * G.Nx)));
    size_t sh = (2 * (size_t)6 * nseq + 1) * G.Nx * sizeof(C);
    if (G.Nx == 256) {
      k_fft_x_c2r6_256<T><<<(unsigned)((pairs + C2R256_P - 1) / C2R256_P), 192, 0, g->s>>>(
          in[0], in[1], in[2], in[3], in[4], in[5], dst, rows, (const C*)g->twx);
      return;
    }
    if (G.Nx == 512) {
      k_fft_x_c2r6_512<T><<<(unsigned)pairs, 192, 0, g->s>>>(in[0], in[1], in[2], in[3], in[4], in[5], dst,
                                                                rows, (const C*)g->twx);
      return;
    }
    k_fft_x_c2r6<T><<<nblk(pairs, nseq), 256, sh, g->s>>>(in[0], in[1], in[2], in[3], in[4], in[5], dst, rows,
                                                            G.Nx, nseq, (const C*)g->twx);
  }
  // six field spectra (outs) -> interleaved real node records F6
  static void fft_inv6(gempic* g) {
    const Geom& G = g->g;
    if (G.Ny > 1)
      for (int q = 0; q < 6; ++q) fft_y(g, (C*)g->outs[q], G.Nz, 1);
    const C* in[6];
    for (int q = 0; q < 6; ++q) in[q] = (const C*)g->outs[q];
    c2r6(g, in, (T*)g->F6, (int64_t)G.Nz * G.Ny);
  }

  // ---- field update: FFT(J) -> march -> iFFT ------------------------------
  // The solver filters the current itself unless the denoiser has already
  // produced the current it is to use (filter passes 0 in the march).
  static void field_update(gempic* g, bool with_current, T Delta) {
    const Geom& G = g->g;
    MarchArgs<T> a;
    a.g = G;
    bool den = with_current && g->dn;
    if (den) a.g.P = 0;
    for (int q = 0; q < 3; ++q) {
      if (with_current) fft_fwd(g, (const T*)(den ? g->Jd[q] : g->J[q]), (C*)g->Jhat[q], G.NPF);
      a.J[q] = with_current ? (const C*)g->Jhat[q] : nullptr;
    }
    for (int q = 0; q < 4; ++q) a.st[q] = (C*)g->st[q];
    for (int q = 0; q < 6; ++q) a.out[q] = (C*)g->outs[q];
    a.L[0] = (C*)g->Lsp[0];
    a.L[1] = (C*)g->Lsp[1];
    a.Delta = Delta;
    int64_t M = (int64_t)G.Ny * G.Nxh;
    if (a.g.P == 0) k_march<T, 0><<<nblk(M, 64), 64, 0, g->s>>>(a);
    else if (a.g.P == 1) k_march<T, 1><<<nblk(M, 64), 64, 0, g->s>>>(a);
    else k_march<T, 2><<<nblk(M, 64), 64, 0, g->s>>>(a);
    fft_inv6(g);
  }

  // ---- sort + window injection of batch b --------------------------------
  static int sort_and_inject(gempic* g, int64_t b) {
    const Geom& G = g->g;
    int A = g->cur, B = 1 - g->cur;
    ChunkTab& oldt = g->ct[g->ctc];
    ChunkTab& newt = g->ct[1 - g->ctc];
    SortArgs sa;
    sa.g = G;
    sa.ct = oldt;
    sa.cell = (const int32_t*)g->part[A][0];
    sa.px = (const float*)g->part[A][1];
    sa.py = (const float*)g->part[A][2];
    sa.pz = (const float*)g->part[A][3];
    sa.code = g->code;
    sa.counts = g->counts;
    sa.err = g->err_dev;
    k_sort_rank<<<g->max_chunks, 64, 0, g->s>>>(sa);

    k_fill<int32_t><<<nblk(G.NT, 256), 256, 0, g->s>>>(g->inj_count, G.NT, 0);
    InjArgs ia;
    int64_t nm = 0;
    if (g->cfg.n_e > 0.0) {
      double lo = g->L + (double)b * G.dtau;
      double hi = g->L + (double)(b + 1) * G.dtau;
      int64_t m0 = (int64_t)(G.Nzp - 1) * g->ppcz;
      int64_t m_lo = b > 0 ? std::max<int64_t>(m0, (int64_t)std::floor(lo / g->hz) - 1) : m0;
      int64_t m_hi = (int64_t)std::floor(hi / g->hz) + 1;
      nm = m_hi - m_lo + 1;
      if (nm > g->max_nm) return fail(g, GEMPIC_EDEVICE, "internal: window batch larger than staging");
      ia.g = G;
      ia.ppcx = g->ppcx; ia.ppcy = g->ppcy; ia.ppcz = g->ppcz;
      ia.quiet = g->quiet;
      ia.key = g->key;
      ia.b = (int)b;
      ia.m_lo = m_lo; ia.m_hi = m_hi;
      ia.lo = lo; ia.hi = hi; ia.hz = g->hz;
      ia.shift = (double)b * G.dtau;
      ia.stage_per_tile = g->stage_per_tile;
      ia.inj_count = g->inj_count;
      ia.stage_g = g->stage_g;
      ia.gflag = g->ids[0] ? g->gflag : nullptr;
      k_inject<T><<<G.nTx * G.nTy, 256, 0, g->s>>>(ia, staging(g));
      if (g->ids[0]) {
        int64_t ng = nm * G.Ny * G.Nx * g->ppcx * g->ppcy;
        k_scan_flags<<<1, 1024, 0, g->s>>>(ng, g->gflag, g->grank, nullptr);
      }
    }
    OffArgs oa;
    oa.g = G;
    oa.ct = oldt;
    oa.counts = g->counts;
    oa.offs = g->offs;
    oa.inj_count = g->inj_count;
    oa.inj_off = g->inj_off;
    oa.tile_count = g->tile_count;
    k_tile_offsets<<<(unsigned)((G.NT + 4 * OFF_TPW - 1) / (4 * OFF_TPW)), 256, 0, g->s>>>(oa);
    scan_tiles(g, newt);
    k_build_chunks<<<nblk(G.NT, 128), 128, 0, g->s>>>(G.NT, g->tile_base, g->tile_count, newt,
                                                       g->max_chunks);
    ScatArgs<T> sc;
    sc.g = G;
    sc.ct = oldt;
    sc.code = g->code;
    sc.offs = g->offs;
    sc.tile_base = g->tile_base;
    sc.capacity = g->capacity;
    sc.err = g->err_dev;
    if (G.dims == 3)
      k_scatter<T, 3><<<g->max_chunks, 256, 0, g->s>>>(sc, parts(g, A), parts(g, B));
    else
      k_scatter<T, 2><<<g->max_chunks, 256, 0, g->s>>>(sc, parts(g, A), parts(g, B));
    if (g->cfg.n_e > 0.0) {
      InjCopyArgs ca;
      ca.g = G;
      ca.inj_count = g->inj_count;
      ca.inj_off = g->inj_off;
      ca.tile_base = g->tile_base;
      ca.stage_per_tile = g->stage_per_tile;
      ca.stage_g = g->stage_g;
      ca.grank = g->grank;
      ca.next_id = g->next_id;
      ca.capacity = g->capacity;
      ca.err = g->err_dev;
      if (G.dims == 3)
        k_inject_copy<T, 3><<<G.nTx * G.nTy, 256, 0, g->s>>>(ca, staging(g), parts(g, B));
      else
        k_inject_copy<T, 2><<<G.nTx * G.nTy, 256, 0, g->s>>>(ca, staging(g), parts(g, B));
      if (g->ids[0]) {
        int64_t ng = nm * G.Ny * G.Nx * g->ppcx * g->ppcy;
        // next_id += number of selected candidates (a scan of the flags adds the total)
        k_scan_flags<<<1, 1024, 0, g->s>>>(ng, g->gflag, g->grank, g->next_id);
      }
    }
    g->cur = B;
    g->ctc = 1 - g->ctc;
    return GEMPIC_OK;
  }

  static PushArgs<T> push_args(gempic* g) {
    const Geom& G = g->g;
    PushArgs<T> a;
    a.g = G;
    a.F6 = (const T*)g->F6;
    for (int q = 0; q < 3; ++q) a.J[q] = (T*)g->J[q];
    for (int q = 0; q < 3; ++q) a.Jfix[q] = (unsigned long long*)g->Jfix[q];
    a.rho0 = g->cfg.deposit_rho ? (T*)g->rho[0] : nullptr;
    a.rho1 = g->cfg.deposit_rho ? (T*)g->rho[1] : nullptr;
    double q = -1.0;
    double dtau = G.dtau;
    a.eps = (T)(0.5 * q * dtau);
    a.ax = (T)(dtau / G.hx);
    a.ay = (T)(dtau / G.hy);
    a.az = (T)(dtau / G.h);
    double qw = G.qw;
    if (G.dims == 3) {
      a.cx = (T)(-qw / (dtau * G.hy * G.h));
      a.cy = (T)(-qw / (dtau * G.hx * G.h));
      a.cz = (T)(-qw / (dtau * G.hx * G.hy));
      a.cjy = (T)0;
    } else {
      a.cx = (T)(-qw / (dtau * G.h));
      a.cy = (T)0;
      a.cz = (T)(-qw / (dtau * G.hx));
      a.cjy = (T)(qw / (G.hx * G.h));
    }
    a.crho = (T)(qw / G.V);
    // FP32 fixed-point scale: every single contribution is bounded by
    // max(|cx|, |cy|, |cz| + |crho|, |cjy|) and is converted through int32
    // below 2^30; a node receives at most one contribution per particle, so
    // the 64-bit sums hold 2^33 particles.  FP64 accumulates in FP64 (scale 1).
    double cmax = std::max(std::max(std::fabs((double)a.cx), std::fabs((double)a.cy)),
                           std::max(std::fabs((double)a.cz) + std::fabs((double)a.crho),
                                    std::fabs((double)a.cjy)));
    cmax = std::max(cmax, std::fabs((double)a.crho));
    // driver-beam particles carry rb times the plasma weight
    a.rb = (T)(g->wb > 0 ? g->wb / g->w : 1.0);
    a.dtau = (T)G.dtau;
    if (g->wb > 0) cmax *= std::max(1.0, g->wb / g->w);
    double sc = cmax > 0 ? std::ldexp(1.0, 30) / (cmax * 1.01) : 1.0;
    int e2 = sizeof(T) == 4 ? (int)std::floor(std::log2(sc)) : 0;
    a.fscale = (T)std::ldexp(1.0, e2);
    a.finv = (T)std::ldexp(1.0, -e2);
    a.tile_base = g->tile_base;
    a.tile_count = g->tile_count;
    a.total = g->total;
    // zeta segments: enough work-groups to fill the chip several times over,
    // segments long enough that most current planes are carried, not flushed,
    // and short enough (at most 32 tiles) that the last work-groups leave no
    // long tail; with a driver beam, whose tiles hold up to ~1e5 particles each,
    // 4 tiles, so that one work-group does not walk all of them in turn
    int ncol = G.nTx * G.nTy;
    const int seg_target = g->cfg.beam_np > 0 ? 4 : 32;
    int nseg = std::max((G.nTz + seg_target - 1) / seg_target, (8192 + ncol - 1) / ncol);
    nseg = std::min(G.nTz, std::max(1, nseg));
    a.seg_len = (G.nTz + nseg - 1) / nseg;
    a.nseg = (G.nTz + a.seg_len - 1) / a.seg_len;
    a.err = g->err_dev;
    return a;
  }

  static unsigned push_blocks(const PushArgs<T>& a) {
    int nitem = a.g.nTx * a.g.nTy * a.nseg;
    return (unsigned)(8 * ((nitem + 7) / 8));
  }

  static size_t colnode_lds(const Geom& G) {
    return (12 * (size_t)(G.Ny + FFTY_PAD) + (size_t)G.Ny) * sizeof(C);
  }

  static void set_lds_limits() {
    int lim = 160 * 1024;
    (void)hipFuncSetAttribute((const void*)k_mz_colnode<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_fft_x_r2c<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_fft_x_c2r6<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_fft_y<T>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  }

  // work-group size: the register budget (about 96 VGPRs) allows five waves
  // per SIMD, so small tiles (whose LDS footprint allows five work-groups per
  // CU) run one wave per SIMD per work-group
  template <int DIM, int TX, int TY, int TZ>
  static void push_tile(gempic* g, const PushArgs<T>& a, PartPtrs<T> P, bool rho) {
    unsigned nb = push_blocks(a);
    constexpr int NTHR = TZ == 8 ? 512 : 256;
    if constexpr (std::is_same<T, float>::value) {
      if (g->det) {   // no driver beam (rejected when the mode is set)
        constexpr bool A3 = DIM == 3;   // absolute positions: 3-D only
        if (A3 && g->g.abs_pos) {
          if (rho) k_push_deposit<T, DIM, true, TX, TY, TZ, NTHR, false, A3, true><<<nb, NTHR, 0, g->s>>>(a, P);
          else k_push_deposit<T, DIM, false, TX, TY, TZ, NTHR, false, A3, true><<<nb, NTHR, 0, g->s>>>(a, P);
        } else {
          if (rho) k_push_deposit<T, DIM, true, TX, TY, TZ, NTHR, false, false, true><<<nb, NTHR, 0, g->s>>>(a, P);
          else k_push_deposit<T, DIM, false, TX, TY, TZ, NTHR, false, false, true><<<nb, NTHR, 0, g->s>>>(a, P);
        }
        return;
      }
    }
    if constexpr (DIM == 3) {
      if (g->cfg.beam_np > 0) {
        if (rho) k_push_deposit<T, DIM, true, TX, TY, TZ, NTHR, true, false><<<nb, NTHR, 0, g->s>>>(a, P);
        else k_push_deposit<T, DIM, false, TX, TY, TZ, NTHR, true, false><<<nb, NTHR, 0, g->s>>>(a, P);
        return;
      }
      if constexpr (std::is_same<T, float>::value) {
        if (g->g.abs_pos) {
          if (rho) k_push_deposit<T, DIM, true, TX, TY, TZ, NTHR, false, true><<<nb, NTHR, 0, g->s>>>(a, P);
          else k_push_deposit<T, DIM, false, TX, TY, TZ, NTHR, false, true><<<nb, NTHR, 0, g->s>>>(a, P);
          return;
        }
      }
    }
    if (rho) k_push_deposit<T, DIM, true, TX, TY, TZ, NTHR, false, false><<<nb, NTHR, 0, g->s>>>(a, P);
    else k_push_deposit<T, DIM, false, TX, TY, TZ, NTHR, false, false><<<nb, NTHR, 0, g->s>>>(a, P);
  }

  static void launch_push(gempic* g) {
    const Geom& G = g->g;
    bool rho = g->cfg.deposit_rho != 0;
    PushArgs<T> a = push_args(g);
    PartPtrs<T> P = parts(g, g->cur);
    if (G.dims == 3) {
      if (G.Tx == 8 && G.Tz == 8) push_tile<3, 8, 8, 8>(g, a, P, rho);
      else if (G.Tx == 8) push_tile<3, 8, 8, 4>(g, a, P, rho);
      else push_tile<3, 4, 4, 4>(g, a, P, rho);
    } else {
      if (G.Tx == 8 && G.Tz == 8) push_tile<2, 8, 1, 8>(g, a, P, rho);
      else if (G.Tx == 8) push_tile<2, 8, 1, 4>(g, a, P, rho);
      else push_tile<2, 4, 1, 4>(g, a, P, rho);
    }
  }

  static int mark(gempic* g, int k) {
    if (!g->timing) return GEMPIC_OK;
    size_t i = (size_t)g->tsteps * 5 + k;
    while (g->ev.size() <= i) {
      hipEvent_t e;
      HIPCHK(g, hipEventCreate(&e));
      g->ev.push_back(e);
    }
    HIPCHK(g, hipEventRecord(g->ev[i], g->s));
    return GEMPIC_OK;
  }

  static int one_step(gempic* g) {
    const Geom& G = g->g;
    int64_t nJ = (int64_t)G.NPJ * G.Ny * G.Nx;
    int rc = mark(g, 0);
    if (rc) return rc;
    Range range("gempic.clear");
    if (g->det) {
      // the conversion below writes every node of J
      for (int q = 0; q < 3; ++q)
        k_fill<int64_t><<<nblk(nJ, 256), 256, 0, g->s>>>((int64_t*)g->Jfix[q], nJ, 0);
    } else {
      for (int q = 0; q < 3; ++q) fill(g, g->J[q], nJ);
    }
    if (g->cfg.deposit_rho) { fill(g, g->rho[0], nJ); fill(g, g->rho[1], nJ); }
    if ((rc = launch_check(g, "clearing the current"))) return rc;
    if ((rc = mark(g, 1))) return rc;
    range.next("gempic.push_deposit");
    launch_push(g);
    if constexpr (std::is_same<T, float>::value) {
      if (g->det) {
        const PushArgs<T> a = push_args(g);
        for (int q = 0; q < 3; ++q)
          k_fix_to_float<<<nblk(nJ, 256), 256, 0, g->s>>>((const unsigned long long*)g->Jfix[q], (float*)g->J[q],
                                                          nJ, a.finv);
      }
    }
    if ((rc = launch_check(g, "push and deposit"))) return rc;
    if ((rc = mark(g, 2))) return rc;
    range.next("gempic.sort_window");
    (void)hipMemcpyAsync(g->pushed, g->total, 8, hipMemcpyDeviceToDevice, g->s);
    rc = sort_and_inject(g, g->step + 1);
    if (rc) return rc;
    if ((rc = launch_check(g, "sort and window"))) return rc;
    if ((rc = mark(g, 3))) return rc;
    if (g->dn) {
      range.next("gempic.denoise");
      if (sizeof(T) != 4) return fail(g, GEMPIC_EINVAL, "denoiser needs FP32");
      const double hs[3] = {G.hx, G.hy, G.h};
      const float* J[3] = {(const float*)g->J[0], (const float*)g->J[1], (const float*)g->J[2]};
      float* Jf[3] = {(float*)g->Jf[0], (float*)g->Jf[1], (float*)g->Jf[2]};
      float* Jd[3] = {(float*)g->Jd[0], (float*)g->Jd[1], (float*)g->Jd[2]};
      float* Jt[3] = {(float*)g->Jt[0], (float*)g->Jt[1], (float*)g->Jt[2]};
      rc = dn_step(g->dn, g->s, G.NPJ, G.Ny, G.Nx, J, Jf, Jd, Jt, g->cfg.n_e, hs, G.P, g->dn_thr,
                   g->dn_fallbacks, g->dn_rel);
      if (rc) return fail(g, rc, std::string("denoiser: ") + dn_error(g->dn));
    }
    range.next("gempic.fields");
    field_update(g, true, (T)G.dtau);
    if ((rc = launch_check(g, "field update"))) return rc;
    if ((rc = mark(g, 4))) return rc;
    if (g->timing) g->tsteps += 1;
    g->step += 1;
    return GEMPIC_OK;
  }

  // ---- creation: load plasma, batch 0, laser -------------------------------
  static int init_state(gempic* g) {
    const Geom& G = g->g;
    // chunk table of the loaded (full-cell) particles: closed-form tile counts
    std::vector<int64_t> cnt(G.NT, 0), base(G.NT, 0);
    int64_t tot = 0;
    if (g->cfg.n_e > 0.0) {
      for (int t = 0; t < G.NT; ++t) {
        int tz = t / (G.nTx * G.nTy);
        int z0 = tz * G.Tz, zend = std::min(z0 + G.Tz, G.Nzp - 1);
        int64_t n = zend > z0 ? (int64_t)(zend - z0) * g->ppcz * G.Ty * G.Tx * g->ppcx * g->ppcy : 0;
        cnt[t] = n;
        base[t] = tot;
        tot += n;
      }
    }
    // driver beam: sampled on the host, placed behind the plasma particles of
    // its tiles (sample order within a tile)
    HostBeam hb;
    if (g->cfg.beam_np > 0) {
      sample_beam(g, &hb);
      std::vector<int64_t> bcnt(G.NT, 0);
      for (int64_t i = 0; i < hb.n; ++i) bcnt[hb.tile[i]] += 1;
      tot = 0;
      for (int t = 0; t < G.NT; ++t) {
        base[t] = tot;
        tot += cnt[t] + bcnt[t];
      }
      std::vector<int64_t> fill_(G.NT, 0);
      hb.dst.resize(hb.n);
      for (int64_t i = 0; i < hb.n; ++i) {
        int t = hb.tile[i];
        hb.dst[i] = base[t] + cnt[t] + fill_[t]++;
      }
      for (int t = 0; t < G.NT; ++t) cnt[t] += bcnt[t];
    }
    if (tot > g->capacity) return fail(g, GEMPIC_EINVAL, "capacity too small for the initial load");
    HIPCHK(g, hipMemcpyAsync(g->tile_count, cnt.data(), G.NT * 8, hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->tile_base, base.data(), G.NT * 8, hipMemcpyHostToDevice, g->s));
    if (tot > 0) {
      LoadArgs la;
      la.g = G;
      la.ppcx = g->ppcx; la.ppcy = g->ppcy; la.ppcz = g->ppcz;
      la.quiet = g->quiet;
      la.key = g->key;
      la.tile_base = g->tile_base;
      k_load_full<T><<<G.NT, 256, 0, g->s>>>(la, parts(g, g->cur));
    }
    BeamArgs ba{};
    if (hb.n > 0) {
      int64_t n = hb.n;
      ba.n = n;
      int32_t* dc = (int32_t*)g->dev.alloc(n * 4);
      double* doff = (double*)g->dev.alloc(3 * n * 8);
      double* duz = (double*)g->dev.alloc(n * 8);
      int64_t* ddst = (int64_t*)g->dev.alloc(n * 8);
      if (!dc || !doff || !duz || !ddst) return fail(g, GEMPIC_ENOMEM, "beam staging buffers");
      HIPCHK(g, hipMemcpyAsync(dc, hb.cell.data(), n * 4, hipMemcpyHostToDevice, g->s));
      HIPCHK(g, hipMemcpyAsync(doff, hb.off.data(), 3 * n * 8, hipMemcpyHostToDevice, g->s));
      HIPCHK(g, hipMemcpyAsync(duz, hb.uz.data(), n * 8, hipMemcpyHostToDevice, g->s));
      HIPCHK(g, hipMemcpyAsync(ddst, hb.dst.data(), n * 8, hipMemcpyHostToDevice, g->s));
      ba.cell = dc;
      ba.off = doff;
      ba.uz = duz;
      ba.dst = ddst;
      ba.id0 = tot - n;
      k_place_beam<T><<<nblk(n, 256), 256, 0, g->s>>>(ba, parts(g, g->cur), G.dims);
      g->nbeam = n;
    }
    ChunkTab& t0 = g->ct[g->ctc];
    scan_tiles(g, t0);
    k_build_chunks<<<nblk(G.NT, 128), 128, 0, g->s>>>(G.NT, g->tile_base, g->tile_count, t0,
                                                       g->max_chunks);
    if (g->ids[0]) HIPCHK(g, hipMemcpyAsync(g->next_id, &tot, 8, hipMemcpyHostToDevice, g->s));
    int rc = sort_and_inject(g, 0);
    if (rc) return rc;

    // laser: R_pol = 2 E_pol on the field nodes, then a march with Delta = 0
    int64_t nxy = (int64_t)G.Ny * G.Nx;
    int64_t nsp = (int64_t)G.Nz * G.Ny * G.Nxh;
    for (int q = 0; q < 4; ++q) fill(g, g->st[q], 2 * nsp);
    if (g->cfg.a0 != 0.0) {
      std::vector<double> lon(G.Nz), tra(nxy);
      for (int n = 0; n < G.Nz; ++n) {
        double zeta = (double)n * G.h;
        double phi = zeta - g->zeta_c;
        lon[n] = g->cfg.a0 * std::cos(phi) * std::exp(-(phi * phi) / (g->Tlas * g->Tlas));
      }
      for (int j = 0; j < G.Ny; ++j)
        for (int i = 0; i < G.Nx; ++i) {
          double X = (double)i * G.hx - (double)(G.Nx / 2) * G.hx;
          double Y = G.dims == 3 ? (double)j * G.hy - (double)(G.Ny / 2) * G.hy : 0.0;
          tra[(int64_t)j * G.Nx + i] = g->waist > 0.0 ? std::exp(-(X * X + Y * Y) / (g->waist * g->waist)) : 1.0;
        }
      double* dl = (double*)g->dev.alloc(lon.size() * 8);
      double* dt = (double*)g->dev.alloc(tra.size() * 8);
      if (!dl || !dt) return fail(g, GEMPIC_ENOMEM, "laser buffers");
      HIPCHK(g, hipMemcpyAsync(dl, lon.data(), lon.size() * 8, hipMemcpyHostToDevice, g->s));
      HIPCHK(g, hipMemcpyAsync(dt, tra.data(), tra.size() * 8, hipMemcpyHostToDevice, g->s));
      k_laser<T><<<nblk((int64_t)G.Nz * nxy, 256), 256, 0, g->s>>>((T*)g->J[0], dl, dt, G.Nz, nxy);
      fft_fwd(g, (const T*)g->J[0], (C*)g->st[g->cfg.pol == 0 ? 0 : 1], G.Nz);
    }
    if (hb.n > 0) {
      // the bunch's own field: charge on the nodes, transverse Poisson solve
      // per zeta node, R_perp += 2 E_perp
      int64_t nf = (int64_t)G.Nz * nxy;
      fill(g, g->J[1], nf);
      k_beam_rho<T><<<nblk(hb.n, 256), 256, 0, g->s>>>(ba, G, -g->wb / G.V, (T*)g->J[1]);
      fft_fwd(g, (const T*)g->J[1], (C*)g->outs[0], G.Nz);
      k_beam_R<T><<<nblk(nsp, 256), 256, 0, g->s>>>((const C*)g->outs[0], (C*)g->st[0], (C*)g->st[1], G.Nz,
                                                     G.Ny, G.Nxh, G.hx, G.hy, G.P);
      // its current J_z = rhobar enters the consistency march
      int64_t nJ = (int64_t)G.NPJ * nxy;
      fill(g, g->J[0], nJ);
      fill(g, g->J[2], nJ);
      k_beam_jz<T><<<nblk((int64_t)(G.Nz + 1) * nxy, 256), 256, 0, g->s>>>((const T*)g->J[1], (T*)g->J[2],
                                                                           G.Nz, nxy);
      fill(g, g->J[1], nJ);
      HIPCHK(g, hipStreamSynchronize(g->s));
      for (void* p : {(void*)ba.cell, (void*)ba.off, (void*)ba.uz, (void*)ba.dst}) g->dev.free(p);
    }
    field_update(g, hb.n > 0, (T)0);
    int64_t nJ = (int64_t)G.NPJ * nxy;
    for (int q = 0; q < 3; ++q) fill(g, g->J[q], nJ);
    if (g->cfg.deposit_rho) { fill(g, g->rho[0], nJ); fill(g, g->rho[1], nJ); }
    int rc2 = launch_check(g, "initial state");
    if (rc2) return rc2;
    HIPCHK(g, hipStreamSynchronize(g->s));
    return GEMPIC_OK;
  }

  // ---- zeta march ----------------------------------------------------------
  static MzParts<T> mzp(gempic* g, int k) {
    MzParts<T> P;
    P.cell = (int32_t*)g->mz_part[k][0];
    P.ox = (T*)g->mz_part[k][1];
    P.oy = (T*)g->mz_part[k][2];
    P.oz = (T*)g->mz_part[k][3];
    P.ux = (T*)g->mz_part[k][4];
    P.uy = (T*)g->mz_part[k][5];
    P.uz = (T*)g->mz_part[k][6];
    P.w = (T*)g->mz_part[k][7];
    P.b = (T*)g->mz_part[k][8];
    P.id = (int64_t*)g->mz_part[k][9];
    return P;
  }
  enum { MZ_PARK = 0, MZ_STOP = 1, MZ_ACT = 2 };
  enum { C_ACT = 0, C_STOP = 2, C_LEFT = 3, C_PARK = 4 };

  // stopped particles -> parked store sorted by zeta cell
  static void mz_sort(gempic* g) {
    const Geom& G = g->g;
    const int nxy = G.Nx * G.Ny;
    k_fill<int32_t><<<nblk(G.Nz, 256), 256, 0, g->s>>>(g->mz_pcount, G.Nz, 0);
    k_mz_count<<<256, 256, 0, g->s>>>((const int32_t*)g->mz_part[MZ_STOP][0], g->mz_cnt + C_STOP, g->mz_cap,
                                       nxy, g->mz_pcount);
    k_mz_scan<<<1, 1024, 0, g->s>>>(g->mz_pcount, G.Nz, g->mz_pstart, g->mz_cursor, g->mz_cnt + C_PARK);
    k_mz_scatter<T><<<256, 256, 0, g->s>>>(mzp(g, MZ_STOP), g->mz_cnt + C_STOP, g->mz_cap, nxy, g->mz_cursor,
                                            mzp(g, MZ_PARK));
  }

  static MzBatchArgs mz_batch_args(gempic* g, int64_t row, double zeta_abs, double b0, int base, int64_t id0) {
    const Geom& G = g->g;
    MzBatchArgs ba;
    ba.g = G;
    ba.ppcx = g->ppcx;
    ba.ppcy = g->ppcy;
    ba.quiet = g->quiet;
    ba.key = sm_mix(g->cfg.seed ^ (2ull << 56));
    ba.row = row;
    // cell n with zeta_n < zeta <= zeta_{n+1}, offset in (0, 1]
    int n = (int)(std::lower_bound(g->zn.begin(), g->zn.end(), zeta_abs) - g->zn.begin()) - 1;
    n = std::max(0, std::min(n, G.Nz - 1));
    ba.iz = n;
    ba.oz = (zeta_abs - g->zn[n]) / (g->zn[n + 1] - g->zn[n]);
    ba.n_e = g->cfg.n_e;
    ba.ratio = g->cfg.ch_ratio;
    ba.R = g->cfg.ch_radius * g->cfg.length_unit;
    ba.Delta = g->Delta;
    ba.b0 = b0;
    ba.base = base;
    ba.id0 = id0;
    ba.capacity = g->mz_cap;
    ba.err = g->err_dev;
    return ba;
  }

  static MzNodeArgs<T> mz_node_args(gempic* g, int n, T D) {
    const Geom& G = g->g;
    MzNodeArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.g = G;
    a.n = n;
    a.h = (T)(g->zn[n + 1] - g->zn[n]);
    a.D = D;
    a.first = g->mz_first;
    for (int q = 0; q < 2; ++q) a.j0[q] = (C*)g->mz_j0[q];
    for (int q = 0; q < 4; ++q) a.st[q] = (C*)g->st[q];
    a.L[0] = (C*)g->Lsp[0];
    a.L[1] = (C*)g->Lsp[1];
    return a;
  }

  // creation: laser (Sec. 6, eq. E_laser) on the nodes zeta_n as a forward
  // wave, the consistency march with Delta = 0 node by node, real fields,
  // and (GT1, Delta < L) the batches already in the box
  static int mz_init(gempic* g) {
    const Geom& G = g->g;
    int64_t nxy = (int64_t)G.Ny * G.Nx;
    int64_t M = (int64_t)G.Ny * G.Nxh;
    int64_t nsp = (int64_t)G.Nz * M;
    for (int q = 0; q < 4; ++q) fill(g, g->st[q], 2 * nsp);
    for (int q = 0; q < 2; ++q) fill(g, g->Lsp[q], 2 * nsp);
    for (int q = 0; q < 2; ++q) fill(g, g->mz_j0[q], 2 * (nsp + M));
    fill(g, g->mz_dep, 3 * nxy);
    if (g->cfg.a0 != 0.0) {
      std::vector<double> lon(G.Nz), tra(nxy);
      for (int n = 0; n < G.Nz; ++n) {
        double phi = g->zn[n] - g->zeta_c;
        lon[n] = g->cfg.a0 * std::cos(phi) * std::exp(-(phi * phi) / (g->Tlas * g->Tlas));
      }
      for (int j = 0; j < G.Ny; ++j)
        for (int i = 0; i < G.Nx; ++i) {
          double X = (double)i * G.hx - (double)(G.Nx / 2) * G.hx;
          double Y = G.dims == 3 ? (double)j * G.hy - (double)(G.Ny / 2) * G.hy : 0.0;
          tra[(int64_t)j * G.Nx + i] = g->waist > 0.0 ? std::exp(-(X * X + Y * Y) / (g->waist * g->waist)) : 1.0;
        }
      double* dl = (double*)g->dev.alloc(lon.size() * 8);
      double* dt = (double*)g->dev.alloc(tra.size() * 8);
      if (!dl || !dt) return fail(g, GEMPIC_ENOMEM, "laser buffers");
      HIPCHK(g, hipMemcpyAsync(dl, lon.data(), lon.size() * 8, hipMemcpyHostToDevice, g->s));
      HIPCHK(g, hipMemcpyAsync(dt, tra.data(), tra.size() * 8, hipMemcpyHostToDevice, g->s));
      k_laser<T><<<nblk((int64_t)G.Nz * nxy, 256), 256, 0, g->s>>>((T*)g->J[0], dl, dt, G.Nz, nxy);
      fft_fwd(g, (const T*)g->J[0], (C*)g->st[g->cfg.pol == 0 ? 0 : 1], G.Nz);
      HIPCHK(g, hipStreamSynchronize(g->s));
      g->dev.free(dl);
      g->dev.free(dt);
      fill(g, g->J[0], (int64_t)G.NPJ * nxy);
    }
    g->mz_first = 1;
    for (int n = G.Nz - 1; n >= 0; --n) {
      MzNodeArgs<T> a = mz_node_args(g, n, (T)0);
      for (int q = 0; q < 6; ++q) a.out[q] = (C*)g->outs[q] + (int64_t)n * M;
      k_mz_node<T><<<nblk(M, 256), 256, 0, g->s>>>(a);
    }
    fft_inv6(g);
    // particles already in the box (GT1): batches at L - m Delta, budget 0
    k_fill<int32_t><<<1, 64, 0, g->s>>>(g->mz_cnt, 8, 0);
    const double L = g->zn[G.Nz];
    int64_t nb = 0;
    if (g->cfg.n_e > 0.0 && g->scheme == 1) {
      for (int64_t m = 1; L - (double)m * g->Delta > 0.0; ++m) {
        MzBatchArgs ba = mz_batch_args(g, -m, L - (double)m * g->Delta, 0.0, (int)((m - 1) * g->nperp),
                                       (m - 1) * g->nperp);
        k_mz_batch<T><<<nblk(g->nperp, 256), 256, 0, g->s>>>(ba, mzp(g, MZ_STOP));
        nb = m;
      }
    }
    g->mz_batches = nb;
    int cnt = (int)(nb * g->nperp);
    HIPCHK(g, hipMemcpyAsync(g->mz_cnt + C_STOP, &cnt, sizeof(int), hipMemcpyHostToDevice, g->s));
    mz_sort(g);
    int rc = launch_check(g, "zeta-march initial state");
    if (rc) return rc;
    // GT2: the plasma's current of the level of creation (j^0 of the first
    // step) from the startup march (plasma at rest streams through the box
    // at fixed s~); GT1's first step uses j^1 for both levels (mz_first)
    if (g->cfg.n_e > 0.0 && g->scheme == 2 && (rc = mz_step(g, true))) return rc;
    HIPCHK(g, hipStreamSynchronize(g->s));
    return GEMPIC_OK;
  }

  template <int DIM>
  static void mz_stage(gempic* g, int n, T D, bool pred) {
    const Geom& G = g->g;
    MzStageArgs<T> a;
    a.g = G;
    a.n = n;
    a.hn = (T)(g->zn[n + 1] - g->zn[n]);
    a.hx = (T)G.hx;
    a.hy = (T)(G.dims == 3 ? G.hy : 1.0);
    a.D = D;
    a.ds_perp = (T)(0.5 * (G.dims == 3 ? std::min(G.hx, G.hy) : G.hx));
    a.scheme = g->scheme;
    a.pred = pred ? 1 : 0;
    a.cap = g->mz_subcap;
    a.capacity = g->mz_cap;
    // node n: the old level in the predictor, the predicted new level in the
    // corrector (without plasma there is no predictor and no particle)
    a.F0 = (const T*)(pred || g->nperp == 0 ? g->F6 : g->F6b);
    a.F1 = (const T*)g->F6b;
    a.dep = (T*)g->mz_dep;
    a.in = mzp(g, MZ_ACT + (n & 1));
    a.in_count = g->mz_cnt + C_ACT + (n & 1);
    a.park = mzp(g, MZ_PARK);
    a.pstart = g->mz_pstart;
    a.pcount = g->mz_pcount;
    a.out = mzp(g, MZ_ACT + ((n + 1) & 1));
    a.out_count = g->mz_cnt + C_ACT + ((n + 1) & 1);
    a.stop = mzp(g, MZ_STOP);
    a.stop_count = g->mz_cnt + C_STOP;
    a.left_count = g->mz_cnt + C_LEFT;
    a.err = g->err_dev;
    k_mz_stage<T, DIM><<<g->mz_stage_blocks, 256, 0, g->s>>>(a);
  }

  // one slow step of the zeta march; startup (GT2, at creation): the
  // startup march that gives the plasma's current of the level of creation
  // (j^0 of the first step) and the fields with its response -- node solves
  // of zero slow step, one fresh batch pushed through and discarded, nothing
  // advanced
  static int mz_step(gempic* g, bool startup = false) {
    Range range(startup ? "gempic.zeta_march_startup" : "gempic.zeta_march_step");
    const Geom& G = g->g;
    const int Nz = G.Nz;
    const int64_t M = (int64_t)G.Ny * G.Nxh;
    const int64_t nxy = (int64_t)G.Ny * G.Nx;
    const T D = (T)g->Delta;
    const T Dn = startup ? (T)0 : D;          // slow step of the node solves
    int rc = mark(g, 0);
    if (rc) return rc;
    const int fresh = g->cfg.n_e > 0.0 ? (int)g->nperp : 0;
    k_mz_begin<T><<<256, 256, 0, g->s>>>(mzp(g, MZ_PARK), g->mz_cnt + C_PARK, g->mz_cap, D,
                                          g->mz_cnt + C_ACT + ((Nz - 1) & 1), fresh,
                                          g->mz_cnt + C_ACT + (Nz & 1), g->mz_cnt + C_STOP, g->mz_cnt + C_LEFT);
    if (fresh) {
      MzBatchArgs ba = mz_batch_args(g, g->step, g->zn[Nz], g->Delta, 0,
                                     (g->mz_batches + g->step) * g->nperp);
      k_mz_batch<T><<<nblk(g->nperp, 256), 256, 0, g->s>>>(ba, mzp(g, MZ_ACT + ((Nz - 1) & 1)));
    }
    if ((rc = launch_check(g, "zeta-march step start"))) return rc;
    if ((rc = mark(g, 1))) return rc;
    C* out6[6];
    const C* in6[6];
    for (int q = 0; q < 6; ++q) {
      out6[q] = (C*)g->mz_out6 + q * M;
      in6[q] = out6[q];
    }
    // predictor-corrector stages: with plasma, each stage first pushes and
    // deposits with node n at the old level and solves node n (records
    // only), then pushes again with that node and solves for good
    const int passes = g->nperp > 0 ? 2 : 1;
    for (int n = Nz - 1; n >= 0; --n) {
      for (int pass = 2 - passes; pass < 2; ++pass) {
        const bool pred = pass == 0;
        if (G.dims == 3) mz_stage<3>(g, n, D, pred);
        else mz_stage<2>(g, n, D, pred);
        MzNodeArgs<T> a = mz_node_args(g, n, Dn);
        a.jhat = (const C*)g->mz_jhat;
        for (int q = 0; q < 6; ++q) a.out[q] = out6[q];
        a.dep = (T*)g->mz_dep;
        a.pred = pred ? 1 : 0;
        if (!pred) {
          for (int q = 0; q < 3; ++q) a.jrec[q] = (T*)g->J[q] + (int64_t)(n + 2) * nxy;
          a.zero_count = g->mz_cnt + C_ACT + (n & 1);
        }
        if (G.Ny > 1 && G.Ny != 256 && G.Ny != 512) {
          // x transform of the deposit, then one work-group per kx column:
          // y transform, node solve and inverse y transforms in LDS (where
          // no four-step y transform exists; with one, its coalesced
          // launches are faster than a work-group per column)
          fft_xfwd(g, (const T*)g->mz_dep, (C*)g->mz_jhat, 3);
          k_mz_colnode<T><<<(unsigned)G.Nxh, 256, colnode_lds(G), g->s>>>(a, (const C*)g->mz_jhat,
                                                                           (const C*)g->twy);
        } else {
          fft_fwd(g, (const T*)g->mz_dep, (C*)g->mz_jhat, 3);
          k_mz_node<T><<<nblk(std::max<int64_t>(M, 3 * nxy / 8), 256), 256, 0, g->s>>>(a);
          if (G.Ny > 1) fft_y(g, out6[0], 6, 1);
        }
        c2r6(g, in6, (T*)g->F6b + (int64_t)n * nxy * 6, G.Ny);
      }
    }
    if ((rc = launch_check(g, "zeta-march stages"))) return rc;
    if (startup) {
      // the batch's particles are dropped: the next step's k_mz_begin resets
      // the active, stopped and left counters, and no parked store changed
      std::swap(g->F6, g->F6b);
      g->mz_first = 0;
      return GEMPIC_OK;
    }
    if ((rc = mark(g, 2))) return rc;
    mz_sort(g);
    std::swap(g->F6, g->F6b);
    g->mz_first = 0;
    g->s_total += g->Delta;
    if ((rc = launch_check(g, "zeta-march parking"))) return rc;
    if ((rc = mark(g, 3))) return rc;
    if ((rc = mark(g, 4))) return rc;
    if (g->timing) g->tsteps += 1;
    g->step += 1;
    return GEMPIC_OK;
  }

  static int mz_diag(gempic* g, gempic_diag* d) {
    const Geom& G = g->g;
    int cnt[5] = {0, 0, 0, 0, 0};
    HIPCHK(g, hipMemcpyAsync(cnt, g->mz_cnt, sizeof(cnt), hipMemcpyDeviceToHost, g->s));
    k_mz_wsum<T><<<DIAG_BLOCKS, 256, 0, g->s>>>((const T*)g->mz_part[MZ_PARK][7], g->mz_cnt + C_PARK,
                                                 g->partial);
    k_final<<<1, 256, 0, g->s>>>(g->partial, DIAG_BLOCKS, 1, g->dres + 1);
    k_mz_energy<T><<<DIAG_BLOCKS, 256, 0, g->s>>>((const T*)g->F6, g->mz_hnode, G.Nz, (int64_t)G.Ny * G.Nx,
                                                  g->partial + 2 * DIAG_BLOCKS);
    k_final<<<1, 256, 0, g->s>>>(g->partial + 2 * DIAG_BLOCKS, DIAG_BLOCKS, 1, g->dres);
    double res[2] = {0, 0};
    HIPCHK(g, hipMemcpyAsync(res, g->dres, 16, hipMemcpyDeviceToHost, g->s));
    HIPCHK(g, hipStreamSynchronize(g->s));
    d->tau = g->s_total;
    d->step = g->step;
    d->n_particles = cnt[C_PARK];
    d->field_energy = 0.5 * res[0] * G.hx * (G.dims == 3 ? G.hy : 1.0);
    d->charge_particles = -1.0 * res[1];
    d->charge_grid = 0.0;
    d->continuity_rel = 0.0;
    d->fallbacks = 0;
    d->denoise_rel = 0.0;
    return GEMPIC_OK;
  }

  static int bunch(gempic* g, double gamma_min, gempic_bunch* out) {
    const Geom& G = g->g;
    BunchArgs<T> a;
    a.g = G;
    a.gamma_min = gamma_min;
    a.partial = g->partial;
    if (g->scheme) {
      MzParts<T> P = mzp(g, MZ_PARK);
      a.count32 = g->mz_cnt + C_PARK;
      a.count64 = nullptr;
      a.capacity = g->mz_cap;
      a.cell = P.cell; a.ox = P.ox; a.oy = P.oy; a.oz = P.oz; a.ux = P.ux; a.uy = P.uy; a.uz = P.uz;
      a.w = P.w;
      a.w_plasma = a.w_beam = 0.0;
      a.zn = g->mz_zn;
    } else {
      PartPtrs<T> P = parts(g, g->cur);
      a.count32 = nullptr;
      a.count64 = g->total;
      a.capacity = (int)g->capacity;
      a.cell = P.cell; a.ox = P.ox; a.oy = P.oy; a.oz = P.oz; a.ux = P.ux; a.uy = P.uy; a.uz = P.uz;
      a.w = nullptr;
      a.w_plasma = g->w;
      a.w_beam = g->wb > 0 ? g->wb : g->w;
      a.zn = nullptr;
    }
    const int nb = 96;   // 96 * BUNCH_NS partials fit the diagnostics buffer (6 * DIAG_BLOCKS)
    k_bunch<T><<<nb, 256, 0, g->s>>>(a);
    k_final<<<1, 256, 0, g->s>>>(g->partial, nb, BUNCH_NS, g->partial + nb * BUNCH_NS);
    double r[BUNCH_NS];
    HIPCHK(g, hipMemcpyAsync(r, g->partial + nb * BUNCH_NS, sizeof(r), hipMemcpyDeviceToHost, g->s));
    HIPCHK(g, hipStreamSynchronize(g->s));
    std::memset(out, 0, sizeof(*out));
    const double W = r[0];
    out->n_macro = (int64_t)std::llround(r[15]);
    out->charge = -1.0 * W;
    if (!(W > 0)) return GEMPIC_OK;
    auto mean = [&](int k) { return r[k] / W; };
    auto var = [&](int k2, int k1a, int k1b) { return r[k2] / W - mean(k1a) * mean(k1b); };
    out->gamma_mean = mean(1);
    out->gamma_rms = std::sqrt(std::max(var(2, 1, 1), 0.0));
    out->mean[0] = mean(3);
    out->mean[1] = mean(5);
    out->mean[2] = mean(7);
    out->sigma[0] = std::sqrt(std::max(var(4, 3, 3), 0.0));
    out->sigma[1] = std::sqrt(std::max(var(6, 5, 5), 0.0));
    out->sigma[2] = std::sqrt(std::max(var(8, 7, 7), 0.0));
    const double vx = var(4, 3, 3), vux = var(10, 9, 9), cx = var(11, 3, 9);
    const double vy = var(6, 5, 5), vuy = var(13, 12, 12), cy = var(14, 5, 12);
    out->emittance[0] = std::sqrt(std::max(vx * vux - cx * cx, 0.0));
    out->emittance[1] = std::sqrt(std::max(vy * vuy - cy * cy, 0.0));
    return GEMPIC_OK;
  }

  static int diag(gempic* g, gempic_diag* d) {
    const Geom& G = g->g;
    int64_t n = 0, np = 0;
    HIPCHK(g, hipMemcpyAsync(&n, g->total, 8, hipMemcpyDeviceToHost, g->s));
    HIPCHK(g, hipMemcpyAsync(&np, g->pushed, 8, hipMemcpyDeviceToHost, g->s));
    int64_t nf = (int64_t)G.Nz * G.Ny * G.Nx;
    k_partial<T><<<DIAG_BLOCKS, 256, 0, g->s>>>((const T*)g->F6, nullptr, nullptr, nullptr, nullptr,
                                                nullptr, 1, 6 * nf, 1, g->partial);
    k_final<<<1, 256, 0, g->s>>>(g->partial, DIAG_BLOCKS, 1, g->dres);
    double res[4] = {0, 0, 0, 0};
    int64_t nJ = (int64_t)G.NPJ * G.Ny * G.Nx;
    d->fallbacks = 0;
    d->denoise_rel = 0.0;
    if (g->dn_fallbacks) {
      HIPCHK(g, hipMemcpyAsync(&d->fallbacks, g->dn_fallbacks, 8, hipMemcpyDeviceToHost, g->s));
      HIPCHK(g, hipMemcpyAsync(&d->denoise_rel, g->dn_rel, 8, hipMemcpyDeviceToHost, g->s));
    }
    if (g->cfg.deposit_rho) {
      k_partial<T><<<DIAG_BLOCKS, 256, 0, g->s>>>((const T*)g->rho[1], nullptr, nullptr, nullptr, nullptr,
                                                  nullptr, 1, nJ, 0, g->partial + 2 * DIAG_BLOCKS);
      k_final<<<1, 256, 0, g->s>>>(g->partial + 2 * DIAG_BLOCKS, DIAG_BLOCKS, 1, g->dres + 1);
      k_continuity<T><<<DIAG_BLOCKS, 256, 0, g->s>>>(G, (const T*)g->rho[0], (const T*)g->rho[1],
                                                     (const T*)g->J[0], (const T*)g->J[1],
                                                     (const T*)g->J[2], g->partial + 4 * DIAG_BLOCKS);
      k_final<<<1, 256, 0, g->s>>>(g->partial + 4 * DIAG_BLOCKS, DIAG_BLOCKS, 2, g->dres + 2);
    }
    HIPCHK(g, hipMemcpyAsync(res, g->dres, 32, hipMemcpyDeviceToHost, g->s));
    HIPCHK(g, hipStreamSynchronize(g->s));
    d->tau = (double)g->step * G.dtau;
    d->step = g->step;
    d->n_particles = n;
    d->field_energy = 0.5 * res[0] * G.V;
    d->charge_grid = g->cfg.deposit_rho ? res[1] * G.V : 0.0;
    d->continuity_rel = g->cfg.deposit_rho && res[3] > 0 ? std::sqrt(res[2]) / std::sqrt(res[3]) : 0.0;
    d->charge_particles = G.qw * (double)np;
    if (g->bcount) {
      // beam particles counted in the buffer after the step
      unsigned long long nb = 0;
      HIPCHK(g, hipMemsetAsync(g->bcount, 0, 8, g->s));
      k_count_beam<<<256, 256, 0, g->s>>>((const int32_t*)g->part[g->cur][0], g->total, g->bcount);
      HIPCHK(g, hipMemcpyAsync(&nb, g->bcount, 8, hipMemcpyDeviceToHost, g->s));
      HIPCHK(g, hipStreamSynchronize(g->s));
      d->charge_particles = G.qw * (double)(np - (int64_t)nb) - g->wb * (double)nb;
    }
    return GEMPIC_OK;
  }
};

// ---------------------------------------------------------------------------
static int check_errors(gempic* g) {
  int e = 0;
  HIPCHK(g, hipMemcpyAsync(&e, g->err_dev, sizeof(int), hipMemcpyDeviceToHost, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  if (e & ERR_CFL) return fail(g, GEMPIC_ECFL, "a particle crossed more than one cell in a step");
  if (e & ERR_NUMERIC) return fail(g, GEMPIC_ENUMERIC, "non-finite particle momentum");
  if (e & ERR_CAPACITY) return fail(g, GEMPIC_ECAPACITY, "particle buffer capacity exceeded");
  if (e & ERR_TILE) return fail(g, GEMPIC_EDEVICE, "internal: particle outside its tile or chunk too long");
  if (e & ERR_MARCH) return fail(g, GEMPIC_EDEVICE, "internal: a particle exceeded the sub-step bound of a zeta-march stage");
  return GEMPIC_OK;
}

static int validate(const gempic_config* c, Geom* G, std::string* why) {
  if (c->abi_version != GEMPIC_ABI_VERSION) { *why = "abi_version mismatch"; return GEMPIC_EABI; }
  if (c->dims != 2 && c->dims != 3) { *why = "dims must be 2 or 3"; return GEMPIC_EINVAL; }
  if (!(c->length_unit > 0)) { *why = "length_unit must be > 0"; return GEMPIC_EINVAL; }
  if (c->precision != GEMPIC_FP64 && c->precision != GEMPIC_FP32_CELL && c->precision != GEMPIC_FP32_ABS) {
    *why = "unknown precision";
    return GEMPIC_EINVAL;
  }
  if (c->precision == GEMPIC_FP32_ABS && (c->dims != 3 || c->beam_np > 0)) {
    *why = "GEMPIC_FP32_ABS needs dims = 3 and no driver beam";
    return GEMPIC_EINVAL;
  }
  if (c->filter_passes < 0 || c->filter_passes > 2) { *why = "filter_passes must be 0, 1 or 2"; return GEMPIC_EINVAL; }
  if (c->scheme < 0 || c->scheme > 2) { *why = "scheme must be 0 (tau), 1 (GT1 zeta march) or 2 (GT2)"; return GEMPIC_EINVAL; }
  double lu = c->length_unit;
  G->dims = c->dims;
  G->Nx = c->n[0];
  G->Ny = c->dims == 3 ? c->n[1] : 1;
  G->Nz = c->n[2];
  if (!pow2(G->Nx) || !pow2(G->Nz) || !pow2(G->Ny) || G->Nx < 2 || G->Nz < 2 || (c->dims == 3 && G->Ny < 2)) {
    *why = "grid sizes must be powers of two (>= 2)";
    return GEMPIC_EINVAL;
  }
  G->Tx = c->tile[0];
  G->Ty = c->dims == 3 ? c->tile[1] : 1;
  G->Tz = c->tile[2];
  bool tile_ok = (c->dims == 2 || G->Ty == G->Tx) &&
                 ((G->Tx == 8 && (G->Tz == 8 || G->Tz == 4)) || (G->Tx == 4 && G->Tz == 4));
  if (!tile_ok || G->Nx % G->Tx || G->Ny % G->Ty || G->Nz % G->Tz) {
    *why = "tile must be 8x8x8, 8x8x4 or 4x4x4 (2-D: 8x1x8, 8x1x4 or 4x1x4) and divide the grid";
    return GEMPIC_EINVAL;
  }
  G->lnx = 0; while ((1 << G->lnx) < G->Nx) ++G->lnx;
  G->lny = 0; while ((1 << G->lny) < G->Ny) ++G->lny;
  G->hx = c->d[0] * lu;
  G->hy = c->dims == 3 ? c->d[1] * lu : 1.0;
  G->h = c->d[2] * lu;
  if (!(G->hx > 0 && G->hy > 0 && G->h > 0)) { *why = "grid steps must be > 0"; return GEMPIC_EINVAL; }
  if (c->n_e < 0) { *why = "n_e must be >= 0"; return GEMPIC_EINVAL; }
  if (c->scheme == 0) {
    G->dtau = c->dtau * lu;
    if (G->dtau == 0.0) G->dtau = 0.5 * G->h;
    if (!(G->dtau > 0)) { *why = "dtau must be >= 0"; return GEMPIC_EINVAL; }
    if (2.0 * G->dtau > G->h * (1.0 + 1e-12)) { *why = "slow step too large: need 2 dtau <= h"; return GEMPIC_ECFL; }
    if (c->n_e > 0.0 && G->dtau * G->h > 4.0 / c->n_e) { *why = "slow step violates Delta*h <= 4/omega_p^2"; return GEMPIC_ECFL; }
  } else {
    G->dtau = 0.5 * G->h;   // unused by the zeta march
    if (c->precision == GEMPIC_FP32_ABS) { *why = "the zeta march needs precision FP64 or FP32_CELL"; return GEMPIC_EINVAL; }
    if (c->beam_np != 0) { *why = "the zeta march takes no driver beam"; return GEMPIC_EINVAL; }
    if (c->deposit_rho) { *why = "the zeta march deposits no charge (deposit_rho = 0)"; return GEMPIC_EINVAL; }
    if (G->Nz > 65536) { *why = "the zeta march needs n[2] <= 65536"; return GEMPIC_EINVAL; }
    if (!(c->delta > 0)) { *why = "the zeta march needs delta > 0"; return GEMPIC_EINVAL; }
    double hmax = G->h;
    if (c->zeta_nodes) {
      const double* zn = c->zeta_nodes;
      if (zn[0] != 0.0) { *why = "zeta_nodes must start at 0"; return GEMPIC_EINVAL; }
      hmax = 0.0;
      for (int n = 0; n < G->Nz; ++n) {
        double hn = zn[n + 1] - zn[n];
        if (!(hn > 0)) { *why = "zeta_nodes must increase"; return GEMPIC_EINVAL; }
        hmax = std::max(hmax, hn * lu);
      }
    }
    if (c->n_e > 0.0 && c->delta * lu * hmax > 4.0 / c->n_e) {
      *why = "slow step violates Delta*h <= 4/omega_p^2";
      return GEMPIC_ECFL;
    }
    if (c->ch_ratio < 0 || (c->ch_ratio > 0 && c->ch_ratio != 1.0 && !(c->ch_radius > 0))) {
      *why = "channel needs ch_ratio >= 0 and ch_radius > 0";
      return GEMPIC_EINVAL;
    }
  }
  if (c->ppc[0] < 1 || c->ppc[2] < 1 || (c->dims == 3 && c->ppc[1] < 1)) { *why = "ppc must be >= 1"; return GEMPIC_EINVAL; }
  if (c->pol != 0 && c->pol != 1) { *why = "pol must be 0 or 1"; return GEMPIC_EINVAL; }
  G->P = c->filter_passes;
  G->ext = G->P + 3;
  G->Nzp = G->Nz + G->ext;
  G->NPJ = G->Nz + G->ext + 4;
  G->NPF = G->Nz + 3 + G->P;
  G->nTx = G->Nx / G->Tx;
  G->nTy = G->Ny / G->Ty;
  G->nTz = (G->Nzp + G->Tz - 1) / G->Tz;
  G->NT = G->nTx * G->nTy * G->nTz;
  G->Nxh = G->Nx / 2;
  if ((int64_t)G->Nzp * G->Ny * G->Nx >= (1ll << 30)) { *why = "grid too large: cells must stay below 2^30"; return GEMPIC_EINVAL; }
  // the transverse transforms hold whole rows of six components in LDS; sizes
  // up to 512 are the ones the parity tests cover
  if (G->Nx > 512 || G->Ny > 512) {
    *why = "transverse grid too large: Nx, Ny <= 512";
    return GEMPIC_EINVAL;
  }
  if (c->beam_np < 0) { *why = "beam_np must be >= 0"; return GEMPIC_EINVAL; }
  if (c->beam_np > 0) {
    if (c->dims != 3) { *why = "a driver beam needs dims = 3"; return GEMPIC_EINVAL; }
    if (!(c->n_e > 0)) { *why = "a driver beam needs a plasma (n_e > 0)"; return GEMPIC_EINVAL; }
    if (!(c->beam_n > 0 && c->beam_sr > 0 && c->beam_sz > 0 && c->beam_gamma > 1 && c->beam_dgamma >= 0)) {
      *why = "beam needs beam_n, beam_sr, beam_sz > 0, beam_gamma > 1, beam_dgamma >= 0";
      return GEMPIC_EINVAL;
    }
    if (c->beam_np > (1ll << 28)) { *why = "beam_np too large"; return GEMPIC_EINVAL; }
  }
  if ((int64_t)G->NT > (int64_t)SCAN_PER * SCAN_MAXB) { *why = "too many tiles"; return GEMPIC_EINVAL; }
  G->abs_pos = c->precision == GEMPIC_FP32_ABS ? 1 : 0;
  G->ihx = (float)(1.0 / G->hx);
  G->ihy = (float)(1.0 / G->hy);
  G->ih = (float)(1.0 / G->h);
  G->Lx = (float)((double)G->Nx * G->hx);
  G->Ly = (float)((double)G->Ny * G->hy);
  return GEMPIC_OK;
}

static int upload_twiddles(gempic* g) {
  const Geom& G = g->g;
  auto twiddles = [&](int N, void* dst) -> int {
    int hN = std::max(1, N / 2);
    std::vector<double> tw(2 * hN);
    for (int t = 0; t < hN; ++t) {
      double a = -2.0 * M_PI * (double)t / (double)N;
      tw[2 * t] = std::cos(a);
      tw[2 * t + 1] = std::sin(a);
    }
    if (g->prec == 0) return (int)hipMemcpy(dst, tw.data(), tw.size() * 8, hipMemcpyHostToDevice);
    std::vector<float> f(tw.begin(), tw.end());
    return (int)hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
  };
  if (twiddles(G.Nx, g->twx) || twiddles(std::max(G.Ny, 2), g->twy) ||
      hipMemset(g->err_dev, 0, sizeof(int)) != hipSuccess)
    return fail(g, GEMPIC_EDEVICE, "initial device copies failed");
  return GEMPIC_OK;
}

// sub-step bound of a zeta-march stage: every sub-step that neither reaches
// the node nor ends the budget advances time by the transverse limit and
// either zeta or the budget by at least half of it (GT1: all of it)
static void march_subcap(gempic* g) {
  const Geom& G = g->g;
  double hmax = 0.0;
  for (int n = 0; n < G.Nz; ++n) hmax = std::max(hmax, g->zn[n + 1] - g->zn[n]);
  double dsp = 0.5 * (G.dims == 3 ? std::min(G.hx, G.hy) : G.hx);
  g->mz_subcap = (int)std::min(1e8, 2.0 * std::ceil((hmax + g->Delta) / dsp) + 8.0);
}

// creation of a zeta-march handle (scheme 1, 2)
static int create_march(gempic* g) {
  const gempic_config* cfg = &g->cfg;
  const Geom& G = g->g;
  const double lu = cfg->length_unit;
  g->zn.resize(G.Nz + 1);
  for (int n = 0; n <= G.Nz; ++n) g->zn[n] = cfg->zeta_nodes ? cfg->zeta_nodes[n] * lu : (double)n * G.h;
  g->Delta = cfg->delta * lu;
  g->nperp = cfg->n_e > 0.0 ? (int64_t)G.Nx * G.Ny * g->ppcx * g->ppcy : 0;
  // room for the batches of a slow step down to Delta / 4 (gempic_set_slow_step)
  const double L = g->zn[G.Nz];
  int64_t mb = (int64_t)std::ceil(4.0 * L / g->Delta) + 1;
  int64_t cap = g->nperp * (mb + 3) + g->nperp / 2 + 4096;
  if (cap > (int64_t)INT32_MAX) return fail(g, GEMPIC_EINVAL, "zeta-march particle capacity beyond 2^31 - 1");
  g->mz_cap = (int)cap;
  g->mz_stage_blocks = (int)std::max<int64_t>(64, std::min<int64_t>(4096, (2 * g->nperp + 255) / 256));
  march_subcap(g);
  Dev& d = g->dev;
  bool ok = true;
  size_t es = g->esz;
  auto A = [&](size_t bytes) { void* p = d.alloc(bytes); ok = ok && p; return p; };
  for (int k = 0; k < 4; ++k) {
    g->mz_part[k][0] = A((size_t)cap * 4);
    for (int q = 1; q <= 8; ++q) g->mz_part[k][q] = A((size_t)cap * es);
    g->mz_part[k][9] = cfg->track_ids ? A((size_t)cap * 8) : nullptr;
  }
  g->mz_cnt = (int*)A(8 * sizeof(int));
  g->mz_pstart = (int*)A((size_t)G.Nz * 4);
  g->mz_pcount = (int*)A((size_t)G.Nz * 4);
  g->mz_cursor = (int*)A((size_t)G.Nz * 4);
  int64_t nxy = (int64_t)G.Ny * G.Nx;
  int64_t M = (int64_t)G.Ny * G.Nxh;
  int64_t nsp = (int64_t)G.Nz * M;
  int64_t nf = (int64_t)G.Nz * nxy;
  g->mz_dep = A((size_t)3 * nxy * es);
  g->mz_jhat = A((size_t)3 * M * 2 * es);
  g->mz_out6 = A((size_t)6 * M * 2 * es);
  for (int q = 0; q < 2; ++q) g->mz_j0[q] = A((size_t)(nsp + M) * 2 * es);
  g->F6 = A((size_t)6 * nf * es);
  g->F6b = A((size_t)6 * nf * es);
  for (int q = 0; q < 3; ++q) g->J[q] = A((size_t)G.NPJ * nxy * es);
  for (int q = 0; q < 4; ++q) g->st[q] = A((size_t)nsp * 2 * es);
  for (int q = 0; q < 6; ++q) g->outs[q] = A((size_t)nsp * 2 * es);
  for (int q = 0; q < 2; ++q) g->Lsp[q] = A((size_t)nsp * 2 * es);
  g->twx = A((size_t)std::max(1, G.Nx / 2) * 2 * es);
  g->twy = A((size_t)std::max(1, G.Ny / 2) * 2 * es);
  g->partial = (double*)A(6 * DIAG_BLOCKS * 8);
  g->dres = (double*)A(4 * 8);
  g->err_dev = (int*)A(sizeof(int));
  g->mz_hnode = (double*)A((size_t)G.Nz * 8);
  g->mz_zn = (double*)A((size_t)(G.Nz + 1) * 8);
  if (!ok) return fail(g, GEMPIC_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(d.last));
  int rc = upload_twiddles(g);
  if (rc) return rc;
  std::vector<double> hnode(G.Nz);
  for (int n = 0; n < G.Nz; ++n) {
    double hl = n > 0 ? g->zn[n] - g->zn[n - 1] : g->zn[1] - g->zn[0];
    hnode[n] = 0.5 * (hl + (g->zn[n + 1] - g->zn[n]));
  }
  HIPCHK(g, hipMemcpy(g->mz_hnode, hnode.data(), G.Nz * 8, hipMemcpyHostToDevice));
  HIPCHK(g, hipMemcpy(g->mz_zn, g->zn.data(), (G.Nz + 1) * 8, hipMemcpyHostToDevice));
  if (g->prec == 0) Impl<double>::set_lds_limits(); else Impl<float>::set_lds_limits();
  for (int q = 0; q < 3; ++q) {
    if (g->prec == 0) Impl<double>::fill(g, g->J[q], (int64_t)G.NPJ * nxy);
    else Impl<float>::fill(g, g->J[q], (int64_t)G.NPJ * nxy);
  }
  rc = g->prec == 0 ? Impl<double>::mz_init(g) : Impl<float>::mz_init(g);
  if (rc == GEMPIC_OK) rc = check_errors(g);
  return rc;
}

extern "C" {

const char* gempic_strerror(int code) {
  switch (code) {
    case GEMPIC_OK: return "ok";
    case GEMPIC_EINVAL: return "invalid argument";
    case GEMPIC_ENOMEM: return "out of device memory";
    case GEMPIC_EDEVICE: return "device error";
    case GEMPIC_ECFL: return "slow step too large (more than one cell crossing)";
    case GEMPIC_ENUMERIC: return "non-finite value";
    case GEMPIC_ESTATE: return "call not allowed in this state";
    case GEMPIC_EABI: return "ABI version mismatch";
    case GEMPIC_ECAPACITY: return "particle capacity exceeded";
    default: return "unknown error";
  }
}

const char* gempic_last_error(const gempic_t* g) {
  return g ? g->err.c_str() : g_create_error.c_str();
}

void gempic_destroy(gempic_t* g) {
  if (!g) return;
  if (g->s) (void)hipStreamSynchronize(g->s);
  for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
  g->dev.release();
  delete g;
}

int gempic_create(const gempic_config* cfg, gempic_t** out) {
  if (!out) { g_create_error = "out is NULL"; return GEMPIC_EINVAL; }
  *out = nullptr;
  if (!cfg) { g_create_error = "cfg is NULL"; return GEMPIC_EINVAL; }
  Geom G;
  std::memset(&G, 0, sizeof(G));
  std::string why;
  int rc = validate(cfg, &G, &why);
  if (rc) { g_create_error = why; return rc; }
  gempic* g = new gempic();
  g->cfg = *cfg;
  g->s = (hipStream_t)cfg->stream;
  g->prec = cfg->precision == GEMPIC_FP64 ? 0 : 1;
  g->esz = g->prec == 0 ? 8 : 4;
  g->ppcx = cfg->ppc[0];
  g->ppcy = cfg->dims == 3 ? cfg->ppc[1] : 1;
  g->ppcz = cfg->ppc[2];
  g->quiet = cfg->load == 1;
  g->key = sm_mix(cfg->seed ^ (0ull << 56));
  double lu = cfg->length_unit;
  int ppc = g->ppcx * g->ppcy * g->ppcz;
  double hy_eff = G.dims == 3 ? G.hy : 1.0;
  g->w = cfg->n_e * G.hx * hy_eff * G.h / (double)ppc;
  // driver beam: the bunch holds beam_n (2 pi)^(3/2) sr^2 sz electrons, shared
  // equally by beam_np macro-particles
  g->nbeam = 0;
  g->wb = cfg->beam_np > 0 ? cfg->beam_n * std::pow(2.0 * M_PI, 1.5) * (cfg->beam_sr * lu) *
                                 (cfg->beam_sr * lu) * (cfg->beam_sz * lu) / (double)cfg->beam_np
                           : 0.0;
  G.qw = -1.0 * g->w;
  G.V = G.hx * hy_eff * G.h;
  g->L = (double)(G.Nz - 1 + G.ext) * G.h;
  g->hz = G.h / (double)g->ppcz;
  double fwhm = cfg->fwhm * lu;
  g->Tlas = fwhm > 0 ? fwhm / std::sqrt(2.0 * std::log(2.0)) : 0.0;
  g->zeta_c = std::isnan(cfg->zeta_c) ? (double)(G.Nz - 1) * G.h - 2.0 * g->Tlas : cfg->zeta_c * lu;
  g->waist = cfg->waist * lu;
  if (cfg->a0 != 0.0 && !(g->Tlas > 0)) { delete g; g_create_error = "laser needs fwhm > 0"; return GEMPIC_EINVAL; }
  g->g = G;
  g->step = 0;
  g->failed = false;
  g->timing = false;
  g->tsteps = 0;
  g->cur = 0;
  g->ctc = 0;
  g->scheme = cfg->scheme;
  g->s_total = 0.0;
  if (g->scheme != 0) {
    rc = create_march(g);
    if (rc) {
      g_create_error = g->err;
      gempic_destroy(g);
      return rc;
    }
    *out = g;
    return GEMPIC_OK;
  }

  // capacities
  int64_t ncell_p = (int64_t)G.Nzp * G.Ny * G.Nx;
  int64_t n0 = cfg->n_e > 0 ? ncell_p * ppc : 0;
  g->capacity = n0 + n0 / 4 + 4096 + cfg->beam_np;
  g->max_nm = (int64_t)std::ceil(G.dtau * g->ppcz / G.h) + 5;
  g->stage_per_tile = g->max_nm * G.Ty * G.Tx * g->ppcx * g->ppcy;
  // particle indices, chunk starts and the sort's ranks are int32
  if (g->capacity > (int64_t)INT32_MAX || (int64_t)G.NT + g->capacity / GP_CHUNK + 1 > (int64_t)INT32_MAX) {
    delete g;
    g_create_error = "particle capacity beyond 2^31 - 1 (int32 particle indices)";
    return GEMPIC_EINVAL;
  }
  g->max_chunks = (int)(G.NT + g->capacity / GP_CHUNK + 1);

  Dev& d = g->dev;
  size_t es = g->esz;
  bool ok = true;
  auto A = [&](size_t bytes) { void* p = d.alloc(bytes); ok = ok && p; return p; };
  for (int b = 0; b < 2; ++b) {
    g->part[b][0] = G.abs_pos ? nullptr : A(g->capacity * 4);
    for (int q = 1; q < 7; ++q) g->part[b][q] = (q == 2 && G.dims == 2) ? nullptr : A(g->capacity * es);
    g->ids[b] = cfg->track_ids ? (int64_t*)A(g->capacity * 8) : nullptr;
  }
  int64_t nstage = (int64_t)G.nTx * G.nTy * g->stage_per_tile;
  g->stage[0] = A(nstage * 4);
  for (int q = 1; q < 7; ++q) g->stage[q] = (q == 2 && G.dims == 2) ? nullptr : A(nstage * es);
  g->stage_g = (int32_t*)A(nstage * 4);
  for (int b = 0; b < 2; ++b) {
    g->ct[b].tile = (int32_t*)A((size_t)g->max_chunks * 4);
    g->ct[b].start = (int32_t*)A((size_t)g->max_chunks * 4);
    g->ct[b].end = (int32_t*)A((size_t)g->max_chunks * 4);
    g->ct[b].first = (int32_t*)A((size_t)G.NT * 4);
    g->ct[b].count = (int32_t*)A((size_t)G.NT * 4);
    g->ct[b].n = (int32_t*)A(4);
  }
  g->code = (int32_t*)A(g->capacity * 4);
  g->counts = (int32_t*)A((size_t)g->max_chunks * NCODE * 4);
  g->offs = (int32_t*)A((size_t)g->max_chunks * NCODE * 4);
  g->inj_count = (int32_t*)A((size_t)G.NT * 4);
  g->inj_off = (int32_t*)A((size_t)G.NT * 4);
  int64_t ng = g->max_nm * G.Ny * G.Nx * g->ppcx * g->ppcy;
  g->gflag = cfg->track_ids ? (int32_t*)A(ng * 4) : nullptr;
  g->grank = cfg->track_ids ? (int32_t*)A(ng * 4) : nullptr;
  g->tile_count = (int64_t*)A((size_t)G.NT * 8);
  g->tile_base = (int64_t*)A((size_t)G.NT * 8);
  g->scan_part = (int64_t*)A((size_t)2 * SCAN_MAXB * 8);
  g->total = (int64_t*)A(8);
  g->next_id = (int64_t*)A(8);
  g->inj_total = (int64_t*)A(8);
  g->pushed = (int64_t*)A(8);
  g->err_dev = (int*)A(sizeof(int));
  g->bcount = cfg->beam_np > 0 ? (unsigned long long*)A(8) : nullptr;
  int64_t nf = (int64_t)G.Nz * G.Ny * G.Nx;
  int64_t nJ = (int64_t)G.NPJ * G.Ny * G.Nx;
  int64_t nsp = (int64_t)G.Nz * G.Ny * G.Nxh;
  int64_t nJs = (int64_t)G.NPF * G.Ny * G.Nxh;
  g->F6 = A(6 * nf * es);
  for (int q = 0; q < 3; ++q) g->J[q] = A(nJ * es);
  for (int q = 0; q < 2; ++q) g->rho[q] = cfg->deposit_rho ? A(nJ * es) : nullptr;
  for (int q = 0; q < 3; ++q) g->Jhat[q] = A(nJs * 2 * es);
  for (int q = 0; q < 4; ++q) g->st[q] = A(nsp * 2 * es);
  for (int q = 0; q < 6; ++q) g->outs[q] = A(nsp * 2 * es);
  for (int q = 0; q < 2; ++q) g->Lsp[q] = A(nsp * 2 * es);
  g->twx = A((size_t)std::max(1, G.Nx / 2) * 2 * es);
  g->twy = A((size_t)std::max(1, G.Ny / 2) * 2 * es);
  g->partial = (double*)A(6 * DIAG_BLOCKS * 8);
  g->dres = (double*)A(4 * 8);
  if (!ok) {
    std::string m = std::string("device allocation failed: ") + hipGetErrorString(d.last);
    gempic_destroy(g);
    g_create_error = m;
    return GEMPIC_ENOMEM;
  }
  // twiddles exp(-2 pi i t / N), computed in FP64 on the host
  auto twiddles = [&](int N, void* dst) -> int {
    int hN = std::max(1, N / 2);
    std::vector<double> tw(2 * hN);
    for (int t = 0; t < hN; ++t) {
      double a = -2.0 * M_PI * (double)t / (double)N;
      tw[2 * t] = std::cos(a);
      tw[2 * t + 1] = std::sin(a);
    }
    if (g->prec == 0) return (int)hipMemcpy(dst, tw.data(), tw.size() * 8, hipMemcpyHostToDevice);
    std::vector<float> f(tw.begin(), tw.end());
    return (int)hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
  };
  int e0 = 0;
  if (twiddles(G.Nx, g->twx) || twiddles(std::max(G.Ny, 2), g->twy) ||
      hipMemset(g->err_dev, 0, sizeof(int)) != hipSuccess ||
      hipMemset(g->next_id, 0, 8) != hipSuccess) {
    gempic_destroy(g);
    g_create_error = "initial device copies failed";
    return GEMPIC_EDEVICE;
  }
  (void)e0;
  if (g->prec == 0) Impl<double>::set_lds_limits(); else Impl<float>::set_lds_limits();
  rc = g->prec == 0 ? Impl<double>::init_state(g) : Impl<float>::init_state(g);
  if (rc == GEMPIC_OK) rc = check_errors(g);
  if (rc) {
    g_create_error = g->err;
    gempic_destroy(g);
    return rc;
  }
  *out = g;
  return GEMPIC_OK;
}

int gempic_step(gempic_t* g, int32_t nsteps, gempic_diag* diag) {
  if (!g) return GEMPIC_EINVAL;
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  if (nsteps < 0) return fail(g, GEMPIC_EINVAL, "nsteps < 0");
  for (int k = 0; k < nsteps; ++k) {
    int rc;
    if (g->scheme) rc = g->prec == 0 ? Impl<double>::mz_step(g) : Impl<float>::mz_step(g);
    else rc = g->prec == 0 ? Impl<double>::one_step(g) : Impl<float>::one_step(g);
    if (rc) return rc;
  }
  int rc = check_errors(g);
  if (rc) return rc;
  if (diag) {
    if (g->scheme) rc = g->prec == 0 ? Impl<double>::mz_diag(g, diag) : Impl<float>::mz_diag(g, diag);
    else rc = g->prec == 0 ? Impl<double>::diag(g, diag) : Impl<float>::diag(g, diag);
    if (rc) return rc;
  }
  return GEMPIC_OK;
}

size_t gempic_fields_bytes(const gempic_t* g, uint32_t mask) {
  if (!g) return 0;
  const Geom& G = g->g;
  size_t nf = (size_t)G.Nz * G.Ny * G.Nx, nJ = (size_t)G.NPJ * G.Ny * G.Nx;
  size_t b = 0;
  for (int q = 0; q < 10; ++q)
    if (mask & (1u << q)) b += (q < 6 ? nf : nJ) * g->esz;
  return b;
}

int gempic_fields(gempic_t* g, uint32_t mask, int32_t on_device, void* dst, size_t dst_bytes) {
  if (!g || !dst) return GEMPIC_EINVAL;
  if (mask >= (1u << 10)) return fail(g, GEMPIC_EINVAL, "unknown field bits");
  if (dst_bytes < gempic_fields_bytes(g, mask)) return fail(g, GEMPIC_EINVAL, "dst_bytes too small");
  if ((mask & GEMPIC_RHO) && !g->cfg.deposit_rho) return fail(g, GEMPIC_EINVAL, "rho needs deposit_rho = 1");
  const Geom& G = g->g;
  size_t nf = (size_t)G.Nz * G.Ny * G.Nx, nJ = (size_t)G.NPJ * G.Ny * G.Nx;
  char* o = (char*)dst;
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int q = 0; q < 10; ++q) {
    if (!(mask & (1u << q))) continue;
    const void* src = q < 6 ? g->outs[0] : (q < 9 ? g->J[q - 6] : g->rho[1]);
    if (q < 6) {
      // the fields live as interleaved node records; outs[0] is scratch here
      if (g->prec == 0)
        k_deinterleave<double><<<nblk(nf, 256), 256, 0, g->s>>>((const double*)g->F6, (double*)g->outs[0], q, nf);
      else
        k_deinterleave<float><<<nblk(nf, 256), 256, 0, g->s>>>((const float*)g->F6, (float*)g->outs[0], q, nf);
    }
    size_t bytes = (q < 6 ? nf : nJ) * g->esz;
    HIPCHK(g, hipMemcpyAsync(o, src, bytes, kind, g->s));
    o += bytes;
  }
  HIPCHK(g, hipStreamSynchronize(g->s));
  return GEMPIC_OK;
}

int gempic_axis_field(gempic_t* g, int32_t component, double* dst, size_t n) {
  if (!g || !dst) return GEMPIC_EINVAL;
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  if (component < 0 || component > 5) return fail(g, GEMPIC_EINVAL, "component must be 0 .. 5 (Ex .. Bz)");
  const Geom& G = g->g;
  if (n < (size_t)G.Nz) return fail(g, GEMPIC_EINVAL, "n smaller than the zeta planes");
  // outs[0] (Nz Ny Nx elements of the mode's precision) holds the Nz doubles
  const int64_t plane = (int64_t)G.Ny * G.Nx, col = (int64_t)(G.Ny / 2) * G.Nx + G.Nx / 2;
  double* tmp = (double*)g->outs[0];
  if (g->prec == 0)
    k_axis<double><<<nblk(G.Nz, 256), 256, 0, g->s>>>((const double*)g->F6, tmp, component, G.Nz, plane, col);
  else
    k_axis<float><<<nblk(G.Nz, 256), 256, 0, g->s>>>((const float*)g->F6, tmp, component, G.Nz, plane, col);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipMemcpyAsync(dst, tmp, (size_t)G.Nz * 8, hipMemcpyDeviceToHost, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  return GEMPIC_OK;
}

static int march_particles(gempic_t* g, int32_t on_device, int32_t* cell, void* off, void* u, int64_t* id,
                           void* w, void* b, size_t capacity, size_t* count) {
  int n = 0;
  HIPCHK(g, hipMemcpyAsync(&n, g->mz_cnt + 4, sizeof(int), hipMemcpyDeviceToHost, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  *count = (size_t)n;
  if ((size_t)n > capacity) return fail(g, GEMPIC_EINVAL, "capacity smaller than the particle count");
  if (id && !g->mz_part[0][9]) return fail(g, GEMPIC_EINVAL, "ids need track_ids = 1");
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  size_t es = g->esz;
  if (cell) HIPCHK(g, hipMemcpyAsync(cell, g->mz_part[0][0], (size_t)n * 4, kind, g->s));
  for (int q = 0; q < 3; ++q) {
    if (off) HIPCHK(g, hipMemcpyAsync((char*)off + q * capacity * es, g->mz_part[0][1 + q], (size_t)n * es, kind, g->s));
    if (u) HIPCHK(g, hipMemcpyAsync((char*)u + q * capacity * es, g->mz_part[0][4 + q], (size_t)n * es, kind, g->s));
  }
  if (w) HIPCHK(g, hipMemcpyAsync(w, g->mz_part[0][7], (size_t)n * es, kind, g->s));
  if (b) HIPCHK(g, hipMemcpyAsync(b, g->mz_part[0][8], (size_t)n * es, kind, g->s));
  if (id) HIPCHK(g, hipMemcpyAsync(id, g->mz_part[0][9], (size_t)n * 8, kind, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  return GEMPIC_OK;
}

int gempic_particles(gempic_t* g, int32_t on_device, int32_t* cell, void* off, void* u, int64_t* id,
                     size_t capacity, size_t* count) {
  if (!g || !count) return GEMPIC_EINVAL;
  if (g->scheme) return march_particles(g, on_device, cell, off, u, id, nullptr, nullptr, capacity, count);
  int64_t n = 0;
  HIPCHK(g, hipMemcpyAsync(&n, g->total, 8, hipMemcpyDeviceToHost, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  *count = (size_t)n;
  if ((size_t)n > capacity) return fail(g, GEMPIC_EINVAL, "capacity smaller than the particle count");
  if (id && !g->ids[0]) return fail(g, GEMPIC_EINVAL, "ids need track_ids = 1");
  hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  int b = g->cur;
  size_t es = g->esz;
  if (cell && g->g.abs_pos) {
    // cells decoded from the absolute positions, staged in the sort-code array
    k_abs_cells<<<nblk(n, 256), 256, 0, g->s>>>(g->g, (const float*)g->part[b][1], (const float*)g->part[b][2],
                                                 (const float*)g->part[b][3], n, g->code);
    HIPCHK(g, hipMemcpyAsync(cell, g->code, n * 4, kind, g->s));
  } else if (cell) {
    HIPCHK(g, hipMemcpyAsync(cell, g->part[b][0], n * 4, kind, g->s));
  }
  for (int q = 0; q < 3; ++q) {
    char* o = off ? (char*)off + q * capacity * es : nullptr;
    char* v = u ? (char*)u + q * capacity * es : nullptr;
    if (o) {
      if (g->part[b][1 + q]) HIPCHK(g, hipMemcpyAsync(o, g->part[b][1 + q], n * es, kind, g->s));
      else if (on_device) HIPCHK(g, hipMemsetAsync(o, 0, n * es, g->s));
      else std::memset(o, 0, n * es);
    }
    if (v) HIPCHK(g, hipMemcpyAsync(v, g->part[b][4 + q], n * es, kind, g->s));
  }
  if (id) HIPCHK(g, hipMemcpyAsync(id, g->ids[b], n * 8, kind, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  return GEMPIC_OK;
}

int gempic_march_particles(gempic_t* g, int32_t on_device, void* w, void* b, size_t capacity, size_t* count) {
  if (!g || !count) return GEMPIC_EINVAL;
  if (!g->scheme) return fail(g, GEMPIC_EINVAL, "weights and budgets belong to the zeta march");
  return march_particles(g, on_device, nullptr, nullptr, nullptr, nullptr, w, b, capacity, count);
}

int gempic_bunch_diag(gempic_t* g, double gamma_min, gempic_bunch* out) {
  if (!g || !out) return GEMPIC_EINVAL;
  if (g->g.abs_pos) return fail(g, GEMPIC_EINVAL, "bunch diagnostics need cell + offset positions");
  return g->prec == 0 ? Impl<double>::bunch(g, gamma_min, out) : Impl<float>::bunch(g, gamma_min, out);
}

int gempic_set_slow_step(gempic_t* g, double delta) {
  if (!g) return GEMPIC_EINVAL;
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  if (!g->scheme) return fail(g, GEMPIC_EINVAL, "the tau scheme's slow step is fixed at creation (dtau)");
  if (!(delta > 0)) return fail(g, GEMPIC_EINVAL, "delta must be > 0");
  double D = delta * g->cfg.length_unit;
  double hmax = 0.0;
  for (int n = 0; n < g->g.Nz; ++n) hmax = std::max(hmax, g->zn[n + 1] - g->zn[n]);
  if (g->cfg.n_e > 0.0 && D * hmax > 4.0 / g->cfg.n_e)
    return fail(g, GEMPIC_EINVAL, "slow step violates Delta*h <= 4/omega_p^2");
  // the particle buffers hold the batches of Delta / 4 of the creation's Delta
  const double L = g->zn[g->g.Nz];
  int64_t mb = (int64_t)std::ceil(L / D) + 1;
  if (g->nperp * (mb + 3) + g->nperp / 2 + 4096 > (int64_t)g->mz_cap)
    return fail(g, GEMPIC_EINVAL, "delta below a quarter of the creation's delta (particle buffers)");
  g->Delta = D;
  march_subcap(g);
  return GEMPIC_OK;
}

int gempic_set_state(gempic_t* g, int64_t step, const int32_t* cell, const void* off, const void* u,
                     const int64_t* id, size_t count, const void* spectral, size_t spectral_bytes) {
  if (!g) return GEMPIC_EINVAL;
  if (g->scheme) return fail(g, GEMPIC_EINVAL, "gempic_set_state serves the tau scheme");
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  const Geom& G = g->g;
  size_t es = g->esz;
  int64_t nsp = (int64_t)G.Nz * G.Ny * G.Nxh;
  if ((int64_t)count > g->capacity) return fail(g, GEMPIC_EINVAL, "count exceeds capacity");
  if (spectral && spectral_bytes < (size_t)(6 * nsp * 2) * es) return fail(g, GEMPIC_EINVAL, "spectral_bytes too small");
  if (id && !g->ids[0]) return fail(g, GEMPIC_EINVAL, "ids need track_ids = 1");
  if (count > 0 && (!cell || !off || !u)) return fail(g, GEMPIC_EINVAL, "particle arrays missing");
  // tile counts from the cells; the order must already be sorted by tile
  std::vector<int64_t> cnt(G.NT, 0);
  int prev = -1;
  int64_t maxid = -1;
  for (size_t i = 0; i < count; ++i) {
    int c = cell[i];
    if (c >= 0 && (c & GEMPIC_BEAM_BIT)) {
      if (g->cfg.beam_np <= 0) return fail(g, GEMPIC_EINVAL, "beam particle on a handle without a beam");
      c &= ~GEMPIC_BEAM_BIT;
    }
    if (c < 0 || c >= G.Nzp * G.Ny * G.Nx) return fail(g, GEMPIC_EINVAL, "cell out of range");
    int ix = c % G.Nx, r = c / G.Nx, iy = r % G.Ny, iz = r / G.Ny;
    int t = ((iz / G.Tz) * G.nTy + iy / G.Ty) * G.nTx + ix / G.Tx;
    if (t < prev) return fail(g, GEMPIC_EINVAL, "particles not sorted by tile");
    prev = t;
    cnt[t] += 1;
    if (id) maxid = std::max<int64_t>(maxid, id[i]);
  }
  int b = g->cur;
  if (G.abs_pos) {
    // the cells must be those the absolute positions decode to
    const float* px = (const float*)off;
    for (size_t i = 0; i < count; ++i) {
      float o;
      float x = px[i], y = px[count + i], z = px[2 * count + i];
      int ix = (int)std::floor(x * G.ihx), iy = (int)std::floor(y * G.ihy), iz = (int)std::floor(z * G.ih);
      (void)o;
      if (ix >= G.Nx) ix -= G.Nx;
      if (iy >= G.Ny) iy -= G.Ny;
      if (iz >= G.Nzp) iz = G.Nzp - 1;
      if (cell[i] != (iz * G.Ny + iy) * G.Nx + ix) return fail(g, GEMPIC_EINVAL, "cell does not match the absolute position");
    }
  } else {
    HIPCHK(g, hipMemcpyAsync(g->part[b][0], cell, count * 4, hipMemcpyHostToDevice, g->s));
  }
  for (int q = 0; q < 3; ++q) {
    if (g->part[b][1 + q])
      HIPCHK(g, hipMemcpyAsync(g->part[b][1 + q], (const char*)off + q * count * es, count * es,
                               hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->part[b][4 + q], (const char*)u + q * count * es, count * es,
                             hipMemcpyHostToDevice, g->s));
  }
  if (id) {
    HIPCHK(g, hipMemcpyAsync(g->ids[b], id, count * 8, hipMemcpyHostToDevice, g->s));
    int64_t nid = maxid + 1;
    HIPCHK(g, hipMemcpyAsync(g->next_id, &nid, 8, hipMemcpyHostToDevice, g->s));
  }
  HIPCHK(g, hipMemcpyAsync(g->tile_count, cnt.data(), G.NT * 8, hipMemcpyHostToDevice, g->s));
  ChunkTab& t0 = g->ct[g->ctc];
  scan_tiles(g, t0);
  k_build_chunks<<<nblk(G.NT, 128), 128, 0, g->s>>>(G.NT, g->tile_base, g->tile_count, t0, g->max_chunks);
  if (spectral) {
    const char* sp = (const char*)spectral;
    size_t bytes = (size_t)nsp * 2 * es;
    // Rx, Ry, Lx, Ly, Ez, Bz -> state (Rx, Ry, Ez, Bz) and L
    HIPCHK(g, hipMemcpyAsync(g->st[0], sp + 0 * bytes, bytes, hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->st[1], sp + 1 * bytes, bytes, hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->Lsp[0], sp + 2 * bytes, bytes, hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->Lsp[1], sp + 3 * bytes, bytes, hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->st[2], sp + 4 * bytes, bytes, hipMemcpyHostToDevice, g->s));
    HIPCHK(g, hipMemcpyAsync(g->st[3], sp + 5 * bytes, bytes, hipMemcpyHostToDevice, g->s));
    if (g->prec == 0) {
      using C = cplx<double>;
      k_state_to_fields<double><<<nblk(nsp, 256), 256, 0, g->s>>>(
          (C*)g->st[0], (C*)g->st[1], (C*)g->Lsp[0], (C*)g->Lsp[1], (C*)g->st[2], (C*)g->st[3],
          (C*)g->outs[0], (C*)g->outs[1], (C*)g->outs[2], (C*)g->outs[3], (C*)g->outs[4], (C*)g->outs[5], nsp);
      Impl<double>::fft_inv6(g);
    } else {
      using C = cplx<float>;
      k_state_to_fields<float><<<nblk(nsp, 256), 256, 0, g->s>>>(
          (C*)g->st[0], (C*)g->st[1], (C*)g->Lsp[0], (C*)g->Lsp[1], (C*)g->st[2], (C*)g->st[3],
          (C*)g->outs[0], (C*)g->outs[1], (C*)g->outs[2], (C*)g->outs[3], (C*)g->outs[4], (C*)g->outs[5], nsp);
      Impl<float>::fft_inv6(g);
    }
  }
  g->step = step;
  HIPCHK(g, hipStreamSynchronize(g->s));
  return check_errors(g);
}

int gempic_timing(gempic_t* g, int32_t enable) {
  if (!g) return GEMPIC_EINVAL;
  HIPCHK(g, hipStreamSynchronize(g->s));
  g->timing = enable != 0;
  if (enable) g->tsteps = 0;
  return GEMPIC_OK;
}

int gempic_get_timing(gempic_t* g, double* ms, int64_t* steps) {
  if (!g || !ms) return GEMPIC_EINVAL;
  HIPCHK(g, hipStreamSynchronize(g->s));
  for (int k = 0; k < 5; ++k) ms[k] = 0.0;
  for (int64_t s = 0; s < g->tsteps; ++s) {
    float t;
    for (int k = 0; k < 4; ++k) {
      HIPCHK(g, hipEventElapsedTime(&t, g->ev[s * 5 + k], g->ev[s * 5 + k + 1]));
      ms[k] += t;
    }
    HIPCHK(g, hipEventElapsedTime(&t, g->ev[s * 5], g->ev[s * 5 + 4]));
    ms[4] += t;
  }
  if (steps) *steps = g->tsteps;
  return GEMPIC_OK;
}

int gempic_set_fields(gempic_t* g, const void* fields, size_t bytes) {
  if (!g || !fields) return GEMPIC_EINVAL;
  if (g->scheme) return fail(g, GEMPIC_EINVAL, "gempic_set_fields serves the tau scheme");
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  const Geom& G = g->g;
  size_t nb = (size_t)G.Nz * G.Ny * G.Nx * g->esz;
  if (bytes < 6 * nb) return fail(g, GEMPIC_EINVAL, "bytes too small");
  int64_t nf = (int64_t)G.Nz * G.Ny * G.Nx;
  for (int q = 0; q < 6; ++q) {
    HIPCHK(g, hipMemcpyAsync(g->outs[0], (const char*)fields + q * nb, nb, hipMemcpyHostToDevice, g->s));
    if (g->prec == 0)
      k_interleave<double><<<nblk(nf, 256), 256, 0, g->s>>>((double*)g->F6, (const double*)g->outs[0], q, nf);
    else
      k_interleave<float><<<nblk(nf, 256), 256, 0, g->s>>>((float*)g->F6, (const float*)g->outs[0], q, nf);
  }
  HIPCHK(g, hipStreamSynchronize(g->s));
  return GEMPIC_OK;
}

int gempic_set_deterministic(gempic_t* g, int32_t on) {
  if (!g) return GEMPIC_EINVAL;
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  if (!on) { g->det = false; return GEMPIC_OK; }
  if (g->scheme) return fail(g, GEMPIC_EINVAL, "the deterministic deposit serves the tau scheme");
  if (g->prec != 1)
    return fail(g, GEMPIC_EINVAL, "the deterministic deposit needs an FP32 mode (FP64 tiles sum in FP64 atomics)");
  if (g->cfg.beam_np > 0) return fail(g, GEMPIC_EINVAL, "the deterministic deposit does not take a driver beam");
  const Geom& G = g->g;
  int64_t nJ = (int64_t)G.NPJ * G.Ny * G.Nx;
  if (!g->Jfix[0]) {
    bool ok = true;
    for (int q = 0; q < 3; ++q) {
      g->Jfix[q] = g->dev.alloc(nJ * 8);
      ok = ok && g->Jfix[q];
    }
    if (!ok) return fail(g, GEMPIC_ENOMEM, "deterministic current buffers");
  }
  g->det = true;
  return GEMPIC_OK;
}

int gempic_set_denoiser(gempic_t* g, gempic_dn_t* d, double threshold) {
  if (!g) return GEMPIC_EINVAL;
  if (g->failed) return fail(g, GEMPIC_ESTATE, "handle failed earlier: " + g->err);
  const Geom& G = g->g;
  if (!d) { g->dn = nullptr; return GEMPIC_OK; }
  if (g->scheme) return fail(g, GEMPIC_EINVAL, "the denoiser serves the tau scheme");
  if (g->prec != 1 || G.dims != 3) return fail(g, GEMPIC_EINVAL, "the denoiser needs an FP32 3-D simulation");
  if (G.Nx % 16 || G.Ny % 8) return fail(g, GEMPIC_EINVAL, "the denoiser needs Nx % 16 == 0 and Ny % 8 == 0");
  if (!(g->cfg.n_e > 0)) return fail(g, GEMPIC_EINVAL, "the denoiser needs a plasma (n_e > 0)");
  if (threshold != threshold) return fail(g, GEMPIC_EINVAL, "threshold is NaN");
  int64_t nJ = (int64_t)G.NPJ * G.Ny * G.Nx;
  if (!g->Jf[0]) {
    bool ok = true;
    for (int q = 0; q < 3; ++q) {
      g->Jf[q] = g->dev.alloc(nJ * 4);
      g->Jd[q] = g->dev.alloc(nJ * 4);
      g->Jt[q] = g->dev.alloc(nJ * 4);
      ok = ok && g->Jf[q] && g->Jd[q] && g->Jt[q];
    }
    g->dn_fallbacks = (int64_t*)g->dev.alloc(8);
    g->dn_rel = (double*)g->dev.alloc(8);
    if (!ok || !g->dn_fallbacks || !g->dn_rel) return fail(g, GEMPIC_ENOMEM, "denoiser current buffers");
    k_fill<int64_t><<<1, 64, 0, g->s>>>(g->dn_fallbacks, 1, 0);
    k_fill<double><<<1, 64, 0, g->s>>>(g->dn_rel, 1, 0.0);
  }
  int rc = dn_reserve(d, nJ);
  if (rc) return fail(g, rc, std::string("denoiser: ") + dn_error(d));
  HIPCHK(g, hipStreamSynchronize(g->s));
  g->dn = d;
  g->dn_thr = threshold;
  return GEMPIC_OK;
}

int gempic_get_spectral(gempic_t* g, void* spectral, size_t spectral_bytes) {
  if (!g || !spectral) return GEMPIC_EINVAL;
  const Geom& G = g->g;
  size_t bytes = (size_t)G.Nz * G.Ny * G.Nxh * 2 * g->esz;
  if (spectral_bytes < 6 * bytes) return fail(g, GEMPIC_EINVAL, "spectral_bytes too small");
  char* o = (char*)spectral;
  const void* src[6] = {g->st[0], g->st[1], g->Lsp[0], g->Lsp[1], g->st[2], g->st[3]};
  for (int q = 0; q < 6; ++q)
    HIPCHK(g, hipMemcpyAsync(o + q * bytes, src[q], bytes, hipMemcpyDeviceToHost, g->s));
  HIPCHK(g, hipStreamSynchronize(g->s));
  return GEMPIC_OK;
}

}  // extern "C"
