/* gempic.h -- C ABI of the MI355X (gfx950) Galilean PIC step.
 *
 * One step advances a plasma and its electromagnetic field by one slow step
 * dtau in the Galilean coordinates (x, y, zeta = z - c t, tau = t) of
 * Pukhov, Elkina & Wilson, "Galilean Electromagnetic Particle-in-Cell Code"
 * (arXiv 2509.16793):
 *   - field gather and relativistic push along the characteristics of the
 *     transformed Vlasov equation, d zeta / d tau = v_z - c (Sec. 5, eq:Vlasov1
 *     and its characteristics);
 *   - charge-conserving deposition of the beam-particle current j = q n v with
 *     macro-particle charge Q_b = q n h_x h_y h (Sec. 5.1);
 *   - the semi-implicit FD-spectral field update: transverse Fourier transform
 *     (Sec. 3.1), universal reduced system (eq:RxGu .. eq:EzGu), node scheme
 *     RxN .. eqall marched from the right boundary (Sec. 4.1) with the analytic
 *     node solution of App. B;
 *   - moving-window injection of the fresh plasma the domain sweeps over
 *     (Sec. 5.1; here every particle carries Q_b and is pushed in tau);
 *   - or, with scheme = 1 (GT1) or 2 (GT2), the paper's own slow step: the
 *     particles are integrated along zeta (Sec. 5, stop rules eq:trap1 and
 *     eq:trap2), fresh plasma of weight Q_f = q n h_x h_y Delta enters at the
 *     right edge every step and deposits j = (Q / (h_x h_y h)) v ds / Delta
 *     (Sec. 5.1), interleaved with the right-to-left node march (Sec. 4.1),
 *     so that Delta may exceed h by far; Delta may change between steps and
 *     h may vary along zeta (Sec. 7).
 * Units are the paper's normalised ones (Sec. 3): c = 1, lengths in c/omega_0,
 * fields in m c omega_0 / e, densities in units of the critical density.
 *
 * Conventions
 *   - Every function returns a gempic_status (0 = success, negative = error);
 *     nothing throws or aborts across this boundary.  gempic_last_error()
 *     returns a human-readable reason for the last failure on a handle.
 *   - The handle owns every device allocation it makes (hipMalloc).  Getters
 *     copy into caller-owned buffers; no internal pointer escapes.
 *   - All device work is enqueued on cfg.stream (a hipStream_t; NULL = the
 *     legacy default stream).  Getters and gempic_step synchronise that stream
 *     before returning.
 *   - Thread-compatible, not thread-safe: one handle per host thread.
 *   - After GEMPIC_EDEVICE, GEMPIC_ECFL, GEMPIC_ENUMERIC or GEMPIC_ECAPACITY the
 *     handle is "failed": the particle/field state is undefined (a step may
 *     have been applied partially; the step keeps no copy of the pre-step
 *     state, which would double the particle memory) and only getters,
 *     gempic_last_error and gempic_destroy are accepted.  The flags are read
 *     once per gempic_step call, after its last step.
 */
#ifndef GEMPIC_H
#define GEMPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEMPIC_ABI_VERSION 3

/* Bit of a particle's cell word that marks a driver-beam electron (gempic_particles,
 * gempic_set_state); the cell index itself is the word without this bit. */
#define GEMPIC_BEAM_BIT (1 << 30)

typedef struct gempic gempic_t;

typedef enum {
  GEMPIC_OK = 0,
  GEMPIC_EINVAL = -1,     /* bad argument or configuration                         */
  GEMPIC_ENOMEM = -2,     /* device allocation failed                              */
  GEMPIC_EDEVICE = -3,    /* a HIP call failed                                     */
  GEMPIC_ECFL = -4,       /* slow step too large / a particle crossed > 1 cell     */
  GEMPIC_ENUMERIC = -5,   /* NaN or Inf in the state                               */
  GEMPIC_ESTATE = -6,     /* call not allowed in the handle's state                */
  GEMPIC_EABI = -7,       /* abi_version mismatch                                  */
  GEMPIC_ECAPACITY = -8   /* particle buffer capacity exceeded                     */
} gempic_status;

typedef enum {
  GEMPIC_FP64 = 0,        /* every particle and field quantity in FP64             */
  GEMPIC_FP32_CELL = 1,   /* int32 cell + FP32 offsets/momenta/fields; FP64 tau,
                             window thresholds and diagnostics                    */
  GEMPIC_FP32_ABS = 2     /* FP32 absolute positions (x, y, zeta from the grid
                             origin, normalised units) + FP32 momenta/fields, 24 B
                             per particle: the precision-study mode.  A particle's
                             cell is floor(x * (1/h_x)) in FP32 (1/h_x rounded to
                             FP32), the move x += v dtau is done in FP32.  No
                             driver beam in this mode.                            */
} gempic_precision;

/* Configuration.  Lengths and times in "config units": multiplied by
 * length_unit they become c/omega_0 (length_unit = 2 pi for lengths given in
 * laser wavelengths, 1 when already normalised). */
typedef struct {
  int32_t abi_version;      /* must equal GEMPIC_ABI_VERSION                            */
  int32_t dims;             /* 2 = (x, zeta), 3 = (x, y, zeta)                          */
  int32_t n[3];             /* Nx, Ny (ignored in 2-D), Nzeta: powers of two, >= 2;
                               Nx, Ny <= 512 (the transverse transforms hold whole
                               rows in LDS)                                             */
  double  d[3];             /* hx, hy (ignored in 2-D), h (zeta step), config units     */
  double  length_unit;      /* > 0                                                      */
  double  dtau;             /* slow step, config units; 0 selects h / 2.  2 dtau > h or
                               dtau * h > 4 / n_e is rejected with GEMPIC_ECFL          */
  int32_t precision;        /* gempic_precision                                         */
  int32_t tile[3];          /* particle tile in cells: 8x8x8, 8x8x4 or 4x4x4 (2-D:
                               8x1x8, 8x1x4 or 4x1x4); must divide n                     */
  double  n_e;              /* electron density (units of the critical density); 0 = vacuum */
  int32_t ppc[3];           /* macro-particles per cell along x, y, zeta (2-D: ppc[1]=1) */
  int32_t load;             /* 0 = stratified random (SplitMix64), 1 = quiet lattice    */
  double  a0;               /* laser amplitude; 0 = no laser                            */
  double  waist;            /* 1/e field radius R, config units; 0 = plane wave         */
  double  fwhm;             /* intensity FWHM duration, config units                    */
  double  zeta_c;           /* pulse centre, config units; NaN = (Nzeta-1) h - 2 T      */
  int32_t pol;              /* 0 = E along x, 1 = E along y                             */
  uint64_t seed;
  int32_t filter_passes;    /* binomial 1-2-1 passes per axis: 0, 1 or 2                */
  int32_t track_ids;        /* 1: keep a per-particle id array (tests, checkpoints)     */
  int32_t deposit_rho;      /* 1: also deposit charge (diagnostics: continuity, charge) */
  /* Electron driver beam (3-D only; beam_np = 0: none).  beam_np macro-particles
   * sample the density beam_n exp(-r^2 / (2 beam_sr^2)) exp(-(zeta - beam_zc)^2 /
   * (2 beam_sz^2)) (rms sizes; r from the axis at node (Nx/2, Ny/2); density in
   * the units of n_e), each carrying an equal share of the bunch charge; u_perp
   * = 0, gamma normal with mean beam_gamma and deviation beam_dgamma.  Sampled on
   * the host in FP64: SplitMix64 uniforms keyed by (seed, particle, draw) and
   * the Box-Muller transform; particles outside the field box in zeta are not
   * created.  The bunch's own field starts as the field of a charge moving at c:
   * per zeta node the transverse Poisson solution E_perp = -grad phi, phi^ =
   * rho^ / K^2, as a forward wave (R_perp = 2 E_perp, L = 0), made consistent by
   * one march with Delta = 0 like the laser.  Beam particles are pushed and
   * deposited like plasma ones with their own weight; their cell words carry
   * GEMPIC_BEAM_BIT. */
  double  beam_n;           /* peak density                                             */
  double  beam_sr;          /* rms radius, config units                                 */
  double  beam_sz;          /* rms length, config units                                 */
  double  beam_zc;          /* centre, config units; NaN = (Nzeta - 1) h - 6 beam_sz    */
  double  beam_gamma;       /* mean Lorentz factor (> 1)                                */
  double  beam_dgamma;      /* rms spread of gamma                                      */
  int64_t beam_np;          /* macro-particles                                          */
  /* Slow-step scheme.  0: every particle pushed in tau with slow step dtau
   * (the fields above).  1, 2: the zeta march (GT1, GT2; Sec. 5): per slow
   * step `delta` the particles of each zeta cell, right to left, take
   * midpoint sub-steps along zeta (or, limited by the remaining slow budget
   * or by half a transverse cell, in lab time) until they reach the node
   * below, exhaust the budget (they are then parked in the box for the next
   * step; GT1 counts the budget in time, GT2 in lab z) or leave at zeta = 0;
   * each cell's currents are complete before its node is solved.  Fields
   * inside a cell are linear in zeta between the new level above and the old
   * level below.  One batch of fresh particles (ppc[0] x ppc[1] per
   * transverse cell, u = 0, offsets as in `load`) enters at the right edge
   * per step; GT1 also loads, at creation, batches every delta below the
   * edge.  GT2 creation ends with a startup march (one fresh batch pushed
   * through the initial fields with node solves of zero slow step, its
   * particles then dropped): the initial fields include the plasma's
   * response and its current is the old-level current of the first step
   * (Sec. 4.1); GT1's first step takes the new-level current for both.  Needs n[2] <= 65536, no driver beam, precision FP64 or FP32_CELL;
   * dtau, ppc[2], deposit_rho and the zeta passes of the filter are unused
   * (the transverse filter factor cos^2(k h / 2) per pass remains). */
  int32_t scheme;
  double  delta;            /* slow step Delta of the zeta march, config units          */
  const double* zeta_nodes; /* nullable: n[2] + 1 increasing zeta node positions from 0
                               (config units; copied at creation): a variable fast step
                               h_n = zeta_{n+1} - zeta_n; NULL = uniform d[2]           */
  double  ch_ratio;         /* Gaussian plasma channel (Sec. 6, eq. n_plasma): density on
                               the axis over n_e; 0 or 1 = uniform (zeta march only)      */
  double  ch_radius;        /* channel radius R_ch, config units                        */
  void*   stream;           /* hipStream_t or NULL                                      */
} gempic_config;

/* FP64 diagnostics of the last step (filled by gempic_step when requested). */
typedef struct {
  double  tau;              /* slow time after the step                                  */
  int64_t step;             /* steps done since creation                                 */
  int64_t n_particles;      /* macro-particles in the box (plasma and beam)              */
  double  charge_particles; /* sum of q w over the macro-particles                       */
  double  charge_grid;      /* sum of rho V over the grid (needs deposit_rho)            */
  double  field_energy;     /* 1/2 sum (E^2 + B^2) V over the field nodes                */
  double  continuity_rel;   /* ||(rho1-rho0)/dtau - D rhobar + D.J|| / ||(rho1-rho0)/dtau||
                               of the raw deposit (needs deposit_rho)                    */
  int64_t fallbacks;        /* steps whose denoised current failed the continuity test
                               (gempic_denoise.h); 0 without a denoiser                  */
  double  denoise_rel;      /* that test's ratio in the last step                        */
} gempic_diag;

/* Field selector bits for gempic_fields. */
#define GEMPIC_EX  (1u << 0)
#define GEMPIC_EY  (1u << 1)
#define GEMPIC_EZ  (1u << 2)
#define GEMPIC_BX  (1u << 3)
#define GEMPIC_BY  (1u << 4)
#define GEMPIC_BZ  (1u << 5)
#define GEMPIC_JX  (1u << 6)   /* raw deposited currents of the last step, lab frame    */
#define GEMPIC_JY  (1u << 7)
#define GEMPIC_JZ  (1u << 8)
#define GEMPIC_RHO (1u << 9)   /* charge density after the last push (deposit_rho = 1)  */

/* Create a simulation: validates the configuration, allocates device memory,
 * loads the plasma at tau = 0 and initialises the laser (Sec. 6, E_laser) as a
 * pure forward wave.  *out = NULL on error (the reason is returned by
 * gempic_last_error(NULL) until the next call). */
int gempic_create(const gempic_config* cfg, gempic_t** out);

/* Advance nsteps slow steps (Sec. 4.1: the slow coordinate s = tau advances by
 * Delta = dtau per step).  Each step gathers the level-k node fields, pushes
 * every particle along the characteristics of eq:Vlasov1 (Sec. 5), deposits
 * the beam-particle current j = q n v of Sec. 5.1 in charge-conserving form,
 * injects the fresh plasma the window sweeps over, and marches the node
 * system RxN .. eqall right to left with the App. B solution.
 * diag (nullable) receives the FP64 diagnostics of the last step; computing
 * them adds reductions to that step only.  Errors: GEMPIC_ESTATE on a failed
 * handle, GEMPIC_ECFL (a particle crossed more than one cell), GEMPIC_ENUMERIC
 * (a non-finite momentum), GEMPIC_ECAPACITY, GEMPIC_EDEVICE; each fails the
 * handle. */
int gempic_step(gempic_t* g, int32_t nsteps, gempic_diag* diag);

/* Copy the selected real-space fields, in bit order, each as one array of the
 * handle's precision (double for GEMPIC_FP64, float otherwise).  E and B are
 * the node fields of the current slow level, E_x = (R_x + L_x)/2,
 * B_y = (R_x - L_x)/2, E_y = (R_y + L_y)/2, B_x = (L_y - R_y)/2 (Sec. 3.1,
 * eq:Rx .. eq:Ly), transformed back from the transverse spectrum:
 *   E, B:   [Nzeta][Ny][Nx]            node (i, j, n) at (i hx, j hy, n h)
 *   J, rho: [Nzeta + filter_passes + 7][Ny][Nx]; plane p holds node n = p - 2
 *           (J_x at x index i is J_x(i + 1/2); J_y at y index j is J_y(j + 1/2)
 *           in 3-D; J_z at plane p is J_z(n + 1/2)).
 * on_device = 1: dst is device memory, else host memory.  dst_bytes too small
 * gives GEMPIC_EINVAL. */
int gempic_fields(gempic_t* g, uint32_t mask, int32_t on_device, void* dst, size_t dst_bytes);

/* Number of bytes gempic_fields needs for mask. */
size_t gempic_fields_bytes(const gempic_t* g, uint32_t mask);

/* Copy the particles (structure of arrays, in the handle's sorted order) --
 * the macro-particles of Sec. 5.1 (plasma electrons of weight Q_b / ppc and
 * driver-beam electrons), at the current slow level:
 * cell[i] = (iz * Ny + iy) * Nx + ix (int32), with GEMPIC_BEAM_BIT set for
 * driver-beam electrons; off = 3 planes of
 * capacity entries (offset in [0,1) along x, y, zeta); u = 3 planes of
 * capacity entries (momentum gamma v); id (nullable) = capacity int64 ids
 * (needs track_ids).  Offsets and momenta are double for GEMPIC_FP64, float
 * otherwise.  GEMPIC_FP32_ABS: off holds the absolute positions (x, y, zeta)
 * and cell the cells they decode to.  *count receives the particle count; GEMPIC_EINVAL if capacity
 * is smaller (then nothing is copied). */
int gempic_particles(gempic_t* g, int32_t on_device, int32_t* cell, void* off, void* u,
                     int64_t* id, size_t capacity, size_t* count);

/* Replace the state (checkpoint restore and tests).  particles: count entries
 * in the layout of gempic_particles (must be sorted by tile, stable order
 * within a tile as a step leaves it); spectral: six arrays R_x, R_y, L_x,
 * L_y, E_z, B_z of [Nzeta][Ny][Nx/2] complex (interleaved re, im) in the
 * handle's precision: the transverse modes k_x = 2 pi i / (Nx hx),
 * i = 0 .. Nx/2 - 1, and k_y = 2 pi fftfreq(Ny, hy) of the forward transform
 * sum f exp(-i k.r).  step sets the step counter (tau = step * dtau).  Host
 * memory.  ids (nullable) as in gempic_particles.  GEMPIC_FP32_ABS: off holds
 * absolute positions and cell must equal the cells they decode to. */
int gempic_set_state(gempic_t* g, int64_t step, const int32_t* cell, const void* off,
                     const void* u, const int64_t* id, size_t count, const void* spectral,
                     size_t spectral_bytes);

/* Overwrite the six real-space node fields the next push gathers from
 * (E_x, E_y, E_z, B_x, B_y, B_z, each [Nzeta][Ny][Nx] in the handle's
 * precision, host memory).  For tests that feed identical fields to the GPU
 * push and to a reference; the spectral state is left unchanged. */
int gempic_set_fields(gempic_t* g, const void* fields, size_t bytes);

/* Read the spectral state (same layout as gempic_set_state) into host memory. */
int gempic_get_spectral(gempic_t* g, void* spectral, size_t spectral_bytes);

/* Per-phase GPU time measured with HIP events on the handle's stream,
 * accumulated over the steps taken while enabled (for benchmarks; timing adds
 * five event records per step).  enable = 1 starts (and resets) the
 * accumulation, 0 stops it.  Phases of ms[5]: 0 = clearing the current
 * arrays, 1 = gather + push + deposit kernel, 2 = sort + window injection,
 * 3 = field update (FFT, march, inverse FFT), 4 = whole step.  *steps = steps
 * accumulated.  gempic_get_timing synchronises the stream. */
int gempic_timing(gempic_t* g, int32_t enable);
int gempic_get_timing(gempic_t* g, double* ms, int64_t* steps);

/* On-axis field (FP64 diagnostics; the wake's E_z is the quantity that Sec. 6
 * and the denoiser's accuracy measure): component (0 .. 5 = Ex, Ey, Ez, Bx,
 * By, Bz) at the node column (Nx/2, Ny/2) (2-D: Nx/2), for the zeta planes
 * 0 .. Nz - 1, converted to FP64 into the caller's host buffer dst[n].
 * GEMPIC_EINVAL for another component or n < Nz.  Synchronises the stream. */
int gempic_axis_field(gempic_t* g, int32_t component, double* dst, size_t n);

/* Deterministic deposit (tau scheme, FP32 modes, no driver beam; for tests
 * and reproducible runs).  The charge-conserving current of Sec. 5.1 is
 * summed per tile in 64-bit fixed point in either mode; by default each tile
 * then adds its FP32 values to the global current with floating-point
 * atomics, so a node that up to four tiles reach depends on their order in
 * its last bits.  With on = 1 the tiles add their fixed-point sums to 64-bit
 * integer arrays (3 x 8 bytes per node, allocated at the first call and held
 * until gempic_destroy) and one pass converts them: the current, and so every
 * later field and particle, is then the same bit for bit from run to run.
 * It costs integer atomics and a conversion pass per step.  on = 0 returns to
 * the default.  The charge arrays of deposit_rho keep FP32 atomics.
 * GEMPIC_EINVAL for the zeta march, FP64, or a driver beam; GEMPIC_ENOMEM
 * when the arrays cannot be allocated. */
int gempic_set_deterministic(gempic_t* g, int32_t on);

/* Witness-bunch diagnostics in the style of Table 1 (Sec. 6): over the
 * macro-particles with gamma >= gamma_min, weighted by their electrons w,
 * the charge q sum w, the mean and rms of gamma (energy gamma m c^2), the
 * weighted means and rms sizes of x, y (from the axis node (Nx/2, Ny/2)) and
 * zeta (from zeta = 0), and the normalised rms emittances
 * eps = sqrt(<dx^2><du_x^2> - <dx du_x>^2) (u = gamma v in units of c;
 * lengths in the normalised unit).  FP64, two-pass and deterministic.  Both
 * schemes; GEMPIC_EINVAL in the FP32-absolute mode. */
typedef struct {
  double  charge;
  int64_t n_macro;
  double  gamma_mean, gamma_rms;
  double  mean[3];
  double  sigma[3];
  double  emittance[2];
} gempic_bunch;
int gempic_bunch_diag(gempic_t* g, double gamma_min, gempic_bunch* out);

/* Zeta march (scheme 1, 2): slow step Delta (config units) of the following
 * steps (Sec. 7: Delta may change from one step to the next; the new step's
 * fresh particles carry the new Q_f).  Delta h_max <= 4 / n_e is required
 * (Sec. 4.2), and Delta at least a quarter of the creation's delta (the
 * particle buffers are sized for that many batches in the box).
 * GEMPIC_EINVAL for the tau scheme or an invalid Delta. */
int gempic_set_slow_step(gempic_t* g, double delta);

/* Zeta march: weights w (electrons per macro-particle) and remaining slow
 * budgets b (normalised time, <= 0 for a particle whose budget ran out,
 * the rest carried into the next step) of the particles, in the order of
 * gempic_particles, in the handle's precision.  Host or device memory. */
int gempic_march_particles(gempic_t* g, int32_t on_device, void* w, void* b, size_t capacity, size_t* count);

void gempic_destroy(gempic_t* g);

const char* gempic_strerror(int code);
const char* gempic_last_error(const gempic_t* g);

#ifdef __cplusplus
}
#endif

#endif /* GEMPIC_H */
