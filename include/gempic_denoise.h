/* gempic_denoise.h -- C ABI of the learned current denoiser (gfx950).
 *
 * The Galilean PIC step of gempic.h deposits a current that is noisy when few
 * macro-particles share a cell.  The paper's solver smooths it with the
 * binomial filter of its field update; this library adds a small network
 * that corrects the filtered current:
 *
 *     J = F(J_raw) + s * curl(A),   A = net(J_raw / n_e),   s = n_e * h,
 *
 * net: four 3x3x3 convolutions 3 -> 16 -> 32 -> 16 -> 3 with ReLU after the
 * first three, "same" padding periodic in x and y and zero in zeta, BF16
 * weights and activations with FP32 accumulation (MFMA).  A lives on cell
 * faces and curl is the staggered curl matching the deposit's staggering
 * (J_x at (i+1/2, j, n), J_y at (i, j+1/2, n), J_z at (i, j, n+1/2)), so the
 * correction is divergence-free and leaves the discrete continuity equation
 * of the filtered current (Sec. 5.1 beam current, charge-conserving deposit)
 * unchanged up to rounding.  The continuity test
 *
 *     rel = ||D.(J - F(J_raw))|| / ||D.F(J_raw)||
 *
 * falls back to F(J_raw) when rel exceeds a threshold or is not finite.
 * D.curl vanishes identically, so for a finite network output rel is FP32
 * rounding: this test is a finiteness guard.  The filtered current also
 * bounds the network's correction: the step falls back as well when
 * ||s curl(A)|| > ||F(J_raw)||, a correction larger than the current it
 * corrects, which catches a finite but wrong output.
 * F is one (or two) 1-2-1 passes along x, y (periodic) and zeta (zero
 * outside the box).
 *
 * Boxes are (Z, Y, X) voxels: Z >= 1 zeta planes, Y a multiple of 8, X a
 * multiple of 16, x and y periodic.  Currents are FP32 device arrays laid
 * out [3][Z][Y][X] (components x, y, z).  Parameters are FP32, layer by layer
 * W[Cout][Cin][kz][ky][kx] (tap (kz, ky, kx) reads the voxel at offset
 * (kz-1, ky-1, kx-1)) followed by b[Cout]; gempic_dn_nparams() of them.
 *
 * Every function returns a gempic_status (gempic.h).  A handle owns its
 * device memory; it is used on the stream given at creation (NULL = legacy
 * default stream) and is thread-compatible, not thread-safe.  Buffers grow
 * on demand to the largest box seen.
 */
#ifndef GEMPIC_DENOISE_H
#define GEMPIC_DENOISE_H

#include <stddef.h>
#include <stdint.h>

#include "gempic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gempic_dn gempic_dn_t;

/* Number of FP32 parameters of the network (30307). */
size_t gempic_dn_nparams(void);

/* Create a denoiser with host parameters theta[n] (n = gempic_dn_nparams())
 * and zero Adam moments.  *out = NULL on error (EINVAL, ENOMEM, EDEVICE). */
int gempic_dn_create(const float* theta, size_t n, void* stream, gempic_dn_t** out);

void gempic_dn_destroy(gempic_dn_t* d);
const char* gempic_dn_last_error(const gempic_dn_t* d);

/* Copy the current FP32 parameters / the gradient of the last
 * gempic_dn_train call to host memory (n >= gempic_dn_nparams()). */
int gempic_dn_params(gempic_dn_t* d, float* theta, size_t n);
int gempic_dn_grad(gempic_dn_t* d, float* grad, size_t n);

/* Denoise one box.  jraw, jout: device [3][Z][Y][X]; aout: nullable device
 * [3][Z][Y][X] receiving the network output A.  h = (h_x, h_y, h_zeta) grid
 * steps, n_e > 0 the plasma density (both in the units of the current),
 * passes in 0..2 filter passes, threshold the continuity-test bound.
 * used (host, nullable) = 1 when the corrected current was kept, 0 when the
 * filtered one was returned; rel (host, nullable) = the test ratio.
 * Synchronises the stream. */
int gempic_dn_apply(gempic_dn_t* d, const int32_t box[3], const float* jraw, double n_e, const double h[3],
                    int32_t passes, double threshold, float* jout, float* aout, int32_t* used, double* rel);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as gempic_dn_apply, with every per-box buffer (activations, A,
 * the filtered current, the filter's second pass, the test's partial sums)
 * taken from a static device array of 43,057,664 bytes that each GPU the
 * library runs on holds until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine.  Boxes beyond 2^18 voxels
 * (Z * Y * X > 262144) give GEMPIC_EINVAL.  Every call on a GPU shares that
 * GPU's array and the handle's stream: calls that overlap on one GPU (from
 * several threads or streams) race.  Same arguments, results and
 * synchronisation as gempic_dn_apply. */
int gempic_dn_apply_noalloc(gempic_dn_t* d, const int32_t box[3], const float* jraw, double n_e,
                            const double h[3], int32_t passes, double threshold, float* jout, float* aout,
                            int32_t* used, double* rel);

/* One training step over nbatch boxes: jraw and jtarget are device arrays
 * [nbatch][3][Z][Y][X] holding the raw deposits of a low- and a high-ppc run;
 * the loss is mean over the batch and over planes region[0] <= z < region[1]
 * of the three components of ((J - F(jtarget)) / n_e)^2, with J the denoised
 * current of jraw.  The gradient (readable with gempic_dn_grad) is that of
 * this loss; when lr > 0 one Adam step (beta 0.9, 0.999, eps 1e-8, bias
 * corrected) updates the parameters.  loss (host, nullable) receives the
 * batch loss (synchronises the stream). */
int gempic_dn_train(gempic_dn_t* d, const int32_t box[3], int32_t nbatch, const float* jraw,
                    const float* jtarget, double n_e, const double h[3], int32_t passes, const int32_t region[2],
                    double lr, double* loss);

/* Attach a denoiser to an FP32 3-D simulation (NULL detaches).  Each later
 * step then hands the field solver F(J_raw) + s curl(A) over all current
 * planes, or F(J_raw) when the continuity test exceeds threshold (counted
 * in gempic_diag.fallbacks); the solver's own filter is then not applied
 * again.  A negative threshold forces the filtered current every step.
 * The simulation does not own d; d must outlive the attachment.
 * EINVAL for FP64 or 2-D simulations, Nx not a multiple of 16 or Ny not a
 * multiple of 8. */
int gempic_set_denoiser(gempic_t* g, gempic_dn_t* d, double threshold);

#ifdef __cplusplus
}
#endif

#endif
