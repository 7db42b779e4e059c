// Internal interface between the PIC step and the current denoiser.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct gempic_dn;

// Make sure the denoiser's buffers hold a box of `voxels` (inference only).
int dn_reserve(gempic_dn* d, int64_t voxels);

// Denoised current of one step on the box (Z, Y, X) (x, y periodic, zero
// beyond the Z planes), all FP32 planar arrays [Z][Y][X]:
//   Jf = F^passes(J)                                  (binomial filter)
//   Jd = Jf + n_e h * curl(A(J / n_e))                (network correction)
// then, on the device, Jd = Jf where the continuity test fails
// (||D.(Jd - Jf)|| / ||D.Jf|| > thr or not finite); fallbacks[0] counts
// those steps and rel[0] keeps the last ratio.  tmp: scratch planar arrays
// (needed when passes == 2).  Enqueued on `s`, no synchronisation.
int dn_step(gempic_dn* d, hipStream_t s, int Z, int Y, int X, const float* const J[3],
            float* const Jf[3], float* const Jd[3], float* const tmp[3], double n_e,
            const double hs[3], int passes, double thr, int64_t* fallbacks, double* rel);

const char* dn_error(const gempic_dn* d);
