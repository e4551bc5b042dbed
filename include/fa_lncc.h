/*
 * fa_lncc.h -- the fused LNCC cost and its Gateaux gradient as a stateless
 * call, for use as a differentiable loss outside the registration driver.
 *
 * For a fixed image I, a moving image I_m and a displacement d (voxel units),
 * the call evaluates, in one streaming pass over the volume,
 *
 *   J(x)  = I_m(x + d(x))                    trilinear, zero outside the grid
 *   L     = -(1/N) sum_x cc(x)               cc = cross^2 / (v_I v_J + eps)
 *   dL/dd = dL/dJ (x) * grad I_m (x + d(x))  (Section 4.4.2: the gradient of
 *                                             the cost with respect to the
 *                                             warp, without the Jacobian term)
 *
 * over windows of w^3 voxels clipped to the grid and normalised by their
 * voxel count.  This is the computation of one iteration of Algorithm 1 up to
 * the optimiser, with the same kernels and the same readings as fa.h
 * (cross, v_I, v_J are sum-form window (co)variances; eps is added to their
 * product; the derivative at an integer sample position is the one-sided
 * derivative of the cell holding it).
 *
 * Conventions as in fa.h: float32 volumes in C order [n0][n1][n2] in device
 * memory, displacement SoA [3][n0][n1][n2]; work is enqueued on the stream
 * given at creation; every call returns an fa_status and never aborts.
 */
#ifndef FA_LNCC_H_
#define FA_LNCC_H_

#include "fa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fa_lncc_s* fa_lncc;   /* opaque; owns its reduction buffers */

/* Create an evaluator for volumes of `shape` (every dimension >= 2,
 * n0*n1*n2 < 2^29), window w (odd, 1..9) and eps >= 0.  Allocates a copy of
 * the moving image with a two-voxel zero border, (n0+4)(n1+4)(n2+4) floats,
 * the same grid as corner quads (four times that, for volumes whose quad copy
 * stays below 4 GiB), plus a few KB of device memory; work is enqueued on
 * `hip_stream` (NULL = null stream). */
fa_status fa_lncc_create(fa_shape shape, int window, float cc_eps, void* hip_stream, fa_lncc* out);

/* Evaluate at (fixed, moving, d), all device pointers of the evaluator's shape.
 *   loss_dev:  device float receiving L (may be NULL).
 *   grad_dev:  device [3][n0][n1][n2] receiving dL/dd, or NULL for the loss only.
 *   grad_scale_dev: device float multiplying the gradient (the upstream
 *              derivative of a chain rule), or NULL for 1.
 * At least one of loss_dev and grad_dev must be non-NULL.  Enqueued; calls on
 * one evaluator must not overlap (they share its reduction buffers). */
fa_status fa_lncc_eval(fa_lncc h, const float* fixed, const float* moving, const float* d,
                       float* loss_dev, float* grad_dev, const float* grad_scale_dev);

/* Destroy (synchronises the stream).  NULL is a no-op. */
void fa_lncc_destroy(fa_lncc h);

/* Size in bytes of the library's fixed device scratch array used by
 * fa_lncc_eval_noalloc (one copy per GPU, held until the process ends). */
#define FA_LNCC_NOALLOC_SCRATCH_BYTES (32u << 20)

/* fa_lncc_eval without an evaluator, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It computes exactly what fa_lncc_create(shape, window,
 * cc_eps, hip_stream) followed by fa_lncc_eval(fixed, moving, d, loss_dev,
 * grad_dev, grad_scale_dev) computes (same arithmetic in the same launch
 * shapes, so the same bits: the evaluator samples the corner-quad copy and
 * this call the scalar zero-bordered copy, which give every trilinear sample
 * the same corner values), with arguments as documented there.
 *
 * It calls no hipMalloc, hipFree or other allocating routine.  Every buffer
 * besides the caller's inputs and outputs (control block, reduction partials,
 * zero-bordered copy of the moving image) lives in a fixed device array of
 * FA_LNCC_NOALLOC_SCRATCH_BYTES; a call needs about 4 (n0+4)(n1+4)(n2+4)
 * bytes of it plus a few KB (160x192x224 takes 29.3 MB).  A larger volume is
 * rejected with FA_EINVAL before any work is enqueued.  The first call on a
 * device looks up the array's address on that device (hipGetSymbolAddress).
 *
 * Every call on one GPU shares that GPU's array, and each call overwrites
 * what the last one left there before reading it.  Calls on one GPU that
 * overlap in time (different streams, or different host threads without
 * ordering) race on the array and must be serialised by the caller.
 * Enqueued on hip_stream (NULL = null stream); returns an fa_status. */
fa_status fa_lncc_eval_noalloc(fa_shape shape, int window, float cc_eps, const float* fixed, const float* moving,
                               const float* d, float* loss_dev, float* grad_dev, const float* grad_scale_dev,
                               void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FA_LNCC_H_ */
