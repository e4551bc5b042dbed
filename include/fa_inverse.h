/*
 * fa_inverse.h -- the post hoc inverse of a warp.
 *
 * The paper (Section 4.4.3, "Alternative formulations for Eulerian
 * differential") computes phi^{-1} after a registration as the minimiser over
 * diffeomorphisms psi of
 *     sum_x |psi(phi(x)) - x|^2 + |phi(psi(x)) - x|^2,
 * with a multi-scale objective like the image-matching one, and uses the same
 * routine for the final transform of its symmetric registration.
 *
 * Here psi = id + e is fitted by Algorithm 1's own loop with that cost (taken
 * as a mean over the voxels of the level): Gateaux gradient, Adam, smoothing
 * with sigma_grad, step scaled to eta / (2 max |s|), composition
 * psi o (id + u), smoothing with sigma_warp, over a pyramid whose levels carry
 * the warp's field like an image (blur with sigma = s/2, corner-aligned
 * trilinear resampling, each component divided by (n_fine - 1)/(n_coarse - 1)).
 * Displacements are in voxels, sampled trilinearly, zero outside the grid.
 *
 * Every step of an iteration runs on the GPU on the handle's stream: a splat
 * kernel (the derivative of |psi(phi(x)) - x|^2, scattered with 64-bit
 * fixed-point atomics, so results do not depend on the order of the atomics
 * and are bitwise reproducible), a kernel for the derivative of
 * |phi(psi(x)) - x|^2 plus Adam, and the registration's smoothing and
 * composition kernels.  The splat accumulates in units of 2^-32 and holds
 * sums of magnitude below 2^31, which bounds |d| and |e| far beyond any
 * volume's size.
 */
#ifndef FA_INVERSE_H_
#define FA_INVERSE_H_

#include "fa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fa_inverse_s* fa_inverse;

/* d: device pointer, the warp's displacement phi - id in voxels, float32
 * [3][n0][n1][n2] (component-major: all of d_0, then d_1, then d_2); copied,
 * the caller keeps ownership.  params: eta, sigma_grad, sigma_warp and the
 * Adam constants are used (cc_window, cc_eps and use_jac must be valid and
 * are ignored).  stream: a hipStream_t (NULL = the default stream) that
 * receives all of the handle's work.  FA_EINVAL (NULL d or out, bad
 * parameters), FA_ESHAPE, FA_ENOMEM, FA_EHIP. */
fa_status fa_inverse_create(const float* d, fa_shape shape, const fa_params* params, void* stream,
                            fa_inverse* out);

/* Pyramid: n_levels in [1, 16] levels, scales[i] in [1, 20] (a level's grid is
 * max(1, floor(n / s + 1/2)) per axis and must be at least 2), iters[i] >= 0
 * iterations.  Resets psi to the identity, the Adam state and the loss
 * history.  Host arrays.  FA_EINVAL, FA_ESHAPE, FA_ENOMEM, FA_EHIP. */
fa_status fa_inverse_set_schedule(fa_inverse h, int n_levels, const float* scales, const int* iters);

/* Runs up to max_iters iterations (moving to the next level when one is
 * done).  *iters_done and *finished (may be NULL) receive the iterations run
 * and whether the schedule is complete.  Enqueued; does not synchronise.
 * FA_EINVAL, FA_ESTATE (no schedule), FA_EHIP. */
fa_status fa_inverse_step(fa_inverse h, int max_iters, int* iters_done, int* finished);

/* Copies e = psi - id at the current level to dev_out (device, float32
 * [3][n0][n1][n2] of that level's grid; NULL only queries).  *level and
 * *shape (may be NULL) receive the level index and its grid.  Enqueued.
 * FA_EINVAL, FA_ESTATE, FA_EHIP. */
fa_status fa_inverse_get_field(fa_inverse h, float* dev_out, int* level, fa_shape* shape);

/* The cost (mean of |psi(phi(x)) - x|^2 + |phi(psi(x)) - x|^2 over the level's
 * voxels, before the iteration's update) of every iteration run so far, into
 * host_out (capacity floats).  *n_written (may be NULL) receives the count.
 * Synchronises with the handle's stream.  FA_EINVAL, FA_EHIP. */
fa_status fa_inverse_get_loss(fa_inverse h, float* host_out, int capacity, int* n_written);

/* dU/de at the current level for the current e, into g_dev (device, float32
 * [3][n0][n1][n2]), and U into *loss_host (may be NULL; synchronises when
 * given).  Changes no state.  FA_EINVAL, FA_ESTATE, FA_EHIP. */
fa_status fa_inverse_eval_gradient(fa_inverse h, float* g_dev, float* loss_host);

/* Splat form (a tuning and test switch): 0 (default) sums each brick's
 * contributions in LDS and adds each touched node once; 1 adds every
 * contribution with its own global atomic.  Both add the same fixed-point
 * integers, so results are bitwise equal.  FA_EINVAL. */
fa_status fa_inverse_set_splat(fa_inverse h, int direct);

/* Releases the handle (synchronises with its stream first).  NULL is a
 * no-op. */
void fa_inverse_destroy(fa_inverse h);

#ifdef __cplusplus
}
#endif

#endif /* FA_INVERSE_H_ */
