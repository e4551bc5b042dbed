/*
 * fa_symmetric.h -- symmetric registration.
 *
 * The paper reports a symmetric variant of its registration (Table
 * "timingbrain", "Ours (symmetric)") whose transform is
 * phi = phi_M o phi_F^{-1}, with phi_F^{-1} from the post hoc inverse
 * (Section 4.4.3, "Alternative formulations for Eulerian differential").
 *
 * Here two half-way warps phi_F = id + d_F and phi_M = id + d_M minimise the
 * LNCC cost between the two warped images, C(I_F o phi_F, I_M o phi_M), so the
 * images meet in between.  LNCC is symmetric in its images, so each half's
 * gradient is the registration's fused gradient with the other half's warped
 * image as the fixed image, both taken at the same pair of warps.  Each half
 * is then advanced by Algorithm 1's steps (its own Adam moments and step norm
 * M; a shared step count, pyramid and level transitions).  fa_sym_finish
 * fits psi = phi_F^{-1} (fa_inverse.h) and returns d(x) = e(x) + d_M(x + e(x)),
 * the displacement of phi_M o psi, so that I_M(x + d(x)) ~ I_F(x) as for an
 * asymmetric registration.
 *
 * All work runs on the handle's stream.  An iteration is two warps (each half's
 * image by its own warp), then the fused gradient + Adam, smoothing and
 * composition kernels, each as one batched launch over both halves (the
 * launches of fa_batch_step_fused).
 */
#ifndef FA_SYMMETRIC_H_
#define FA_SYMMETRIC_H_

#include "fa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fa_sym_s* fa_sym;

/* fixed, moving: device pointers, float32 [n0][n1][n2] (copied; the caller
 * keeps ownership).  params as for fa_pair_create (cc_window, cc_eps, eta,
 * sigma_grad, sigma_warp, Adam, use_jac: the same for both halves).  stream: a
 * hipStream_t (NULL = the default stream).  FA_EINVAL, FA_ESHAPE, FA_ENOMEM,
 * FA_EHIP. */
fa_status fa_sym_create(const float* fixed, const float* moving, fa_shape shape, const fa_params* params,
                        void* stream, fa_sym* out);

/* The pyramid of the half-way problem, as fa_pair_set_schedule.  Resets both
 * halves to the identity and the loss history.  FA_EINVAL, FA_ESHAPE,
 * FA_ENOMEM, FA_EHIP. */
fa_status fa_sym_set_schedule(fa_sym h, int n_levels, const float* scales, const int* iters);

/* Runs up to max_iters iterations of both halves.  *iters_done and *finished
 * (may be NULL) as fa_pair_step.  Synchronises with the stream when the level
 * changes (the batched launches' tables are uploaded then) and before it
 * returns.  FA_EINVAL, FA_ESTATE, FA_ENOMEM, FA_EHIP. */
fa_status fa_sym_step(fa_sym h, int max_iters, int* iters_done, int* finished);

/* The half-way displacements d_F and d_M at the current level into dF_dev and
 * dM_dev (device, float32 [3][n0][n1][n2] of that grid; either may be NULL);
 * *level and *shape (may be NULL) receive the level and its grid.  Enqueued.
 * FA_EINVAL, FA_ESTATE, FA_EHIP. */
fa_status fa_sym_get_halfway(fa_sym h, float* dF_dev, float* dM_dev, int* level, fa_shape* shape);

/* The cost -mean cc(I_F o phi_F, I_M o phi_M) before each iteration's update,
 * into host_out (capacity floats); *n_written (may be NULL) gets the count.
 * Synchronises.  FA_EINVAL, FA_EHIP. */
fa_status fa_sym_get_loss(fa_sym h, float* host_out, int capacity, int* n_written);

/* After the schedule is complete: psi = phi_F^{-1} fitted with inv_params
 * (eta, sigmas, Adam) over the given inverse schedule (as
 * fa_inverse_set_schedule), then d_out = the displacement of phi_M o psi
 * (device, float32 [3][n0][n1][n2] of the input grid).  *inv_cost (may be
 * NULL) receives the inverse fit's last cost.  Synchronises.  FA_EINVAL,
 * FA_ESTATE (schedule not complete), FA_ENOMEM, FA_EHIP. */
fa_status fa_sym_finish(fa_sym h, const fa_params* inv_params, int n_levels, const float* scales,
                        const int* iters, float* d_out, float* inv_cost);

/* Releases the handle (synchronises first).  NULL is a no-op. */
void fa_sym_destroy(fa_sym h);

#ifdef __cplusplus
}
#endif

#endif /* FA_SYMMETRIC_H_ */
