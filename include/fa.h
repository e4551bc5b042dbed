/*
 * fa.h -- C ABI of the MI355X-native FireANTs dense matching step.
 *
 * The library registers a moving volume to a fixed volume with the method of
 * "FireANTs: Adaptive Riemannian Optimization for Multi-Scale Diffeomorphic
 * Matching" (arXiv 2404.01249):
 *
 *   phi* = argmin_phi C(I_f, I_m o phi) + R(phi)          Eq. (image-reg)
 *
 * with C = local normalized cross-correlation (LNCC), R = 0 (regularisation
 * comes from Gaussian smoothing of the gradient and of the warp, as in the
 * paper's hyperparameter study), and phi optimised by Algorithm 1: on each
 * level of a multi-scale pyramid, every iteration computes the Gateaux
 * gradient of the cost (Jacobian-free Eulerian descent, Section 4.4.2), passes
 * it through Adam (Section 4.4, "Adaptive optimization on diffeomorphisms"),
 * smooths it, scales it by eta / LP(v) (Appendix E) and applies it by
 * composition phi <- phi o (id + u).  Between levels the warp and the Adam
 * moments are upsampled trilinearly (Section 4.5).
 *
 * Conventions (all calls):
 *   - Volumes are float32, C order [n0][n1][n2], n2 contiguous, in device
 *     memory of the current HIP device.
 *   - Displacement fields are float32 structure-of-arrays [3][n0][n1][n2] in
 *     voxel units of their level; component c moves along axis c;
 *     phi(x) = x + d(x).
 *   - Work is enqueued on the HIP stream given at creation; calls return
 *     without synchronising unless stated.
 *   - No call throws or aborts.  Every call returns an fa_status; on a
 *     non-OK status fa_last_error() returns a message (thread-local).
 *   - A pair is not thread-safe: calls on one pair must not overlap.
 */
#ifndef FA_H_
#define FA_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fa_pair_s* fa_pair;   /* opaque; owns every buffer it allocates */

typedef enum {
  FA_OK = 0,
  FA_EINVAL = -1,   /* bad argument: null pointer, bad parameter value          */
  FA_ESHAPE = -2,   /* a volume or pyramid level has an unsupported size        */
  FA_ENOMEM = -3,   /* device allocation failed                                  */
  FA_EHIP = -4,     /* a HIP runtime call failed (message has hipGetErrorString) */
  FA_ESTATE = -5    /* call not valid in the pair's current state                */
} fa_status;

typedef struct { int n0, n1, n2; } fa_shape;   /* C order, n2 contiguous */

/* Hyperparameters.  Algorithm 1 inputs plus the smoothing widths and window
 * size of the hyperparameter study ("FireANTs enables rapid prototyping and
 * hyperparameter tuning"). */
typedef struct {
  float eta;          /* step size: max |u| per iteration is eta/2 voxels (Appendix E,
                         LP(v) <= 2 sup|v|/|dx| with dx = 1 voxel); > 0            */
  float sigma_grad;   /* Gaussian on the Adam direction, voxels of the level;
                         <= 0 disables; radius ceil(3 sigma) must be <= 24         */
  float sigma_warp;   /* Gaussian on the composed displacement; same rules         */
  int   cc_window;    /* LNCC window w = 2r+1; odd, 1..9                            */
  float cc_eps;       /* added to the product of the sum-form window variances; >= 0 */
  float adam_beta1;   /* Adam (Kingma & Ba) constants, bias corrected; the step     */
  float adam_beta2;   /*   count continues across levels                            */
  float adam_eps;
  int   use_jac;      /* Algorithm 1's use_jac: 0 = Jacobian-free descent (the
                         Gateaux gradient, as in all of the paper's experiments);
                         1 = Eulerian descent, direction J(phi)^T dU/dphi with
                         J(phi) = I + grad d by central differences inside the grid
                         and one-sided differences on its faces (Section 4.4.2)    */
} fa_params;

/* Default parameters: eta 0.5, sigma_grad 1.0, sigma_warp 0.5, window 5,
 * cc_eps 1e-5, beta1 0.9, beta2 0.999, adam_eps 1e-8, use_jac 0. */
fa_status fa_params_default(fa_params* out);

/* Create a registration pair: the fixed image I_f and moving image I_m of
 * Eq. (image-reg), which are Algorithm 1's first two inputs.
 *   fixed_dev, moving_dev: device pointers to float32 volumes of `shape`;
 *     copied on `hip_stream` (stream order), so the caller may release them
 *     once that copy has run.
 *   shape: every dimension >= 2; n0*n1*n2 < 2^29 (512^3 fits).
 *   p: parameters (copied).  hip_stream: a hipStream_t (NULL = null stream).
 *   out: receives the handle.  Nothing is allocated on failure. */
fa_status fa_pair_create(const float* fixed_dev, const float* moving_dev, fa_shape shape,
                         const fa_params* p, void* hip_stream, fa_pair* out);

/* Set the multi-scale schedule (Algorithm 1 inputs [s_1..s_n], [T_1..T_n],
 * coarsest first) and reset the state: phi = id at level 1, Adam moments 0,
 * step count 0, loss history empty.  Builds the image pyramid: level l has
 * size max(1, floor(n / s_l + 1/2)) per axis and holds the input blurred with
 * sigma = s_l/2 (none at s_l = 1) and resampled trilinearly at corner-aligned
 * positions (Section 4.5).  scales and iters are host arrays of n_levels
 * entries; scales >= 1; iters >= 0; every level dimension >= 2.
 * May be called again to restart.  The pyramid build and the state reset are
 * enqueued on the stream.  When the level grids differ from the previous
 * schedule's (or on the first call), the call also synchronises the pair's
 * stream (the previous pyramid is released first) and allocates device memory
 * with hipMalloc; it does the same when the new schedule needs larger state,
 * history or tap-table buffers than the pair holds.  A schedule with the same
 * level grids reuses every buffer and returns without waiting. */
fa_status fa_pair_set_schedule(fa_pair pair, int n_levels, const float* scales, const int* iters);

/* Run up to max_iters iterations of Algorithm 1 (crossing level boundaries
 * and upsampling warp and Adam state as needed).  *iters_done receives the
 * number run, *finished 1 once the whole schedule is done (either pointer may
 * be NULL).  Enqueued; does not synchronise.  FA_ESTATE before a schedule. */
fa_status fa_pair_step(fa_pair pair, int max_iters, int* iters_done, int* finished);

/* Copy the loss history (one value per completed iteration: the cost
 * -mean(LNCC) at the warp before that iteration's update, Algorithm 1's U_i
 * with C of Eq. (image-reg)) to host memory.
 * Synchronises the stream.  Writes min(capacity, count) values; *n_written
 * receives that number. */
fa_status fa_pair_get_loss(fa_pair pair, float* host_out, int capacity, int* n_written);

/* Copy the current displacement d of phi = id + d (Algorithm 1's output once
 * the schedule is finished; the warp at the current level before that) into
 * dev_out.
 * layout 0: SoA [3][n0][n1][n2]; layout 1: [n0][n1][n2][3].  *level (0-based)
 * and *shape receive the level and its size (either may be NULL); with
 * dev_out NULL only those are returned.  Enqueued. */
fa_status fa_pair_get_field(fa_pair pair, float* dev_out, int layout, int* level, fa_shape* shape);

/* J = I_m o phi at the current level, the warped image whose cost Algorithm 1
 * evaluates (Eq. (image-reg); the pushforward image of Section 4.4.3),
 * sampled trilinearly with zero outside the grid, into dev_out ([n0][n1][n2]
 * of the current level).  Enqueued. */
fa_status fa_pair_get_warped(fa_pair pair, float* dev_out);

/* Destroy a pair (synchronises its stream, frees everything).  NULL is a no-op. */
void fa_pair_destroy(fa_pair pair);

/* Message for the last non-OK status returned on this thread. */
const char* fa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FA_H_ */
