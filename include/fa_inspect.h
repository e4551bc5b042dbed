/*
 * fa_inspect.h -- state access and intermediate readback for a registration
 * pair (include/fa.h).  These calls let a caller check each step of one
 * iteration of Algorithm 1 on its own, resume from a saved state, or evaluate
 * the cost and its gradient without stepping.  Same conventions as fa.h.
 */
#ifndef FA_INSPECT_H_
#define FA_INSPECT_H_

#include "fa.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Current level (0-based), iterations completed at that level, and the Adam
 * step count t (iterations completed since the schedule was set, across
 * levels).  Any pointer may be NULL.  Host-side only; no synchronisation. */
fa_status fa_pair_get_progress(fa_pair pair, int* level, int* iter_in_level, int* t_done);

/* Overwrite the optimiser state at the current level: displacement d and the
 * Adam moments m (EMA of the gradient) and v (EMA of its square), each a
 * device SoA array [3][n0][n1][n2] of the current level (NULL leaves that
 * array unchanged), and the Adam step count t_done (>= 0; the next iteration
 * uses step t_done + 1 in the bias corrections).  The loss history and the
 * schedule position are not changed.
 * Section 4.5 keeps m and v at the scale of the warp, so they are set with
 * it.  Enqueued.  FA_ESTATE before a schedule. */
fa_status fa_pair_set_state(fa_pair pair, const float* d, const float* m, const float* v, int t_done);

/* Copy d, m, v of the current level into device arrays (NULL skips). Enqueued. */
fa_status fa_pair_get_state(fa_pair pair, float* d, float* m, float* v);

/* Evaluate, at the current state and level and without changing it, the
 * cost L = -mean LNCC(I_f, I_m o phi) and its Gateaux derivative dL/dphi
 * (the Jacobian-free descent direction of Section 4.4.2, up to sign) into
 * g_dev (device SoA [3][n0][n1][n2]; NULL: loss only).  *loss_host receives L
 * (may be NULL).  Synchronises the stream when loss_host is given. */
fa_status fa_pair_eval_gradient(fa_pair pair, float* g_dev, float* loss_host);

/* The Adam direction a = mhat / (sqrt(vhat) + eps) of the last iteration
 * (device SoA, current level) into dev_out.  Enqueued. */
fa_status fa_pair_get_direction(fa_pair pair, float* dev_out);

/* M = max_x |G_sigma_grad * a| of the last iteration (the scale of
 * Appendix E: u = -eta s / (2M)).  Synchronises the stream. */
fa_status fa_pair_get_step_norm(fa_pair pair, float* m_host);

/* Pyramid image of level `level` (0-based): which = 0 fixed, 1 moving.
 * dev_out NULL returns only the shape.  Enqueued. */
fa_status fa_pair_get_level_image(fa_pair pair, int level, int which, float* dev_out, fa_shape* shape);

/* Kernel timing.  While enabled (enable = 1), every iteration records HIP
 * events on the pair's stream around each of its kernels; kind as in
 * fa_pair_set_tuning: 0 = gradient (warp, LNCC, adjoint, Adam), 1 = smoothed
 * direction and its maximum norm, 2 = warp smoothing, 3 = composition (the
 * launches run in the order 0, 1, 3, 2).  fa_pair_get_profile synchronises the stream and
 * returns, for level `level` and kernel `kind`, the summed duration in
 * milliseconds and the number of launches recorded since profiling was last
 * enabled.  Enabling clears the totals. */
fa_status fa_pair_profile(fa_pair pair, int enable);
fa_status fa_pair_get_profile(fa_pair pair, int level, int kind, double* total_ms, int* launches);

/* Launch-shape override for tuning.  kind 0 = gradient kernel, 1 = the
 * sigma_grad smoothing kernel (smoothed direction and its maximum norm),
 * 2 = the sigma_warp smoothing kernel, 3 = the composition kernel.  ty x tx
 * is the in-plane tile (n1 x n2): 16x32 or 8x32 for every kind, 8x64 also for
 * kinds 1 to 3, or 0x0 for the automatic choice; zc is the number of n0 planes
 * per workgroup (0 = automatic).  Volumes of at most 300,000 voxels take
 * 4x8x16 bricks processed whole in LDS instead of the march along n0
 * (kind 0: windows 1 to 5; kinds 1 and 2: radii up to 3).  variant, kind 0: 0 automatic, 1 the
 * march with next-plane gathers overlapped with the LDS passes, 2 the march
 * with them issued after the passes, 3 bricks; kinds 1 to 3: 0 automatic,
 * 1 the march, 2 bricks where supported.
 * Takes effect at the next fa_pair_set_schedule.  Results do not depend on
 * the launch shape beyond floating-point summation order. */
fa_status fa_pair_set_tuning(fa_pair pair, int kind, int ty, int tx, int zc, int variant);

/* A launch-shape autotuner: for every level of the schedule and each of the
 * four kernels (kinds as in fa_pair_set_tuning), times candidate launch shapes
 * on this GPU and keeps the fastest for that level.  Candidates: the automatic
 * shape; the 16x32 and 8x32 tiles (8x64 too for kinds 1 to 3) at chunk
 * lengths giving 1/2, 2/3, 1, 3/2 and 2 times their automatic number of
 * chunks; bricks where they exist, for volumes up to 1.2 M voxels.  Each is
 * timed with HIP events, as the fastest of three runs of `trials` launches
 * (in [1, 100]) after one warm-up, on the level's images with every output, the Adam moments and the
 * control block redirected to scratch: the pair's state (d, m, v, step
 * count, loss history) is unchanged.  Batched launches keep tuned chunks.
 * Call after fa_pair_set_schedule.  The choices are also kept for the
 * process, per device, kernel, level grid and kernel form (window, Gaussian
 * radius, composition form): every later fa_pair_set_schedule with such a
 * level uses them unless fa_pair_set_tuning overrides that kernel, so one
 * call tunes all later registrations of those shapes.  Synchronises.  Results do not depend on the shapes beyond floating-point
 * summation order (bricks sum the gradient's window statistics in another
 * order).  FA_EINVAL, FA_ESTATE (no schedule), FA_ENOMEM, FA_EHIP. */
fa_status fa_pair_autotune(fa_pair pair, int trials);

/* Forgets every launch shape fa_pair_autotune has kept for the process
 * (pairs already scheduled keep theirs). */
void fa_autotune_clear(void);

/* The launch shape in use for kernel `kind` (as in fa_pair_set_tuning) at
 * `level`: in-plane tile ty x tx, planes per workgroup zc, and whether it is a
 * brick launch (*brick = 1; then ty, tx, zc are the brick's extents).  Any
 * output may be NULL.  FA_EINVAL, FA_ESTATE. */
fa_status fa_pair_get_tiling(fa_pair pair, int level, int kind, int* ty, int* tx, int* zc, int* brick);

/* Host-only view of the automatic march launch shapes (no GPU involved).
 * kind as in fa_pair_set_tuning; shapes: n volumes (host array).
 * batched = 0: each volume's own launch (the chunk fa_pair_step uses);
 * batched = 1: the chunks of one batched launch over all n volumes, as
 * fa_batch_step_fused chooses them, with `halo` planes recomputed per chunk
 * (4 * (window / 2) for kind 0, 2 * radius for kinds 1 and 2, 2 for kind 3).
 * zc_out and blocks_out (host, n ints each, may be NULL) receive the planes
 * per workgroup and the workgroups of each volume.  FA_EINVAL for a bad kind,
 * n < 1, halo < 0 or NULL shapes; FA_ESHAPE for an invalid shape. */
fa_status fa_plan_tiling(int kind, int n, const fa_shape* shapes, int halo, int batched, int* zc_out,
                         int* blocks_out);

#ifdef __cplusplus
}
#endif

#endif /* FA_INSPECT_H_ */
