/*
 * fa_eval.h -- evaluation of a registration result: nearest-neighbour label
 * transfer, per-class overlap counts for the Dice score, and the Jacobian
 * determinant of the transformation.
 *
 * These are the quantities behind the paper's accuracy measures: the
 * per-region target overlap TO_r = |S_r n T_r| / |T_r| and mean overlap (Dice)
 * MO_r = 2 |S_r n T_r| / (|S_r| + |T_r|) of transferred label maps (appendix
 * "Datasets and Evaluation Metrics", in-vivo brain MRI), and the singularity
 * error, the fraction of voxels where the transformation is not locally
 * invertible, det(D phi) <= 0 (Results, lung CT benchmarks).
 *
 * Conventions as in fa.h: C order [n0][n1][n2]; displacement SoA
 * [3][n0][n1][n2] in voxel units (phi(x) = x + d(x)); device pointers; work
 * enqueued on `hip_stream` (NULL = null stream).  Every call returns an
 * fa_status and never aborts.  Calls that return host results synchronise
 * the stream.  Scratch for the reductions is allocated and freed per call.
 */
#ifndef FA_EVAL_H_
#define FA_EVAL_H_

#include <stdint.h>

#include "fa.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Transfer labels through phi: out(x) = labels(round(x + d(x))), each
 * coordinate rounded half up (floor(p + 1/2), decided exactly from the fp32
 * displacement), and -1 where the rounded position leaves the grid or d is
 * not finite.  labels and out are int8 volumes of `shape` (labels >= 0 are
 * classes); out must not alias labels.  Enqueued. */
fa_status fa_warp_labels(const int8_t* labels_dev, const float* d_dev, fa_shape shape, int8_t* out_dev,
                         void* hip_stream);

/* Per-class overlap of two int8 label volumes of n voxels:
 *   counts_host[3 r + 0] = |{x : a(x) = r}|, [3 r + 1] = |{x : b(x) = r}|,
 *   counts_host[3 r + 2] = |{x : a(x) = r and b(x) = r}|   for r in [0, n_classes).
 * With a the transferred source labels S and b the target labels T:
 * MO_r = 2 counts[3r+2] / (counts[3r] + counts[3r+1]), TO_r = counts[3r+2] /
 * counts[3r+1].  Labels outside
 * [0, n_classes) are not counted.  1 <= n_classes <= 127, n >= 0.
 * counts_host is a host array of 3 n_classes values.  Synchronises. */
fa_status fa_label_overlap(const int8_t* a_dev, const int8_t* b_dev, int64_t n, int n_classes,
                           int64_t* counts_host, void* hip_stream);

/* det(I + grad d) at the interior voxels (1 <= x_a <= n_a - 2), grad by
 * central differences, evaluated in double precision:
 *   det_dev (may be NULL): double [n0-2][n1-2][n2-2];
 *   *n_nonpos_host (may be NULL): number of interior voxels with det <= 0;
 *   *n_interior_host (may be NULL): (n0-2)(n1-2)(n2-2).
 * Shapes with a dimension < 3 have no interior: counts 0, nothing written.
 * Synchronises when a count is requested, else enqueued. */
fa_status fa_jacobian_det(const float* d_dev, fa_shape shape, double* det_dev, int64_t* n_nonpos_host,
                          int64_t* n_interior_host, void* hip_stream);

/* out = u + d(x + u): the displacement of (id + d) o (id + u), with d sampled
 * trilinearly per component and zero outside the grid (the composition of
 * Algorithm 1's retraction).  With u a registration's result and d the warp
 * that made the moving image from the fixed one (moving(x) = fixed(x + d(x))),
 * out is the registration's residual: zero where it recovered that warp
 * exactly.  u, d, out: device float32 [3][n0][n1][n2]; out must not alias d.
 * Enqueued.  FA_EINVAL (NULL pointer), FA_ESHAPE. */
fa_status fa_compose_fields(const float* u_dev, const float* d_dev, fa_shape shape, float* out_dev,
                            void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FA_EVAL_H_ */
