/*
 * fa_batch.h -- several registrations advanced together, for the throughput
 * use of the method: many pairs, or one pair under many hyperparameter
 * settings, as in the paper's grid searches (Results, "FireANTs enables rapid
 * prototyping and hyperparameter tuning").
 *
 * Each pair keeps its own state, schedule, step norm M and loss history.
 * fa_batch_step runs each pair's kernels on the HIP stream it was created
 * with, so pairs created on different streams run concurrently on the GPU;
 * fa_batch_step_fused runs one launch per kernel for the whole batch.  Either
 * way the coarse pyramid levels of one registration, which leave most of the
 * chip idle, are filled by the other registrations.
 */
#ifndef FA_BATCH_H_
#define FA_BATCH_H_

#include "fa.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Advance every pair of `pairs` (n entries, each with a schedule set) by up to
 * max_iters iterations, one iteration per pair in turn, so that the streams
 * receive their work interleaved.  *n_finished (may be NULL) receives the
 * number of pairs whose schedule is complete.  Enqueued; does not
 * synchronise.  Results are those of fa_pair_step on each pair alone.  A pair
 * must not appear twice.  On an error no further pair is advanced. */
fa_status fa_batch_step(fa_pair* pairs, int n, int max_iters, int* n_finished);

/* The same advance with batched launches: each kernel of an iteration of
 * Algorithm 1 (fused gradient + Adam, sigma_grad smoothing with the max norm,
 * composition, sigma_warp smoothing with the loss record) runs as ONE launch
 * for all the pairs that share its template parameters -- cost window, Gaussian
 * radius, composition form and the tile form of the pair's current level --
 * and as one launch per such group otherwise.  Pairs may differ in size,
 * level, schedule and every parameter; each keeps its own M, Adam step count
 * and loss history (per-pair control blocks), and its results are bitwise
 * those of fa_pair_step on the pair alone.  The use_jac direction stays one
 * launch per pair.
 *
 * Streams: all the work of the call is enqueued on pairs[0]'s stream, which
 * first waits for the work already queued on the other pairs' streams; at the
 * end those streams wait for it.  The call synchronises with that stream when
 * the batch's composition changes (a level transition or a finished pair:
 * the launch tables are uploaded then) and before it returns.  All pairs must
 * be on one device.  The per-kernel timing of fa_pair_profile does not cover
 * iterations run here.  Errors: FA_EINVAL (NULL or repeated pair, n < 0,
 * max_iters < 0, pairs on different devices), FA_ESTATE (a pair without a
 * schedule), FA_ENOMEM (launch tables), FA_EHIP; after an error the pairs
 * already advanced keep their progress. */
fa_status fa_batch_step_fused(fa_pair* pairs, int n, int max_iters, int* n_finished);

/* Process-wide switch for fa_batch_step_fused (off by default).  On: the call
 * runs on a private non-blocking stream (joined to the pairs' streams by
 * events at entry and exit); the first iteration of each batch composition
 * runs eagerly, its launches are then captured once into a HIP graph, and the
 * graph replays every later iteration until the composition changes.  The
 * iteration's per-step values live in the pairs' control blocks on the
 * device, so a replay needs no host input.  Results are those of the eager
 * form. */
void fa_batch_use_graphs(int enable);

#ifdef __cplusplus
}
#endif

#endif /* FA_BATCH_H_ */
