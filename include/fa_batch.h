/*
 * fa_batch.h -- several registrations advanced together, for the throughput
 * use of the method: many pairs, or one pair under many hyperparameter
 * settings, as in the paper's grid searches (Results, "FireANTs enables rapid
 * prototyping and hyperparameter tuning").
 *
 * Each pair keeps its own state, schedule, step norm M and loss history, and
 * runs its kernels on the HIP stream it was created with.  Pairs created on
 * different streams therefore run concurrently on the GPU: the coarse pyramid
 * levels of one registration leave most of the chip idle, and the other
 * registrations fill it.
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

#ifdef __cplusplus
}
#endif

#endif /* FA_BATCH_H_ */
