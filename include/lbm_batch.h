/*
 * lbm_batch.h - many independent simulations advanced together: one set of
 * kernel launches per time step runs the update of section 4.3 (criterion,
 * activation, initialisation of new blocks, the fused step) over the merged
 * list of every member's active blocks, and the steps are replayed from a
 * captured HIP graph.  Each member computes exactly what lbm_step would
 * compute for it alone (same kernels, same arithmetic).
 *
 * Members are existing handles (lbm.h) after lbm_set_geometry (and, for a
 * progressive mesh, after their first blocks were activated).  They must
 * share the storage format, the number of components, the mesh mode
 * (static or progressive), the access pattern and their step count; the batch keeps pointers to
 * them, so they must outlive it.  While a batch steps, the members are
 * ordered after the work already queued on their own streams, and work
 * queued on their streams afterwards waits for the batch.  Members can still
 * be used alone (lbm_step, lbm_moments, ...) between batch calls.
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_batch lbm_batch_t;

/* Creates a batch of n >= 1 handles (the handle array is copied).  The
 * learned proposal (lbm_mlp.h) must be disabled on every member.  Errors:
 * LBM_EINVAL (mismatched members, a member with the proposal enabled, the
 * same handle twice, NULL),
 * LBM_ESTATE (a member without geometry), LBM_EHIP (device allocation). */
int lbm_batch_create(lbm_t* const* handles, int32_t n, lbm_batch_t** out);

/* Advances every member by nsteps steps.  use_graph = 1 replays the steps
 * from a HIP graph captured on the first call (two steps, one per buffer
 * parity); 0 launches them one by one.  Asynchronous like lbm_step.
 * Errors: LBM_EINVAL, LBM_ESTATE (members no longer at the same step),
 * LBM_EHIP (a launch or the capture failed: the members then count only the
 * steps enqueued before the failure; the message is on the first member). */
int lbm_batch_step(lbm_batch_t* b, int32_t nsteps, int32_t use_graph);

/* Schedule of the step kernel (a performance setting; the results are the
 * same bits either way).  persistent = 0 (the default): one workgroup per
 * (block, part) item of the merged active list.  persistent = 1: a resident
 * grid (as many workgroups as the GPU holds at once) whose workgroups take
 * items from one queue per XCD, their own first, then steal from the
 * others, until every queue is empty.  Applies to the two-buffer pattern;
 * the work split is the first member's (lbm_set_split).  Errors: LBM_EINVAL. */
int lbm_batch_schedule(lbm_batch_t* b, int32_t persistent);

/* Releases the batch (not the members); waits for its work. */
int lbm_batch_destroy(lbm_batch_t* b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_BATCH_H */
