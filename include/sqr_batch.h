/*
 * sqr_batch.h -- batched calls of libsqr (serving many bases at once).
 *
 * One sqr_batch call runs several orthogonalisations (Algorithm 1 with the
 * CholQR3 start, as sqr_orth) and appends (Algorithm 2 / Prop. 2.1, as
 * sqr_append) of different sizes together: the passes of all calls advance
 * in step, and every kernel launch of a pass covers all calls that use that
 * kernel at that point of their pass.  Each call keeps its own route, grid,
 * partial-Gram slots and device-side decisions, so its result is bit for bit
 * the one of the same call made alone (sqr_orth / sqr_append).  Calls that
 * finish early exit at once from the later launches.
 */
#ifndef SQR_BATCH_H
#define SQR_BATCH_H

#include <stdint.h>

#include "sqr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SQR_BATCH_ORTH    0
#define SQR_BATCH_APPEND  1

typedef struct sqr_batch_item {
  int32_t kind;            /* SQR_BATCH_ORTH or SQR_BATCH_APPEND                 */
  int32_t rc;              /* out: as sqr_orth / sqr_append would return it      */
  sqr_basis* basis;        /* append: the basis to extend (in);
                              orth: the new handle (out, on rc >= 0)             */
  const double* in;        /* A (orth, m x cols) or W (append, basis m x cols),
                              column-major device memory, read only              */
  int64_t ld_in;
  int64_t m;               /* orth: rows (append: the basis's)                   */
  int64_t cols;            /* orth: n; append: p                                 */
  int64_t cap;             /* orth: column capacity of Q and R                   */
  double* Q; int64_t ldq;  /* orth: m x cap output                               */
  double* R; int64_t ldr;  /* orth: cap x cap output                             */
  sqr_info info;           /* out: outcome of the call                           */
} sqr_batch_item;

/*
 * sqr_batch -- run `count` calls on `stream` and wait for all of them.
 *   opts   options of the orthogonalisations (NULL = defaults); appends use
 *          the options of their basis.
 *   items  per call; usage errors of one item (negative rc, with the checks
 *          of sqr_orth / sqr_append; SQR_EOPT also for a second append to the
 *          same basis in one batch) leave the other items running.
 * Appends run on block_pass only: an append whose basis is too wide for it
 * (see sqr_append) or whose block has more than 528 columns gets SQR_EDIM;
 * run it with sqr_append.  Orthogonalisations take cap <= 528.
 * An append with rc = SQR_OK and info.status = SQR_OK grows its basis by p;
 * on any other status the width is unchanged.  The call returns after the
 * work of the batch has finished on `stream` (the argument tables it stages
 * are reused by the next batch).
 * Returns SQR_OK, SQR_ENULL (items NULL or count < 1), SQR_EOPT (bad opts)
 * or SQR_EHIP (then every item that was started has rc = SQR_EHIP).
 */
int sqr_batch(const sqr_opts* opts, sqr_batch_item* items, int32_t count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SQR_BATCH_H */
