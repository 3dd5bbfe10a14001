/*
 * sqr_prof.h -- measurement hooks of libsqr (timing of the streaming kernel).
 *
 * When enabled, the library records a pair of HIP events on the call's stream
 * around every launch of its streaming kernel (the per-16-column-block pass
 * over the tall operands) and keeps the algorithmic HBM bytes of the launch:
 *   Gram-only launch : 8 m (s + b)   bytes,
 *   apply launch     : 8 m (s + 2 b) bytes,
 * with s the columns of the basis and same-pass prefix it reads and b the
 * columns of the block.  Launches that a finished call turned into no-ops are
 * not counted.  Host-side, process-wide; not thread-safe.
 */
#ifndef SQR_PROF_H
#define SQR_PROF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sqr_prof {
  int64_t launches[2];  /* [0] Gram-only launches, [1] apply launches        */
  double  ms[2];        /* summed event-measured durations, milliseconds     */
  double  bytes[2];     /* summed algorithmic bytes                          */
} sqr_prof;

/* Start (on != 0) or stop recording.  Starting discards earlier records. */
void sqr_prof_enable(int on);

/* Synchronise the recorded events, fold them into *out and clear them.
 * Returns 0, or SQR_EHIP / SQR_ENULL (see sqr.h). */
int sqr_prof_read(sqr_prof* out);

#ifdef __cplusplus
}
#endif

#endif /* SQR_PROF_H */
