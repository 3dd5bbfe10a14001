/*
 * sqr.h -- shifted Cholesky QR and Cholesky QR block append on AMD MI355X.
 *
 * C ABI of libsqr.so.  All matrices are FP64, column-major, in device memory
 * (HBM) of the current HIP device; every call is stream-ordered on the HIP
 * stream it is given.  The library never allocates or frees caller buffers.
 *
 * Method: Bindhak, Pelling & Saak, "Towards an Efficient Shifted Cholesky QR
 * for Applications in Model Order Reduction using pyMOR", arXiv 2507.07788.
 *   - sqr_orth   : Algorithm 1 (iterated Cholesky QR with shift recomputation)
 *                  started as shiftedCholeskyQR3 (Sec. 3.1, algorithm list,
 *                  item 2): pass 1 shifted, passes 2-3 plain unless the
 *                  factorisation breaks down, then Algorithm 1's test.
 *   - sqr_append : Algorithm 2 (cholQRUpdate) built on Proposition 2.1:
 *                  [Q_in Q] [[R_in B],[0 R]] = [Q_in R_in, A_in].
 *   - repeated sqr_append calls from an empty or orthonormalised start are
 *     Algorithm 3 (pnCholQR, the panel scheme).
 */
#ifndef SQR_H
#define SQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes.  Negative: usage errors found before any work is enqueued;
 * nothing was modified.  Positive: numerical outcome of the algorithm. */
#define SQR_OK             0
#define SQR_NOT_CONVERGED  1  /* max_iter passes without ||X - I||_F < tol    */
#define SQR_BREAKDOWN      2  /* shifted Cholesky failed after max_escalations */
#define SQR_ENONFINITE     3  /* a Gramian held NaN or Inf                     */
#define SQR_ENULL         (-1) /* a required pointer is NULL                   */
#define SQR_EDIM          (-2) /* inconsistent sizes or leading dimensions     */
#define SQR_EHIP          (-3) /* HIP runtime error or device out of memory    */
#define SQR_EOPT          (-4) /* an option value outside its documented range */
#define SQR_ELIMIT        (-5) /* sqr_orth_noalloc: the call needs more than its
                                  static scratch holds                         */

/* Limits of sqr_orth_noalloc: columns, and bytes of its per-GPU scratch. */
#define SQR_NOALLOC_MAX_COLS       128
#define SQR_NOALLOC_SCRATCH_BYTES  (24ll << 20)

/* Options.  Defaults (sqr_default_opts) are the paper's experimental settings
 * (Sec. 3.1: tolerance 1e-13 on ||I - Q^T Q||_F, at most 10 iterations). */
typedef struct sqr_opts {
  int32_t precision;        /* 0 = FP64 throughout.  1 = mixed form of sqr_orth
                               (n <= 256): the Gramians of the shifted passes
                               and of the first unshifted pass are formed on
                               FP32 MFMA from the FP32-rounded iterate; applies,
                               shift estimates, Cholesky and the Gramians of the
                               final pass and of the check stay FP64.  An FP32
                               Gramian never ends the iteration; its shift is
                               n u32 ||X||_2 (u32 = 2^-24, floor 2 u32), x10 on
                               breakdown.  sqr_append always runs in FP64.     */
  int32_t first_pass_shift; /* 1 = CholQR3 start (shifted pass 1); 0 = Alg. 1   */
  int32_t min_passes;       /* passes run before the stopping test is consulted;
                               3 for CholQR3, 0 for Algorithm 1 as printed      */
  int32_t max_iter;         /* cap on Cholesky QR passes (1..64), default 10    */
  double  tol;              /* stop when ||X - I||_F < tol, default 1e-13       */
  double  unit_roundoff;    /* u in the shift formulas, default 2^-53           */
  int32_t max_escalations;  /* cap on the x10 shift escalations, default 32     */
  int32_t power_steps;      /* power-iteration steps for ||X||_2 from the
                               all-ones vector, 1..1000, default 30 (for
                               p <= 64 the same iterate X^s 1 is formed from
                               powers of X by repeated squaring)              */
  int32_t shift_policy;     /* sqr_orth only (sqr_append always follows
                               Algorithm 2), the variants of Sec. 3.1:
                               0 = Algorithm 1: on a breakdown the shift is
                                   recomputed from the current Gramian (x10
                                   escalation if the shifted factorisation
                                   still breaks down), default;
                               1 = no shift: a breakdown ends the call with
                                   SQR_BREAKDOWN, and a shifted first pass
                                   does not escalate (CholQR: max_iter = 1,
                                   CholQR2: 2, shiftedCholeskyQR3: 3 with
                                   first_pass_shift = 1);
                               2 = isCholQR: one shift, computed from the
                                   input Gramian (||A||^2), is used for every
                                   breakdown; if it fails, SQR_BREAKDOWN.
                               1 and 2 need precision = 0.                   */
  int32_t append_shift_dim; /* sqr_append: the width d in Algorithm 2's first
                               shift 11 (m d + d (d+1)) u ||X||: 0 = q, the
                               basis width, as printed (default); 1 = p, the
                               block width; 2 = q + p                         */
} sqr_opts;

/* Outcome of one call (host struct). */
typedef struct sqr_info {
  int32_t status;        /* SQR_OK / SQR_NOT_CONVERGED / SQR_BREAKDOWN / ...    */
  int32_t passes;        /* Cholesky QR passes executed (apply steps)           */
  int32_t chol_attempts; /* Cholesky factorisations tried, failed ones included */
  int32_t converged;     /* 1 if the stopping test was met                      */
  double  orth_fro;      /* last ||X - I||_F of the block's Gramian             */
  double  sigma[16];     /* shift of pass k+1 (0 = unshifted), first 16 passes  */
} sqr_info;

/* Opaque basis handle: (m, n, cap), borrowed Q and R, options and workspace. */
typedef struct sqr_basis sqr_basis;

/* Fill *o with the defaults listed above. */
void sqr_default_opts(sqr_opts* o);

/*
 * sqr_orth -- Q R = A for a tall A (m x n, m >= n >= 1); Algorithm 1 with the
 * CholQR3 start (see above).
 *
 *   out      receives a new handle describing the basis Q[:, 0:n] (required).
 *   opts     options, or NULL for the defaults.
 *   A, lda   m x n input, lda >= m; read only, never written.
 *   Q, ldq   m x cap output, ldq >= m, cap >= n; columns [0, n) receive Q,
 *            columns [n, cap) are reserved for later sqr_append calls.
 *   R, ldr   cap x cap output, ldr >= cap; R[0:n, 0:n] receives the upper
 *            triangular factor, its strictly lower part is written as zero.
 *   stream   hipStream_t to run on (NULL = the null stream).
 *   info     host struct, or NULL.  Non-NULL: the call waits until the
 *            device has decided the outcome (it publishes it to pinned host
 *            memory) and returns the numerical status; kernels of the call
 *            that have nothing left to do may still be queued, so Q and R are
 *            complete for later work on `stream`, and for the host or other
 *            streams once `stream` is synchronised.  NULL: the call returns
 *            after enqueueing; sqr_last_info synchronises and reports.
 *
 * Status: SQR_OK and SQR_NOT_CONVERGED leave the last pass's factors in Q
 * and R.  After SQR_BREAKDOWN or SQR_ENONFINITE their contents are
 * unspecified (with at most 16 columns, the passes before the first one
 * that can end the call recompute their input from A and do not write Q).
 *
 * Ownership: A, Q and R are borrowed and must stay allocated until the work
 * enqueued on `stream` completes.  The handle owns only its workspace.
 * Streams: a later call on the handle may use another stream; it first makes
 * that stream wait for all work of the handle's previous call (an event),
 * so the calls of one handle are always ordered.  A handle must not be used
 * by two host threads at once.
 * Widths: n up to cap (16384).  Blocks of more than 528 columns are applied
 * in superblocks of 128 columns, their Gramian is formed as one matrix, and
 * the small matrices (Cholesky, shift, R update) are worked on by one
 * workgroup in the handle's workspace; the workspace grows with n (about
 * 6 n^2 doubles beyond 528 columns).
 * Errors: SQR_ENULL, SQR_EDIM (m < 1, n < 1, n > m, lda < m, ldq < m,
 * cap < n, ldr < cap, cap > 16384, lda or ldq > 2^25 - 1), SQR_EOPT (also for
 * precision 1 with n > 256), SQR_EHIP; all
 * before any work is enqueued, except SQR_EHIP from a failed launch.
 */
int sqr_orth(sqr_basis** out, const sqr_opts* opts, int64_t m, int64_t n,
             const double* A, int64_t lda, double* Q, int64_t ldq, int64_t cap,
             double* R, int64_t ldr, void* stream, sqr_info* info);

/*
 * sqr_orth_noalloc -- for callers that cannot allocate device memory (code
 * that a HIP graph captures, tight serving loops, harnesses that forbid
 * hipMalloc): the computation of sqr_orth (same kernels, same options; with
 * the same slot count the result is bit for bit that of sqr_orth) without a
 * handle, without pinned host memory and without any hipMalloc/hipFree.
 * Its workspace (partial Gramians, small matrices, control block) is one
 * static device array of SQR_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * first call on that GPU until the process ends.
 *
 *   A, lda   m x n input (n <= SQR_NOALLOC_MAX_COLS), read only.
 *   Q, ldq   m x n output; R, ldr: n x n output (ldr >= n), as in sqr_orth.
 *   stream   hipStream_t; every pass up to max_iter is enqueued (passes
 *            after the device's decision exit at once).
 *   info     NULL: nothing waits, the call only enqueues work; non-NULL:
 *            the outcome is copied from the device and the stream is
 *            synchronised (not allowed during stream capture).
 *
 * All calls on one GPU share its scratch array and the array keeps the last
 * call's contents (every call starts from its own cleared state): calls that
 * overlap on one GPU -- on different streams, or from different host threads
 * without ordering -- race and give wrong results.  Order them on one stream.
 * The first call on a device looks the array up (hipGetSymbolAddress); make
 * it outside any stream capture.
 * Errors: SQR_ENULL, SQR_EDIM (as sqr_orth with cap = n), SQR_ELIMIT
 * (n > SQR_NOALLOC_MAX_COLS), SQR_EOPT, SQR_EHIP; all before any work is
 * enqueued, except SQR_EHIP from a failed launch.
 */
int sqr_orth_noalloc(const sqr_opts* opts, int64_t m, int64_t n, const double* A, int64_t lda,
                     double* Q, int64_t ldq, double* R, int64_t ldr, void* stream,
                     sqr_info* info);

/*
 * sqr_append -- Algorithm 2: extend the basis Q[:, 0:n] of handle b by the p
 * columns of W (m x p, ldw >= m), writing the new columns to Q[:, n:n+p] and
 * R[0:n+p, n:n+p] (B above R, Prop. 2.1).  On SQR_OK the handle's n grows by
 * p.  On any non-zero status n is unchanged (the reserved columns may hold
 * partial results).  W is read only.  Always waits for the outcome, as
 * sqr_orth does with a non-NULL info (the new width depends on it); `info`
 * may be NULL.  At least one pass runs, so the projection of Prop. 2.1 is
 * applied even when the initial Schur complement already passes the
 * stopping test (W = Q_in C + H, H orthonormal and orthogonal to Q_in).
 * Widths: up to cap (16384).  While the basis and the block fit in 36 tiles
 * of 16 columns (n rounded up to 16, plus p rounded up to 16, at most 576),
 * each pass streams Q_in once per 16-column block of W; a wider basis takes
 * the wide-basis route, which reads Q_in twice per pass (Q_in^T W and
 * W - Q_in B~ as separate tall products).  A block of more than 528 columns
 * is handled as in sqr_orth; the first such block larger than the handle's
 * workspace serves makes the call wait for the handle's earlier work and
 * take a larger workspace.  All routes compute the same method.
 * Errors: SQR_ENULL, SQR_EDIM (p < 1, ldw < m, ldw > 2^25 - 1, n + p > cap,
 * n + p > m).
 */
int sqr_append(sqr_basis* b, const double* W, int64_t p, int64_t ldw,
               void* stream, sqr_info* info);

/*
 * sqr_panel -- Algorithm 3 (pnCholQR, the panel scheme of Sec. 2.3): split A
 * (m x n) into r panels of nearly equal width, columns [e_i, e_{i+1}) with
 * e_i = i n / r rounded to the nearest integer (ties to even), and apply
 * Algorithm 2 to each in turn, starting from an empty basis (the first panel
 * is Algorithm 2 with q = 0: its first shift is the 2u floor).
 *
 *   out, opts, A, lda, Q, ldq, cap, R, ldr, stream: as sqr_orth; A is read
 *            only, Q[:, 0:n] and R[0:n, 0:n] receive the factors.
 *   r        number of panels, 1 <= r <= n.
 *   info     outcome of the last panel's call (required to be waited for:
 *            every panel waits for the device's decision).
 * On a non-zero status of panel i the handle keeps the basis of panels
 * 0..i-1 (sqr_cols tells its width) and the later panels are not run.
 * Widths: n up to cap (16384), panels of any width (as sqr_append).
 * Errors: as sqr_orth, and SQR_EDIM for r < 1 or r > n, SQR_EOPT for
 * precision 1 (the append always runs in FP64).
 */
int sqr_panel(sqr_basis** out, const sqr_opts* opts, int64_t m, int64_t n, const double* A, int64_t lda,
              int64_t r, double* Q, int64_t ldq, int64_t cap, double* R, int64_t ldr, void* stream,
              sqr_info* info);

/* Outcome of the handle's last sqr_orth / sqr_append call; synchronises the
 * stream of that call.  Returns the status, or SQR_ENULL. */
int sqr_last_info(sqr_basis* b, sqr_info* info);

/* Current basis width n of the handle (0 for NULL). */
int64_t sqr_cols(const sqr_basis* b);

/* Release the handle and its workspace after the work on its stream ends.
 * Caller buffers are not touched.  NULL is a no-op. */
void sqr_free(sqr_basis* b);

/* Return the handle's workspace (partial-Gramian slots, small-matrix arena,
 * pinned state) to the library's pool once the work on its stream has ended,
 * keeping the handle, its basis width and its last outcome (sqr_last_info
 * still answers).  The next sqr_append takes a workspace from the pool again
 * (or allocates one).  For servers that keep many bases resident between
 * calls: idle handles then hold no scratch memory.  The pool keeps at most 16
 * workspaces per process, releasing the smallest first.
 * Returns SQR_OK, SQR_ENULL or SQR_EHIP (the stream reported an error). */
int sqr_park(sqr_basis* b);

#ifdef __cplusplus
}
#endif

#endif /* SQR_H */
