// sqr_device.h -- argument blocks shared by the HIP kernels and the host
// driver of libsqr (not part of the public ABI).
#pragma once
#include <stdint.h>

namespace sqr {

// Largest block width p handled by small_step's LDS vectors, and largest
// number of columns of S (basis plus same-pass prefix) in one block launch.
constexpr int kMaxCols = 1024;
constexpr int kMaxSCols = 528;
// Blocks wider than kMaxSCols are applied in superblocks of kSuper columns
// (block_pass inside a superblock, proj_pass for the earlier ones); the C_J
// of one superblock take kSuperBneg doubles (16-column blocks 0..31).
constexpr int kSuper = 128;
constexpr int64_t kSuperBneg = 16 * 8 * (int64_t)(kSuper / 16) * (kSuper / 16 - 1);

// Device-resident state of one sqr_orth / sqr_append call.  Kernels read
// `done` first and exit at once when it is set, so the host may enqueue more
// passes than the method needs without waiting for the device.
struct Ctrl {
  int32_t done;           // 1 once the call converged or failed
  int32_t status;         // SQR_* code
  int32_t passes;         // Cholesky QR passes executed so far
  int32_t chol_attempts;  // factorisations tried, failed ones included
  int32_t converged;
  int32_t gram32;         // mixed form: the next pass forms an FP32 Gramian
  int32_t chol_fail;      // blocks wider than kMaxSCols: the factorisation
                          // run by the band kernels met a breakdown
  int32_t att_shifted;    // ... and whether its diagonal was shifted
  double orth_fro;        // last ||X - I||_F
  double sigma[16];       // shift of each pass (0 = unshifted)
  double sigma_fixed;     // isCholQR: the shift of the input Gramian
  double att_sigma;       // the shift of that factorisation
  int64_t stamp;          // host copy only: call id * 256 + phase of the last
                          // small_step that published this state
};

// One launch of block_pass: 16-column block J of a pass.
struct BlockPassArgs {
  const double* win;  int64_t ldw;   // input block (pb real columns)
  double* yout;       int64_t ldy;   // output block (apply mode)
  const double* s1;   int64_t ld1;  int32_t n1;   // basis segment of S
  const double* s2;   int64_t ld2;  int32_t n2;   // same-pass prefix of S
  int32_t pb;                         // real columns of the block (1..16)
  int64_t m;                          // rows
  const double* bneg;                 // (n1 rounded up to 16, + n2) x 16, row-major: C_J
  const double* rinv;                 // 16 x 16 row-major inverse of the diagonal block
  double* part; int64_t part_stride; int64_t part_off;  // slot b at part + b*stride + off
  const int32_t* done;                // NULL in the initial Gram pass of a call
  const int32_t* passes;
  int32_t copy_if_done;
};

// One launch of wide_pass: a whole pass of an orth call with 2..8 blocks.
struct WidePassArgs {
  const double* win;  int64_t ldw;   // input (m x n)
  double* yout;       int64_t ldy;   // output (apply mode; may equal win)
  int32_t n;                          // columns, 16 (NB - 1) < n <= 16 NB
  int64_t m;
  const double* bneg;                 // C_J of each block, row-major (16 J x 16)
  const double* rinv;                 // D_J of each block, 16 x 16 row-major
  double* part; int64_t part_stride;  // slot b at part + b * part_stride
  const int32_t* done;                // NULL in the initial Gram pass of a call
  const int32_t* passes;
  int32_t copy_if_done;
  // mixed form: the launch runs only if *gram32 equals the variant's Gramian
  // precision (1 = FP32); NULL: it always runs
  const int32_t* gram32;
  // narrow_pass apply: the input is multiplied by `levels` inverse factors in
  // turn (rinv + 256 l, l = 0 .. levels - 1), so a pass can recompute its
  // input from A instead of reading the previous pass's result; `store`
  // writes the result (passes that cannot end the call skip it)
  int32_t levels, store;
};

// Slots of inverse factors kept by the one-block orthogonalisation: the
// factor used by pass k is in slot min(k - 1, kNarrowSlots - 1), and passes
// up to kNarrowSlots - 1 recompute their input from A through slots 0 .. k-1.
constexpr int kNarrowSlots = 4;

// One launch of reduce_slots: sum nslots partial slots (stride doubles apart)
// of len doubles each into out, in a fixed order.
struct ReduceArgs {
  const double* in; int64_t stride; int64_t len;
  double* out;
  const int32_t* done;   // NULL in the initial Gram pass of a call
  int32_t nslots;
};

// Appends whose basis is too wide for block_pass's S (more than kBlockTiles
// 16-column tiles with the block): the basis part of a pass runs as
// GEMM-shaped launches.  B~ is kept row-major, rows16 = q rounded up to 16
// rows of `pitch` = p rounded up to 16 doubles (padding rows and columns 0).
constexpr int kBlockTiles = 36;

// cross_pass: partial B~ = X^T Y over one row chunk per slot.
struct CrossArgs {
  const double* x; int64_t ldx; int32_t nx;   // m x nx basis (Q_in)
  const double* y; int64_t ldy; int32_t ny;   // m x ny block
  int64_t m;
  double* part; int64_t part_stride;          // slot s: part + s * part_stride
  int32_t pitch, rows16;
  int32_t tiles_b;                            // column tiles of 16 NB
  int32_t ntiles;                             // row tiles (of 128) * tiles_b
  int32_t nslots;
  int32_t sym;                                // X = Y: tiles strictly below the
                                              // diagonal are skipped (not written)
  const int32_t* done;                        // NULL in the initial Gram pass
};

// proj_pass: Z = W - X T (Z may be W), T row-major with row stride ldt:
// rows16 rows (B~ of an append: q rounded up to 16, padding rows zero; a
// superblock: the rows of R~ above it) and p columns.
struct ProjArgs {
  const double* win; int64_t ldw;
  double* yout; int64_t ldy;
  const double* x; int64_t ldx; int32_t nx;
  const double* bt; int64_t ldt; int32_t rows16;
  int32_t p;
  int64_t m;
  int32_t tiles_b;
  const int32_t* done;
};

// btb_pass: out = B~^T B~ (p x p, row-major, both triangles).
struct BtbArgs {
  const double* bt; int32_t pitch, rows16, p;
  double* out;
  const int32_t* done;
};

// bacc_pass: B <- B + B~ R_old (B = R[0:q, q:q+p]); at phase 0 B <- B~ and
// the block R[q:q+p, 0:q] <- 0.
struct BaccArgs {
  const double* bt; int32_t pitch;
  const double* rold;                 // p x p row-major (upper triangular)
  double* R; int64_t ldr;
  int32_t q, p, phase;
  const int32_t* done;
};

// The kernels around small_step for blocks wider than kMaxSCols (p x p
// row-major matrices in the workspace).
struct BigArgs {
  double* X;              // the Schur complement (symmetric)
  double* M;              // X + sigma I, then its upper Cholesky factor
  int32_t p;
  int32_t k0;             // chol_*: first row of the band
  Ctrl* ctrl;
  double* rinv;           // inverses of the 16x16 diagonal blocks
  double* rold;           // R_old (the identity at phase 0)
  double* R; int64_t ldr; int32_t q; int32_t phase;
  double* rt;             // R~ row-major, zero below the diagonal
  double* bneg;           // C_J per superblock
  // xfill_pass: X = G - B~^T B~ from the reduced Gramian E (row-major, pitch
  // p rounded up to 16, upper tiles valid) and btb (appends), and one partial
  // sum of squares of X - I per workgroup
  const double* E;
  const double* btb;      // NULL without a basis
  double* errpart;
};

// Argument table of a batched launch: call c owns workgroups start[c] ..
// start[c+1]-1 of the grid and reads args[c] (device memory).
template <class T>
struct BatchTable {
  const T* args;
  const int32_t* start;   // ncalls + 1 entries
  int32_t ncalls;
};

// One launch of small_step: finish a pass of an orth or append call.
struct SmallArgs {
  const double* E;       // reduced partial Gramians of the pass, block after block
  int32_t mode;          // 0 = orth (Algorithm 1, CholQR3 start), 1 = append (Algorithm 2)
  int32_t q;             // basis width (append), 0 for orth
  int32_t p;             // block width being orthogonalised
  int32_t nblk;          // 16-column blocks of p
  int64_t m;
  int32_t phase;         // 0 = after the initial Gram, k = after pass k
  // caller R (column-major, ldr): orth uses R[0:p,0:p]; append writes
  // B = R[0:q, q:q+p] and the new diagonal block R[q:q+p, q:q+p]
  double* R; int64_t ldr;
  // workspace arena for the small matrices when they do not fit in LDS:
  // X, M, old R block (p x p each), B~ (q x p), scratch (row-major)
  double* X;
  double* bneg;          // per block J: (q + 16J rounded up to 4) x 16, row-major
  double* rinv;          // per block J: 16 x 16
  Ctrl* ctrl;
  Ctrl* hctrl;           // pinned host mirror (device address), or NULL
  int64_t stamp_base;    // call id * 256
  int32_t publish_from;  // first phase whose state the host waits for
  // options
  int32_t first_pass_shift, min_passes, max_iter, max_escalations, power_steps;
  int32_t shift_policy;  // orth: 0 recompute (Algorithm 1), 1 none, 2 fixed
  int32_t shift_dim;     // append: first shift with 0 q, 1 p, 2 q + p
  double tol, u;
  int32_t mixed;         // orth in the mixed FP32/FP64 form
  int32_t lds_matrices;  // 1: the small matrices live in LDS, not in X;
                         // 2: only the factor M (p x p) lives in LDS
  // ext bit 0 (the basis part outside, an append with a wide basis):
  // B~^T B~ from btb_pass, and where the old diagonal block of R goes for
  // bacc_pass.  ext bit 1 (a block wider than kMaxSCols): E is one row-major
  // Gramian, R~ is written to rt (row-major p x p) for proj_pass.
  int32_t ext;
  // blocks wider than kMaxSCols: 0 = the whole step; 1 = up to the shift of
  // the first factorisation (the band kernels factor X + sigma I); 2 = from
  // that factorisation's outcome on (further attempts in this workgroup; the
  // R update and C_J by trmm_pass / cj_pass)
  int32_t stage;
  const double* btb;
  double* rold;
  double* rt;
  double* vec;           // 2 p doubles for blocks wider than kMaxCols
  // ext bit 1: X already formed by xfill_pass, with nerr partial sums of
  // squares of X - I (0: this kernel forms X)
  const double* errpart;
  int32_t nerr;
};

}  // namespace sqr
