// sqr_api.hip -- host driver of libsqr: the C ABI declared in include/sqr.h.
//
// A call enqueues, on the caller's stream, an initial Gram pass and then
// Cholesky QR passes: the streaming kernels of the pass, a fixed-order
// reduction of the per-workgroup partial Gramians (reduce_slots) and one
// small_step.  The streaming kernels of a pass, by call and width (16-column
// blocks P):
//   orth, P = 1              narrow_pass (apply and Gramian in one launch;
//                            FP32 Gramian variant for the mixed form)
//   orth, P = 2..7           wide_pass (one launch per pass)
//   orth, P = 8..16          wide_apply, then gram_pass (FP32 variant for
//                            the mixed form's early passes)
//   appends; orth, P > 16    block_pass, one launch per block
// The convergence decision is taken on the device; kernels of later passes
// exit at once after it.  With a host `info` the driver enqueues the passes
// the method normally needs, reads the device state once, and adds passes
// only when the device asks for them.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <mutex>
#include <vector>

#include "../../include/sqr.h"
#include "../../include/sqr_prof.h"
#include "../../include/sqr_batch.h"

#include "sqr_kernels.hip"

using namespace sqr;

namespace {

constexpr int kMaxSlots = 1024;
// Largest column capacity of a handle (appends beyond kMaxSCols columns run
// with the wide-basis route), and the bytes of cross_pass slots per handle.
constexpr int64_t kMaxCap = 16384;
constexpr size_t kCrossBudget = 512ull << 20;
// bytes of cross_pass slots for the Gramian of a block wider than kMaxSCols
constexpr size_t kGramBudget = 4ull << 30;
// workgroups a cross_pass launch aims at (about eight per CU)
constexpr int64_t kCrossWant = 2048;
// Leading dimensions below 2^25 keep every per-lane buffer offset inside a
// 16-column tile, (15 ld + m) * 8 bytes, below 4 GiB.
constexpr int64_t kMaxLd = ((int64_t)1 << 25) - 1;
constexpr size_t kPartBudget = 256ull << 20;   // bytes of partial slots per handle
// small_step arena in LDS up to this (its static LDS, about 25 KB, comes on top)
constexpr size_t kSmallLdsBytes = 128 * 1024;
size_t g_small_lds = kSmallLdsBytes;

// ---- measurement records (sqr_prof.h) ----
struct ProfRec { hipEvent_t e0, e1; int kind; double bytes; int64_t call; int phase; int real; };
std::vector<ProfRec> g_prof;             // guarded by g_prof_mu
std::vector<hipEvent_t> g_event_pool;    // guarded by g_prof_mu
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::atomic<int64_t> g_call_id{0};

// Caller holds g_prof_mu.
hipEvent_t take_event() {
  if (g_event_pool.empty()) {
    // timing only: no system-scope fence (cache writeback) at the record,
    // which would otherwise stall the stream between the measured kernels;
    // the records are read after the stream has been synchronised
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = g_event_pool.back();
  g_event_pool.pop_back();
  return e;
}

// Mark the records of call `id`: launches of passes after the last executed
// one were no-ops of a finished call.
void prof_finalize(int64_t id, int passes) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (ProfRec& r : g_prof)
    if (r.call == id && r.real < 0) r.real = (r.phase <= passes) ? 1 : 0;
}

// Event pair around the launches of one streaming step (when recording).
ProfRec prof_begin(int kind, double bytes, int64_t call, int phase, hipStream_t s) {
  ProfRec rec{};
  if (!g_prof_on || call < 0) return rec;   // call < 0: a call that records nothing
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    rec.e0 = take_event();
    rec.e1 = take_event();
  }
  rec.kind = kind; rec.bytes = bytes; rec.call = call; rec.phase = phase; rec.real = -1;
  if (rec.e0) (void)hipEventRecord(rec.e0, s);
  return rec;
}
void prof_end(const ProfRec& rec, hipStream_t s) {
  if (!rec.e0 || !rec.e1) return;
  (void)hipEventRecord(rec.e1, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(rec);
}

// ---- workspace pool: device buffers (and the pinned state) of freed or
// parked handles are kept for later handles on the same device; at most
// kPoolEntries are held, the smallest are released first ----
std::mutex g_cache_mu;
struct CachedWs { void* ptr = nullptr; size_t bytes = 0; int device = -1; void* pinned = nullptr; };
std::vector<CachedWs> g_pool;
constexpr size_t kPoolEntries = 16;

bool pool_take(int device, size_t need, CachedWs* out) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  int best = -1;
  for (int i = 0; i < (int)g_pool.size(); ++i)
    if (g_pool[i].device == device && g_pool[i].bytes >= need &&
        (best < 0 || g_pool[i].bytes < g_pool[best].bytes))
      best = i;
  if (best < 0) return false;
  *out = g_pool[best];
  g_pool.erase(g_pool.begin() + best);
  return true;
}

void pool_put(const CachedWs& e) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_pool.push_back(e);
  while (g_pool.size() > kPoolEntries) {
    int small = 0;
    for (int i = 1; i < (int)g_pool.size(); ++i)
      if (g_pool[i].bytes < g_pool[small].bytes) small = i;
    (void)hipFree(g_pool[small].ptr);
    if (g_pool[small].pinned) (void)hipHostFree(g_pool[small].pinned);
    g_pool.erase(g_pool.begin() + small);
  }
}

int64_t round4(int64_t v) { return (v + 3) & ~int64_t(3); }
// The basis segment of S is padded to whole 16-column tiles.
int64_t round16(int64_t v) { return (v + 15) & ~int64_t(15); }
int64_t nblocks(int64_t p) { return (p + 15) / 16; }
// Doubles of the reduced partial Gramians of a call with basis q and block p.
int64_t total_len(int64_t q, int64_t p) {
  const int64_t P = nblocks(p);
  return 16 * (P * (round16(q) + 16) + 8 * P * (P - 1));
}
int64_t e_off(int64_t q, int64_t J) { return 16 * (J * (round16(q) + 16) + 8 * J * (J - 1)); }
int64_t bneg_off(int64_t q, int64_t J) { return 16 * (J * round16(q) + 8 * J * (J - 1)); }
int64_t bneg_len(int64_t q, int64_t p) { return bneg_off(q, nblocks(p)); }
// Widest basis an append with block p can have on block_pass (S = basis
// tiles plus the block's tiles, at most kBlockTiles); wider bases take the
// wide-basis route (mode 2 of small_step).
int64_t q_fit(int64_t p) { return 16 * (int64_t)kBlockTiles - 16 * nblocks(p); }
bool wide_basis(int64_t q, int64_t p) { return q > q_fit(p); }
// Blocks that take the wide-block route (Gramian by cross_pass, apply in
// superblocks): those wider than kMaxSCols.  (Between 256 and 528 columns
// the per-block route measured faster or equal.)
bool big_block(int64_t p) { return p > kMaxSCols; }

}  // namespace

struct sqr_basis {
  int64_t m = 0, n = 0, cap = 0;
  double* Q = nullptr; int64_t ldq = 0;
  double* R = nullptr; int64_t ldr = 0;
  sqr_opts opts;
  int device = 0;
  hipStream_t stream = nullptr;      // stream of the last call
  bool used = false;                 // a call has been enqueued on `stream`
  hipEvent_t order_ev = nullptr;     // orders a call after the previous one
  int64_t call_id = 0;               // id of the last call (measurement records)
  size_t ws_bytes = 0;
  int slots = 0;                     // partial-Gram slots (workgroups of block_pass)
  void* ws = nullptr;
  Ctrl* ctrl = nullptr;
  Ctrl last{};                       // outcome of the last call (kept while parked)
  bool parked = false;               // workspace returned to the pool
  bool noprof = false;               // never recorded by the profiling hooks
  int publish_from = 0;              // first phase the host waits for (small_step
                                     // publishes its state from there on, and at the end)
  Ctrl* ctrl_host = nullptr;         // pinned, written by small_step
  Ctrl* ctrl_host_dev = nullptr;     // its device address
  double *part = nullptr, *stage = nullptr;
  double *X = nullptr;
  double *bneg = nullptr, *rinv = nullptr;
  // wide-basis appends: cross_pass slots, reduced B~, B~^T B~, R_old
  int slots_c = 0;
  double *partc = nullptr, *stage_bt = nullptr, *btb = nullptr, *rold = nullptr;
  // blocks wider than kMaxSCols (up to pbig columns): cross_pass slots of the
  // Gramian, the reduced Gramian, R~ (row-major), vectors of the small step
  int slots_g = 0;
  int64_t pbig = 0;
  double *partg = nullptr, *stage_g = nullptr, *rt = nullptr, *vec = nullptr;
  double* errpart = nullptr;         // xfill_pass: one partial sum per tile
};

namespace {

typedef void (*BlockKernel)(BlockPassArgs);
typedef void (*BlockBatchKernel)(BatchTable<BlockPassArgs>);
// nt = S tiles per wave, wpt = waves sharing a row tile (4 / wpt row tiles
// in flight per workgroup); a variant covers nt * wpt tiles of S.  Every
// kernel comes with its batched form (the same work for several calls in one
// launch).  The Gram-only pass takes two waves per row tile up to 12 tiles of
// S (two row tiles in flight per workgroup; measured 7 % faster than four
// waves per tile on the growth workload), the apply four from 5 tiles on (its
// members' partial Y meet at a barrier every step; fewer, wider members
// measured slower).  Variants that serve only the Gram-only pass have no
// apply kernel.
struct Variant { int nt, wpt; BlockKernel gram, apply; BlockBatchKernel gram_b, apply_b; };
int g_occ[2][32];     // workgroups per CU of each variant (gram, apply)
int g_ncu = 0;
#define SQR_VARIANT(NT, W) {NT, W, block_pass<NT, W, false>, block_pass<NT, W, true>, \
                            block_pass_batch<NT, W, false>, block_pass_batch<NT, W, true>}
#define SQR_GVARIANT(NT, W) {NT, W, block_pass<NT, W, false>, nullptr, \
                             block_pass_batch<NT, W, false>, nullptr}
const Variant kVariants[] = {
  SQR_VARIANT(1, 1), SQR_VARIANT(1, 2), SQR_VARIANT(2, 2),
  SQR_GVARIANT(3, 2), SQR_GVARIANT(4, 2), SQR_GVARIANT(5, 2), SQR_GVARIANT(6, 2),
  SQR_VARIANT(2, 4), SQR_VARIANT(3, 4), SQR_VARIANT(4, 4), SQR_VARIANT(5, 4),
  SQR_VARIANT(6, 4), SQR_VARIANT(7, 4), SQR_VARIANT(8, 4), SQR_VARIANT(9, 4),
};
#undef SQR_VARIANT
#undef SQR_GVARIANT

// Whole-pass kernels of orth calls with up to 8 column blocks (FP64 calls use
// them from 2 blocks on; the mixed form from 1), with FP64 or FP32 Gramians.
typedef void (*WideKernel)(WidePassArgs);
typedef void (*WideBatchKernel)(BatchTable<WidePassArgs>);
struct WideVariant { WideKernel k[2][2]; WideBatchKernel kb[2][2]; };   // [fp32 gram][apply]
#define SQR_WIDE(NB) {{{wide_pass<NB, false, false>, wide_pass<NB, true, false>}, \
                       {wide_pass<NB, false, true>, wide_pass<NB, true, true>}}, \
                      {{wide_pass_batch<NB, false, false>, wide_pass_batch<NB, true, false>}, \
                       {wide_pass_batch<NB, false, true>, wide_pass_batch<NB, true, true>}}}
constexpr int kWideMin = 1, kWideMax = 8;
const WideVariant kWide[] = {SQR_WIDE(1), SQR_WIDE(2), SQR_WIDE(3), SQR_WIDE(4),
                             SQR_WIDE(5), SQR_WIDE(6), SQR_WIDE(7), SQR_WIDE(8)};
#undef SQR_WIDE
int g_wide_occ[2][2][kWideMax - kWideMin + 1];   // [fp32][apply][nb]

// FP64 orth calls of one block (at most 16 columns): [Gram only, apply].
const WideKernel kNarrow[2][2] = {{narrow_pass<false, false>, narrow_pass<true, false>},     // FP64 Gramian
                                  {narrow_pass<false, true>, narrow_pass<true, true>}};      // FP32
const WideBatchKernel kNarrowB[2][2] = {{narrow_pass_batch<false, false>, narrow_pass_batch<true, false>},
                                        {narrow_pass_batch<false, true>, narrow_pass_batch<true, true>}};
int g_narrow_occ[2];   // [apply]: the smaller of the two Gramian precisions

// Orth calls of 8..16 blocks: a whole-pass apply and a Gramian kernel
// (FP64, and FP32 for the mixed form).
typedef void (*SplitKernel)(WidePassArgs);
struct SplitVariant { SplitKernel apply, gram, gram32; WideBatchKernel apply_b, gram_b, gram32_b; };
#define SQR_SPLIT(NB) {wide_apply<NB>, gram_pass<NB, false>, gram_pass<NB, true>, \
                       wide_apply_batch<NB>, gram_pass_batch<NB, false>, gram_pass_batch<NB, true>}
constexpr int kSplitMin = 8, kSplitMax = 16;
const SplitVariant kSplit[] = {SQR_SPLIT(8), SQR_SPLIT(9), SQR_SPLIT(10), SQR_SPLIT(11), SQR_SPLIT(12),
                               SQR_SPLIT(13), SQR_SPLIT(14), SQR_SPLIT(15), SQR_SPLIT(16)};
#undef SQR_SPLIT
int g_split_occ[3][kSplitMax - kSplitMin + 1];   // [0 gram, 1 apply, 2 gram32][nb]

// Wide-basis appends: cross_pass / proj_pass by block columns per tile (1..8).
typedef void (*CrossKernel)(CrossArgs);
typedef void (*ProjKernel)(ProjArgs);
const CrossKernel kCross[8] = {cross_pass<1>, cross_pass<2>, cross_pass<3>, cross_pass<4>,
                               cross_pass<5>, cross_pass<6>, cross_pass<7>, cross_pass<8>};
const ProjKernel kProj[8] = {proj_pass<1>, proj_pass<2>, proj_pass<3>, proj_pass<4>,
                             proj_pass<5>, proj_pass<6>, proj_pass<7>, proj_pass<8>};
size_t split_lds_bytes(int nb, bool apply) {
  return 8 * (size_t)(apply ? apply_lds_doubles(nb) : gram_op_doubles(nb));
}
size_t gram32_lds_bytes(int nb) { return 4 * (size_t)gram_op_doubles(nb); }
size_t wide_lds_bytes(int nb, bool apply) {
  return 8 * ((size_t)(apply ? wide_panel_doubles(nb) : 0) + (size_t)wide_op_doubles(nb));
}

// Smallest variant of the pass kind whose S capacity covers ns tiles (each
// kind's variants are listed by capacity).
const Variant* pick_variant(int ns, bool apply) {
  for (const Variant& v : kVariants) {
    if (apply ? !v.apply : (v.wpt == 4 && v.nt <= 3)) continue;
    if (v.nt * v.wpt >= std::max(ns, 1)) return &v;
  }
  return nullptr;
}

size_t block_lds_bytes(const Variant& v, bool apply) {
  // main loop: partial T tiles + transposition tiles; the apply adds its
  // operands C_J (16 nt wpt rows) and D_J.  The final cross-group reduction
  // (groups x (nt wpt + 1) tiles) reuses the area from its start.
  const size_t groups = kWaves / v.wpt;
  const size_t red = groups > 1 ? groups * (size_t)(v.nt * v.wpt + 1) * kTPart : 0;
  const size_t loop = (size_t)2 * kWaves * kTPart + (size_t)kWaves * 16 * kYPitch +
                      (apply ? (size_t)v.nt * v.wpt * 256 + 256 : 0);
  return 8 * std::max(loop, red);
}

// Kernel attributes and occupancies, once per process (std::call_once: the
// serving loop calls the library from several threads at once).
std::once_flag g_attr_once;
void set_kernel_attributes_once() {
  auto lds_attr = [](const void* k, int bytes) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
  for (const Variant& v : kVariants) {
    lds_attr((const void*)v.gram, 120 * 1024);
    lds_attr((const void*)v.gram_b, 120 * 1024);
    if (v.apply) {
      lds_attr((const void*)v.apply, 120 * 1024);
      lds_attr((const void*)v.apply_b, 120 * 1024);
    }
  }
  if (hipFuncSetAttribute((const void*)small_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kSmallLdsBytes) != hipSuccess ||
      hipFuncSetAttribute((const void*)small_step_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kSmallLdsBytes) != hipSuccess) {
    (void)hipGetLastError();   // consumed here: arenas then live in the workspace
    g_small_lds = 0;
  }
  for (int nb = kWideMin; nb <= kWideMax; ++nb)
    for (int g32 = 0; g32 < 2; ++g32)
      for (int ap = 0; ap < 2; ++ap) {
        lds_attr((const void*)kWide[nb - kWideMin].k[g32][ap], (int)wide_lds_bytes(nb, ap != 0));
        lds_attr((const void*)kWide[nb - kWideMin].kb[g32][ap], (int)wide_lds_bytes(nb, ap != 0));
      }
  for (int nb = kSplitMin; nb <= kSplitMax; ++nb) {
    const SplitVariant& v = kSplit[nb - kSplitMin];
    lds_attr((const void*)v.apply, (int)split_lds_bytes(nb, true));
    lds_attr((const void*)v.gram, (int)split_lds_bytes(nb, false));
    lds_attr((const void*)v.gram32, (int)gram32_lds_bytes(nb));
    lds_attr((const void*)v.apply_b, (int)split_lds_bytes(nb, true));
    lds_attr((const void*)v.gram_b, (int)split_lds_bytes(nb, false));
    lds_attr((const void*)v.gram32_b, (int)gram32_lds_bytes(nb));
  }
  for (int nb = 1; nb <= 8; ++nb) {
    lds_attr((const void*)kCross[nb - 1], 8 * cross_lds_doubles(nb));
    lds_attr((const void*)kProj[nb - 1], 8 * proj_lds_doubles(nb));
  }
  (void)hipGetLastError();
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&g_ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      g_ncu < 1)
    g_ncu = 256;
  int i = 0;
  for (const Variant& v : kVariants) {
    for (int ap = 0; ap < 2; ++ap) {
      int n = 1;
      if (ap && !v.apply) {   // a Gram-only variant
        g_occ[ap][i] = 1;
        continue;
      }
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)(ap ? v.apply : v.gram),
                                                        kThreads, block_lds_bytes(v, ap != 0)) != hipSuccess ||
          n < 1)
        n = 1;
      g_occ[ap][i] = n;
    }
    ++i;
  }
  for (int nb = kWideMin; nb <= kWideMax; ++nb)
    for (int g32 = 0; g32 < 2; ++g32)
      for (int ap = 0; ap < 2; ++ap) {
        int n = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, (const void*)kWide[nb - kWideMin].k[g32][ap], kThreads,
                wide_lds_bytes(nb, ap != 0)) != hipSuccess ||
            n < 1)
          n = 1;
        g_wide_occ[g32][ap][nb - kWideMin] = n;
      }
  for (int nb = kSplitMin; nb <= kSplitMax; ++nb) {
    int n = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)kSplit[nb - kSplitMin].apply,
                                                      kThreads, split_lds_bytes(nb, true)) != hipSuccess ||
        n < 1)
      n = 1;
    g_split_occ[1][nb - kSplitMin] = n;
    n = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)kSplit[nb - kSplitMin].gram,
                                                      kGramThreads, split_lds_bytes(nb, false)) != hipSuccess ||
        n < 1)
      n = 1;
    g_split_occ[0][nb - kSplitMin] = n;
    n = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)kSplit[nb - kSplitMin].gram32,
                                                      kGramThreads, gram32_lds_bytes(nb)) != hipSuccess ||
        n < 1)
      n = 1;
    g_split_occ[2][nb - kSplitMin] = n;
  }
  for (int ap = 0; ap < 2; ++ap) {
    g_narrow_occ[ap] = 1 << 30;
    for (int g32 = 0; g32 < 2; ++g32) {
      int n = 1;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)kNarrow[g32][ap], kThreads, 0) != hipSuccess ||
          n < 1)
        n = 1;
      g_narrow_occ[ap] = std::min(g_narrow_occ[ap], n);
    }
  }
}
void set_kernel_attributes() { std::call_once(g_attr_once, set_kernel_attributes_once); }

// Sizes (doubles) of the workspace regions of a handle.  bt, pp and slots_c
// serve appends with a wide basis; g, rt, vec and slots_g blocks wider than
// kMaxSCols (zero where the handle never takes that route).
struct WsSizes { int64_t tl, arena, bneg, rinv, bt, pp, g, rt, vec, errp; int slots_c, slots_g; };

// Every call with a block of up to kMaxSCols columns a handle of capacity
// cap can make (q + p <= cap): on block_pass the sizes grow with q, so the
// widest basis that route takes decides; the wide-basis route needs its
// block regions for q = 0 (covered) and B~ for the widest basis.  Blocks
// on the wide-block route are covered up to pbig columns (0: none).
WsSizes handle_sizes(int64_t cap, int64_t pbig) {
  WsSizes z{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t pmax = std::min<int64_t>(cap, kMaxSCols);
  for (int64_t p = 1; p <= pmax; ++p) {
    const int64_t q1 = std::min(cap - p, q_fit(p));
    z.tl = std::max(z.tl, total_len(q1, p));
    z.arena = std::max<int64_t>(z.arena, small_arena((int)q1, (int)p));
    z.bneg = std::max(z.bneg, bneg_len(q1, p));
    if (wide_basis(cap - p, p)) {
      z.bt = std::max(z.bt, round16(cap - p) * round16(p));
      z.pp = std::max(z.pp, p * p);
    }
  }
  z.rinv = std::max<int64_t>(nblocks(pmax), kNarrowSlots) * 256;
  pbig = std::min(pbig, cap);
  if (pbig > 0) {
    // superblocks on block_pass, the Gramian from cross_pass, the small
    // matrices in the workspace; a basis beside the block at most cap - pbig
    const int64_t p = pbig, p16 = round16(p);
    z.tl = std::max(z.tl, total_len(0, kSuper));
    z.arena = std::max<int64_t>(z.arena, small_arena(0, (int)p));
    z.bneg = std::max<int64_t>(z.bneg, ((p + kSuper - 1) / kSuper) * kSuperBneg);
    z.rinv = std::max(z.rinv, nblocks(p) * 256);
    z.g = p16 * p16;
    z.rt = p * p;
    z.vec = p > kMaxCols ? 2 * p : 0;
    z.errp = ((p + 31) / 32) * ((p + 31) / 32);   // xfill_pass partial sums
    z.pp = std::max(z.pp, p * p);   // R_old (and B~^T B~ with a basis)
    if (cap - p > 0) {
      // any block of more than kMaxSCols columns with a basis beside it
      for (int64_t pb = kMaxSCols + 1; pb <= p; ++pb)
        z.bt = std::max(z.bt, round16(cap - pb) * round16(pb));
    }
    z.slots_g = (int)std::max<int64_t>(1, std::min<int64_t>(64, (int64_t)(kGramBudget / (8 * (size_t)z.g))));
  }
  if (z.bt > 0)
    z.slots_c = (int)std::max<int64_t>(1, std::min<int64_t>(64, (int64_t)(kCrossBudget / (8 * (size_t)z.bt))));
  return z;
}

// One orthogonalisation of n <= kMaxSCols columns (no later appends).
WsSizes orth_sizes(int64_t n) {
  return WsSizes{total_len(0, n), small_arena(0, (int)n), bneg_len(0, n),
                 std::max<int64_t>(nblocks(n), kNarrowSlots) * 256, 0, 0, 0, 0, 0, 0, 0, 0};
}

// Partial-Gram slots for m rows: one per resident workgroup at most, within
// the slot budget.
int default_slots(int64_t m, int64_t tl) {
  const int64_t tiles = (m + 15) / 16;
  int64_t slots = std::min<int64_t>(kMaxSlots, (tiles + kWaves - 1) / kWaves);
  slots = std::min<int64_t>(slots, std::max<int64_t>(16, kPartBudget / (8 * tl)));
  return (int)std::max<int64_t>(1, slots);
}

// Lay the regions out from `base` (NULL: only measure); returns the doubles
// used.  Sets the handle's region pointers when base is not NULL.
size_t carve_workspace(sqr_basis* b, double* base, const WsSizes& z, int slots) {
  size_t doubles = 0;
  auto take = [&](int64_t n) { size_t off = doubles; doubles += (size_t)round4(n) + 32; return off; };
  const size_t o_part = take((int64_t)slots * z.tl);
  const size_t o_stage = take(z.tl);        // reduced Gramian blocks of a pass
  const size_t o_X = take(z.arena);
  const size_t o_bneg = take(z.bneg);
  const size_t o_rinv = take(z.rinv);
  const size_t o_ctrl = take((sizeof(Ctrl) + 7) / 8);
  const bool wb = z.bt > 0, big = z.g > 0;
  const size_t o_partc = wb ? take((int64_t)z.slots_c * z.bt) : 0;
  const size_t o_bt = wb ? take(z.bt) : 0;
  const size_t o_btb = z.pp ? take(z.pp) : 0;
  const size_t o_rold = z.pp ? take(z.pp) : 0;
  const size_t o_partg = big ? take((int64_t)z.slots_g * z.g) : 0;
  const size_t o_g = big ? take(z.g) : 0;
  const size_t o_rt = big ? take(z.rt) : 0;
  const size_t o_vec = z.vec ? take(z.vec) : 0;
  const size_t o_errp = z.errp ? take(z.errp) : 0;
  if (base) {
    b->slots = slots;
    b->part = base + o_part; b->stage = base + o_stage;
    b->X = base + o_X;
    b->bneg = base + o_bneg; b->rinv = base + o_rinv;
    b->ctrl = (Ctrl*)(base + o_ctrl);
    b->slots_c = wb ? z.slots_c : 0;
    b->partc = wb ? base + o_partc : nullptr;
    b->stage_bt = wb ? base + o_bt : nullptr;
    b->btb = z.pp ? base + o_btb : nullptr;
    b->rold = z.pp ? base + o_rold : nullptr;
    b->slots_g = big ? z.slots_g : 0;
    b->partg = big ? base + o_partg : nullptr;
    b->stage_g = big ? base + o_g : nullptr;
    b->rt = big ? base + o_rt : nullptr;
    b->vec = z.vec ? base + o_vec : nullptr;
    b->errpart = z.errp ? base + o_errp : nullptr;
  }
  return doubles;
}

// pbig: the widest block above kMaxSCols columns the workspace must serve
// (0: none).
int alloc_workspace(sqr_basis* b, int64_t pbig) {
  const WsSizes z = handle_sizes(b->cap, pbig);
  const int slots = default_slots(b->m, z.tl);
  const size_t doubles = carve_workspace(b, nullptr, z, slots);
  {
    CachedWs e;
    if (pool_take(b->device, doubles * 8, &e)) {
      b->ws = e.ptr; b->ws_bytes = e.bytes;
      b->ctrl_host = (Ctrl*)e.pinned;
    }
  }
  if (!b->ws) {
    if (hipMalloc(&b->ws, doubles * 8) != hipSuccess) { b->ws = nullptr; return SQR_EHIP; }
    b->ws_bytes = doubles * 8;
  }
  carve_workspace(b, (double*)b->ws, z, slots);
  b->pbig = z.g > 0 ? std::min(pbig, b->cap) : 0;
  if (!b->ctrl_host &&
      hipHostMalloc((void**)&b->ctrl_host, sizeof(Ctrl),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    b->ctrl_host = nullptr; return SQR_EHIP;
  }
  memset(b->ctrl_host, 0, sizeof(Ctrl));
  if (hipHostGetDevicePointer((void**)&b->ctrl_host_dev, b->ctrl_host, 0) != hipSuccess)
    return SQR_EHIP;
  return SQR_OK;
}

struct Call {
  int mode;             // 0 orth, 1 append
  int64_t q, p;
  const double* win; int64_t ldw;  // caller input block
  double* y; int64_t ldy;          // output block
};

int variant_index(const Variant* v) { return (int)(v - kVariants); }

// Orthogonalisations of one block (at most 16 columns; FP64 or mixed) run
// whole passes in narrow_pass.
bool narrow_route(const Call& c, int64_t P, bool /*mixed*/) { return c.mode == 0 && P == 1; }
// The first pass that can end the call (and so writes its result): the stop
// test runs from pass min_passes on, the last pass is max_iter; at most
// kNarrowSlots - 1, the passes whose input is recomputed from A.
int narrow_depth(const sqr_opts& o) {
  return std::max(1, std::min({std::max(o.min_passes, 1), kNarrowSlots - 1, o.max_iter}));
}
// Slot of the inverse factor used by pass k (k >= 1).
int narrow_slot(int k) { return std::min(k - 1, kNarrowSlots - 1); }

// One kernel launch of a pass, with its single-call and batched kernels.
struct Launch {
  enum Kind { kBlock, kWide, kReduce, kSmall, kCross, kProj, kBtb, kBacc, kBig } kind;
  const void* k1;          // kernel of one call (arguments by value)
  const void* kb;          // the same kernel for a batch of calls
  union {
    BlockPassArgs bp;
    WidePassArgs wp;
    ReduceArgs ra;
    SmallArgs sa;
    CrossArgs cr;
    ProjArgs pj;
    BtbArgs bb;
    BaccArgs ba;
    BigArgs bg;
  } u;
  int64_t grid;            // workgroups of this call
  int threads;
  size_t lds;              // dynamic LDS bytes
  int prof_kind;           // streaming step record: 0 Gram, 1 apply, -1 none
  double prof_bytes;       // algorithmic bytes of the record
  bool prof_join;          // belongs to the previous launch's record
};

size_t launch_arg_bytes(Launch::Kind k) {
  switch (k) {
    case Launch::kBlock: return sizeof(BlockPassArgs);
    case Launch::kWide: return sizeof(WidePassArgs);
    case Launch::kReduce: return sizeof(ReduceArgs);
    case Launch::kCross: return sizeof(CrossArgs);
    case Launch::kProj: return sizeof(ProjArgs);
    case Launch::kBtb: return sizeof(BtbArgs);
    case Launch::kBacc: return sizeof(BaccArgs);
    case Launch::kBig: return sizeof(BigArgs);
    default: return sizeof(SmallArgs);
  }
}

// Launches of one pass of a call whose block is wider than kMaxSCols columns
// (p <= b->pbig): the apply in superblocks of kSuper columns, Z_K = W_K -
// Q_in B~_K - Y_<K R~_<K,K by proj_pass, then block_pass on the superblock's
// own 16-column blocks; the Gramian of the result (upper tiles) and, for an
// append, B~ = Q_in^T Y by cross_pass; their fixed-order reductions,
// btb_pass, small_step (full-Gramian form) and bacc_pass.
int plan_big(sqr_basis* b, const Call& c, int phase, std::vector<Launch>& out) {
  const int64_t P = nblocks(c.p), p16 = round16(c.p);
  const bool apply = phase > 0;
  const bool basis = c.mode == 1 && c.q > 0;
  const int64_t m = b->m;
  const int64_t tiles = (m + 15) / 16;
  const int64_t steps64 = (tiles + kWaves - 1) / kWaves;
  const int pitch_bt = (int)round16(c.p), rows_bt = (int)round16(c.q);
  const double pass_bytes = 8.0 * (double)m * (double)(c.q + (apply ? 2 : 1) * c.p);
  if (c.p > b->pbig || !b->stage_g || (basis && !b->stage_bt)) return SQR_EDIM;
  bool first = true;   // the pass's streaming launches form one measured record
  auto record = [&](Launch& L) {
    L.prof_kind = apply ? 1 : 0; L.prof_bytes = pass_bytes; L.prof_join = !first;
    first = false;
  };
  auto proj = [&](const double* win, int64_t ldw, double* yout, const double* x, int64_t ldx, int nx,
                  const double* t, int64_t ldt, int rows16, int cols) {
    const int nb8 = (int)std::min<int64_t>(nblocks(cols), 8);
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kProj; L.k1 = (const void*)kProj[nb8 - 1]; L.kb = nullptr;
    ProjArgs& a = L.u.pj;
    a.win = win; a.ldw = ldw; a.yout = yout; a.ldy = c.ldy;
    a.x = x; a.ldx = ldx; a.nx = nx;
    a.bt = t; a.ldt = ldt; a.rows16 = rows16;
    a.p = cols; a.m = m;
    a.tiles_b = (int)((nblocks(cols) + nb8 - 1) / nb8);
    a.done = &b->ctrl->done;
    L.grid = ((m + kProjRows - 1) / kProjRows) * a.tiles_b; L.threads = kThreads; L.lds = 8 * (size_t)proj_lds_doubles(nb8);
    record(L);
    out.push_back(L);
  };
  if (apply) {
    // where Z lives: the caller's block until something has been written
    const bool from_y0 = phase > 1 || basis;
    if (basis)
      proj(phase > 1 ? c.y : c.win, phase > 1 ? c.ldy : c.ldw, c.y, b->Q, b->ldq, (int)c.q,
           b->stage_bt, pitch_bt, rows_bt, (int)c.p);
    for (int64_t k0 = 0; k0 < c.p; k0 += kSuper) {
      const int64_t w = std::min<int64_t>(kSuper, c.p - k0), PK = nblocks(w);
      const bool from_y = from_y0 || k0 > 0;
      if (k0 > 0)
        proj(from_y0 ? c.y + k0 * c.ldy : c.win + k0 * c.ldw, from_y0 ? c.ldy : c.ldw, c.y + k0 * c.ldy,
             c.y, c.ldy, (int)k0, b->rt + k0, c.p, (int)k0, (int)w);
      int64_t nwg = b->slots;
      for (int64_t J = 0; J < PK; ++J) {
        const Variant* v = pick_variant((int)J, true);
        nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * g_occ[1][variant_index(v)]);
        nwg = std::min<int64_t>(nwg, (tiles + (kWaves / v->wpt) - 1) / (kWaves / v->wpt));
      }
      nwg = std::max<int64_t>(nwg, 1);
      for (int64_t Jl = 0; Jl < PK; ++Jl) {
        const int64_t J = k0 / 16 + Jl;
        Launch L;
        memset(&L, 0, sizeof(L));
        BlockPassArgs& a = L.u.bp;
        const double* src = from_y ? c.y : c.win;
        const int64_t lds = from_y ? c.ldy : c.ldw;
        a.win = src + J * 16 * lds; a.ldw = lds;
        a.yout = c.y + J * 16 * c.ldy; a.ldy = c.ldy;
        a.s1 = c.y; a.ld1 = c.ldy; a.n1 = 0;
        a.s2 = c.y + k0 * c.ldy; a.ld2 = c.ldy; a.n2 = (int)(16 * Jl);
        a.pb = (int)std::min<int64_t>(16, c.p - 16 * J);
        a.m = m;
        a.bneg = b->bneg + (k0 / kSuper) * kSuperBneg + bneg_off(0, Jl);
        a.rinv = b->rinv + 256 * J;
        // (its Gramian partials are not used: the Gramian comes from cross_pass)
        a.part = b->part; a.part_stride = total_len(0, kSuper); a.part_off = e_off(0, Jl);
        a.done = &b->ctrl->done;
        a.passes = &b->ctrl->passes;
        a.copy_if_done = 0;
        const Variant* v = pick_variant((int)Jl, true);
        L.kind = Launch::kBlock;
        L.k1 = (const void*)v->apply; L.kb = (const void*)v->apply_b;
        L.grid = nwg; L.threads = kThreads; L.lds = block_lds_bytes(*v, true);
        record(L);
        out.push_back(L);
      }
    }
  }
  const double* src = apply ? c.y : c.win;
  const int64_t lsrc = apply ? c.ldy : c.ldw;
  auto cross = [&](const double* x, int64_t ldx, int nx, int rows16, int pitch, double* part, int slots_max,
                   bool sym) -> int {
    const int nb8 = (int)std::min<int64_t>(P, 8);
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kCross; L.k1 = (const void*)kCross[nb8 - 1]; L.kb = nullptr;
    CrossArgs& a = L.u.cr;
    a.x = x; a.ldx = ldx; a.nx = nx;
    a.y = src; a.ldy = lsrc; a.ny = (int)c.p;
    a.m = m; a.pitch = pitch; a.rows16 = rows16;
    a.tiles_b = (int)((P + nb8 - 1) / nb8);
    const int64_t ta = (rows16 + 16 * kCrossA - 1) / (16 * kCrossA);
    a.ntiles = (int)(ta * a.tiles_b);
    // tiles that work (sym: at or above the diagonal; 16 NB = 128 columns here)
    const int64_t busy = sym ? ta * (ta + 1) / 2 : a.ntiles;
    const int64_t want = (kCrossWant + busy - 1) / busy;
    a.nslots = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)slots_max, steps64, want}));
    a.sym = sym ? 1 : 0;
    a.part = part; a.part_stride = (int64_t)rows16 * pitch;
    a.done = apply ? &b->ctrl->done : nullptr;
    L.grid = (int64_t)a.ntiles * a.nslots; L.threads = kGramThreads; L.lds = 8 * (size_t)cross_lds_doubles(nb8);
    record(L);
    out.push_back(L);
    return a.nslots;
  };
  const int ns_b = basis ? cross(b->Q, b->ldq, (int)c.q, rows_bt, pitch_bt, b->partc, b->slots_c, false) : 0;
  const int ns_g = cross(src, lsrc, (int)c.p, (int)p16, (int)p16, b->partg, b->slots_g, true);
  auto reduce = [&](const double* in, int nslots, int64_t len, double* dst) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kReduce; L.k1 = (const void*)reduce_slots; L.kb = (const void*)reduce_slots_batch;
    ReduceArgs& r = L.u.ra;
    r.in = in; r.nslots = nslots; r.stride = len; r.len = len; r.out = dst;
    r.done = apply ? &b->ctrl->done : nullptr;
    L.grid = (len + kRedElems - 1) / kRedElems; L.threads = 64 * kRedWaves; L.lds = 0;
    L.prof_kind = -1;
    out.push_back(L);
  };
  if (basis) {
    reduce(b->partc, ns_b, (int64_t)rows_bt * pitch_bt, b->stage_bt);
    Launch B;
    memset(&B, 0, sizeof(B));
    B.kind = Launch::kBtb; B.k1 = (const void*)btb_pass; B.kb = nullptr;
    BtbArgs& t = B.u.bb;
    t.bt = b->stage_bt; t.pitch = pitch_bt; t.rows16 = rows_bt; t.p = (int)c.p;
    t.out = b->btb;
    t.done = apply ? &b->ctrl->done : nullptr;
    B.grid = P * (P + 1) / 2; B.threads = kThreads; B.lds = 0;
    B.prof_kind = -1;
    out.push_back(B);
  }
  reduce(b->partg, ns_g, p16 * p16, b->stage_g);
  // small_step in two stages around the band factorisation, then the R
  // update and the operands of the next pass
  SmallArgs k;
  memset(&k, 0, sizeof(k));
  k.E = b->stage_g;
  k.mode = c.mode; k.ext = 2 | (basis ? 1 : 0); k.q = (int)c.q; k.p = (int)c.p; k.nblk = (int)P;
  k.btb = b->btb; k.rold = b->rold; k.rt = b->rt; k.vec = b->vec;
  k.m = m; k.phase = phase;
  k.R = b->R; k.ldr = b->ldr;
  k.X = b->X;
  k.bneg = b->bneg; k.rinv = b->rinv; k.ctrl = b->ctrl;
  k.hctrl = b->ctrl_host_dev; k.stamp_base = b->call_id * 256; k.publish_from = b->publish_from;
  k.first_pass_shift = b->opts.first_pass_shift; k.min_passes = b->opts.min_passes;
  k.max_iter = b->opts.max_iter; k.max_escalations = b->opts.max_escalations;
  k.power_steps = b->opts.power_steps; k.tol = b->opts.tol; k.u = b->opts.unit_roundoff;
  k.shift_policy = b->opts.shift_policy; k.shift_dim = b->opts.append_shift_dim;
  k.mixed = 0;
  k.lds_matrices = 0;   // the small matrices of a wide block live in the workspace
  k.errpart = b->errpart; k.nerr = (int)(((c.p + 31) / 32) * ((c.p + 31) / 32));   // X from xfill_pass
  auto small = [&](int stage) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kSmall; L.k1 = (const void*)small_step; L.kb = (const void*)small_step_batch;
    L.u.sa = k;
    L.u.sa.stage = stage;
    L.lds = 0; L.grid = 1; L.threads = kSmallThreads;
    L.prof_kind = -1;
    out.push_back(L);
  };
  BigArgs g;
  memset(&g, 0, sizeof(g));
  g.X = b->X; g.M = b->X + (int64_t)c.p * c.p; g.p = (int)c.p; g.ctrl = b->ctrl;
  g.rinv = b->rinv; g.rold = b->rold; g.R = b->R; g.ldr = b->ldr; g.q = (int)c.q; g.phase = phase;
  g.rt = b->rt; g.bneg = b->bneg;
  g.E = b->stage_g; g.btb = basis ? b->btb : nullptr; g.errpart = b->errpart;
  auto big = [&](const void* kern, int64_t grid, int threads, int k0) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kBig; L.k1 = kern; L.kb = nullptr;
    L.u.bg = g;
    L.u.bg.k0 = k0;
    L.grid = grid; L.threads = threads; L.lds = 0;
    L.prof_kind = -1;
    out.push_back(L);
  };
  const int64_t tp = (c.p + 31) / 32;
  big((const void*)xfill_pass, tp * tp, kThreads, 0);
  small(1);
  big((const void*)mfill_pass, tp * tp, kThreads, 0);
  for (int64_t k0 = 0; k0 < c.p; k0 += kBand) {
    const int64_t k1 = std::min<int64_t>(c.p, k0 + kBand);
    big((const void*)chol_diag, 1, kSmallThreads, (int)k0);
    if (k1 < c.p) {
      big((const void*)chol_panel, (c.p - k1 + kSmallThreads - 1) / kSmallThreads, kSmallThreads, (int)k0);
      const int64_t T = (c.p - k1 + 15) / 16;
      big((const void*)chol_trail, (T * (T + 1) / 2 + kWaves - 1) / kWaves, kThreads, (int)k0);
    }
  }
  small(2);
  big((const void*)trmm_pass, (P * P + kWaves - 1) / kWaves, kThreads, 0);
  big((const void*)cj_pass, P, kSmallThreads, 0);
  if (basis) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kBacc; L.k1 = (const void*)bacc_pass; L.kb = nullptr;
    BaccArgs& a = L.u.ba;
    a.bt = b->stage_bt; a.pitch = pitch_bt; a.rold = b->rold;
    a.R = b->R; a.ldr = b->ldr; a.q = (int)c.q; a.p = (int)c.p; a.phase = phase;
    a.done = &b->ctrl->done;
    L.grid = (nblocks(c.q) * P + kWaves - 1) / kWaves; L.threads = kThreads; L.lds = 0;
    L.prof_kind = -1;
    out.push_back(L);
  }
  return SQR_OK;
}

// The launches of pass `phase` of a call, in order: the streaming kernels
// (by route), the fixed-order reduction of the slots, the small step.
int plan_pass(sqr_basis* b, const Call& c, int phase, std::vector<Launch>& out) {
  if (big_block(c.p)) return plan_big(b, c, phase, out);
  const int64_t P = nblocks(c.p);
  // wide basis: block_pass sees only the block (q = 0 layouts), the basis
  // part runs in proj_pass / cross_pass / btb_pass / bacc_pass
  const bool wideb = c.mode == 1 && wide_basis(c.q, c.p);
  const int64_t qb = wideb ? 0 : c.q;
  const int64_t tl = total_len(qb, c.p);
  const int64_t tiles = (b->m + 15) / 16;
  const bool apply = phase > 0;
  int64_t nwg = b->slots;
  const bool mixed = c.mode == 0 && b->opts.precision == 1;
  auto push_wide = [&](const void* k1, const void* kb, const WidePassArgs& w, int64_t grid, int threads,
                       size_t lds, int kind, double bytes, bool join) {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kWide; L.k1 = k1; L.kb = kb; L.u.wp = w;
    L.grid = grid; L.threads = threads; L.lds = lds;
    L.prof_kind = kind; L.prof_bytes = bytes; L.prof_join = join;
    out.push_back(L);
  };
  if (c.mode == 0 && P >= kSplitMin && P <= kSplitMax) {
    // apply (from pass 1 on), then the Gramian of its result
    const int idx = (int)P - kSplitMin;
    const SplitVariant& sv = kSplit[idx];
    const int64_t steps = (tiles + kWaves - 1) / kWaves;
    WidePassArgs w;
    memset(&w, 0, sizeof(w));
    w.n = (int)c.p; w.m = b->m;
    w.bneg = b->bneg; w.rinv = b->rinv;
    w.part = b->part; w.part_stride = tl;
    w.done = phase > 0 ? &b->ctrl->done : nullptr;
    w.passes = &b->ctrl->passes;
    if (apply) {
      w.win = (phase > 1) ? c.y : c.win;
      w.ldw = (phase > 1) ? c.ldy : c.ldw;
      w.yout = c.y; w.ldy = c.ldy;
      w.copy_if_done = (phase == 1);
      const int64_t ga = std::max<int64_t>(1, std::min<int64_t>((int64_t)g_ncu * g_split_occ[1][idx], steps));
      push_wide((const void*)sv.apply, (const void*)sv.apply_b, w, ga, kThreads, split_lds_bytes((int)P, true),
                1, 16.0 * (double)b->m * (double)c.p, false);
    }
    // the Gramian of the pass's result (of the input at phase 0); the mixed
    // form launches the FP32 variant at phase 0 and both variants later, the
    // one that does not match the device's choice (ctrl->gram32) exits at
    // once.  Both fill the same nwg slots and count as one measured launch.
    w.win = apply ? c.y : c.win;
    w.ldw = apply ? c.ldy : c.ldw;
    w.copy_if_done = 0;
    const int occ = mixed ? std::min(g_split_occ[0][idx], g_split_occ[2][idx]) : g_split_occ[0][idx];
    nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * occ);
    nwg = std::max<int64_t>(1, std::min<int64_t>(nwg, steps));
    w.gram32 = (mixed && phase > 0) ? &b->ctrl->gram32 : nullptr;
    const double gb = 8.0 * (double)b->m * (double)c.p;
    if (mixed)
      push_wide((const void*)sv.gram32, (const void*)sv.gram32_b, w, nwg, kGramThreads, gram32_lds_bytes((int)P),
                0, gb, false);
    if (!(mixed && phase == 0))
      push_wide((const void*)sv.gram, (const void*)sv.gram_b, w, nwg, kGramThreads, split_lds_bytes((int)P, false),
                0, gb, mixed);
  } else if (narrow_route(c, P, mixed)) {
    // one block: the whole pass in one launch, every wave on its own tiles.
    // Passes up to S = narrow_depth recompute their input from A through the
    // inverse factors of the passes before (the same products in the same
    // order as reading the stored result, so the same values), and only
    // passes from S on, the ones that can end the call, write their result:
    // CholQR3 moves 5 m n words instead of 7 m n.
    nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * g_narrow_occ[apply ? 1 : 0]);
    nwg = std::max<int64_t>(1, std::min<int64_t>(nwg, (tiles + kWaves - 1) / kWaves));
    const int S = narrow_depth(b->opts);
    const bool from_a = !apply || phase <= S;
    WidePassArgs w;
    memset(&w, 0, sizeof(w));
    w.win = from_a ? c.win : c.y;
    w.ldw = from_a ? c.ldw : c.ldy;
    w.yout = c.y; w.ldy = c.ldy;
    w.n = (int)c.p; w.m = b->m;
    w.rinv = b->rinv + 256 * (from_a ? 0 : narrow_slot(phase));
    w.levels = apply ? (from_a ? phase : 1) : 0;
    w.store = apply && phase >= S;
    w.part = b->part; w.part_stride = tl;
    w.done = phase > 0 ? &b->ctrl->done : nullptr;
    w.passes = &b->ctrl->passes;
    w.copy_if_done = (phase == 1);
    // mixed form: phase 0 forms an FP32 Gramian; later phases launch both
    // precisions and the one the device did not choose exits at once
    bool join = false;
    for (int g32 = mixed ? 1 : 0; g32 >= 0; --g32) {
      if (mixed && phase == 0 && g32 == 0) break;
      w.gram32 = (mixed && phase > 0) ? &b->ctrl->gram32 : nullptr;
      push_wide((const void*)kNarrow[g32][apply ? 1 : 0], (const void*)kNarrowB[g32][apply ? 1 : 0], w, nwg,
                kThreads, 0, apply ? 1 : 0, 8.0 * (double)b->m * (double)c.p * (apply ? 2.0 : 1.0), join);
      join = true;
    }
  } else if (c.mode == 0 && P <= kWideMax && (P >= 2 || mixed)) {
    // the whole pass in one launch (mixed form: one launch per Gramian
    // precision from pass 1 on; the one that does not match the device's
    // choice exits at once)
    const int idx = (int)P - kWideMin;
    const int64_t steps = (tiles + kWaves - 1) / kWaves;
    const int occ = std::min(g_wide_occ[0][apply ? 1 : 0][idx], g_wide_occ[1][apply ? 1 : 0][idx]);
    nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * occ);
    nwg = std::max<int64_t>(1, std::min<int64_t>(nwg, steps));
    WidePassArgs w;
    memset(&w, 0, sizeof(w));
    w.win = (apply && phase > 1) ? c.y : c.win;
    w.ldw = (apply && phase > 1) ? c.ldy : c.ldw;
    w.yout = c.y; w.ldy = c.ldy;
    w.n = (int)c.p; w.m = b->m;
    w.bneg = b->bneg; w.rinv = b->rinv;
    w.part = b->part; w.part_stride = tl;
    w.done = phase > 0 ? &b->ctrl->done : nullptr;
    w.passes = &b->ctrl->passes;
    w.copy_if_done = (phase == 1);
    const double bytes = 8.0 * (double)b->m * (double)c.p * (apply ? 2.0 : 1.0);
    bool join = false;
    for (int g32 = mixed ? 1 : 0; g32 >= 0; --g32) {
      // phase 0 of the mixed form is an FP32 Gramian; later phases follow the
      // device (ctrl->gram32); FP64 calls launch the FP64 variant only
      if (mixed && phase == 0 && g32 == 0) break;
      w.gram32 = (mixed && phase > 0) ? &b->ctrl->gram32 : nullptr;
      push_wide((const void*)kWide[idx].k[g32][apply ? 1 : 0], (const void*)kWide[idx].kb[g32][apply ? 1 : 0], w,
                nwg, kThreads, wide_lds_bytes((int)P, apply), apply ? 1 : 0, bytes, join);
      join = true;
    }
  } else {
    const int nb8 = (int)std::min<int64_t>(P, 8);
    const int tiles_b = (int)((P + nb8 - 1) / nb8);
    const int pitch = (int)round16(c.p), rows16 = (int)round16(c.q);
    const double pass_bytes = 8.0 * (double)b->m * (double)(c.q + (apply ? 2 : 1) * c.p);
    if (wideb && apply) {
      // Z = W - Q_in B~ into the new columns (in place from pass 2 on)
      Launch L;
      memset(&L, 0, sizeof(L));
      L.kind = Launch::kProj; L.k1 = (const void*)kProj[nb8 - 1]; L.kb = nullptr;
      ProjArgs& a = L.u.pj;
      a.win = (phase > 1) ? c.y : c.win; a.ldw = (phase > 1) ? c.ldy : c.ldw;
      a.yout = c.y; a.ldy = c.ldy;
      a.x = b->Q; a.ldx = b->ldq; a.nx = (int)c.q;
      a.bt = b->stage_bt; a.ldt = pitch; a.rows16 = rows16;
      a.p = (int)c.p; a.m = b->m; a.tiles_b = tiles_b;
      a.done = &b->ctrl->done;
      L.grid = ((b->m + kProjRows - 1) / kProjRows) * tiles_b; L.threads = kThreads; L.lds = 8 * (size_t)proj_lds_doubles(nb8);
      L.prof_kind = 1; L.prof_bytes = pass_bytes; L.prof_join = false;
      out.push_back(L);
    }
    // One grid size for every block of the pass (the slots are reduced
    // together): resident workgroups of the most demanding block's variant,
    // capped by the slot capacity and by the row tiles available.
    for (int64_t J = 0; J < P; ++J) {
      const int ks = (int)round16(qb) + (int)(16 * J);
      const Variant* v = pick_variant((ks + 15) / 16, apply);
      if (!v) return SQR_EDIM;
      const int occ = g_occ[apply ? 1 : 0][variant_index(v)];
      nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * occ);
      nwg = std::min<int64_t>(nwg, (tiles + (kWaves / v->wpt) - 1) / (kWaves / v->wpt));
    }
    nwg = std::max<int64_t>(nwg, 1);
    for (int64_t J = 0; J < P; ++J) {
      Launch L;
      memset(&L, 0, sizeof(L));
      BlockPassArgs& a = L.u.bp;
      // (wide basis: the apply reads Z, which proj_pass left in the output)
      const bool from_y = apply && (phase > 1 || wideb);
      const double* src = from_y ? c.y : c.win;
      const int64_t lds = from_y ? c.ldy : c.ldw;
      a.win = src + J * 16 * lds; a.ldw = lds;
      a.yout = c.y + J * 16 * c.ldy; a.ldy = c.ldy;
      a.s1 = b->Q; a.ld1 = b->ldq; a.n1 = (int)qb;
      // same-pass prefix: new values after an apply, the input for the first Gram
      a.s2 = apply ? c.y : c.win; a.ld2 = apply ? c.ldy : c.ldw; a.n2 = (int)(16 * J);
      a.pb = (int)std::min<int64_t>(16, c.p - 16 * J);
      a.m = b->m;
      a.bneg = b->bneg + bneg_off(qb, J);
      a.rinv = b->rinv + 256 * J;
      a.part = b->part; a.part_stride = tl; a.part_off = e_off(qb, J);
      a.done = phase > 0 ? &b->ctrl->done : nullptr;  // phase 0 starts the call
      a.passes = &b->ctrl->passes;
      a.copy_if_done = (phase == 1) && !wideb;
      const int ks = (int)round16(a.n1) + a.n2;   // columns of S with the padding
      const Variant* v = pick_variant((ks + 15) / 16, apply);
      L.kind = Launch::kBlock;
      L.k1 = (const void*)(apply ? v->apply : v->gram);
      L.kb = (const void*)(apply ? v->apply_b : v->gram_b);
      L.grid = nwg; L.threads = kThreads; L.lds = block_lds_bytes(*v, apply);
      // algorithmic bytes: the real columns of S (no padding), the block read,
      // and (apply) the block written
      L.prof_kind = apply ? 1 : 0;
      L.prof_bytes = 8.0 * (double)b->m * (double)(a.n1 + a.n2 + (apply ? 2 : 1) * a.pb);
      if (wideb) {
        // one record for the whole pass of a wide-basis append
        L.prof_join = apply || J > 0;
        L.prof_bytes = pass_bytes;
      }
      out.push_back(L);
    }
    if (wideb) {
      // B~ = Q_in^T Y (of W at phase 0), one row chunk per slot
      Launch L;
      memset(&L, 0, sizeof(L));
      L.kind = Launch::kCross; L.k1 = (const void*)kCross[nb8 - 1]; L.kb = nullptr;
      CrossArgs& a = L.u.cr;
      a.x = b->Q; a.ldx = b->ldq; a.nx = (int)c.q;
      a.y = apply ? c.y : c.win; a.ldy = apply ? c.ldy : c.ldw; a.ny = (int)c.p;
      a.m = b->m;
      a.pitch = pitch; a.rows16 = rows16;
      a.tiles_b = tiles_b;
      a.ntiles = (int)((rows16 + 16 * kCrossA - 1) / (16 * kCrossA)) * tiles_b;
      const int64_t steps = (tiles + kWaves - 1) / kWaves;
      const int64_t want = (kCrossWant + a.ntiles - 1) / a.ntiles;
      a.nslots = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)b->slots_c, steps, want}));
      a.part = b->partc; a.part_stride = (int64_t)rows16 * pitch;
      a.done = phase > 0 ? &b->ctrl->done : nullptr;
      L.grid = (int64_t)a.ntiles * a.nslots; L.threads = kGramThreads; L.lds = 8 * (size_t)cross_lds_doubles(nb8);
      L.prof_kind = apply ? 1 : 0; L.prof_join = true;
      out.push_back(L);
    }
  }
  {
    // Fixed-order reduction of the nwg slots into the pass's Gramian blocks.
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kReduce; L.k1 = (const void*)reduce_slots; L.kb = (const void*)reduce_slots_batch;
    ReduceArgs& r = L.u.ra;
    r.in = b->part; r.nslots = (int)nwg; r.stride = tl; r.len = tl; r.out = b->stage;
    r.done = phase > 0 ? &b->ctrl->done : nullptr;
    L.grid = (tl + kRedElems - 1) / kRedElems; L.threads = 64 * kRedWaves; L.lds = 0;
    L.prof_kind = -1;
    out.push_back(L);
  }
  if (wideb) {
    // the cross_pass slots into B~, then B~^T B~
    const Launch& X = out[out.size() - 2];   // the cross_pass launch
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kReduce; L.k1 = (const void*)reduce_slots; L.kb = (const void*)reduce_slots_batch;
    ReduceArgs& r = L.u.ra;
    r.in = b->partc; r.nslots = X.u.cr.nslots; r.stride = X.u.cr.part_stride; r.len = r.stride;
    r.out = b->stage_bt;
    r.done = phase > 0 ? &b->ctrl->done : nullptr;
    L.grid = (r.len + kRedElems - 1) / kRedElems; L.threads = 64 * kRedWaves; L.lds = 0;
    L.prof_kind = -1;
    out.push_back(L);
    Launch B;
    memset(&B, 0, sizeof(B));
    B.kind = Launch::kBtb; B.k1 = (const void*)btb_pass; B.kb = nullptr;
    BtbArgs& t = B.u.bb;
    t.bt = b->stage_bt; t.pitch = (int)round16(c.p); t.rows16 = (int)round16(c.q); t.p = (int)c.p;
    t.out = b->btb;
    t.done = phase > 0 ? &b->ctrl->done : nullptr;
    B.grid = P * (P + 1) / 2; B.threads = kThreads; B.lds = 0;
    B.prof_kind = -1;
    out.push_back(B);
  }
  {
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kSmall; L.k1 = (const void*)small_step; L.kb = (const void*)small_step_batch;
    SmallArgs& k = L.u.sa;
    k.E = b->stage;
    k.mode = c.mode; k.ext = wideb ? 1 : 0; k.q = (int)c.q; k.p = (int)c.p; k.nblk = (int)P;
    k.btb = b->btb; k.rold = b->rold;
    k.m = b->m; k.phase = phase;
    k.R = b->R; k.ldr = b->ldr;
    k.X = b->X;
    k.bneg = b->bneg; k.rinv = b->rinv; k.ctrl = b->ctrl;
    // one-block orthogonalisation: the factor for pass phase + 1 goes to its slot
    if (narrow_route(c, P, mixed)) k.rinv = b->rinv + 256 * narrow_slot(phase + 1);
    k.hctrl = b->ctrl_host_dev; k.stamp_base = b->call_id * 256; k.publish_from = b->publish_from;
    k.first_pass_shift = b->opts.first_pass_shift; k.min_passes = b->opts.min_passes;
    k.max_iter = b->opts.max_iter; k.max_escalations = b->opts.max_escalations;
    k.power_steps = b->opts.power_steps; k.tol = b->opts.tol; k.u = b->opts.unit_roundoff;
    k.shift_policy = b->opts.shift_policy; k.shift_dim = b->opts.append_shift_dim;
    k.mixed = mixed ? 1 : 0;
    const size_t arena = 8 * (size_t)small_arena((int)qb, (int)c.p);
    const size_t mbytes = 8 * (size_t)c.p * (size_t)c.p;
    k.lds_matrices = (arena <= g_small_lds) ? 1 : (mbytes <= g_small_lds ? 2 : 0);
    L.lds = k.lds_matrices == 1 ? arena : (k.lds_matrices == 2 ? mbytes : 0);
    L.grid = 1; L.threads = kSmallThreads;
    L.prof_kind = -1;
    out.push_back(L);
  }
  if (wideb) {
    // B <- B + B~ R_old (phase 0: B <- B~), after the device's decision
    Launch L;
    memset(&L, 0, sizeof(L));
    L.kind = Launch::kBacc; L.k1 = (const void*)bacc_pass; L.kb = nullptr;
    BaccArgs& a = L.u.ba;
    a.bt = b->stage_bt; a.pitch = (int)round16(c.p); a.rold = b->rold;
    a.R = b->R; a.ldr = b->ldr; a.q = (int)c.q; a.p = (int)c.p; a.phase = phase;
    a.done = &b->ctrl->done;
    L.grid = (nblocks(c.q) * P + kWaves - 1) / kWaves; L.threads = kThreads; L.lds = 0;
    L.prof_kind = -1;
    out.push_back(L);
  }
  return SQR_OK;
}

// Enqueue the launches of one call's pass on s, with the measurement records.
int exec_single(sqr_basis* b, int phase, const std::vector<Launch>& L, hipStream_t s) {
  for (size_t i = 0; i < L.size();) {
    size_t j = i + 1;   // launches i .. j-1 share one measurement record
    if (L[i].prof_kind >= 0)
      while (j < L.size() && L[j].prof_join) ++j;
    ProfRec rec{};
    if (L[i].prof_kind >= 0) rec = prof_begin(L[i].prof_kind, L[i].prof_bytes, b->noprof ? -1 : b->call_id, phase, s);
    for (size_t k = i; k < j; ++k) {
      void* args[] = {(void*)&L[k].u};
      if (hipLaunchKernel(L[k].k1, dim3((unsigned)L[k].grid), dim3(L[k].threads), args, L[k].lds, s) != hipSuccess)
        return SQR_EHIP;
    }
    if (L[i].prof_kind >= 0) prof_end(rec, s);
    i = j;
  }
  return SQR_OK;
}

int launch_gram(sqr_basis* b, const Call& c, int phase, hipStream_t s) {
  std::vector<Launch> L;
  int rc = plan_pass(b, c, phase, L);
  if (rc) return rc;
  return exec_single(b, phase, L, s);
}

int fetch(sqr_basis* /*b*/, hipStream_t s) {
  if (hipStreamSynchronize(s) != hipSuccess) return SQR_EHIP;
  return SQR_OK;
}

// Wait until the device has published the outcome of phase `enq` of the
// current call, or an earlier decision (done).  small_step writes the state
// into pinned host memory, so the host polls it instead of copying it and
// waiting for the stream to drain; it still checks the stream now and then
// for errors, and after kSpinLimit falls back to a blocking stream wait.
int wait_phase(sqr_basis* b, hipStream_t s, int enq) {
  constexpr double kSpinLimitUs = 2000.0;
  volatile Ctrl* h = b->ctrl_host;
  const int64_t want = b->call_id * 256;
  auto ready = [&]() {
    const int64_t st = __atomic_load_n(&b->ctrl_host->stamp, __ATOMIC_ACQUIRE);
    return st >= want && st < want + 256 && (h->done || st - want >= enq);
  };
  const auto t0 = std::chrono::steady_clock::now();
  for (int it = 1;; ++it) {
    if (ready()) return SQR_OK;
    if ((it & 1023) == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e != hipSuccess && e != hipErrorNotReady) return SQR_EHIP;
      const double us = std::chrono::duration<double, std::micro>(
                            std::chrono::steady_clock::now() - t0).count();
      if (e == hipSuccess || us > kSpinLimitUs) break;
    }
    __builtin_ia32_pause();
  }
  if (fetch(b, s)) return SQR_EHIP;
  return ready() ? SQR_OK : SQR_EHIP;
}

void fill_info(const Ctrl* c, sqr_info* info) {
  info->status = c->status;
  info->passes = c->passes;
  info->chol_attempts = c->chol_attempts;
  info->converged = c->converged;
  info->orth_fro = c->orth_fro;
  for (int i = 0; i < 16; ++i) info->sigma[i] = c->sigma[i];
}

// Run one call.  sync: enqueue `spec` passes, then add passes one by one while
// the device reports neither convergence nor failure.
// A call of the handle on stream s starts after all work of its previous
// call: kernels of that call (no-op launches of a finished call among them)
// may still be queued on its stream and read the control block that the new
// call resets, so s waits for an event recorded there.
int order_after_previous(sqr_basis* b, hipStream_t s) {
  if (b->used && s != b->stream) {
    if (!b->order_ev && hipEventCreateWithFlags(&b->order_ev, hipEventDisableTiming) != hipSuccess) {
      b->order_ev = nullptr;
      return SQR_EHIP;
    }
    if (hipEventRecord(b->order_ev, b->stream) != hipSuccess ||
        hipStreamWaitEvent(s, b->order_ev, 0) != hipSuccess)
      return SQR_EHIP;
  }
  b->used = true;
  b->stream = s;
  b->call_id = ++g_call_id;
  return SQR_OK;
}

int run_call(sqr_basis* b, const Call& c, hipStream_t s, bool sync, int spec) {
  int rc = order_after_previous(b, s);
  if (rc) return rc;
  const int maxit = b->opts.max_iter;
  const int first = sync ? std::min(spec, maxit) : maxit;
  b->publish_from = sync ? first : maxit + 1;   // async: only the end is published
  rc = launch_gram(b, c, 0, s);
  if (rc) return rc;
  int enq = 0;
  for (; enq < first; ++enq)
    if ((rc = launch_gram(b, c, enq + 1, s))) return rc;
  if (!sync) return SQR_OK;
  if ((rc = wait_phase(b, s, enq))) return rc;
  while (!b->ctrl_host->done && enq < maxit) {
    if ((rc = launch_gram(b, c, ++enq, s))) return rc;
    if ((rc = wait_phase(b, s, enq))) return rc;
  }
  if (g_prof_on) prof_finalize(b->call_id, b->ctrl_host->passes);
  return SQR_OK;
}

// ---- batched calls (sqr_batch): the passes of several calls advance
// together; each launch of a pass carries one kernel for every call whose
// pass uses it at that position (the same route, the same grid per call as
// alone), reading the calls' argument blocks from a table in device memory.
// Argument tables are staged in pinned host memory and copied with one
// transfer per round of passes.
struct BatchStage {
  char* host = nullptr;   // pinned
  char* dev = nullptr;
  size_t bytes = 0;
  int device = -1;
};
std::mutex g_stage_mu;
std::vector<BatchStage> g_stages;   // idle staging buffers

BatchStage take_stage(int device, size_t need) {
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (size_t i = 0; i < g_stages.size(); ++i)
      if (g_stages[i].device == device && g_stages[i].bytes >= need) {
        BatchStage st = g_stages[i];
        g_stages.erase(g_stages.begin() + i);
        return st;
      }
  }
  BatchStage st;
  const size_t bytes = std::max<size_t>(need, 1 << 20);
  if (hipHostMalloc((void**)&st.host, bytes, hipHostMallocDefault) != hipSuccess) return BatchStage{};
  if (hipMalloc((void**)&st.dev, bytes) != hipSuccess) {
    (void)hipHostFree(st.host);
    return BatchStage{};
  }
  st.bytes = bytes;
  st.device = device;
  return st;
}

void put_stage(const BatchStage& st) {
  if (!st.host) return;
  std::lock_guard<std::mutex> lk(g_stage_mu);
  g_stages.push_back(st);
  while (g_stages.size() > 4) {
    (void)hipHostFree(g_stages.front().host);
    (void)hipFree(g_stages.front().dev);
    g_stages.erase(g_stages.begin());
  }
}

struct BatchCall {
  sqr_basis* b;
  Call c;
  int enq;      // passes enqueued after the initial Gram pass
  int spec;     // passes enqueued before the first wait
};

// Enqueue pass `phase[i]` of every call i in `who` as batched launches.
// `off` is the running offset into the staging buffers.
int enqueue_round(std::vector<BatchCall>& calls, const std::vector<int>& who, const std::vector<int>& phase,
                  BatchStage& st, size_t& off, hipStream_t s) {
  std::vector<std::vector<Launch>> plans(who.size());
  size_t maxstream = 0;
  for (size_t i = 0; i < who.size(); ++i) {
    BatchCall& bc = calls[who[i]];
    const int rc = plan_pass(bc.b, bc.c, phase[i], plans[i]);
    if (rc) return rc;
    maxstream = std::max(maxstream, plans[i].size() - 2);
  }
  struct Group { const void* kb; size_t args_off, start_off; int n; int64_t grid; int threads; size_t lds; };
  std::vector<Group> groups;
  const size_t off0 = off;
  auto align = [&](size_t a) { off = (off + a - 1) / a * a; };
  // one group per batched kernel at each launch position, in call order
  auto build = [&](const std::vector<std::pair<size_t, const Launch*>>& members) -> int {
    std::vector<const void*> kernels;
    for (const auto& mb : members)
      if (std::find(kernels.begin(), kernels.end(), mb.second->kb) == kernels.end())
        kernels.push_back(mb.second->kb);
    for (const void* kb : kernels) {
      std::vector<const Launch*> ls;
      for (const auto& mb : members)
        if (mb.second->kb == kb) ls.push_back(mb.second);
      const size_t asz = launch_arg_bytes(ls[0]->kind);
      Group g;
      g.kb = kb; g.n = (int)ls.size(); g.threads = ls[0]->threads; g.lds = 0; g.grid = 0;
      align(256);
      g.args_off = off;
      if (off + asz * ls.size() > st.bytes) return SQR_EHIP;
      for (size_t k = 0; k < ls.size(); ++k) memcpy(st.host + off + k * asz, &ls[k]->u, asz);
      off += asz * ls.size();
      align(16);
      g.start_off = off;
      if (off + 4 * (ls.size() + 1) > st.bytes) return SQR_EHIP;
      int32_t* start = (int32_t*)(st.host + off);
      int64_t acc = 0;
      for (size_t k = 0; k < ls.size(); ++k) {
        start[k] = (int32_t)acc;
        acc += ls[k]->kind == Launch::kSmall ? 1 : ls[k]->grid;
        g.lds = std::max(g.lds, ls[k]->lds);
      }
      start[ls.size()] = (int32_t)acc;
      off += 4 * (ls.size() + 1);
      g.grid = acc;
      groups.push_back(g);
    }
    return SQR_OK;
  };
  int rc;
  for (size_t pos = 0; pos < maxstream; ++pos) {
    std::vector<std::pair<size_t, const Launch*>> members;
    for (size_t i = 0; i < who.size(); ++i)
      if (pos + 2 < plans[i].size()) members.push_back({i, &plans[i][pos]});
    if ((rc = build(members))) return rc;
  }
  for (int tail = 2; tail >= 1; --tail) {   // the reductions, then the small steps
    std::vector<std::pair<size_t, const Launch*>> members;
    for (size_t i = 0; i < who.size(); ++i) members.push_back({i, &plans[i][plans[i].size() - tail]});
    if ((rc = build(members))) return rc;
  }
  if (hipMemcpyAsync(st.dev + off0, st.host + off0, off - off0, hipMemcpyHostToDevice, s) != hipSuccess)
    return SQR_EHIP;
  for (const Group& g : groups) {
    BatchTable<char> t;   // the same layout for every argument type
    t.args = st.dev + g.args_off;
    t.start = (const int32_t*)(st.dev + g.start_off);
    t.ncalls = g.n;
    void* args[] = {&t};
    if (hipLaunchKernel(g.kb, dim3((unsigned)g.grid), dim3(g.threads), args, g.lds, s) != hipSuccess)
      return SQR_EHIP;
  }
  return SQR_OK;
}

// Run the calls: every call's initial Gram pass and its first `spec` passes
// as batched rounds, then, after the device has decided, further rounds for
// the calls that ask for more passes.
int run_batch(std::vector<BatchCall>& calls, hipStream_t s, BatchStage& st) {
  size_t off = 0;
  int maxspec = 0;
  for (BatchCall& bc : calls) {
    const int rc = order_after_previous(bc.b, s);
    if (rc) return rc;
    bc.enq = 0;
    bc.b->publish_from = bc.spec;
    maxspec = std::max(maxspec, bc.spec);
  }
  for (int ph = 0; ph <= maxspec; ++ph) {
    std::vector<int> who, phase;
    for (size_t i = 0; i < calls.size(); ++i)
      if (ph == 0 || ph <= calls[i].spec) {
        who.push_back((int)i);
        phase.push_back(ph);
        if (ph > 0) calls[i].enq = ph;
      }
    const int rc = enqueue_round(calls, who, phase, st, off, s);
    if (rc) return rc;
  }
  for (;;) {
    std::vector<int> who, phase;
    for (size_t i = 0; i < calls.size(); ++i) {
      BatchCall& bc = calls[i];
      const int rc = wait_phase(bc.b, s, bc.enq);
      if (rc) return rc;
      if (!bc.b->ctrl_host->done && bc.enq < bc.b->opts.max_iter) {
        who.push_back((int)i);
        phase.push_back(++bc.enq);
      }
    }
    if (who.empty()) break;
    const int rc = enqueue_round(calls, who, phase, st, off, s);
    if (rc) return rc;
  }
  return SQR_OK;
}

// ---- the allocation-free orthogonalisation (sqr_orth_noalloc): its
// workspace is one file-scope device array per GPU, `scratch`.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in
// symbol, not a device address): the device address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr int64_t kScratchDoubles = SQR_NOALLOC_SCRATCH_BYTES / 8;
__device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (NULL on failure).
double* scratch_on_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  return g_scratch_ptr[dev];
}

bool opts_ok(const sqr_opts& o) {
  return (o.precision == 0 || o.precision == 1) && o.max_iter >= 1 && o.max_iter <= 64 && o.min_passes >= 0 &&
         o.tol > 0.0 && o.unit_roundoff > 0.0 && o.max_escalations >= 0 &&
         o.power_steps >= 1 && o.power_steps <= 1000 && o.shift_policy >= 0 && o.shift_policy <= 2 &&
         (o.shift_policy == 0 || o.precision == 0) && o.append_shift_dim >= 0 && o.append_shift_dim <= 2;
}

}  // namespace

extern "C" {

void sqr_default_opts(sqr_opts* o) {
  if (!o) return;
  o->precision = 0;
  o->first_pass_shift = 1;
  o->min_passes = 3;
  o->max_iter = 10;
  o->tol = 1e-13;
  o->unit_roundoff = 1.1102230246251565e-16;  // 2^-53
  o->max_escalations = 32;
  o->power_steps = 30;
  o->shift_policy = 0;
  o->append_shift_dim = 0;
}

int sqr_orth(sqr_basis** out, const sqr_opts* opts, int64_t m, int64_t n,
             const double* A, int64_t lda, double* Q, int64_t ldq, int64_t cap,
             double* R, int64_t ldr, void* stream, sqr_info* info) {
  if (!out || !A || !Q || !R) return SQR_ENULL;
  if (m < 1 || n < 1 || n > m || lda < m || ldq < m || cap < n || ldr < cap)
    return SQR_EDIM;
  if (cap > kMaxCap || lda > kMaxLd || ldq > kMaxLd) return SQR_EDIM;
  sqr_opts o;
  sqr_default_opts(&o);
  if (opts) o = *opts;
  if (!opts_ok(o)) return SQR_EOPT;
  if (o.precision == 1 && n > 16 * kSplitMax) return SQR_EOPT;   // mixed form up to 256 columns
  set_kernel_attributes();
  sqr_basis* b = new sqr_basis();
  b->m = m; b->n = n; b->cap = cap; b->Q = Q; b->ldq = ldq; b->R = R; b->ldr = ldr;
  b->opts = o;
  (void)hipGetDevice(&b->device);
  int rc = alloc_workspace(b, big_block(n) ? n : 0);
  if (rc) { sqr_free(b); return rc; }
  Call c{0, 0, n, A, lda, Q, ldq};
  hipStream_t s = (hipStream_t)stream;
  const int spec = std::max(o.min_passes, 1);
  rc = run_call(b, c, s, info != nullptr, spec);
  if (rc) { (void)hipStreamSynchronize(s); sqr_free(b); return rc; }
  *out = b;
  if (info) {
    fill_info(b->ctrl_host, info);
    return info->status;
  }
  return SQR_OK;
}

int sqr_orth_noalloc(const sqr_opts* opts, int64_t m, int64_t n, const double* A, int64_t lda,
                     double* Q, int64_t ldq, double* R, int64_t ldr, void* stream, sqr_info* info) {
  if (!A || !Q || !R) return SQR_ENULL;
  if (m < 1 || n < 1 || n > m || lda < m || ldq < m || ldr < n) return SQR_EDIM;
  if (lda > kMaxLd || ldq > kMaxLd) return SQR_EDIM;
  if (n > SQR_NOALLOC_MAX_COLS) return SQR_ELIMIT;
  sqr_opts o;
  sqr_default_opts(&o);
  if (opts) o = *opts;
  if (!opts_ok(o)) return SQR_EOPT;
  set_kernel_attributes();
  // A handle on the host stack whose regions lie in this device's scratch
  // array; no pinned mirror (the outcome is copied from the device), no
  // measurement records.
  sqr_basis b;
  b.m = m; b.n = n; b.cap = n; b.Q = Q; b.ldq = ldq; b.R = R; b.ldr = ldr;
  b.opts = o;
  b.noprof = true;
  if (hipGetDevice(&b.device) != hipSuccess) return SQR_EHIP;
  double* base = scratch_on_device(b.device);
  if (!base) return SQR_EHIP;
  const WsSizes z = orth_sizes(n);
  // as many slots as sqr_orth would take, as far as the array holds them
  // (then the reduction order, and so the result, is the same)
  int slots = default_slots(m, z.tl);
  const size_t fixed = carve_workspace(&b, nullptr, z, 0);
  const int64_t fit = ((int64_t)kScratchDoubles - (int64_t)fixed - 64) / (z.tl + 1);
  if (fit < 1) return SQR_ELIMIT;
  slots = (int)std::min<int64_t>(slots, fit);
  if ((int64_t)carve_workspace(&b, nullptr, z, slots) > kScratchDoubles) return SQR_ELIMIT;
  carve_workspace(&b, base, z, slots);
  Call c{0, 0, n, A, lda, Q, ldq};
  hipStream_t s = (hipStream_t)stream;
  // every pass up to max_iter is enqueued; those after the device's decision
  // exit at once
  int rc = run_call(&b, c, s, false, 0);
  if (rc) return rc;
  if (!info) return SQR_OK;
  Ctrl st;
  if (hipMemcpyAsync(&st, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SQR_EHIP;
  fill_info(&st, info);
  return info->status;
}

int sqr_append(sqr_basis* b, const double* W, int64_t p, int64_t ldw, void* stream,
               sqr_info* info) {
  if (!b || !W) return SQR_ENULL;
  if (p < 1 || ldw < b->m || ldw > kMaxLd || b->n + p > b->cap || b->n + p > b->m)
    return SQR_EDIM;
  if (b->ws && big_block(p) && p > b->pbig) {
    // a wider block than the workspace serves: give it back (after the
    // handle's queued work) and take one that fits
    if (sqr_park(b)) return SQR_EHIP;
  }
  if (!b->ws) {   // parked: take a workspace again
    const int rc0 = alloc_workspace(b, big_block(p) ? p : 0);
    if (rc0) return rc0;
    b->parked = false;
  }
  hipStream_t s = (hipStream_t)stream;
  Call c{1, b->n, p, W, ldw, b->Q + b->n * b->ldq, b->ldq};
  int rc = run_call(b, c, s, true, 2);
  if (rc) return rc;
  if (b->ctrl_host->status == SQR_OK) b->n += p;
  if (info) fill_info(b->ctrl_host, info);
  return b->ctrl_host->status;
}

int sqr_batch(const sqr_opts* opts, sqr_batch_item* items, int32_t count, void* stream) {
  if (!items || count < 1) return SQR_ENULL;
  sqr_opts o;
  sqr_default_opts(&o);
  if (opts) o = *opts;
  if (!opts_ok(o)) return SQR_EOPT;
  // usage checks of every item, as sqr_orth / sqr_append make them
  for (int32_t i = 0; i < count; ++i) {
    sqr_batch_item& it = items[i];
    it.rc = SQR_OK;
    memset(&it.info, 0, sizeof(it.info));
    if (it.kind == SQR_BATCH_ORTH) {
      const int64_t m = it.m, n = it.cols;
      if (!it.in || !it.Q || !it.R) it.rc = SQR_ENULL;
      else if (m < 1 || n < 1 || n > m || it.ld_in < m || it.ldq < m || it.cap < n || it.ldr < it.cap ||
               it.cap > kMaxSCols || it.ld_in > kMaxLd || it.ldq > kMaxLd)
        it.rc = SQR_EDIM;
      else if (o.precision == 1 && n > 16 * kSplitMax)
        it.rc = SQR_EOPT;
    } else if (it.kind == SQR_BATCH_APPEND) {
      sqr_basis* b = it.basis;
      if (!b || !it.in) it.rc = SQR_ENULL;
      else if (it.cols < 1 || it.cols > kMaxSCols || it.ld_in < b->m || it.ld_in > kMaxLd ||
               b->n + it.cols > b->cap || b->n + it.cols > b->m || wide_basis(b->n, it.cols))
        it.rc = SQR_EDIM;   // (appends with a wide basis run through sqr_append only)
      for (int32_t k = 0; k < i && it.rc == SQR_OK; ++k)   // one call per handle
        if (items[k].kind == SQR_BATCH_APPEND && items[k].basis == b) it.rc = SQR_EOPT;
    } else {
      it.rc = SQR_EOPT;
    }
  }
  bool any = false;
  for (int32_t i = 0; i < count; ++i) any = any || items[i].rc == SQR_OK;
  if (!any) return SQR_OK;   // nothing to run (no HIP call made)
  set_kernel_attributes();
  int device = 0;
  (void)hipGetDevice(&device);
  std::vector<BatchCall> calls;
  std::vector<int> idx;
  size_t need = 0;
  for (int32_t i = 0; i < count; ++i) {
    sqr_batch_item& it = items[i];
    if (it.rc) continue;
    sqr_basis* b;
    Call c;
    int spec;
    if (it.kind == SQR_BATCH_ORTH) {
      b = new sqr_basis();
      b->m = it.m; b->n = it.cols; b->cap = it.cap; b->Q = it.Q; b->ldq = it.ldq; b->R = it.R; b->ldr = it.ldr;
      b->opts = o;
      b->device = device;
      b->noprof = true;
      const int rc = alloc_workspace(b, 0);
      if (rc) { sqr_free(b); it.rc = rc; continue; }
      it.basis = b;
      c = Call{0, 0, it.cols, it.in, it.ld_in, it.Q, it.ldq};
      spec = std::min(std::max(o.min_passes, 1), o.max_iter);
    } else {
      b = it.basis;
      if (!b->ws) {
        const int rc = alloc_workspace(b, 0);
        if (rc) { it.rc = rc; continue; }
        b->parked = false;
      }
      c = Call{1, b->n, it.cols, it.in, it.ld_in, b->Q + b->n * b->ldq, b->ldq};
      spec = std::min(2, b->opts.max_iter);
    }
    calls.push_back(BatchCall{b, c, 0, spec});
    idx.push_back(i);
    // staging bound: every pass of the call, its launches, argument blocks
    // and start entries, with alignment slack
    const int64_t P = nblocks(c.p);
    need += (size_t)(b->opts.max_iter + 1) * (size_t)(P + 4) * (sizeof(Launch) + 8 + 512);
  }
  if (calls.empty()) return SQR_OK;
  hipStream_t s = (hipStream_t)stream;
  BatchStage st = take_stage(device, need + 4096);
  int rc = st.host ? run_batch(calls, s, st) : SQR_EHIP;
  // every queued launch of the batch has read its tables before they are reused
  if (hipStreamSynchronize(s) != hipSuccess && rc == SQR_OK) rc = SQR_EHIP;
  put_stage(st);
  for (size_t k = 0; k < calls.size(); ++k) {
    sqr_batch_item& it = items[idx[k]];
    sqr_basis* b = calls[k].b;
    if (rc) {
      it.rc = rc;
      if (it.kind == SQR_BATCH_ORTH) { sqr_free(b); it.basis = nullptr; }
      continue;
    }
    fill_info(b->ctrl_host, &it.info);
    if (it.kind == SQR_BATCH_APPEND && b->ctrl_host->status == SQR_OK) b->n += it.cols;
  }
  return rc;
}

int sqr_panel(sqr_basis** out, const sqr_opts* opts, int64_t m, int64_t n, const double* A, int64_t lda,
              int64_t r, double* Q, int64_t ldq, int64_t cap, double* R, int64_t ldr, void* stream,
              sqr_info* info) {
  if (!out || !A || !Q || !R) return SQR_ENULL;
  if (m < 1 || n < 1 || n > m || lda < m || ldq < m || cap < n || ldr < cap || r < 1 || r > n)
    return SQR_EDIM;
  if (cap > kMaxCap || lda > kMaxLd || ldq > kMaxLd) return SQR_EDIM;
  // panel i holds columns [e_i, e_{i+1}), e_i = i n / r rounded to the
  // nearest integer (ties to even), e_r = n
  auto edge = [&](int64_t i) -> int64_t {
    return (i >= r) ? n : (int64_t)nearbyint((double)i * ((double)n / (double)r));
  };
  int64_t widest = 0;
  for (int64_t i = 0; i < r; ++i) widest = std::max(widest, edge(i + 1) - edge(i));
  sqr_opts o;
  sqr_default_opts(&o);
  if (opts) o = *opts;
  if (!opts_ok(o) || o.precision != 0) return SQR_EOPT;
  set_kernel_attributes();
  sqr_basis* b = new sqr_basis();
  b->m = m; b->n = 0; b->cap = cap; b->Q = Q; b->ldq = ldq; b->R = R; b->ldr = ldr;
  b->opts = o;
  (void)hipGetDevice(&b->device);
  int rc = alloc_workspace(b, big_block(widest) ? widest : 0);
  if (rc) { sqr_free(b); return rc; }
  hipStream_t s = (hipStream_t)stream;
  int64_t c0 = 0;
  for (int64_t i = 0; i < r; ++i) {
    const int64_t c1 = edge(i + 1);
    const int64_t p = c1 - c0;
    if (p < 1) continue;
    Call c{1, b->n, p, A + c0 * lda, lda, b->Q + b->n * b->ldq, b->ldq};
    rc = run_call(b, c, s, true, 2);
    if (rc) { (void)hipStreamSynchronize(s); sqr_free(b); return rc; }
    if (b->ctrl_host->status != SQR_OK) break;   // the basis keeps the panels done so far
    b->n += p;
    c0 = c1;
  }
  *out = b;
  if (info) fill_info(b->ctrl_host, info);
  return b->ctrl_host->status;
}

int sqr_last_info(sqr_basis* b, sqr_info* info) {
  if (!b || !info) return SQR_ENULL;
  if (b->parked) {
    fill_info(&b->last, info);
    return info->status;
  }
  if (fetch(b, b->stream)) return SQR_EHIP;
  if (g_prof_on) prof_finalize(b->call_id, b->ctrl_host->passes);
  fill_info(b->ctrl_host, info);
  return info->status;
}

int64_t sqr_cols(const sqr_basis* b) { return b ? b->n : 0; }

void sqr_free(sqr_basis* b) {
  if (!b) return;
  (void)sqr_park(b);
  if (b->order_ev) (void)hipEventDestroy(b->order_ev);
  delete b;
}

int sqr_park(sqr_basis* b) {
  if (!b) return SQR_ENULL;
  if (!b->ws && !b->ctrl_host) return SQR_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return SQR_EHIP;
  if (b->ctrl_host) b->last = *b->ctrl_host;   // outcome of the last call
  b->parked = true;
  if (b->ws) {
    CachedWs e;
    e.ptr = b->ws; e.bytes = b->ws_bytes; e.device = b->device; e.pinned = b->ctrl_host;
    pool_put(e);
  } else if (b->ctrl_host) {
    (void)hipHostFree(b->ctrl_host);
  }
  b->ws = nullptr; b->ws_bytes = 0; b->ctrl_host = nullptr; b->ctrl_host_dev = nullptr;
  b->ctrl = nullptr; b->part = b->stage = b->X = b->bneg = b->rinv = nullptr;
  b->partc = b->stage_bt = b->btb = b->rold = nullptr;
  b->partg = b->stage_g = b->rt = b->vec = b->errpart = nullptr;
  b->pbig = 0;
  return SQR_OK;
}

void sqr_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (ProfRec& r : g_prof) { g_event_pool.push_back(r.e0); g_event_pool.push_back(r.e1); }
  g_prof.clear();
  g_prof_on = on != 0;
}

int sqr_prof_read(sqr_prof* out) {
  if (!out) return SQR_ENULL;
  memset(out, 0, sizeof(*out));
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int rc = SQR_OK;
  for (ProfRec& r : g_prof) {
    if (hipEventSynchronize(r.e1) != hipSuccess) { rc = SQR_EHIP; continue; }
    if (r.real == 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) { rc = SQR_EHIP; continue; }
    out->launches[r.kind] += 1;
    out->ms[r.kind] += ms;
    out->bytes[r.kind] += r.bytes;
  }
  for (ProfRec& r : g_prof) { g_event_pool.push_back(r.e0); g_event_pool.push_back(r.e1); }
  g_prof.clear();
  return rc;
}

}  // extern "C"
