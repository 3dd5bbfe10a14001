// sqr_api.hip -- host driver of libsqr: the C ABI declared in include/sqr.h.
//
// A call enqueues, on the caller's stream, an initial Gram pass and then
// Cholesky QR passes: the streaming kernels of the pass, a fixed-order
// reduction of the per-workgroup partial Gramians (reduce_slots) and one
// small_step.  The streaming kernels of a pass, by call and width (16-column
// blocks P):
//   orth, FP64, P = 1        narrow_pass (apply and Gramian in one launch)
//   orth, P = 2..7 (mixed 1..8)  wide_pass (one launch per pass)
//   orth, P = 8..16 (mixed 9..16)  wide_apply, then gram_pass (FP32 variant
//                            for the mixed form's early passes)
//   appends; orth, P > 16    block_pass, one launch per block
// The convergence decision is taken on the device; kernels of later passes
// exit at once after it.  With a host `info` the driver enqueues the passes
// the method normally needs, reads the device state once, and adds passes
// only when the device asks for them.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <vector>

#include "../../include/sqr.h"
#include "../../include/sqr_prof.h"

#include "sqr_kernels.hip"

using namespace sqr;

namespace {

constexpr int kMaxSlots = 1024;
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
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
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
  Ctrl* ctrl_host = nullptr;         // pinned, written by small_step
  Ctrl* ctrl_host_dev = nullptr;     // its device address
  double *part = nullptr, *stage = nullptr;
  double *X = nullptr;
  double *bneg = nullptr, *rinv = nullptr;
};

namespace {

typedef void (*BlockKernel)(BlockPassArgs);
// nt = S tiles per wave, wpt = waves sharing a row tile (4 / wpt row tiles
// in flight per workgroup); a variant covers nt * wpt tiles of S.
struct Variant { int nt, wpt; BlockKernel gram, apply; };
int g_occ[2][32];     // workgroups per CU of each variant (gram, apply)
int g_ncu = 0;
#define SQR_VARIANT(NT, W) {NT, W, block_pass<NT, W, false>, block_pass<NT, W, true>}
const Variant kVariants[] = {
  SQR_VARIANT(1, 1), SQR_VARIANT(1, 2), SQR_VARIANT(2, 2),
  SQR_VARIANT(2, 4), SQR_VARIANT(3, 4), SQR_VARIANT(4, 4), SQR_VARIANT(5, 4),
  SQR_VARIANT(6, 4), SQR_VARIANT(7, 4), SQR_VARIANT(8, 4), SQR_VARIANT(9, 4),
};
#undef SQR_VARIANT

// Whole-pass kernels of orth calls with up to 8 column blocks (FP64 calls use
// them from 2 blocks on; the mixed form from 1), with FP64 or FP32 Gramians.
typedef void (*WideKernel)(WidePassArgs);
struct WideVariant { WideKernel k[2][2]; };   // [fp32 gram][apply]
#define SQR_WIDE(NB) {{{wide_pass<NB, false, false>, wide_pass<NB, true, false>}, \
                       {wide_pass<NB, false, true>, wide_pass<NB, true, true>}}}
constexpr int kWideMin = 1, kWideMax = 8;
const WideVariant kWide[] = {SQR_WIDE(1), SQR_WIDE(2), SQR_WIDE(3), SQR_WIDE(4),
                             SQR_WIDE(5), SQR_WIDE(6), SQR_WIDE(7), SQR_WIDE(8)};
#undef SQR_WIDE
int g_wide_occ[2][2][kWideMax - kWideMin + 1];   // [fp32][apply][nb]

// FP64 orth calls of one block (at most 16 columns): [Gram only, apply].
const WideKernel kNarrow[2] = {narrow_pass<false>, narrow_pass<true>};
int g_narrow_occ[2];

// Orth calls of 8..16 blocks: a whole-pass apply and a Gramian kernel
// (FP64, and FP32 for the mixed form).
typedef void (*SplitKernel)(WidePassArgs);
struct SplitVariant { SplitKernel apply, gram, gram32; };
#define SQR_SPLIT(NB) {wide_apply<NB>, gram_pass<NB, false>, gram_pass<NB, true>}
constexpr int kSplitMin = 8, kSplitMax = 16;
const SplitVariant kSplit[] = {SQR_SPLIT(8), SQR_SPLIT(9), SQR_SPLIT(10), SQR_SPLIT(11), SQR_SPLIT(12),
                               SQR_SPLIT(13), SQR_SPLIT(14), SQR_SPLIT(15), SQR_SPLIT(16)};
#undef SQR_SPLIT
int g_split_occ[3][kSplitMax - kSplitMin + 1];   // [0 gram, 1 apply, 2 gram32][nb]
size_t split_lds_bytes(int nb, bool apply) {
  return 8 * (size_t)(apply ? apply_lds_doubles(nb) : gram_op_doubles(nb));
}
size_t gram32_lds_bytes(int nb) { return 4 * (size_t)gram_op_doubles(nb); }
size_t wide_lds_bytes(int nb, bool apply) {
  return 8 * ((size_t)(apply ? wide_panel_doubles(nb) : 0) + (size_t)wide_op_doubles(nb));
}

// Smallest variant whose S capacity covers ns tiles (listed by capacity).
const Variant* pick_variant(int ns) {
  for (const Variant& v : kVariants)
    if (v.nt * v.wpt >= std::max(ns, 1)) return &v;
  return nullptr;
}

size_t block_lds_bytes(const Variant& v, bool apply) {
  // main loop: partial T tiles + transposition tiles (the final cross-group
  // reduction, at most 4 groups x 2 tiles or 2 groups x 5 tiles, fits in
  // them); the apply adds its operands C_J (16 nt wpt rows) and D_J
  return 8 * ((size_t)2 * kWaves * kTPart + (size_t)kWaves * 16 * kYPitch +
              (apply ? (size_t)v.nt * v.wpt * 256 + 256 : 0));
}

// Kernel attributes and occupancies, once per process (std::call_once: the
// serving loop calls the library from several threads at once).
std::once_flag g_attr_once;
void set_kernel_attributes_once() {
  for (const Variant& v : kVariants) {
    (void)hipFuncSetAttribute((const void*)v.gram, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
    (void)hipFuncSetAttribute((const void*)v.apply, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
  }
  if (hipFuncSetAttribute((const void*)small_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kSmallLdsBytes) != hipSuccess) {
    (void)hipGetLastError();   // consumed here: arenas then live in the workspace
    g_small_lds = 0;
  }
  for (int nb = kWideMin; nb <= kWideMax; ++nb)
    for (int g32 = 0; g32 < 2; ++g32)
      for (int ap = 0; ap < 2; ++ap)
        (void)hipFuncSetAttribute((const void*)kWide[nb - kWideMin].k[g32][ap],
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)wide_lds_bytes(nb, ap != 0));
  for (int nb = kSplitMin; nb <= kSplitMax; ++nb) {
    (void)hipFuncSetAttribute((const void*)kSplit[nb - kSplitMin].apply,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)split_lds_bytes(nb, true));
    (void)hipFuncSetAttribute((const void*)kSplit[nb - kSplitMin].gram,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)split_lds_bytes(nb, false));
    (void)hipFuncSetAttribute((const void*)kSplit[nb - kSplitMin].gram32,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)gram32_lds_bytes(nb));
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
    int n = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)kNarrow[ap], kThreads, 0) != hipSuccess || n < 1)
      n = 1;
    g_narrow_occ[ap] = n;
  }
}
void set_kernel_attributes() { std::call_once(g_attr_once, set_kernel_attributes_once); }

// Worst-case sizes over every call the handle can make (q + p <= cap).
int64_t worst_total_len(int64_t cap) {
  int64_t w = 0;
  for (int64_t p = 1; p <= cap; ++p) w = std::max(w, total_len(cap - p, p));
  return w;
}
int64_t worst_bneg_len(int64_t cap) {
  int64_t w = 0;
  for (int64_t p = 1; p <= cap; ++p) w = std::max(w, bneg_len(cap - p, p));
  return w;
}

// Sizes (doubles) of the workspace regions of a handle.
struct WsSizes { int64_t tl, arena, bneg, rinv; };

// Every call a handle of capacity cap can make (q + p <= cap).
WsSizes handle_sizes(int64_t cap) {
  WsSizes z;
  z.tl = worst_total_len(cap);
  z.arena = 0;
  for (int64_t p = 1; p <= cap; ++p) z.arena = std::max<int64_t>(z.arena, small_arena((int)(cap - p), (int)p));
  z.bneg = worst_bneg_len(cap);
  z.rinv = nblocks(cap) * 256;
  return z;
}

// One orthogonalisation of n columns (no later appends).
WsSizes orth_sizes(int64_t n) {
  return WsSizes{total_len(0, n), small_arena(0, (int)n), bneg_len(0, n), nblocks(n) * 256};
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
  if (base) {
    b->slots = slots;
    b->part = base + o_part; b->stage = base + o_stage;
    b->X = base + o_X;
    b->bneg = base + o_bneg; b->rinv = base + o_rinv;
    b->ctrl = (Ctrl*)(base + o_ctrl);
  }
  return doubles;
}

int alloc_workspace(sqr_basis* b) {
  const WsSizes z = handle_sizes(b->cap);
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

int launch_gram(sqr_basis* b, const Call& c, int phase, hipStream_t s) {
  const int64_t P = nblocks(c.p);
  const int64_t tl = total_len(c.q, c.p);
  const int64_t tiles = (b->m + 15) / 16;
  const bool apply = phase > 0;
  int64_t nwg = b->slots;
  const bool mixed = c.mode == 0 && b->opts.precision == 1;
  if (c.mode == 0 && P >= kSplitMin && P <= kSplitMax && (!mixed || P > kWideMax)) {
    // apply (from pass 1 on), then the Gramian of its result
    const int idx = (int)P - kSplitMin;
    const int64_t steps = (tiles + kWaves - 1) / kWaves;
    WidePassArgs w;
    memset(&w, 0, sizeof(w));
    w.n = (int)c.p; w.m = b->m;
    w.bneg = b->bneg; w.rinv = b->rinv;
    w.part = b->part; w.part_stride = tl;
    w.done = phase > 0 ? &b->ctrl->done : nullptr;
    w.passes = &b->ctrl->passes;
    auto launch = [&](const void* k, int64_t grid, int threads, size_t lds) {
      void* args[] = {&w};
      return hipLaunchKernel(k, dim3((unsigned)grid), dim3(threads), args, lds, s) == hipSuccess;
    };
    // launches between one pair of profiling events (the mixed form's two
    // Gramian variants count as one launch: one of them exits at once)
    auto timed = [&](int kind, double bytes, auto&& enqueue) {
      const ProfRec rec = prof_begin(kind, bytes, b->noprof ? -1 : b->call_id, phase, s);
      if (!enqueue()) return false;
      prof_end(rec, s);
      return true;
    };
    if (apply) {
      w.win = (phase > 1) ? c.y : c.win;
      w.ldw = (phase > 1) ? c.ldy : c.ldw;
      w.yout = c.y; w.ldy = c.ldy;
      w.copy_if_done = (phase == 1);
      const int64_t ga = std::max<int64_t>(1, std::min<int64_t>((int64_t)g_ncu * g_split_occ[1][idx], steps));
      if (!timed(1, 16.0 * (double)b->m * (double)c.p, [&] {
            return launch((const void*)kSplit[idx].apply, ga, kThreads, split_lds_bytes((int)P, true));
          }))
        return SQR_EHIP;
    }
    // the Gramian of the pass's result (of the input at phase 0); the mixed
    // form launches the FP32 variant at phase 0 and both variants later, the
    // one that does not match the device's choice (ctrl->gram32) exits at
    // once.  Both fill the same nwg slots.
    w.win = apply ? c.y : c.win;
    w.ldw = apply ? c.ldy : c.ldw;
    w.copy_if_done = 0;
    const int occ = mixed ? std::min(g_split_occ[0][idx], g_split_occ[2][idx]) : g_split_occ[0][idx];
    nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * occ);
    nwg = std::max<int64_t>(1, std::min<int64_t>(nwg, steps));
    w.gram32 = (mixed && phase > 0) ? &b->ctrl->gram32 : nullptr;
    if (!timed(0, 8.0 * (double)b->m * (double)c.p, [&] {
          if (mixed && !launch((const void*)kSplit[idx].gram32, nwg, kGramThreads, gram32_lds_bytes((int)P)))
            return false;
          return (mixed && phase == 0) ||
                 launch((const void*)kSplit[idx].gram, nwg, kGramThreads, split_lds_bytes((int)P, false));
        }))
      return SQR_EHIP;
  } else if (c.mode == 0 && P == 1 && !mixed) {
    // one block: the whole pass in one launch, every wave on its own tiles
    nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * g_narrow_occ[apply ? 1 : 0]);
    nwg = std::max<int64_t>(1, std::min<int64_t>(nwg, (tiles + kWaves - 1) / kWaves));
    WidePassArgs w;
    memset(&w, 0, sizeof(w));
    w.win = (apply && phase > 1) ? c.y : c.win;
    w.ldw = (apply && phase > 1) ? c.ldy : c.ldw;
    w.yout = c.y; w.ldy = c.ldy;
    w.n = (int)c.p; w.m = b->m;
    w.rinv = b->rinv;
    w.part = b->part; w.part_stride = tl;
    w.done = phase > 0 ? &b->ctrl->done : nullptr;
    w.passes = &b->ctrl->passes;
    w.copy_if_done = (phase == 1);
    void* args[] = {&w};
    const ProfRec rec = prof_begin(apply ? 1 : 0, 8.0 * (double)b->m * (double)c.p * (apply ? 2.0 : 1.0),
                                   b->noprof ? -1 : b->call_id, phase, s);
    if (hipLaunchKernel((const void*)kNarrow[apply ? 1 : 0], dim3((unsigned)nwg), dim3(kThreads), args, 0, s) !=
        hipSuccess)
      return SQR_EHIP;
    prof_end(rec, s);
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
    void* args[] = {&w};
    const ProfRec rec = prof_begin(apply ? 1 : 0, 8.0 * (double)b->m * (double)c.p * (apply ? 2.0 : 1.0),
                                   b->noprof ? -1 : b->call_id, phase, s);
    for (int g32 = mixed ? 1 : 0; g32 >= 0; --g32) {
      // phase 0 of the mixed form is an FP32 Gramian; later phases follow the
      // device (ctrl->gram32); FP64 calls launch the FP64 variant only
      if (mixed && phase == 0 && g32 == 0) break;
      w.gram32 = (mixed && phase > 0) ? &b->ctrl->gram32 : nullptr;
      const WideKernel k = kWide[idx].k[g32][apply ? 1 : 0];
      if (hipLaunchKernel((const void*)k, dim3((unsigned)nwg), dim3(kThreads), args,
                          wide_lds_bytes((int)P, apply), s) != hipSuccess)
        return SQR_EHIP;
    }
    prof_end(rec, s);
  } else {
  // One grid size for every block of the pass (the slots are reduced
  // together): resident workgroups of the most demanding block's variant,
  // capped by the slot capacity and by the row tiles available.
  for (int64_t J = 0; J < P; ++J) {
    const int ks = (int)round16(c.q) + (int)(16 * J);
    const Variant* v = pick_variant((ks + 15) / 16);
    if (!v) return SQR_EDIM;
    const int occ = g_occ[apply ? 1 : 0][variant_index(v)];
    nwg = std::min<int64_t>(nwg, (int64_t)g_ncu * occ);
    nwg = std::min<int64_t>(nwg, (tiles + (kWaves / v->wpt) - 1) / (kWaves / v->wpt));
  }
  nwg = std::max<int64_t>(nwg, 1);
  for (int64_t J = 0; J < P; ++J) {
    BlockPassArgs a;
    memset(&a, 0, sizeof(a));
    const double* src = (apply && phase > 1) ? c.y : c.win;
    const int64_t lds = (apply && phase > 1) ? c.ldy : c.ldw;
    a.win = src + J * 16 * lds; a.ldw = lds;
    a.yout = c.y + J * 16 * c.ldy; a.ldy = c.ldy;
    a.s1 = b->Q; a.ld1 = b->ldq; a.n1 = (int)c.q;
    // same-pass prefix: new values after an apply, the input for the first Gram
    a.s2 = apply ? c.y : c.win; a.ld2 = apply ? c.ldy : c.ldw; a.n2 = (int)(16 * J);
    a.pb = (int)std::min<int64_t>(16, c.p - 16 * J);
    a.m = b->m;
    a.bneg = b->bneg + bneg_off(c.q, J);
    a.rinv = b->rinv + 256 * J;
    a.part = b->part; a.part_stride = tl; a.part_off = e_off(c.q, J);
    a.done = phase > 0 ? &b->ctrl->done : nullptr;  // phase 0 starts the call
    a.passes = &b->ctrl->passes;
    a.copy_if_done = (phase == 1);
    const int ks = (int)round16(a.n1) + a.n2;   // columns of S with the padding
    const Variant* v = pick_variant((ks + 15) / 16);
    void* args[] = {&a};
    // algorithmic bytes: the real columns of S (no padding), the block read,
    // and (apply) the block written
    const ProfRec rec = prof_begin(apply ? 1 : 0, 8.0 * (double)b->m * (double)(a.n1 + a.n2 + (apply ? 2 : 1) * a.pb),
                                   b->noprof ? -1 : b->call_id, phase, s);
    if (hipLaunchKernel((const void*)(apply ? v->apply : v->gram), dim3((unsigned)nwg),
                        dim3(kThreads), args, block_lds_bytes(*v, apply), s) != hipSuccess)
      return SQR_EHIP;
    prof_end(rec, s);
  }
  }
  // Fixed-order reduction of the nwg slots into the pass's Gramian blocks.
  hipLaunchKernelGGL(reduce_slots, dim3((unsigned)((tl + kRedElems - 1) / kRedElems)), dim3(64 * kRedWaves), 0, s,
                     (const double*)b->part, (int)nwg, tl, tl, b->stage,
                     phase > 0 ? (const int*)&b->ctrl->done : (const int*)nullptr);
  SmallArgs k;
  memset(&k, 0, sizeof(k));
  k.E = b->stage;
  k.mode = c.mode; k.q = (int)c.q; k.p = (int)c.p; k.nblk = (int)P;
  k.m = b->m; k.phase = phase;
  k.R = b->R; k.ldr = b->ldr;
  k.X = b->X;
  k.bneg = b->bneg; k.rinv = b->rinv; k.ctrl = b->ctrl;
  k.hctrl = b->ctrl_host_dev; k.stamp_base = b->call_id * 256;
  k.first_pass_shift = b->opts.first_pass_shift; k.min_passes = b->opts.min_passes;
  k.max_iter = b->opts.max_iter; k.max_escalations = b->opts.max_escalations;
  k.power_steps = b->opts.power_steps; k.tol = b->opts.tol; k.u = b->opts.unit_roundoff;
  k.shift_policy = b->opts.shift_policy; k.shift_dim = b->opts.append_shift_dim;
  k.mixed = mixed ? 1 : 0;
  const size_t arena = 8 * (size_t)small_arena((int)c.q, (int)c.p);
  const size_t mbytes = 8 * (size_t)c.p * (size_t)c.p;
  k.lds_matrices = (arena <= g_small_lds) ? 1 : (mbytes <= g_small_lds ? 2 : 0);
  const size_t dyn = k.lds_matrices == 1 ? arena : (k.lds_matrices == 2 ? mbytes : 0);
  hipLaunchKernelGGL(small_step, dim3(1), dim3(kSmallThreads), dyn, s, k);
  return hipGetLastError() == hipSuccess ? SQR_OK : SQR_EHIP;
}

int fetch(sqr_basis* b, hipStream_t s) {
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
int run_call(sqr_basis* b, const Call& c, hipStream_t s, bool sync, int spec) {
  if (b->used && s != b->stream) {
    // Kernels of the previous call (no-op launches of a finished call among
    // them) may still be queued on its stream and read the control block
    // that this call resets: this stream waits for all of them.
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
  int rc = launch_gram(b, c, 0, s);
  if (rc) return rc;
  const int maxit = b->opts.max_iter;
  int enq = 0;
  const int first = sync ? std::min(spec, maxit) : maxit;
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
  if (cap > kMaxSCols || lda > kMaxLd || ldq > kMaxLd) return SQR_EDIM;
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
  int rc = alloc_workspace(b);
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
  if (p < 1 || ldw < b->m || ldw > kMaxLd || b->n + p > b->cap || b->n + p > b->m) return SQR_EDIM;
  if (!b->ws) {   // parked: take a workspace again
    const int rc0 = alloc_workspace(b);
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
