// sqr_kernels.hip -- CDNA4 (gfx950) kernels of shifted Cholesky QR and the
// Cholesky QR block append (arXiv 2507.07788, Algorithms 1 and 2).
//
// The tall operands stay in HBM, column-major.  A pass over them is split
// into 16-column blocks.  In the general form (appends, and orthogonalisations
// wider than 256 columns) one launch of `block_pass` per block J streams
// 16-row tiles and, per tile,
//   (1) forms Y_J = W_J D_J + S C_J, where D_J is the inverse of the 16x16
//       diagonal block of R~ and C_J = -[B~_J; R~_<J,J] D_J: the
//       Q <- (Q - Q_in B~) R~^{-1} step of Algorithm 2 (Q <- Q R~^{-1} of
//       Algorithm 1) as a blocked triangular solve whose diagonal blocks are
//       multiplied by their inverses,
//   (2) writes Y_J and accumulates the partial Gramian [S Y_J]^T Y_J of the
//       next pass (Algorithm 1's X <- Q^T Q; Algorithm 2's B~ <- Q_in^T Q and
//       Q^T Q), so every pass reads the tall data once.
// S is the concatenation of the existing basis Q_in and the blocks < J of the
// same pass.  All contractions run on v_mfma_f64_16x16x4f64.  Every workgroup
// writes its partial Gramian to its own slot; `reduce_slots` sums the slots
// in a fixed order (no atomics), so results do not depend on scheduling.
// Orthogonalisations of up to 256 columns have whole-pass kernels with the
// same arithmetic: `narrow_pass` (one block), `wide_pass` (up to 8 blocks),
// `wide_apply` + `gram_pass` (8 to 16 blocks).
//
// `small_step` is a one-workgroup kernel that finishes a pass: from the
// reduced Gramian it forms the Schur complement X = G - B~^T B~ (Prop. 2.1), tests
// ||X - I||_F, picks the shift (Algorithm 1: recomputed from ||X||_2;
// Algorithm 2: x10 escalation), factors X + sigma I, updates R and B, and
// prepares the operands of the next pass.  Control decisions stay on the
// device; later kernels of a finished call exit at once.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "sqr_device.h"

namespace sqr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  // D = A (16x4) * B (4x16) + C.  Lane l supplies A[l%16][l/16] and
  // B[l/16][l%16]; it holds D[l/16 + 4r][l%16] in register r.
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  // FP32 counterpart (same operand lanes); lane l holds D[4 (l/16) + r][l%16]
  // in register r.
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Wave-private LDS hand-off: every lane's earlier LDS writes are complete and
// visible to the other lanes of the wave.
// Buffer descriptor over `bytes` bytes from `base` (range-checked loads past
// the end return zero).  Ranges above 4 GiB are clamped to the 32-bit limit;
// every offset used with a descriptor stays below 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const uint32_t n = bytes <= 0 ? 0u : (bytes >= 0xffffffffLL ? 0xffffffffu : (uint32_t)bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, 0x00020000);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The LDS instructions of one wave are performed in the order they are
// issued, so a wave-private exchange (lanes write, then read what other lanes
// of the same wave wrote) needs no wait for the writes to complete: only the
// compiler must keep the order of the accesses.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Batched launches: the workgroups of call c are start[c] .. start[c+1]-1 of
// the grid; each reads its call's argument block from the table.
template <class T>
__device__ __forceinline__ int batch_call(const BatchTable<T>& t) {
  int lo = 0, hi = t.ncalls - 1;   // largest c with start[c] <= blockIdx.x
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t.start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kWaves = 4;             // waves per workgroup of block_pass
constexpr int kThreads = 64 * kWaves;
constexpr int kYPitch = 17;           // LDS row pitch of a 16x16 tile (doubles)

// S is the concatenation [s1 (n1 columns) | zero padding up to q16 = n1
// rounded up to 16 | s2 (n2 columns, a multiple of 16)], so every 16-column
// tile of S lies in a single segment and is read through one buffer
// descriptor.  ks = q16 + n2 columns in all.
//
// Work split: the four waves of a workgroup form 4/WPT groups of WPT waves;
// each group processes its own 16-row tile per step, so a workgroup keeps
// 4/WPT tiles in flight.  Within a group the 16-column tiles of S are dealt
// out round-robin (tile I -> member I % WPT), so each wave keeps only its
// share of S, of -B~ and of the Gram accumulators in registers.  With
// WPT > 1 the members' partial sums of S B~ meet in LDS (fixed order) and
// every member forms the same Y tile.  Member 0 of a group owns the block
// input, the Y store and Y^T Y.  Groups' Gram partials are summed in group
// order at the end.
constexpr int kTPart = 256;    // doubles per 16x16 tile in LDS

// Waves per SIMD the register allocation must leave room for: three for the
// variants up to 12 S tiles (their LDS allows three workgroups per CU), one
// for the wider ones, two for the Gram-only pairs of 3..6 tiles per wave.
template <int NTW, int WPT, bool APPLY>
__device__ __forceinline__ void block_pass_body(const BlockPassArgs& a, const int bid, const int nwg) {
  // LDS: double-buffered partial T tiles (2 x 4 x 256 doubles), then one
  // 16x17 transposition tile per wave; the final cross-group reduction
  // reuses the area.
  extern __shared__ double lds[];
  constexpr int G = kWaves / WPT;      // row tiles in flight per workgroup
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int grp = wave / WPT;          // row-tile group
  const int mem = wave % WPT;          // member within the group
  const int x = lane & 15;
  const int g = lane >> 4;
  const int64_t tiles = (a.m + 15) / 16;
  // The row tiles are dealt out round-robin: local tile i of this workgroup
  // is row tile i nwg + bid, so the workgroups of the grid stream one band of
  // rows together.
  const int64_t tw = tiles > bid ? (tiles - 1 - bid) / nwg + 1 : 0;
  auto tile_of = [&](int64_t i) { return i * nwg + bid; };

  if (a.done && *a.done) {
    // A finished call: nothing to do, except that the first apply of a call
    // that converged before any pass copies the input block to the output.
    if (APPLY && a.copy_if_done && *a.passes == 0) {
      for (int64_t i = wave; i < tw; i += kWaves) {
        const int64_t row = tile_of(i) * 16 + x;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = g + 4 * r;
          if (row < a.m && col < a.pb)
            a.yout[(int64_t)col * a.ldy + row] = a.win[(int64_t)col * a.ldw + row];
        }
      }
    }
    return;
  }

  const int q16 = (a.n1 + 15) & ~15;   // basis segment padded to whole tiles
  const int ks = q16 + a.n2;            // columns of S (a multiple of 16)
  const int nk = ks >> 2;              // k-slices of four S columns
  const int ns = (ks + 15) >> 4;       // 16-column tiles of S
  double* tpart = lds;                                   // [2][4][256]
  double* tr = lds + 2 * kWaves * kTPart + wave * 16 * kYPitch;
  const int hi1 = a.n1 - 1, hi2 = a.n2 - 1;              // last column of each S segment

  // A operands of the apply, kept in LDS (not registers, for occupancy):
  // the rows of C_J (zero past the end of S) and the inverse diagonal block
  // D_J; k-slice s of C_J is read as C[4s + g][x], k-slice r of D_J as
  // D[g + 4r][x].
  constexpr int kCop = NTW * WPT * 256;   // rows 16 NTW WPT of 16 doubles
  double* cop = lds + 2 * kWaves * kTPart + kWaves * 16 * kYPitch;
  if (APPLY) {
    for (int e = threadIdx.x; e < kCop; e += kThreads) cop[e] = (e < ks * 16) ? a.bneg[e] : 0.0;
    for (int e = threadIdx.x; e < 256; e += kThreads) cop[kCop + e] = a.rinv[e];
    __syncthreads();
  }

  d4 acc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  d4 accg = d4{0.0, 0.0, 0.0, 0.0};

  // Step k of a group handles local tile k G + grp.  The member that owns
  // step k (k mod WPT) adds W_J D_J to the apply, stores Y and accumulates
  // Y^T Y, so this extra work rotates over the members (and their SIMDs).
  // In the apply only the owner needs the block input; in the Gram-only pass
  // every member does (Y = W).
  const int nsteps = (int)((tw + G - 1) / G);   // the same for every wave
  // Loads of one step: my S slices and (if needed) the block input.  One
  // buffer descriptor per 16-column tile: base at the tile's first column,
  // range = bytes up to the end of its segment's last column, so columns past
  // a segment (padding, tiles past the end of S) read zero in hardware.  Lane
  // (x, g) of slice jj adds ((4 jj + g) ld + row) * 8, below 4 GiB for the
  // leading dimensions the library accepts.  A tile past the range is
  // clamped to a valid one and its rows are masked when it is used (keep),
  // not here, so the loads stay in flight until then.
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.win, ((int64_t)(a.pb - 1) * a.ldw + a.m) * 8);
  auto load_step = [&](int k, double (&sreg)[NTW][4], d4& w, uint64_t& keep) {
    const int64_t li = (int64_t)k * G + grp;
    const int64_t row = tile_of(min(li, max(tw - 1, (int64_t)0))) * 16 + x;
    keep = (li < tw && row < a.m) ? ~0ull : 0ull;
    const int64_t rowc = row < a.m ? row : a.m - 1;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const int I = mem + WPT * j;
      const bool first = (16 * I < q16) || a.n2 == 0;
      const int cs = first ? 16 * I : 16 * I - q16;
      const int hi = first ? hi1 : hi2;
      const int64_t ld = first ? a.ld1 : a.ld2;
      const double* base = (first ? a.s1 : a.s2) + (int64_t)cs * ld;
      const int64_t nrec = (hi >= cs) ? (((int64_t)(hi - cs) * ld + a.m) * 8) : 0;
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, nrec);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const uint32_t o = (uint32_t)(((int64_t)(4 * jj + g) * ld + rowc) * 8);
        sreg[j][jj] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)o, 0, 0));
      }
    }
    // block input in D layout: lane (x, g) register r holds W[row x][col
    // g + 4r]; columns past pb lie outside the buffer range and read zero
    if (!APPLY || k % WPT == mem) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t ow = (uint32_t)(((int64_t)(g + 4 * r) * a.ldw + rowc) * 8);
        w[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rw, (int)ow, 0, 0));
      }
    }
  };
  auto masked = [](double v, uint64_t keep) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & keep);
  };

  auto do_step = [&](int k, const double (&sreg)[NTW][4], const d4& wraw, uint64_t keep) {
    const int64_t li = (int64_t)k * G + grp;
    const bool tile_ok = li < tw;
    const int64_t tile = tile_of(li);
    const int64_t row = tile * 16 + x;
    const bool row_ok = keep != 0;
    const bool own = k % WPT == mem;     // wave-uniform
    d4 y;
    if (APPLY) {
      // Partial Y^T over my slices (two chains): Y_J = W_J D_J + S C_J with
      // C_J = -B~_J D_J.  The owner adds D^T W^T: register r of W^T (D
      // layout) is the B operand of k-slice r.
      d4 c0 = d4{0.0, 0.0, 0.0, 0.0};
      d4 c1 = d4{0.0, 0.0, 0.0, 0.0};
      if (own) {
        c0 = mfma(cop[kCop + (g + 0) * 16 + x], masked(wraw[0], keep), c0);
        c1 = mfma(cop[kCop + (g + 4) * 16 + x], masked(wraw[1], keep), c1);
        c0 = mfma(cop[kCop + (g + 8) * 16 + x], masked(wraw[2], keep), c0);
        c1 = mfma(cop[kCop + (g + 12) * 16 + x], masked(wraw[3], keep), c1);
      }
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        if (mem + WPT * j < ns) {   // tile slots past the end of S hold zeros
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const double bv = cop[(16 * (mem + WPT * j) + 4 * jj + g) * 16 + x];
            if (jj & 1) c1 = mfma(bv, sreg[j][jj], c1);
            else        c0 = mfma(bv, sreg[j][jj], c0);
          }
        }
      }
      y = c0 + c1;
      if (WPT > 1) {
        double* tp = tpart + ((k & 1) * kWaves + wave) * kTPart;
#pragma unroll
        for (int r = 0; r < 4; ++r) tp[r * 64 + lane] = y[r];
        __syncthreads();
        // Y^T = sum of the group's partials in member order.
        y = d4{0.0, 0.0, 0.0, 0.0};
        const double* tb = tpart + ((k & 1) * kWaves + grp * WPT) * kTPart;
#pragma unroll
        for (int v = 0; v < WPT; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) y[r] += tb[v * kTPart + r * 64 + lane];
      }
      if (!row_ok) y = d4{0.0, 0.0, 0.0, 0.0};
      if (own && tile_ok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = g + 4 * r;
          if (row_ok && col < a.pb) a.yout[(int64_t)col * a.ldy + row] = y[r];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) y[r] = masked(wraw[r], keep);
    }
    // Y through wave-private LDS: the row index becomes the contraction index
    // (k-slot g of slice u <-> row g + 4u).
#pragma unroll
    for (int r = 0; r < 4; ++r) tr[x * kYPitch + g + 4 * r] = y[r];
    wave_lds_order();
    double yb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) yb[u] = tr[(g + 4 * u) * kYPitch + x];
    wave_lds_order();
    if (own) {
#pragma unroll
      for (int u = 0; u < 4; ++u) accg = mfma(yb[u], yb[u], accg);
    }
    // My S tiles through the same LDS tile: sreg[j][jj] = S[row x][16I + 4jj + g].
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      if (mem + WPT * j >= ns) continue;   // no such tile of S
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) tr[x * kYPitch + 4 * jj + g] = sreg[j][jj];
      wave_lds_order();
      double sa[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) sa[u] = tr[(g + 4 * u) * kYPitch + x];
      wave_lds_order();
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[j] = mfma(sa[u], yb[u], acc[j]);
    }
  };

  // Two register buffers: the loads of step k + 1 land in one while step k
  // computes on the other (no copies, so no wait for the loads in flight).
  double sb0[NTW][4], sb1[NTW][4];
  d4 wb0 = d4{0.0, 0.0, 0.0, 0.0}, wb1 = d4{0.0, 0.0, 0.0, 0.0};
  uint64_t kb0, kb1;
  load_step(0, sb0, wb0, kb0);
  for (int k = 0; k < nsteps; k += 2) {
    load_step(k + 1, sb1, wb1, kb1);
    do_step(k, sb0, wb0, kb0);
    if (k + 1 >= nsteps) break;
    load_step(k + 2, sb0, wb0, kb0);
    do_step(k + 1, sb1, wb1, kb1);
  }
  if (WPT > 1) {
    // Y^T Y partials of the members (each over the steps it owned), summed
    // in member order into member 0 of the group.
    __syncthreads();
    double* ga = lds;
#pragma unroll
    for (int r = 0; r < 4; ++r) ga[wave * kTPart + (g + 4 * r) * 16 + x] = accg[r];
    __syncthreads();
    if (mem == 0) {
      accg = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int v = 0; v < WPT; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) accg[r] += ga[(grp * WPT + v) * kTPart + (g + 4 * r) * 16 + x];
    }
  }

  // Slot layout: rows 0..ks-1 hold S^T Y, rows ks..ks+15 hold Y^T Y, 16
  // doubles per row.  Tile I row (g + 4r) is S column 16I + g + 4r.
  double* out = a.part + (int64_t)bid * a.part_stride + a.part_off;
  if (G == 1) {
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const int I = mem + WPT * j;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = 16 * I + g + 4 * r;
        if (I < ns && rr < ks) out[rr * 16 + x] = acc[j][r];
      }
    }
    if (mem == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(ks + g + 4 * r) * 16 + x] = accg[r];
    }
  } else {
    // Groups hold partials of the same tiles: sum them in group order.
    // red[grp][slot]: slot mem + WPT*j for S tiles, WPT*NTW for Y^T Y.
    constexpr int kSlots = WPT * NTW + 1;
    __syncthreads();
    double* red = lds;
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[(grp * kSlots + mem + WPT * j) * kTPart + (g + 4 * r) * 16 + x] = acc[j][r];
    if (mem == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[(grp * kSlots + WPT * NTW) * kTPart + (g + 4 * r) * 16 + x] = accg[r];
    }
    __syncthreads();
    const int rows = ks + 16;
    for (int e = threadIdx.x; e < rows * 16; e += kThreads) {
      const int rr = e >> 4, c = e & 15;
      const int slot = (rr < ks) ? (rr >> 4) : WPT * NTW;
      const int within = (rr < ks) ? (rr & 15) : (rr - ks);
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < G; ++v) s += red[(v * kSlots + slot) * kTPart + within * 16 + c];
      out[e] = s;
    }
  }
}

template <int NTW, int WPT, bool APPLY>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WPT == 2 && NTW >= 3 ? 2 : (NTW * WPT <= 12 ? 3 : 1))))
void block_pass(BlockPassArgs a) {
  block_pass_body<NTW, WPT, APPLY>(a, blockIdx.x, gridDim.x);
}
template <int NTW, int WPT, bool APPLY>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WPT == 2 && NTW >= 3 ? 2 : (NTW * WPT <= 12 ? 3 : 1))))
void block_pass_batch(BatchTable<BlockPassArgs> t) {
  const int c = batch_call(t);
  block_pass_body<NTW, WPT, APPLY>(t.args[c], blockIdx.x - t.start[c], t.start[c + 1] - t.start[c]);
}


// Sum the nslots partial slots element-wise.  A workgroup covers kRedElems
// elements; lane (sub, e) of wave w reads element e of slots
// 4w + sub + 64k, k = 0, 1, ... (each load instruction takes 128 contiguous
// bytes from four slots), summing them in k order; the four sub-sums of a
// wave are added by a fixed butterfly, and the 16 wave sums in wave order.
// The order of every addition is fixed by nslots alone.
constexpr int kRedWaves = 16;
constexpr int kRedElems = 16;
__device__ __forceinline__ void reduce_slots_body(const ReduceArgs& a, const int bid) {
  const double* __restrict__ in = a.in;
  const int nslots = a.nslots;
  const int64_t stride = a.stride, len = a.len;
  double* __restrict__ out = a.out;
  const int* done = a.done;
  __shared__ double part[kRedWaves][kRedElems];
  if (done && *done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int e = lane & (kRedElems - 1), sub = lane >> 4;
  const int64_t el = (int64_t)bid * kRedElems + e;
  double s = 0.0;
  if (el < len) {
#pragma unroll 4
    for (int i = 4 * wv + sub; i < nslots; i += 4 * kRedWaves) s += in[(int64_t)i * stride + el];
  }
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  if (sub == 0) part[wv][e] = s;
  __syncthreads();
  if (wv == 0 && sub == 0 && el < len) {
    double t = 0.0;
#pragma unroll
    for (int v = 0; v < kRedWaves; ++v) t += part[v][e];
    out[el] = t;
  }
}

__global__ __launch_bounds__(64 * kRedWaves) void reduce_slots(ReduceArgs a) { reduce_slots_body(a, blockIdx.x); }
__global__ __launch_bounds__(64 * kRedWaves) void reduce_slots_batch(BatchTable<ReduceArgs> t) {
  const int c = batch_call(t);
  reduce_slots_body(t.args[c], blockIdx.x - t.start[c]);
}


// Offset (in doubles) of block J's partial Gramian inside a reduced slot:
// block J' holds (q16 + 16 J' + 16) rows of 16 doubles, q16 = q rounded up to
// 16 (rows q..q16-1 belong to the zero padding of S and are ignored).
__device__ __forceinline__ int64_t e_off(int q16, int J) {
  return 16 * ((int64_t)J * (q16 + 16) + 8 * (int64_t)J * (J - 1));
}

// ---------------------------------------------------------------------------
// narrow_pass: one launch per pass of an orth call of at most 16
// columns (G32: the mixed form's FP32 Gramian).  With one block the apply is Y = W D (D the inverse of R~;
// none in the Gram-only pass) and the Gramian is Y^T Y.  With lane (x, g),
// reg s holding W[row x][col 4s + g] (as loaded) and D[4s + g][x],
//   sum_s mfma(w_s, d_s) = W D,     reg r = Y[row g + 4r][col x]
//                                   (the A and B operand layout of Y^T Y),
//   sum_s mfma(d_s, w_s) = D^T W^T, reg r = Y[row x][col g + 4r]
//                                   (the load layout: the earlier factors of
//                                   a recomputed pass).
// The Gram-only pass brings W into the operand layout, and a storing pass
// brings Y back to rows across lanes (coalesced stores), through a
// wave-private 16 x 16 LDS tile rather than a product with I.
// Steps of four row tiles are dealt round-robin over the grid, so that the
// workgroups stream one common window of rows; every wave works on its own
// tile of a step with kNarrowPF tiles in flight, and no barrier until the
// four wave Gramians are summed in wave order into the workgroup's slot.
// ---------------------------------------------------------------------------
constexpr int kNarrowPF = 4;

template <bool APPLY, bool G32>
__device__ __forceinline__ void narrow_pass_body(const WidePassArgs& a, const int bid, const int nwg) {
  __shared__ double red[kWaves * 256];
  __shared__ double trs[kWaves * 16 * kYPitch];   // one 16 x 16 tile per wave
  if (a.gram32 && *a.gram32 != (G32 ? 1 : 0)) return;   // the other variant's pass
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = lane & 15, g = lane >> 4;
  const int64_t tiles = (a.m + 15) / 16;
  // steps of kWaves row tiles dealt round-robin over the grid: local step j
  // is step j nwg + bid, and the wave takes row tile (j nwg + bid) kWaves + wave
  const int64_t steps = (tiles + kWaves - 1) / kWaves;
  const int64_t sw = steps > bid ? (steps - 1 - bid) / nwg + 1 : 0;
  auto tile_of = [&](int64_t j) { return (j * nwg + bid) * kWaves + wave; };

  if (a.done && *a.done) {
    if (APPLY && a.copy_if_done && *a.passes == 0) {
      for (int64_t j = 0; j < sw; ++j) {
        const int64_t t = tile_of(j);
        if (t >= tiles) continue;
        const int64_t row = t * 16 + x;
        if (row >= a.m) continue;
        for (int c = g; c < a.n; c += 4)
          a.yout[(int64_t)c * a.ldy + row] = a.win[(int64_t)c * a.ldw + row];
      }
    }
    return;
  }

  // The apply multiplies the input by the inverse factors of `levels`
  // passes in turn (a pass that recomputes its input from A); dv is the last
  // one (unused in the Gram-only pass), dp[l] the earlier ones.  k-slice s
  // of a factor is read as D[4s + g][x].
  const int lv = APPLY ? a.levels : 1;   // 1 .. kNarrowSlots - 1
  double dv[4], dp[kNarrowSlots - 2][4];
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    dv[s4] = APPLY ? a.rinv[(lv - 1) * 256 + (4 * s4 + g) * 16 + x] : 0.0;
#pragma unroll
    for (int l = 0; l < kNarrowSlots - 2; ++l)
      dp[l][s4] = (APPLY && l + 1 < lv) ? a.rinv[l * 256 + (4 * s4 + g) * 16 + x] : 0.0;
  }

  // W tile: reg r = W[row x][col g + 4r] as loaded; columns past n read
  // zero (buffer range).  Rows past m and steps past the workgroup's last are
  // cleared by the mask `keep` when the tile is used, not at the load, so the
  // loads stay in flight until then.
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.win, ((int64_t)(a.n - 1) * a.ldw + a.m) * 8);
  auto load = [&](int64_t j, d4& w, uint64_t& keep) {
    const int64_t tile = tile_of(j);
    const int64_t row = min(tile, tiles - 1) * 16 + x;
    keep = (row < a.m && tile < tiles && j < sw) ? ~0ull : 0ull;
    const int64_t rowc = row < a.m ? row : a.m - 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t ow = (uint32_t)(((int64_t)(g + 4 * r) * a.ldw + rowc) * 8);
      w[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rw, (int)ow, 0, 0));
    }
  };
  auto masked = [](double v, uint64_t keep) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & keep);
  };

  d4 accg = d4{0.0, 0.0, 0.0, 0.0};
  f4 accg32 = f4{0.f, 0.f, 0.f, 0.f};   // G32: Gramian of the FP32-rounded tiles
  if (sw > 0) {
    d4 wb[kNarrowPF];
    uint64_t kb[kNarrowPF];
    // loads issued slot after slot (as in the loop), so that the waits at
    // the loop head are counted per slot
#pragma unroll
    for (int q = 0; q < kNarrowPF; ++q) {
      load(q, wb[q], kb[q]);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int64_t k0 = 0; k0 < sw; k0 += kNarrowPF) {
#pragma unroll
      for (int q = 0; q < kNarrowPF; ++q) {
        // wb[q] is used first and then refilled with the wave's tile
        // kNarrowPF local steps ahead: the load lands in the same registers, so no copy (and
        // no wait for the loads in flight) is needed at the loop's end.  A
        // tile past the range holds zeros: no branch around the arithmetic.
        const int64_t tile = tile_of(k0 + q);
        const bool tile_ok = k0 + q < sw && tile < tiles;
        __builtin_amdgcn_sched_barrier(0);   // keep this slot's wait here, not hoisted
        d4 w;
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = masked(wb[q][r], kb[q]);
        if (APPLY) {
          // earlier passes' factors: w <- w D_l, kept in the load layout
          // (register r = column 4r + g of row x), the products a pass that
          // reads the stored result of the pass before would take
#pragma unroll
          for (int l = 0; l < kNarrowSlots - 2; ++l) {
            if (l + 1 < lv) {   // uniform
              d4 t = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int s4 = 0; s4 < 4; ++s4) t = mfma(dp[l][s4], w[s4], t);
              w = t;
            }
          }
        }
        {
          d4 ya = d4{0.0, 0.0, 0.0, 0.0};
          if (!APPLY) {
            // Gram-only pass: the tile in the Gramian's operand layout
            // through the wave's LDS tile instead of a product with I
            double* tr = trs + wave * 16 * kYPitch;
#pragma unroll
            for (int r = 0; r < 4; ++r) tr[x * kYPitch + g + 4 * r] = w[r];
            wave_lds_order();
#pragma unroll
            for (int r = 0; r < 4; ++r) ya[r] = tr[(g + 4 * r) * kYPitch + x];
            wave_lds_order();
          } else {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) ya = mfma(w[s4], dv[s4], ya);
          }
          if (APPLY && a.store) {
            // rows across lanes through the wave's LDS tile (ya register r is
            // row g + 4r of column x; yb register r is column g + 4r of row x)
            double* tr = trs + wave * 16 * kYPitch;
#pragma unroll
            for (int r = 0; r < 4; ++r) tr[(g + 4 * r) * kYPitch + x] = ya[r];
            wave_lds_order();
            d4 yb;
#pragma unroll
            for (int r = 0; r < 4; ++r) yb[r] = tr[x * kYPitch + g + 4 * r];
            wave_lds_order();
            const int64_t row = tile * 16 + x;
            if (tile_ok && row < a.m) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int col = g + 4 * r;
                if (col < a.n) a.yout[(int64_t)col * a.ldy + row] = yb[r];
              }
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (G32) {
              const float yf = (float)ya[u];
              accg32 = mfma32(yf, yf, accg32);
            } else {
              accg = mfma(ya[u], ya[u], accg);
            }
          }
        }
        load(k0 + q + kNarrowPF, wb[q], kb[q]);
      }
    }
  }
  // Gramian slot of the workgroup: element (i, j) at i * 16 + j, the wave
  // partials added in wave order (in FP64 for both variants).
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (G32) red[wave * 256 + (4 * g + r) * 16 + x] = (double)accg32[r];
    else     red[wave * 256 + (g + 4 * r) * 16 + x] = accg[r];
  }
  __syncthreads();
  double* out = a.part + (int64_t)bid * a.part_stride;
  for (int e = threadIdx.x; e < 256; e += kThreads) {
    double t = 0.0;
#pragma unroll
    for (int v = 0; v < kWaves; ++v) t += red[v * 256 + e];
    out[e] = t;
  }
}

template <bool APPLY, bool G32>
__global__ __launch_bounds__(kThreads) void narrow_pass(WidePassArgs a) {
  narrow_pass_body<APPLY, G32>(a, blockIdx.x, gridDim.x);
}
template <bool APPLY, bool G32>
__global__ __launch_bounds__(kThreads) void narrow_pass_batch(BatchTable<WidePassArgs> t) {
  const int c = batch_call(t);
  narrow_pass_body<APPLY, G32>(t.args[c], blockIdx.x - t.start[c], t.start[c + 1] - t.start[c]);
}


// ---------------------------------------------------------------------------
// wide_pass: one launch per pass of an orth call whose n columns form NB
// blocks (2 <= NB <= 7 in FP64; 1 <= NB <= 8 in the mixed form).  Same arithmetic as the per-block launches
// (Y_J = W_J D_J + sum_{I<J} Y_I C_IJ, then the Gramian of Y), but a wave
// keeps the Y blocks of its 16-row tile in registers, so the prefix Y_<J is
// never re-read from HBM: the pass reads W once and writes Y once.
//
// Workgroup: four waves, one 16-row tile each (64 rows per step; steps dealt
// round-robin over the grid).  LDS holds
// the operands of the pass (per block J the panel [C_J; D_J], row-major, 16
// columns) and, per step, the transposed Y tiles of all four waves in MFMA
// operand order; each wave then accumulates the Gramian blocks (I, J) it
// owns (pairs dealt out round-robin) over the 64 rows.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int wide_panel_doubles(int nb) { return 128 * nb * (nb + 1); }
constexpr int kOpSlot = 68;   // one 4 x 16 operand slot, rows padded to 17
__host__ __device__ constexpr int wide_op_doubles(int nb) { return kWaves * nb * 4 * kOpSlot; }

template <int NB, bool APPLY, bool G32>
__device__ __forceinline__ void wide_pass_body(const WidePassArgs& a, const int bid, const int nwg) {
  extern __shared__ double lds[];
  constexpr int NP = NB * (NB + 1) / 2;           // Gramian blocks (I <= J)
  constexpr int KP = (NP + kWaves - 1) / kWaves;   // blocks per wave
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = lane & 15, g = lane >> 4;
  const int64_t tiles = (a.m + 15) / 16;
  const int64_t steps = (tiles + kWaves - 1) / kWaves;
  // steps dealt round-robin over the grid: local step i is step i nwg + bid
  const int64_t sw = steps > bid ? (steps - 1 - bid) / nwg + 1 : 0;
  auto step_of = [&](int64_t i) { return i * nwg + bid; };

  if (a.gram32 && *a.gram32 != (G32 ? 1 : 0)) return;   // the other variant's pass
  if (a.done && *a.done) {
    if (APPLY && a.copy_if_done && *a.passes == 0) {
      for (int64_t i = 0; i < sw; ++i) {
        const int64_t t = step_of(i) * kWaves + wave;
        if (t >= tiles) continue;
        const int64_t row = t * 16 + x;
        if (row >= a.m) continue;
        for (int c = g; c < a.n; c += 4)
          a.yout[(int64_t)c * a.ldy + row] = a.win[(int64_t)c * a.ldw + row];
      }
    }
    return;
  }

  double* panel = lds;                                   // APPLY only
  double* op = lds + (APPLY ? wide_panel_doubles(NB) : 0);
  if (APPLY) {
    for (int J = 0; J < NB; ++J) {
      double* P = panel + 128 * J * (J + 1);
      const double* C = a.bneg + 128 * J * (J - 1);
      for (int e = threadIdx.x; e < 256 * J; e += kThreads) P[e] = C[e];
      for (int e = threadIdx.x; e < 256; e += kThreads) P[256 * J + e] = a.rinv[256 * J + e];
    }
  }

  // Input of one tile in D layout: lane (x, g) register r of block J holds
  // W[row x][16 J + g + 4 r]; columns past n read zero (buffer range), rows
  // past m are masked.
  // (rows past m read a clamped row: the consumers zero those rows, so the
  // loads are not masked here and stay in flight until their use)
  auto load_w = [&](int64_t tile, d4 (&w)[NB]) {
    const int64_t row = tile * 16 + x;
    const int64_t rowc = row < a.m ? row : a.m - 1;
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      // one descriptor per 16-column block
      const int64_t nrec = (a.n - 1 >= 16 * J) ? (((int64_t)(a.n - 1 - 16 * J) * a.ldw + a.m) * 8) : 0;
      const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.win + (int64_t)(16 * J) * a.ldw, nrec);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t ow = (uint32_t)(((int64_t)(g + 4 * r) * a.ldw + rowc) * 8);
        w[J][r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rw, (int)ow, 0, 0));
      }
    }
  };

  d4 acc[G32 ? 1 : KP];
  f4 acc32[G32 ? KP : 1];
  int pi[KP], pj[KP];   // owned Gramian blocks (I, J), I <= J
  bool pidx_ok[KP];
#pragma unroll
  for (int k = 0; k < (G32 ? 1 : KP); ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < (G32 ? KP : 1); ++k) acc32[k] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int pidx = wave + kWaves * k;
    pidx_ok[k] = pidx < NP;
    int J = 0;
    while ((J + 1) * (J + 2) / 2 <= pidx && J < NB - 1) ++J;
    pj[k] = J;
    pi[k] = min(pidx - J * (J + 1) / 2, J);
  }

  d4 wnext[NB];
  load_w(min(step_of(0) * kWaves + wave, tiles - 1), wnext);
  __syncthreads();  // panels loaded
  double* myop = op + wave * NB * 4 * kOpSlot;
  for (int64_t i = 0; i < sw; ++i) {
    const int64_t tile = step_of(i) * kWaves + wave;
    const int64_t row = tile * 16 + x;
    const bool row_ok = tile < tiles && row < a.m;
    d4 y[NB];
#pragma unroll
    for (int J = 0; J < NB; ++J) y[J] = wnext[J];
    load_w(min(step_of(i + 1) * kWaves + wave, tiles - 1), wnext);
    if (!APPLY && !row_ok) {
#pragma unroll
      for (int J = 0; J < NB; ++J) y[J] = d4{0.0, 0.0, 0.0, 0.0};
    }
    if (APPLY) {
#pragma unroll
      for (int J = 0; J < NB; ++J) {
        const double* P = panel + 128 * J * (J + 1);
        d4 c0 = d4{0.0, 0.0, 0.0, 0.0};
        d4 c1 = d4{0.0, 0.0, 0.0, 0.0};
        // W_J D_J (block J of y still holds W_J)
        c0 = mfma(P[(16 * J + g) * 16 + x], y[J][0], c0);
        c1 = mfma(P[(16 * J + 4 + g) * 16 + x], y[J][1], c1);
        c0 = mfma(P[(16 * J + 8 + g) * 16 + x], y[J][2], c0);
        c1 = mfma(P[(16 * J + 12 + g) * 16 + x], y[J][3], c1);
        // + Y_I C_IJ for the finished blocks I < J
#pragma unroll
        for (int I = 0; I < J; ++I) {
          c0 = mfma(P[(16 * I + g) * 16 + x], y[I][0], c0);
          c1 = mfma(P[(16 * I + 4 + g) * 16 + x], y[I][1], c1);
          c0 = mfma(P[(16 * I + 8 + g) * 16 + x], y[I][2], c0);
          c1 = mfma(P[(16 * I + 12 + g) * 16 + x], y[I][3], c1);
        }
        y[J] = row_ok ? (c0 + c1) : d4{0.0, 0.0, 0.0, 0.0};
        if (row_ok) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = 16 * J + g + 4 * r;
            if (col < a.n) a.yout[(int64_t)col * a.ldy + row] = y[J][r];
          }
        }
      }
    }
    // Operand order for the Gramian: slot (J, u) holds Y[row 4u + g'][16 J + c]
    // of this wave's tile at g' * 17 + c (padded rows: the transposing
    // stores and the operand loads both spread over the LDS banks).
    if (G32) {
      // mixed form: the Gramian of the FP32-rounded tile, FP32 accumulation
      float* myop32 = reinterpret_cast<float*>(myop);
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          myop32[(J * 4 + (x >> 2)) * kOpSlot + 17 * (x & 3) + g + 4 * r] = (float)y[J][r];
      __syncthreads();
      const float* op32 = reinterpret_cast<const float*>(op);
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        if (pidx_ok[k]) {
          const float* oa = op32 + pi[k] * 4 * kOpSlot + x + 17 * g;
          const float* ob = op32 + pj[k] * 4 * kOpSlot + x + 17 * g;
#pragma unroll
          for (int t = 0; t < kWaves; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u)
              acc32[k] = mfma32(oa[(2 * t * NB * 4 + u) * kOpSlot], ob[(2 * t * NB * 4 + u) * kOpSlot],
                                acc32[k]);
        }
      }
      __syncthreads();
    } else {
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          myop[(J * 4 + (x >> 2)) * kOpSlot + 17 * (x & 3) + g + 4 * r] = y[J][r];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        if (pidx_ok[k]) {
          const double* oa = op + pi[k] * 4 * kOpSlot + x + 17 * g;
          const double* ob = op + pj[k] * 4 * kOpSlot + x + 17 * g;
#pragma unroll
          for (int t = 0; t < kWaves; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u)
              acc[k] = mfma(oa[(t * NB * 4 + u) * kOpSlot], ob[(t * NB * 4 + u) * kOpSlot], acc[k]);
        }
      }
      __syncthreads();
    }
  }

  // Slot: block J holds rows 0..16J+15 of Gramian columns 16J..16J+15.
  double* out = a.part + (int64_t)bid * a.part_stride;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (pidx_ok[k]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (G32)
          out[e_off(0, pj[k]) + (int64_t)(16 * pi[k] + 4 * g + r) * 16 + x] = (double)acc32[k][r];
        else
          out[e_off(0, pj[k]) + (int64_t)(16 * pi[k] + g + 4 * r) * 16 + x] = acc[k][r];
      }
    }
  }
}

template <int NB, bool APPLY, bool G32>
__global__ __launch_bounds__(kThreads) void wide_pass(WidePassArgs a) {
  wide_pass_body<NB, APPLY, G32>(a, blockIdx.x, gridDim.x);
}
template <int NB, bool APPLY, bool G32>
__global__ __launch_bounds__(kThreads) void wide_pass_batch(BatchTable<WidePassArgs> t) {
  const int c = batch_call(t);
  wide_pass_body<NB, APPLY, G32>(t.args[c], blockIdx.x - t.start[c], t.start[c + 1] - t.start[c]);
}


// ---------------------------------------------------------------------------
// Orth calls of 8..16 blocks (113..256 columns): the apply and the Gramian
// of a pass as two launches.  Registers cannot hold a row tile of Y, the
// prefetched input and all Gramian accumulators at once, so
//   wide_apply<NB>: Y = W R~^{-1} with the row tile's Y blocks in registers
//     (as in wide_pass) and the panel [C_J; D_J] of block J staged through
//     LDS while block J-1 is formed (one barrier per block);
//   gram_pass<NB, G32>:  the Gramian of the m x n result (upper 16x16
//     blocks), eight waves, 64-row steps staged in LDS in MFMA operand order,
//     the blocks (I, J) dealt out to the waves; also the initial Gramian of A.
//     G32 (mixed form): the Gramian of the FP32-rounded tiles on FP32 MFMA
//     with FP32 accumulation per workgroup.
// The pass then reads the tall data three times (W, and Y twice) instead of
// re-reading the prefix Y_<J for every block.
// ---------------------------------------------------------------------------
constexpr int kGramWaves = 8;
constexpr int kGramThreads = 64 * kGramWaves;
__host__ __device__ constexpr int gram_op_doubles(int nb) { return kWaves * nb * 4 * kOpSlot; }

// LDS doubles of wide_apply: panels 0..R-1 resident for the whole launch,
// two stream buffers for the later panels (none when all fit).
constexpr int kApplyLdsDoubles = 19968;   // 156 KB
__host__ __device__ constexpr int apply_resident(int nb) {
  int r = nb;
  while (r > 0 && 128 * r * (r + 1) + (r < nb ? 2 * 256 * nb : 0) > kApplyLdsDoubles) --r;
  return r;
}
__host__ __device__ constexpr int apply_lds_doubles(int nb) {
  return 128 * apply_resident(nb) * (apply_resident(nb) + 1) +
         (apply_resident(nb) < nb ? 2 * 256 * nb : 0);
}

// s_waitcnt with vmcnt(n) only (expcnt and lgkmcnt left at their maximum)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

template <int NB>
__device__ __forceinline__ void wide_apply_body(const WidePassArgs& a, const int bid, const int nwg) {
  extern __shared__ double lds[];
  constexpr int R = apply_resident(NB);           // resident panels
  constexpr int NPF = NB <= 10 ? NB : 8;          // blocks of the next tile prefetched
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = lane & 15, g = lane >> 4;
  const int64_t tiles = (a.m + 15) / 16;
  const int64_t steps = (tiles + kWaves - 1) / kWaves;
  const int64_t per = (steps + nwg - 1) / nwg;
  const int64_t s0 = (int64_t)bid * per;
  const int64_t s1 = min(steps, s0 + per);

  if (a.done && *a.done) {
    if (a.copy_if_done && *a.passes == 0) {
      for (int64_t t = s0 * kWaves + wave; t < min(tiles, s1 * kWaves); t += kWaves) {
        const int64_t row = t * 16 + x;
        if (row >= a.m) continue;
        for (int c = g; c < a.n; c += 4)
          a.yout[(int64_t)c * a.ldy + row] = a.win[(int64_t)c * a.ldw + row];
      }
    }
    return;
  }

  // Block J of one tile in D layout (columns past n read zero, rows past m
  // are masked).
  // (rows past m read a clamped row; their outputs are zeroed and not
  // stored, so the loads are not masked and stay in flight until their use)
  auto load_block = [&](int64_t tile, int J) -> d4 {
    const int64_t row = tile * 16 + x;
    const int64_t rowc = row < a.m ? row : a.m - 1;
    // one descriptor per 16-column block
    const int64_t nrec = (a.n - 1 >= 16 * J) ? (((int64_t)(a.n - 1 - 16 * J) * a.ldw + a.m) * 8) : 0;
    const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.win + (int64_t)(16 * J) * a.ldw, nrec);
    d4 w;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t ow = (uint32_t)(((int64_t)(g + 4 * r) * a.ldw + rowc) * 8);
      w[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rw, (int)ow, 0, 0));
    }
    return w;
  };
  // Panel J = [C_J (16 J rows); D_J (16 rows)] x 16, row-major (2 (J + 1)
  // chunks of 1 KB).  Resident panels: plain loads at the start.  Streamed
  // panels: direct global -> LDS loads, chunk c by wave c % 4, lane l moving
  // 16 bytes to chunk base + 16 l; completion is awaited with vmcnt.
  double* stream = lds + 128 * R * (R + 1);
  auto panel_src = [&](int J, int c) -> const double* {
    return (c < 2 * J) ? a.bneg + 128 * J * (J - 1) + 128 * c : a.rinv + 256 * J + 128 * (c - 2 * J);
  };
  auto dma_panel = [&](int J, double* dst) {
#pragma unroll
    for (int i = 0; i < (2 * (J + 1) + kWaves - 1) / kWaves; ++i) {
      const int c = wave + kWaves * i;
      if (c < 2 * (J + 1))
        __builtin_amdgcn_global_load_lds((const void*)(panel_src(J, c) + 2 * lane),
                                         (__attribute__((address_space(3))) void*)(dst + 128 * c),
                                         16, 0, 0);
    }
  };
  for (int J = 0; J < R; ++J) {
    double* P = lds + 128 * J * (J + 1);
    for (int e = threadIdx.x; e < 256 * (J + 1); e += kThreads)
      P[e] = (e < 256 * J) ? a.bneg[128 * J * (J - 1) + e] : a.rinv[256 * J + e - 256 * J];
  }
  __syncthreads();

  d4 wnext[NPF];
#pragma unroll
  for (int J = 0; J < NPF; ++J) wnext[J] = load_block(min(s0 * kWaves + wave, tiles - 1), J);
  for (int64_t s = s0; s < s1; ++s) {
    const int64_t tile = s * kWaves + wave;
    const int64_t row = tile * 16 + x;
    const bool row_ok = tile < tiles && row < a.m;
    d4 y[NB];
#pragma unroll
    for (int J = 0; J < NPF; ++J) y[J] = wnext[J];
#pragma unroll
    for (int J = NPF; J < NB; ++J) y[J] = load_block(min(tile, tiles - 1), J);
    if (R == NB) {
#pragma unroll
      for (int J = 0; J < NPF; ++J) wnext[J] = load_block(min(tile + kWaves, tiles - 1), J);
    }
#pragma clang loop unroll(full)
    for (int J = 0; J < NB; ++J) {
      // keep later blocks' operand loads out of this block (their registers
      // would not fit beside the tile's Y)
      __builtin_amdgcn_sched_barrier(0);
      const bool stage_next = J + 1 >= R && J + 1 < NB;
      if (stage_next) dma_panel(J + 1, stream + ((J + 1) & 1) * 256 * NB);
      // the next tile's prefetch goes out after the last streamed panel, so
      // the panel waits below do not wait for it
      if (R < NB && J == NB - 2) {
#pragma unroll
        for (int J2 = 0; J2 < NPF; ++J2) wnext[J2] = load_block(min(tile + kWaves, tiles - 1), J2);
      }
      const double* P = (J < R) ? lds + 128 * J * (J + 1) : stream + (J & 1) * 256 * NB;
      d4 c0 = d4{0.0, 0.0, 0.0, 0.0};
      d4 c1 = d4{0.0, 0.0, 0.0, 0.0};
      c0 = mfma(P[(16 * J + g) * 16 + x], y[J][0], c0);
      c1 = mfma(P[(16 * J + 4 + g) * 16 + x], y[J][1], c1);
      c0 = mfma(P[(16 * J + 8 + g) * 16 + x], y[J][2], c0);
      c1 = mfma(P[(16 * J + 12 + g) * 16 + x], y[J][3], c1);
#pragma unroll
      for (int I = 0; I < J; ++I) {
        c0 = mfma(P[(16 * I + g) * 16 + x], y[I][0], c0);
        c1 = mfma(P[(16 * I + 4 + g) * 16 + x], y[I][1], c1);
        c0 = mfma(P[(16 * I + 8 + g) * 16 + x], y[I][2], c0);
        c1 = mfma(P[(16 * I + 12 + g) * 16 + x], y[I][3], c1);
      }
      y[J] = row_ok ? (c0 + c1) : d4{0.0, 0.0, 0.0, 0.0};
      if (row_ok) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * J + g + 4 * r;
          if (col < a.n) a.yout[(int64_t)col * a.ldy + row] = y[J][r];
        }
      }
      if (stage_next) {
        // this wave's chunks of panel J + 1 have landed (the prefetch issued
        // after them may still be in flight), then all waves' chunks have
        if (J == NB - 2 && R < NB) wait_vmcnt<4 * NPF>(); else wait_vmcnt<0>();
        __syncthreads();
      }
    }
    if (R < NB) __syncthreads();   // the stream buffers are free for the next step
  }
}

template <int NB>
__global__ __launch_bounds__(kThreads) void wide_apply(WidePassArgs a) {
  wide_apply_body<NB>(a, blockIdx.x, gridDim.x);
}
template <int NB>
__global__ __launch_bounds__(kThreads) void wide_apply_batch(BatchTable<WidePassArgs> t) {
  const int c = batch_call(t);
  wide_apply_body<NB>(t.args[c], blockIdx.x - t.start[c], t.start[c + 1] - t.start[c]);
}


template <int NB, bool G32>
__device__ __forceinline__ void gram_pass_body(const WidePassArgs& a, const int bid, const int nwg) {
  extern __shared__ double lds[];
  using Op = typename std::conditional<G32, float, double>::type;
  using Acc = typename std::conditional<G32, f4, d4>::type;
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int KP = (NP + kGramWaves - 1) / kGramWaves;
  constexpr int H = (NB + 1) / 2;                 // blocks loaded per wave
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tw = wave >> 1, half = wave & 1;      // row tile of the step, half of the blocks
  const int x = lane & 15, g = lane >> 4;
  const int64_t tiles = (a.m + 15) / 16;
  const int64_t steps = (tiles + kWaves - 1) / kWaves;
  const int64_t per = (steps + nwg - 1) / nwg;
  const int64_t s0 = (int64_t)bid * per;
  const int64_t s1 = min(steps, s0 + per);
  if (a.done && *a.done) return;
  if (a.gram32 && *a.gram32 != (G32 ? 1 : 0)) return;   // the other variant's pass

  // (rows past m read a clamped row and are zeroed where the tile is put
  // into LDS, so the loads stay in flight until then)
  auto load_h = [&](int64_t tile, d4 (&w)[H]) {
    const int64_t row = tile * 16 + x;
    const int64_t rowc = row < a.m ? row : a.m - 1;
#pragma unroll
    for (int jj = 0; jj < H; ++jj) {
      // one descriptor per 16-column block
      const int c0 = 16 * (half * H + jj);
      const int64_t nrec = (a.n - 1 >= c0) ? (((int64_t)(a.n - 1 - c0) * a.ldw + a.m) * 8) : 0;
      const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.win + (int64_t)c0 * a.ldw, nrec);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t ow = (uint32_t)(((int64_t)(g + 4 * r) * a.ldw + rowc) * 8);
        w[jj][r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rw, (int)ow, 0, 0));
      }
    }
  };

  Acc acc[KP];
  int pi[KP], pj[KP];
  bool pok[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    acc[k] = Acc{0, 0, 0, 0};
    const int pidx = wave + kGramWaves * k;
    pok[k] = pidx < NP;
    int J = 0;
    while ((J + 1) * (J + 2) / 2 <= pidx && J < NB - 1) ++J;
    pj[k] = J;
    pi[k] = min(pidx - J * (J + 1) / 2, J);
  }

  d4 wnext[H];
  load_h(min(s0 * kWaves + tw, tiles - 1), wnext);
  // operand slots in the Gramian's precision (FP32: half the LDS)
  Op* const ops = reinterpret_cast<Op*>(lds);
  Op* myop = ops + tw * NB * 4 * kOpSlot;
  for (int64_t s = s0; s < s1; ++s) {
    const int64_t tile = s * kWaves + tw;
    const bool tile_ok = tile < tiles && tile * 16 + x < a.m;   // this lane's row exists
    // this step's tile into LDS (operand order), then the next tile's loads
#pragma unroll
    for (int jj = 0; jj < H; ++jj) {
      const int J = half * H + jj;
      if (J < NB) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          myop[(J * 4 + (x >> 2)) * kOpSlot + 17 * (x & 3) + g + 4 * r] = (Op)(tile_ok ? wnext[jj][r] : 0.0);
      }
    }
    load_h(min(tile + kWaves, tiles - 1), wnext);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (pok[k]) {
        const Op* oa = ops + pi[k] * 4 * kOpSlot + x + 17 * g;
        const Op* ob = ops + pj[k] * 4 * kOpSlot + x + 17 * g;
#pragma unroll
        for (int t = 0; t < kWaves; ++t)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if constexpr (G32)
              acc[k] = mfma32(oa[(t * NB * 4 + u) * kOpSlot], ob[(t * NB * 4 + u) * kOpSlot], acc[k]);
            else
              acc[k] = mfma(oa[(t * NB * 4 + u) * kOpSlot], ob[(t * NB * 4 + u) * kOpSlot], acc[k]);
          }
      }
    }
    __syncthreads();
  }
  // Slot: block J holds rows 0..16J+15 of Gramian columns 16J..16J+15 (the
  // two MFMA forms place the 16x16 result differently across lanes).
  double* out = a.part + (int64_t)bid * a.part_stride;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (pok[k]) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (G32)
          out[e_off(0, pj[k]) + (int64_t)(16 * pi[k] + 4 * g + r) * 16 + x] = (double)acc[k][r];
        else
          out[e_off(0, pj[k]) + (int64_t)(16 * pi[k] + g + 4 * r) * 16 + x] = acc[k][r];
      }
    }
  }
}

template <int NB, bool G32>
__global__ __launch_bounds__(kGramThreads) void gram_pass(WidePassArgs a) {
  gram_pass_body<NB, G32>(a, blockIdx.x, gridDim.x);
}
template <int NB, bool G32>
__global__ __launch_bounds__(kGramThreads) void gram_pass_batch(BatchTable<WidePassArgs> t) {
  const int c = batch_call(t);
  gram_pass_body<NB, G32>(t.args[c], blockIdx.x - t.start[c], t.start[c + 1] - t.start[c]);
}


// ---------------------------------------------------------------------------
// Appends whose basis is too wide for block_pass's S (more than kBlockTiles
// tiles with the block).  A pass of Algorithm 2 then runs as
//   proj_pass    Z = W - Q_in B~ (apply phases): a tall product over the q
//                basis columns, written into the new columns;
//   block_pass   Y_J = Z_J D_J + Y_<J C_J and the Gramian G of Y (S holds only
//                the block's own prefix, as for an orthogonalisation);
//   cross_pass   B~ = Q_in^T Y, partial sums of one row chunk per slot;
//   reduce_slots (G and B~), btb_pass (B~^T B~), small_step (mode 2), and
//   bacc_pass    B <- B + B~ R_old.
// Q_in is read twice per pass (proj and cross), not once per 16-column block.
// ---------------------------------------------------------------------------
constexpr int kCrossA = 8;   // basis blocks (16 columns) of a cross_pass tile
__host__ __device__ constexpr int cross_lds_doubles(int nb) { return kWaves * (kCrossA + nb) * 4 * kOpSlot; }

// Partial X^T Y of tile (128 basis columns) x (16 NB block columns) over the
// rows of one slot, eight waves.  32-row steps (two 16-row tiles) are staged
// in LDS in MFMA operand order, double-buffered: while the waves work on
// step s from one buffer they store step s + 1 (loaded two steps earlier
// into registers) into the other, so one barrier per step suffices and the
// staging of one wave overlaps the MFMA work of the others.  Wave w owns the
// WI x WJ block pairs (gi WI + i, gj WJ + j): per k-slice WI + WJ operand
// reads from LDS feed WI WJ MFMAs.
template <int NB>
__device__ __forceinline__ void cross_pass_body(const CrossArgs& a, const int bid) {
  extern __shared__ double lds[];
  constexpr int NBLK = kCrossA + NB;               // blocks staged per row tile
  constexpr int KP = NB;                           // pairs per wave (8 NB pairs)
  constexpr int HB = (NBLK + 3) / 4;               // blocks loaded per wave
  constexpr int BUF = 2 * NBLK * 4 * kOpSlot;      // doubles of one buffer
  constexpr int WI = (NB == 8) ? 2 : 1, WJ = NB / WI;
  static_assert(WI * WJ == KP && (kCrossA / WI) * (NB / WJ) == kGramWaves, "pair split");
  static_assert(2 * BUF == cross_lds_doubles(NB), "LDS size");
  if (a.done && *a.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tr = wave >> 2, qd = wave & 3;          // row tile of a step, block quarter
  const int x = lane & 15, g = lane >> 4;
  const int slot = bid / a.ntiles, tile = bid - slot * a.ntiles;
  const int ta = tile / a.tiles_b, tb = tile - ta * a.tiles_b;
  const int a0 = 16 * kCrossA * ta, b0 = 16 * NB * tb;
  if (a.sym && a0 >= b0 + 16 * NB) return;   // strictly below the diagonal
  const int64_t tiles = (a.m + 15) / 16;
  const int64_t steps = (tiles + 1) / 2;
  const int64_t per = (steps + a.nslots - 1) / a.nslots;
  const int64_t s0 = (int64_t)slot * per;
  const int64_t s1 = min(steps, s0 + per);
  const int gi = wave % (kCrossA / WI), gj = wave / (kCrossA / WI);

  // blocks qd, qd + 4, ... of row tile t: blocks 0..7 are basis columns a0..,
  // blocks 8.. block columns b0..; one descriptor per block (columns past the
  // matrix read zero).  The per-lane offsets ((g + 4r) ld + x) * 8 are formed
  // once; a step adds its first row as the scalar offset, so the loads need
  // no address arithmetic.  Rows past m read the next column's top (or zero
  // past the last column) and are zeroed where the tile goes into LDS; every
  // offset stays below (16 ld + 14) * 8 < 2^32.
  __amdgpu_buffer_rsrc_t rsb[HB];
  uint32_t vo[HB][4];
#pragma unroll
  for (int jj = 0; jj < HB; ++jj) {
    const int blk = qd + 4 * jj;
    const bool isx = blk < kCrossA;
    const int c0 = isx ? a0 + 16 * blk : b0 + 16 * (blk - kCrossA);
    const int nc = isx ? a.nx : a.ny;
    const int64_t ld = isx ? a.ldx : a.ldy;
    const int64_t nrec = (blk < NBLK && nc - 1 >= c0) ? (((int64_t)(nc - 1 - c0) * ld + a.m) * 8) : 0;
    rsb[jj] = make_rsrc((isx ? a.x : a.y) + (int64_t)c0 * ld, nrec);
#pragma unroll
    for (int r = 0; r < 4; ++r) vo[jj][r] = (uint32_t)(((int64_t)(g + 4 * r) * ld + x) * 8);
  }
  auto load = [&](int64_t t, d4 (&w)[HB]) {
    const int so = __builtin_amdgcn_readfirstlane((int)(t * 128));
#pragma unroll
    for (int jj = 0; jj < HB; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        w[jj][r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rsb[jj], (int)vo[jj][r], so, 0));
  };
  auto store = [&](int64_t t, const d4 (&w)[HB], double* buf) {
    double* my = buf + tr * NBLK * 4 * kOpSlot + (x >> 2) * kOpSlot + 17 * (x & 3) + g;
    if ((t + 1) * 16 <= a.m) {   // a whole tile of rows (uniform): no mask
#pragma unroll
      for (int jj = 0; jj < HB; ++jj) {
        const int blk = qd + 4 * jj;
        if (blk < NBLK) {
#pragma unroll
          for (int r = 0; r < 4; ++r) my[blk * 4 * kOpSlot + 4 * r] = w[jj][r];
        }
      }
    } else {
      const bool ok = t < tiles && t * 16 + x < a.m;
#pragma unroll
      for (int jj = 0; jj < HB; ++jj) {
        const int blk = qd + 4 * jj;
        if (blk < NBLK) {
#pragma unroll
          for (int r = 0; r < 4; ++r) my[blk * 4 * kOpSlot + 4 * r] = ok ? w[jj][r] : 0.0;
        }
      }
    }
  };

  d4 acc[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  auto tile_of = [&](int64_t s) { return min(s, s1 - 1) * 2 + tr; };
  auto compute = [&](const double* cur) {
    const double* oa = cur + (gi * WI) * 4 * kOpSlot + x + 17 * g;
    const double* ob = cur + (kCrossA + gj * WJ) * 4 * kOpSlot + x + 17 * g;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double av[WI], bv[WJ];
#pragma unroll
        for (int i = 0; i < WI; ++i) av[i] = oa[((tt * NBLK + i) * 4 + u) * kOpSlot];
#pragma unroll
        for (int j = 0; j < WJ; ++j) bv[j] = ob[((tt * NBLK + j) * 4 + u) * kOpSlot];
#pragma unroll
        for (int i = 0; i < WI; ++i)
#pragma unroll
          for (int j = 0; j < WJ; ++j) acc[i][j] = mfma(av[i], bv[j], acc[i][j]);
      }
  };
  // two register sets: step k's loads land in set k % 2 two steps before it
  // is stored (the loads have two compute phases to arrive)
  double* buf0 = lds;
  double* buf1 = lds + BUF;
  d4 wa[HB], wb[HB];
  if (s0 < s1) {
    load(tile_of(s0), wa);
    load(tile_of(s0 + 1), wb);
    store(tile_of(s0), wa, buf0);
    load(tile_of(s0 + 2), wa);
  }
  __syncthreads();
  for (int64_t s = s0; s < s1; s += 2) {
    if (s + 1 < s1) {
      store(tile_of(s + 1), wb, buf1);
      load(tile_of(s + 3), wb);
    }
    compute(buf0);
    __syncthreads();
    if (s + 1 >= s1) break;
    if (s + 2 < s1) {
      store(tile_of(s + 2), wa, buf0);
      load(tile_of(s + 4), wa);
    }
    compute(buf1);
    __syncthreads();
  }
  // lane (x, g) register r: B~[a0 + 16 I + g + 4r][b0 + 16 J + x]
  double* out = a.part + (int64_t)slot * a.part_stride;
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const int col = b0 + 16 * (gj * WJ + j) + x;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = a0 + 16 * (gi * WI + i) + g + 4 * r;
        if (row < a.rows16 && col < a.pitch) out[(int64_t)row * a.pitch + col] = acc[i][j][r];
      }
    }
}

template <int NB>
__global__ __launch_bounds__(kGramThreads) void cross_pass(CrossArgs a) {
  cross_pass_body<NB>(a, blockIdx.x);
}

// Z = W - X B~ for kProjRows rows (kProjRT 16-row tiles per wave) x 16 NB
// columns.
// B~ streams through LDS in chunks of kProjKC rows (double-buffered, one
// barrier per chunk); the basis operand is loaded straight into registers,
// one chunk ahead.  MFMA roles: A = B~ slice (from LDS), B = X rows, so the
// result lane (x, g) register r is Z[row x][column g + 4r] (stores coalesce
// along rows).
constexpr int kProjKC = 32;
constexpr int kProjRT = 1;                     // 16-row tiles per wave
constexpr int kProjRows = 16 * kProjRT * kWaves;   // rows per workgroup
__host__ __device__ constexpr int proj_pitch(int nb) { return 32 * ((16 * nb + 31) / 32) + 16; }
__host__ __device__ constexpr int proj_lds_doubles(int nb) { return 2 * kProjKC * proj_pitch(nb); }

template <int NB>
__device__ __forceinline__ void proj_pass_body(const ProjArgs& a, const int bid) {
  extern __shared__ double lds[];
  constexpr int LP = proj_pitch(NB);
  constexpr int SL = kProjKC / 4;                 // k-slices per chunk
  constexpr int PER = 2 * NB;                     // B~ doubles per thread per chunk
  if (a.done && *a.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = lane & 15, g = lane >> 4;
  const int rt = bid / a.tiles_b, tb = bid - rt * a.tiles_b;
  const int b0 = 16 * NB * tb;
  const int64_t rbase = (int64_t)rt * kProjRows + wave * 16 * kProjRT;
  const int nch = (a.rows16 + kProjKC - 1) / kProjKC;
  int64_t rowc[kProjRT];
#pragma unroll
  for (int t = 0; t < kProjRT; ++t) rowc[t] = min(rbase + 16 * t + x, a.m - 1);

  // basis operand of chunk ch: lane (x, g), tile t, slice s holds
  // X[row][k0 + 4s + g] (column clamped; zeroed at use past nx)
  auto load_x = [&](int ch, double (&xv)[kProjRT][SL]) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int k = min(ch * kProjKC + 4 * s + g, a.nx - 1);
#pragma unroll
      for (int t = 0; t < kProjRT; ++t) xv[t][s] = a.x[(int64_t)k * a.ldx + rowc[t]];
    }
  };
  // B~ chunk: thread -> row (tid >> 3) of the chunk, columns (tid & 7) * PER ..
  const int brow = threadIdx.x >> 3, bcol = (threadIdx.x & 7) * PER;
  // (row and column clamped to the operand; zeroed where stored)
  auto load_b = [&](int ch, double (&bv)[PER]) {
    const int k = min(ch * kProjKC + brow, a.rows16 - 1);
#pragma unroll
    for (int e = 0; e < PER; ++e) bv[e] = a.bt[(int64_t)k * a.ldt + min(b0 + bcol + e, a.p - 1)];
  };
  auto store_b = [&](int ch, const double (&bv)[PER], double* buf) {
    const bool rok = ch * kProjKC + brow < a.rows16;
#pragma unroll
    for (int e = 0; e < PER; ++e)
      buf[brow * LP + bcol + e] = (rok && b0 + bcol + e < a.p) ? bv[e] : 0.0;
  };
  d4 acc[kProjRT][NB];
#pragma unroll
  for (int t = 0; t < kProjRT; ++t)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[t][c] = d4{0.0, 0.0, 0.0, 0.0};
  auto compute = [&](int ch, const double (&xv)[kProjRT][SL], const double* buf) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const bool kok = ch * kProjKC + 4 * s + g < a.nx;
      double xk[kProjRT];
#pragma unroll
      for (int t = 0; t < kProjRT; ++t) xk[t] = kok ? xv[t][s] : 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double bv = buf[(4 * s + g) * LP + 16 * c + x];
#pragma unroll
        for (int t = 0; t < kProjRT; ++t) acc[t][c] = mfma(bv, xk[t], acc[t][c]);
      }
    }
  };

  double* buf0 = lds;
  double* buf1 = lds + kProjKC * LP;
  double xa[kProjRT][SL], xb[kProjRT][SL];
  double bv[PER];
  load_x(0, xa);
  load_b(0, bv);
  store_b(0, bv, buf0);
  __syncthreads();
  for (int ch = 0; ch < nch; ch += 2) {
    if (ch + 1 < nch) { load_b(ch + 1, bv); load_x(ch + 1, xb); }
    compute(ch, xa, buf0);
    if (ch + 1 < nch) store_b(ch + 1, bv, buf1);
    __syncthreads();
    if (ch + 1 >= nch) break;
    if (ch + 2 < nch) { load_b(ch + 2, bv); load_x(ch + 2, xa); }
    compute(ch + 1, xb, buf1);
    if (ch + 2 < nch) store_b(ch + 2, bv, buf0);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < kProjRT; ++t) {
    const int64_t row = rbase + 16 * t + x;
    if (row >= a.m) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double w[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = b0 + 16 * c + g + 4 * r;
        w[r] = (col < a.p) ? a.win[(int64_t)col * a.ldw + row] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = b0 + 16 * c + g + 4 * r;
        if (col < a.p) a.yout[(int64_t)col * a.ldy + row] = w[r] - acc[t][c][r];
      }
    }
  }
}

template <int NB>
__global__ __launch_bounds__(kThreads) void proj_pass(ProjArgs a) {
  proj_pass_body<NB>(a, blockIdx.x);
}

// B~^T B~: workgroup = one 16x16 block (I <= J) of the p x p result; wave w
// sums the k-slices w, w + 4, ... (two chains), the four wave sums are added
// in wave order; the block and its mirror are stored (exactly symmetric).
__global__ __launch_bounds__(kThreads) void btb_pass(BtbArgs a) {
  __shared__ double red[kWaves * 256];
  if (a.done && *a.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  int J = 0;
  while ((J + 1) * (J + 2) / 2 <= (int)blockIdx.x) ++J;
  const int I = (int)blockIdx.x - J * (J + 1) / 2;
  const int nks = a.rows16 >> 2;
  d4 c0 = d4{0.0, 0.0, 0.0, 0.0}, c1 = d4{0.0, 0.0, 0.0, 0.0};
  int s = wave;
  for (; s + kWaves < nks; s += 2 * kWaves) {
    const double* r0 = a.bt + (int64_t)(4 * s + g) * a.pitch;
    const double* r1 = a.bt + (int64_t)(4 * (s + kWaves) + g) * a.pitch;
    const double a0 = r0[16 * I + x], b0v = r0[16 * J + x];
    const double a1 = r1[16 * I + x], b1v = r1[16 * J + x];
    c0 = mfma(a0, b0v, c0);
    c1 = mfma(a1, b1v, c1);
  }
  if (s < nks) {
    const double* r0 = a.bt + (int64_t)(4 * s + g) * a.pitch;
    c0 = mfma(r0[16 * I + x], r0[16 * J + x], c0);
  }
  const d4 cw = c0 + c1;
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + r * 64 + lane] = cw[r];
  __syncthreads();
  if (wave != 0) return;
  d4 sum = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int w = 0; w < kWaves; ++w)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum[r] += red[w * 256 + r * 64 + lane];
  const int col = 16 * J + x;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * I + g + 4 * r;
    if (row < a.p && col < a.p && (I < J || row <= col)) {
      a.out[(int64_t)row * a.p + col] = sum[r];
      a.out[(int64_t)col * a.p + row] = sum[r];
    }
  }
}

// B <- B + B~ R_old in R[0:q, q:q+p]; one 16x16 block of B per wave.  At
// phase 0 (R_old = I, B = 0): B <- B~, and R[q:q+p, 0:q] <- 0.
__global__ __launch_bounds__(kThreads) void bacc_pass(BaccArgs a) {
  if (a.done && *a.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  const int P = (a.p + 15) >> 4, QT = (a.q + 15) >> 4;
  const int blk = (int)blockIdx.x * kWaves + wave;
  if (blk >= QT * P) return;
  const int rb = blk / P, C = blk - rb * P;
  const int row = 16 * rb + x;
  if (a.phase == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = 16 * C + g + 4 * r;
      if (row < a.q && col < a.p) {
        a.R[row + (int64_t)(a.q + col) * a.ldr] = a.bt[(int64_t)row * a.pitch + col];
        a.R[(a.q + col) + (int64_t)row * a.ldr] = 0.0;
      }
    }
    return;
  }
  // R_old is upper triangular: rows k > 16 C + 15 contribute nothing
  const int kend = min(16 * C + 16, a.pitch);
  const int rowc = min(row, a.q - 1);
  d4 acc = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kend; k0 += 4) {
    const int k = k0 + g;
    const double av = (k < a.p && 16 * C + x < a.p) ? a.rold[(int64_t)k * a.p + 16 * C + x] : 0.0;
    const double bv = a.bt[(int64_t)rowc * a.pitch + k];
    acc = mfma(av, bv, acc);
  }
  // lane (x, g) register r: (B~ R_old)[row][16 C + g + 4r]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int col = 16 * C + g + 4 * r;
    if (row < a.q && col < a.p) a.R[row + (int64_t)(a.q + col) * a.ldr] += acc[r];
  }
}

// ---------------------------------------------------------------------------
// small_step: one workgroup of 256 threads finishes a pass.
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / 64;

// Deterministic workgroup sum: a fixed butterfly inside each wave, then the
// wave sums in wave order.  Every thread gets the result.
// Workgroup barrier.  lds_only: order LDS accesses only, so global stores in
// flight are not waited for (small_step keeps its matrices in LDS and orders
// its few global read-after-write hand-offs with full barriers).
__device__ __forceinline__ void wg_sync(bool lds_only) {
  if (lds_only) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

__device__ double block_sum(double v, double* buf, bool lds_only) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wv = threadIdx.x >> 6;
  wg_sync(lds_only);
  if ((threadIdx.x & 63) == 0) buf[wv] = v;
  wg_sync(lds_only);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kSmallWaves; ++i) s += buf[i];
  return s;
}


// Lane L of each row of 16 lanes to the whole row (DPP row_newbcast), in
// vector registers.
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x150 + L, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x150 + L, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The same double in every lane, as a wave-uniform (scalar) value.
__device__ __forceinline__ double uniform_d(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Row I of the 16x16 wave factorisation below (branch-free apart from the
// uniform tests): pivot check, scaling of row I, and M_lk -= R_Il R_Ik for
// every later row l, R_Il broadcast from lane l.  Entries below the
// diagonal of lane k's column (rows l > k) are updated too and never read.
template <int I, int L>
__device__ __forceinline__ void chol16_update(double (&col)[16]) {
  if constexpr (L > I) col[L] -= row_bcast<L>(col[I]) * col[I];
}
template <int I, int... L>
__device__ __forceinline__ void chol16_row(double (&col)[16], int k, int nb, bool& ok,
                                           std::integer_sequence<int, L...>) {
  if (!ok || I >= nb) return;   // uniform
  const double d = uniform_d(row_bcast<I>(col[I]));
  if (!(d > 0.0) || !isfinite(d)) {
    ok = false;
    return;
  }
  const double r = sqrt(d);
  const double q = col[I] / r;
  col[I] = (k == I) ? r : ((k > I) ? q : col[I]);
  (chol16_update<I, L>(col), ...);
}
template <int... I>
__device__ __forceinline__ bool chol16_rows(double (&col)[16], int k, int nb,
                                            std::integer_sequence<int, I...> seq) {
  bool ok = true;
  (chol16_row<I>(col, k, nb, ok, seq), ...);
  return ok;
}

// Column k of R^{-1} (R the factor above, identity beyond nb) by back
// substitution, row I = 15 .. 0: t_I = (e_k[I] - sum_{L > I} R_IL t_L) / R_II
// with R_IL broadcast from lane L (zero beyond nb, where t_I = e_k[I]).
template <int I, int L>
__device__ __forceinline__ void inv16_term(const double (&col)[16], const double (&t)[16], double& s) {
  if constexpr (L > I) s -= row_bcast<L>(col[I]) * t[L];
}
template <int J, int... L>
__device__ __forceinline__ void inv16_row(const double (&col)[16], double (&t)[16], int k, int nb,
                                          std::integer_sequence<int, L...>) {
  constexpr int I = 15 - J;
  double s = (k == I) ? 1.0 : 0.0;
  if (I < nb) {   // uniform
    (inv16_term<I, L>(col, t, s), ...);
    s = s / row_bcast<I>(col[I]);
  }
  t[I] = s;
}
template <int... J>
__device__ __forceinline__ void inv16_rows(const double (&col)[16], double (&t)[16], int k, int nb,
                                           std::integer_sequence<int, J...> seq) {
  (inv16_row<J>(col, t, k, nb, seq), ...);
}

// In-place upper Cholesky (right-looking) of the nb x nb block at B
// (row-major, pitch ld, nb <= 16) by one wave, in vector registers: every
// row of 16 lanes holds the block, lane k column k; for each row i the pivot
// is checked, row i is scaled (r on the diagonal, the rest divided by r) and
// every later row l takes M_lk -= R_il R_ik, with R_il broadcast from lane l
// by DPP.  Breakdown: a pivot that is not > 0 or not finite (B untouched).
// On success the factor is written back to B and, if given, to copy16
// (pitch 16), and dinv (if given) receives the 16 x 16 inverse of the factor
// padded with the identity beyond nb (row-major).  Padding lanes and rows
// (>= nb) of the factor hold zeros and stay zero.
__device__ __noinline__ bool chol16_wave(double* B, int ld, int nb_in, double* copy16, double* dinv) {
  const int nb = __builtin_amdgcn_readfirstlane(nb_in);
  const int ln = threadIdx.x & 63;
  const int k = ln & 15;
  double col[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) col[i] = (i < nb && k < nb && i <= k) ? B[i * ld + k] : 0.0;
  const bool ok = chol16_rows(col, k, nb, std::make_integer_sequence<int, 16>{});
  if (ok && ln < nb) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i <= ln && i < nb) {
        B[i * ld + ln] = col[i];
        if (copy16) copy16[i * 16 + ln] = col[i];
      }
    }
  }
  if (ok && dinv) {
    double t[16];
    inv16_rows(col, t, k, nb, std::make_integer_sequence<int, 16>{});
    if (ln < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) dinv[i * 16 + ln] = t[i];
    }
  }
  return ok;
}

// dinv = inverse of the nb x nb upper triangular block at B (row-major,
// pitch ld), padded with the identity to 16 x 16 (row-major), by one wave.
__device__ __noinline__ void inv16_wave(const double* B, int ld, int nb_in, double* dinv) {
  const int nb = __builtin_amdgcn_readfirstlane(nb_in);
  const int ln = threadIdx.x & 63;
  const int k = ln & 15;
  double col[16], t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) col[i] = (i < nb && k < nb && i <= k) ? B[i * ld + k] : 0.0;
  inv16_rows(col, t, k, nb, std::make_integer_sequence<int, 16>{});
  if (ln < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) dinv[i * 16 + ln] = t[i];
  }
}

// Upper Cholesky of the p x p matrix M (p <= 16, in LDS) by wave 0; every
// thread receives the outcome.
__device__ bool chol_upper_wave(double* M, int p, int* flag, double* dinv) {
  wg_sync(true);
  if (threadIdx.x < 64) {
    const bool ok = chol16_wave(M, p, p, nullptr, dinv);
    if (threadIdx.x == 0) *flag = ok ? 1 : 0;
  }
  wg_sync(true);
  return *flag != 0;
}

// dst[i * cols + j] = f(i, j) over a rows x cols row-major matrix.  Each
// row is padded to whole 16-column chunks; the padded index space is dealt
// to the threads in batches of eight whose values are all loaded before any
// is stored (dst may alias the sources as far as the compiler knows, which
// would otherwise put every load behind the previous store).
template <class F>
__device__ __forceinline__ void fill_rows(double* dst, int rows, int cols, F f) {
  if (rows * cols <= kSmallThreads * 8) {   // small: one element per thread and step
    for (int e = threadIdx.x; e < rows * cols; e += kSmallThreads) {
      const int i = e / cols;
      dst[e] = f(i, e - i * cols);
    }
    return;
  }
  const int width = (cols + 15) & ~15;
  const int total = rows * width;
  for (int b = threadIdx.x; b < total; b += kSmallThreads * 8) {
    double t[8];
    int ii[8], jj[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b + kSmallThreads * u;
      ii[u] = idx / width;
      jj[u] = idx - ii[u] * width;
      t[u] = (idx < total && jj[u] < cols) ? f(ii[u], jj[u]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b + kSmallThreads * u;
      if (idx < total && jj[u] < cols) dst[(int64_t)ii[u] * cols + jj[u]] = t[u];
    }
  }
}

// In-place upper Cholesky (right-looking) of the row-major p x p matrix M
// for p > 16, band by band of 16 rows:
//   (a) one wave factors the diagonal block M_KK (as it stands after all
//       earlier updates) in registers (chol16_wave) and copies the factor to
//       `blk`; breakdown, a pivot that is not > 0 or not finite, is decided
//       on each pivot in turn;
//   (b) the band's panel R_K,>K = R_KK^{-T} M_K,>K by forward substitution,
//       one column per thread (the operations a column-by-column
//       factorisation applies to those entries, in the same order);
//   (c) every trailing block (I, J), K < I <= J, is updated as
//       M_IJ -= R_KI^T R_KJ on MFMA.
// Three workgroup barriers per band.  M is in LDS or in global memory; blk
// holds 256 doubles of LDS.  Returns false on breakdown; on success dinv
// (global memory) receives the inverses of the 16 x 16 diagonal blocks,
// padded with the identity (row-major, 256 doubles per block).
__device__ bool chol_blocked(double* M, int p, bool lds_only, double* blk, int* flag, double* dinv) {
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63, x = ln & 15, g = ln >> 4;
  const int nbk = (p + 15) >> 4;
  for (int K = 0; K < nbk; ++K) {
    const int b0 = 16 * K, b1 = min(p, b0 + 16), nb = b1 - b0;
    wg_sync(lds_only);   // the trailing update of band K-1 is complete
    if (wv == 0) {
      // (a) diagonal block by one wave, also copied to blk for the panel
      const bool ok = chol16_wave(M + (int64_t)b0 * p + b0, p, nb, blk, nullptr);
      if (ln == 0) *flag = ok ? 1 : 0;
    }
    wg_sync(lds_only);
    if (!*flag) {
      wg_sync(lds_only);   // every thread has read the flag before it is reused
      return false;
    }
    // (b) panel rows b0..b1-1, columns b1..p-1
    for (int c = b1 + tid; c < p; c += kSmallThreads) {
      // keep the reads of blk inside the loop (hoisted, its 136 entries
      // would not fit in registers)
      __asm__ volatile("" ::: "memory");
      double xc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) xc[i] = (i < nb) ? M[(int64_t)(b0 + i) * p + c] : 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i < nb) {
          double s = xc[i];
#pragma unroll
          for (int k = 0; k < i; ++k) s -= blk[k * 16 + i] * xc[k];
          xc[i] = s / blk[i * 16 + i];
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < nb) M[(int64_t)(b0 + i) * p + c] = xc[i];
    }
    wg_sync(lds_only);
    // (c) trailing blocks, one 16x16 tile per wave at a time
    const int rem = nbk - K - 1;
    for (int t = wv; t < rem * (rem + 1) / 2; t += kSmallWaves) {
      int Jr = 0;
      while ((Jr + 1) * (Jr + 2) / 2 <= t) ++Jr;
      const int I = K + 1 + (t - Jr * (Jr + 1) / 2), J = K + 1 + Jr;
      const int ci = 16 * I + x, cj = 16 * J + x;
      d4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + g + 4 * r;
        acc[r] = (row < p && cj < p) ? M[(int64_t)row * p + cj] : 0.0;
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kk = b0 + 4 * s4 + g;
        const double av = (kk < b1 && ci < p) ? -M[(int64_t)kk * p + ci] : 0.0;
        const double bv = (kk < b1 && cj < p) ? M[(int64_t)kk * p + cj] : 0.0;
        acc = mfma(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + g + 4 * r;
        if (row < p && cj < p) M[(int64_t)row * p + cj] = acc[r];
      }
    }
  }
  wg_sync(lds_only);
  // inverses of the diagonal blocks, one block per wave at a time
  for (int K = wv; K < nbk; K += kSmallWaves)
    inv16_wave(M + (int64_t)(16 * K) * p + 16 * K, p, min(16, p - 16 * K), dinv + 256 * K);
  return true;
}

// Doubles small_step keeps in LDS when they fit: X, M, R_old (p x p each),
// B~ (q x p) and a scratch of max(q p, p p).
__host__ __device__ inline int64_t small_arena(int q, int p) {
  const int64_t pp = (int64_t)p * p, qp = (int64_t)q * p;
  return 3 * pp + qp + (qp > pp ? qp : pp);
}

// Copy the call's device state (which thread 0 has just brought up to date)
// to the pinned host mirror, then the stamp (call id and phase), so a host
// that sees the stamp also sees the state.  Only the phases the host waits
// for publish (from a.publish_from on) and the phase that ends the call; the
// mirror always receives the whole state.  Thread 0 only.
__device__ void publish(const SmallArgs& a, const Ctrl* c) {
  Ctrl* h = a.hctrl;
  if (!h || (!c->done && a.phase < a.publish_from)) return;
  h->done = c->done; h->status = c->status; h->converged = c->converged;
  h->passes = c->passes; h->chol_attempts = c->chol_attempts;
  for (int i = 0; i < 16; ++i) h->sigma[i] = c->sigma[i];
  h->orth_fro = c->orth_fro;
  __threadfence_system();
  __hip_atomic_store(&h->stamp, a.stamp_base + a.phase, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void small_step_body(const SmallArgs& a) {
  extern __shared__ double lds[];
  __shared__ double red[kSmallWaves];
  // power-iteration vectors, Schur partial sums, then (up to 8 blocks) the
  // inverted diagonal blocks D_J for forming C_J
  __shared__ double vw[2 * kMaxCols];
  // (blocks wider than kMaxCols keep the two vectors in global memory)
  double* v = (a.p <= kMaxCols) ? vw : a.vec;
  double* w = (a.p <= kMaxCols) ? vw + kMaxCols : a.vec + a.p;
  constexpr int kLdsDBlocks = 2 * kMaxCols / 256;
  __shared__ int cflag;
  Ctrl* c = a.ctrl;
  const int tid = threadIdx.x;
  const bool lo = a.lds_matrices == 1;   // all matrices in LDS: LDS-only barriers
  const bool mlo = a.lds_matrices != 0;  // the factor M in LDS
  int prev_att = 0;  // factorisations of earlier passes (thread 0)
  // mixed form: is the Gramian of this pass an FP32 one?
  const bool cur32 = (a.phase == 0) ? (a.mixed != 0) : (a.mixed != 0 && c->gram32 != 0);
  if (a.phase > 0 || a.stage == 2) {
    if (c->done) return;
    if (tid == 0) prev_att = c->chol_attempts;
  } else if (tid == 0) {
    // first small_step of a call: fresh state
    c->done = 0; c->status = 0; c->passes = 0; c->chol_attempts = 0;
    c->converged = 0; c->orth_fro = 0.0; c->gram32 = a.mixed;
    for (int i = 0; i < 16; ++i) c->sigma[i] = 0.0;
  }
  const int p = a.p, q = a.q;
  // outb: the basis part (B~, B~^T B~, B) lives outside this kernel; the
  // Gramian blocks and C_J cover the block's own columns only.  fullE: the
  // Gramian is one row-major matrix (pitch p rounded up to 16, upper part
  // read), C_J are formed per superblock and R~ goes to a.rt.
  const bool outb = (a.ext & 1) != 0;
  const bool fullE = (a.ext & 2) != 0;
  const int qe = outb ? 0 : q;
  const int64_t pp = (int64_t)p * p, qp = (int64_t)qe * p;
  double* base = lo ? lds : a.X;   // arena (LDS, or workspace)
  double* X = base;
  double* M = (a.lds_matrices == 2) ? lds : X + pp;   // mode 2: only M in LDS
  double* Ro = X + 2 * pp;      // old diagonal block of R (row-major)
  double* Bt = Ro + pp;         // B~ (row-major q x p)
  double* Bo = Bt + qp;         // B before this pass (append), q x p
  double* R = a.R;
  const int64_t ldr = a.ldr;
  const int64_t roff = q + (int64_t)q * ldr;  // R block at (q, q)

  const bool front = a.stage != 2;   // this launch forms X and tests it
  if (a.phase == 0 && outb && front) {
    // the diagonal block only (bacc_pass writes B and the block below R_in)
    for (int e = tid; e < p * p; e += kSmallThreads) {
      const int i = e % p, j = e / p;
      R[roff + i + (int64_t)j * ldr] = (i == j) ? 1.0 : 0.0;
    }
  } else if (a.phase == 0 && front) {
    // Algorithm 1: R = I.  Algorithm 2: B = 0, R = I_p, and the block below
    // the old R is zero in R_out (Prop. 2.1).
    for (int e = tid; e < (q + p) * p; e += kSmallThreads) {
      const int i = e % (q + p), j = e / (q + p);
      R[i + (int64_t)(q + j) * ldr] = (i == q + j) ? 1.0 : 0.0;
    }
    for (int e = tid; e < p * q; e += kSmallThreads) {
      const int i = e % p, j = e / p;
      R[q + i + (int64_t)j * ldr] = 0.0;
    }
  }

  const int q16 = (qe + 15) & ~15;
  const double* E = a.E;
  const int64_t epitch = (p + 15) & ~15;
  const bool ph0 = a.phase == 0;
  const bool xpre = a.nerr > 0;   // X formed by xfill_pass
  if (front && !xpre) {
    // 1. Gramian blocks from the reduced slots: B~ = E[0:q, :],
    //    G = E[q:q+p, :] (upper, mirrored).
    fill_rows(X, p, p, [&](int i, int j) {
      const int lo = min(i, j), hi = max(i, j);
      return fullE ? E[(int64_t)lo * epitch + hi]
                   : E[e_off(q16, hi >> 4) + (int64_t)(q16 + lo) * 16 + (hi & 15)];
    });
    fill_rows(Bt, qe, p, [&](int i, int j) {
      return E[e_off(q16, j >> 4) + (int64_t)i * 16 + (j & 15)];
    });
    // old diagonal block of R and old B, loaded together with the Gramian
    // blocks (at phase 0 they are the identity and zero: step 6 then copies)
    if (!ph0) {
      fill_rows(Ro, p, p, [&](int i, int j) { return R[roff + i + (int64_t)j * ldr]; });
      if (a.mode == 1 && !outb)
        fill_rows(Bo, q, p, [&](int i, int j) { return R[i + (int64_t)(q + j) * ldr]; });
    }
    // phase 0: the stores of R above precede the stores of step 6 by other threads
    wg_sync(lo && a.phase > 0);
    // 2. Schur complement X = G - B~^T B~ (Prop. 2.1).
    //    Upper triangle, each sum split over kSplit interleaved k-ranges whose
    //    partial sums are added in a fixed order; mirrored to the lower part.
    if (outb && q > 0) {
      // B~^T B~ from btb_pass (symmetric, both triangles)
      for (int e = tid; e < pp; e += kSmallThreads) X[e] -= a.btb[e];
      wg_sync(lo);
    }
    if (a.mode == 1 && !outb && q > 0) {
      constexpr int kSplit = 4;
      const bool split = pp * kSplit <= kMaxCols;
      const int S = split ? kSplit : 1;
      for (int t = tid; t < pp * S; t += kSmallThreads) {
        const int e = t / S, sg = t % S;
        const int i = e / p, j = e % p;
        if (i > j) continue;
        double s = 0.0;
#pragma unroll 8
        for (int k = sg; k < q; k += S) s += Bt[(int64_t)k * p + i] * Bt[(int64_t)k * p + j];
        if (split) {
          v[t] = s;
        } else {
          X[e] -= s;
          if (i != j) X[(int64_t)j * p + i] -= s;
        }
      }
      wg_sync(lo);
      if (split) {
        for (int e = tid; e < pp; e += kSmallThreads) {
          const int i = e / p, j = e % p;
          if (i > j) continue;
          double s = 0.0;
#pragma unroll
          for (int sg = 0; sg < kSplit; ++sg) s += v[e * kSplit + sg];
          X[e] -= s;
          if (i != j) X[(int64_t)j * p + i] -= s;
        }
        wg_sync(lo);
      }
    }
  }
  // ||X||_2 by power iteration from the all-ones vector (the paper leaves the
  // estimator open; Appendix A asks only for a rough estimate).  Every thread calls it and
  // receives the estimate.  On a copy of X in LDS when only M lives there: M
  // is rebuilt from X after each use.
  auto xnorm = [&]() -> double {
    const double* Xs = X;
    if (a.lds_matrices == 2) {
      fill_rows(M, p, p, [&](int i, int j) { return X[(int64_t)i * p + j]; });
      Xs = M;
    }
    wg_sync(lo);   // X (or its copy) is complete before any wave reads it
    // X is symmetric (mirrored from its upper triangle), so (X v)_i is read
    // along column i: X[j p + i] over j, coalesced across rows i.
    double lam = 0.0;
    if (p <= 16) {
      // One wave, in registers: X (zero-padded to 16 x 16) is held in the
      // MFMA result layout, reg r of lane (x, g) = X[g + 4r][x].  X is
      // symmetric, so that layout is also the A and B operand layout of a
      // product with X: X^2 is four MFMAs on the registers, and so are
      // X^4, X^8, ...  The steps of the iteration are applied as
      // v = X^s 1 / ||X^s 1||: the first step X 1 explicitly (X 1 = 0 ends
      // the iteration, as in the step-by-step form), then X^(s-1) as the
      // product of the powers X^(2^k) for the set bits k of s - 1 (each
      // power scaled to unit Frobenius norm; scaling only changes the
      // length of the iterate): the same vector as s normalised steps.  The vector is kept as column 0 of a 16 x 16
      // operand, which the MFMA result layout also matches.
      if (tid < 64) {
        const int x = tid & 15, g = tid >> 4;
        auto wsum = [](double t) {
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
          return t;
        };
        auto fro = [&](const d4& t) {
          return sqrt(wsum(t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + t[3] * t[3]));
        };
        auto prod = [&](const d4& pa, const d4& pb) {
          d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int r = 0; r < 4; ++r) acc = mfma(pa[r], pb[r], acc);
          return acc;
        };
        d4 xm;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          xm[r] = (g + 4 * r < p && x < p) ? Xs[(int64_t)(g + 4 * r) * p + x] : 0.0;
        d4 vv;
#pragma unroll
        for (int r = 0; r < 4; ++r) vv[r] = (x == 0 && g + 4 * r < p) ? 1.0 : 0.0;
        // the first step explicitly: X 1 = 0 ends the iteration with 0
        vv = prod(xm, vv);
        const double n1 = fro(vv);
        double lw;
        if (!(n1 > 0.0) || !isfinite(n1)) {
          lw = isfinite(n1) ? 0.0 : __builtin_nan("");
        } else {
          vv = vv * (1.0 / n1);
          const int rest = a.power_steps - 1;
          d4 pw = xm * (1.0 / fro(xm));   // X^(2^k), scaled
          for (int k = 0; (rest >> k) != 0; ++k) {
            if ((rest >> k) & 1) vv = prod(pw, vv);
            if ((rest >> (k + 1)) != 0) {
              pw = prod(pw, pw);
              const double fp = fro(pw);
              pw = pw * (1.0 / fp);
            }
          }
          const double nrm = fro(vv);
          if (!(nrm > 0.0) || !isfinite(nrm)) {
            lw = isfinite(nrm) ? 0.0 : __builtin_nan("");
          } else {
            vv = vv * (1.0 / nrm);
            const d4 xv = prod(xm, vv);
            lw = fabs(wsum(vv[0] * xv[0] + vv[1] * xv[1] + vv[2] * xv[2] + vv[3] * xv[3]));
          }
        }
        if (tid == 0) w[0] = lw;
      }
      wg_sync(lo);
      lam = w[0];
    } else if (p <= 64) {
      // Four waves, the same power scheme on 16 x 16 tiles (nt x nt of
      // them, zero-padded): each power X^(2^k) is formed on MFMA from the
      // previous one (read along columns, which symmetry allows), scaled
      // to unit Frobenius norm and stored row-major in M; the iterate
      // (column 0 of a 16 nt x 16 operand, in v), after the explicit first
      // step X 1, is multiplied by each power whose bit of s - 1 is set as
      // soon as it is formed (powers of X commute).  X itself stays intact
      // for the final Rayleigh quotient.
      const int nt = (p + 15) >> 4;
      const int wv = tid >> 6, x = tid & 15, g = (tid >> 4) & 3;
      const double* src = Xs;   // the current power (X first)
      auto opnd = [&](const double* P, int r, int c) {   // P[r][c], zero padding
        return (r < p && c < p) ? P[(int64_t)r * p + c] : 0.0;
      };
      // v <- P v for the current power P (tile row I = wave), in place
      auto apply_v = [&](const double* P) {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        if (wv < nt) {
          for (int K = 0; K < nt; ++K)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const int kk = 16 * K + 4 * s4 + g;
              const double av = opnd(P, kk, 16 * wv + x);            // P[16wv + x][kk]
              const double bv = (x == 0 && kk < p) ? v[kk] : 0.0;
              acc = mfma(av, bv, acc);
            }
        }
        wg_sync(lo);   // every wave has read v
        if (wv < nt && x == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * wv + g + 4 * r;
            if (row < p) v[row] = acc[r];
          }
        }
        wg_sync(lo);
      };
      for (int i = tid; i < p; i += kSmallThreads) v[i] = 1.0;
      // ||X||_F (scaling only changes lengths)
      double part = 0.0;
      for (int e = tid; e < p * p; e += kSmallThreads) part += Xs[e] * Xs[e];
      const double f = sqrt(block_sum(part, red, lo));
      // the first step explicitly: X 1 = 0 ends the iteration with 0
      apply_v(src);
      double n1 = 0.0;
      for (int i = tid; i < p; i += kSmallThreads) n1 += v[i] * v[i];
      n1 = sqrt(block_sum(n1, red, lo));
      if (!(n1 > 0.0) || !isfinite(n1) || !isfinite(f)) {
        lam = (isfinite(n1) && isfinite(f)) ? 0.0 : __builtin_nan("");
      } else {
        for (int i = tid; i < p; i += kSmallThreads) v[i] = v[i] / n1;
        wg_sync(lo);
        const int rest = a.power_steps - 1;
        double scale = 1.0 / f;   // the current power is scale * src
        for (int k = 0; (rest >> k) != 0; ++k) {
          if ((rest >> k) & 1) apply_v(src);
          if ((rest >> (k + 1)) == 0) break;
          // next power: (scale src)^2, tiles t = wv, wv + 4, ...
          d4 nxt[4];
          double sq = 0.0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            nxt[u] = d4{0.0, 0.0, 0.0, 0.0};
            const int t = wv + kSmallWaves * u;
            if (t < nt * nt) {
              const int I = t / nt, J = t % nt;
              for (int K = 0; K < nt; ++K)
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                  const int kk = 16 * K + 4 * s4 + g;
                  nxt[u] = mfma(opnd(src, kk, 16 * I + x) * scale, opnd(src, kk, 16 * J + x) * scale, nxt[u]);
                }
#pragma unroll
              for (int r = 0; r < 4; ++r) sq += nxt[u][r] * nxt[u][r];
            }
          }
          const double fp = sqrt(block_sum(sq, red, lo));   // also: all reads of src done
          scale = 1.0 / fp;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int t = wv + kSmallWaves * u;
            if (t < nt * nt) {
              const int I = t / nt, J = t % nt;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = 16 * I + g + 4 * r, col = 16 * J + x;
                if (row < p && col < p) M[(int64_t)row * p + col] = nxt[u][r];
              }
            }
          }
          src = M;
          wg_sync(lo);
        }
        // lam = |v^T X v| / (v^T v) with X itself (not a copy that the
        // powers may have overwritten)
        double vv = 0.0;
        for (int i = tid; i < p; i += kSmallThreads) vv += v[i] * v[i];
        const double nv = sqrt(block_sum(vv, red, lo));
        if (!(nv > 0.0) || !isfinite(nv)) {
          lam = isfinite(nv) ? 0.0 : __builtin_nan("");
        } else {
          for (int i = tid; i < p; i += kSmallThreads) w[i] = v[i] / nv;
          wg_sync(lo);
          double rq = 0.0;
          for (int i = tid; i < p; i += kSmallThreads) {
            double t = 0.0;
            for (int j = 0; j < p; ++j) t += X[(int64_t)j * p + i] * w[j];
            rq += w[i] * t;
          }
          lam = fabs(block_sum(rq, red, lo));
        }
      }
    } else {
      // all waves: thread t takes row t mod p and one of H column ranges;
      // the H partial sums of a row are added in range order
      const int H = max(1, kSmallThreads / p);
      for (int i = tid; i < p; i += kSmallThreads) v[i] = 1.0 / sqrt((double)p);
      wg_sync(lo);
      // returns w_i (thread i < p, else 0) with the partial sums in w[]
      auto mv = [&]() {
        for (int t0 = tid; t0 < p * H; t0 += kSmallThreads) {
          const int i = t0 % p, h = t0 / p;
          const int j0 = h * p / H, j1 = (h + 1) * p / H;
          double t = 0.0;
#pragma unroll 16
          for (int j = j0; j < j1; ++j) t += Xs[(int64_t)j * p + i] * v[j];
          w[h * p + i] = t;
        }
        wg_sync(lo);
        double t = 0.0;
        if (tid < p)
          for (int h = 0; h < H; ++h) t += w[h * p + tid];
        return t;
      };
      bool early = false;
      for (int s = 0; s < a.power_steps; ++s) {
        const double t = mv();
        const double nrm = sqrt(block_sum(t * t, red, lo));
        if (!(nrm > 0.0) || !isfinite(nrm)) {
          lam = isfinite(nrm) ? nrm : __builtin_nan("");
          early = true;
          break;
        }
        if (tid < p) v[tid] = t / nrm;
        wg_sync(lo);
      }
      if (!early) {
        const double t = mv();
        lam = fabs(block_sum(tid < p ? v[tid] * t : 0.0, red, lo));
      }
    }
    return lam;
  };
  // 3. ||X - I||_F (the second stage reads the first stage's value).
  double part = 0.0;
  for (int i = (front && !xpre) ? (tid >> 4) : p; i < p; i += kSmallThreads / 16) {
#pragma unroll 4
    for (int j = tid & 15; j < p; j += 16) {
      const double d = X[(int64_t)i * p + j] - (i == j ? 1.0 : 0.0);
      part += d * d;
    }
  }
  if (front && xpre)   // xfill_pass's partial sums, added in a fixed order
    for (int i = tid; i < a.nerr; i += kSmallThreads) part += a.errpart[i];
  const double err = front ? sqrt(block_sum(part, red, lo)) : c->orth_fro;
  // Shift policy of an orth call (appends always follow Algorithm 2):
  // 0 Algorithm 1 (recomputed from the current X, x10 escalation), 1 none
  // (a breakdown ends the call; a shifted first pass does not escalate),
  // 2 isCholQR (one shift from the input Gramian, reapplied on breakdown).
  const int pol = (a.mode == 0) ? a.shift_policy : 0;
  const double mm = (double)a.m;
  if (pol == 2 && ph0 && isfinite(err) && front) {
    // ||X_0|| = ||A||^2: the one shift of the call
    const double lam0 = xnorm();
    if (tid == 0) c->sigma_fixed = fmax(11.0 * (mm * p + (double)p * (p + 1)) * a.u * lam0, 2.0 * a.u);
  }
  // 4. Stopping test (Algorithm 1 with the CholQR3 start; Algorithm 2, whose
  //    first pass always runs: Prop. 2.1 forms the new columns by the
  //    projection, and an initial X = I does not make B~ zero).
  int status = -1;
  if (!front) {
    // decided by the first stage
  } else if (!isfinite(err)) {
    status = 3;  // SQR_ENONFINITE
  } else if ((a.mode == 0) ? (!cur32 && a.phase >= a.min_passes && err < a.tol)
                           : (a.phase >= 1 && err < a.tol)) {
    status = 0;
  } else if (a.phase >= a.max_iter) {
    status = 1;  // SQR_NOT_CONVERGED
  }
  if (status >= 0) {
    if (tid == 0) {
      c->status = status;
      c->converged = (status == 0);
      c->orth_fro = err;
      c->done = 1;
      publish(a, c);
    }
    return;
  }
  const int pass = a.phase + 1;
  // 5. Shift decision and factorisation: an unshifted attempt (except on a
  //    shifted first pass), and after its breakdown, or on a shifted first
  //    pass, the shift from ||X||_2 with x10 escalation.  One factorisation
  //    site for all attempts.
  bool shifted = false;
  bool need_shift = (a.mode == 0 && pass == 1 && a.first_pass_shift);
  int attempts = 0, esc = 0;
  double sigma = 0.0;
  // FP32 Gramian (mixed form): sigma = p u32 ||X||, floor 2 u32
  constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
  const double ufl = cur32 ? kU32 : a.u;
  bool ok = false;
  // stage 2: the first factorisation was run by the band kernels with the
  // shift the first stage chose
  bool ran = a.stage == 2;
  if (ran) {
    ok = c->chol_fail == 0;
    shifted = c->att_shifted != 0;
    sigma = c->att_sigma;
    need_shift = false;
    attempts = 1;
  }
  for (;;) {
    if (ran) {
      ran = false;
      if (ok) break;
      if (!shifted) {
        if (pol == 1) break;
        need_shift = true;
        continue;
      }
      if (pol != 0) break;
      if (esc >= a.max_escalations) break;
      ++esc;
      sigma = fmax(10.0 * sigma, 2.0 * ufl);
    }
    if (need_shift) {
      need_shift = false;
      shifted = true;
      if (pol == 2) {
        sigma = c->sigma_fixed;
      } else {
        const double lam = xnorm();
        // Algorithm 1: the Gramian's own width; Algorithm 2: q as printed,
        // or p, or q + p (option)
        const double d = (a.mode == 0) ? p : (a.shift_dim == 0 ? q : (a.shift_dim == 1 ? p : q + p));
        const double cnt = mm * d + d * (d + 1.0);
        sigma = cur32 ? fmax((double)p * kU32 * lam, 2.0 * kU32)
                      : fmax(11.0 * cnt * a.u * lam, 2.0 * a.u);
      }
    }
    if (a.stage == 1) {
      // the band kernels factor X + sigma I next
      if (tid == 0) {
        c->att_sigma = sigma;
        c->att_shifted = shifted ? 1 : 0;
        c->chol_fail = 0;
        c->orth_fro = err;
      }
      return;
    }
    fill_rows(M, p, p, [&](int i, int j) { return X[(int64_t)i * p + j] + (i == j ? sigma : 0.0); });
    ++attempts;
    ok = (p <= 16 && mlo) ? chol_upper_wave(M, p, &cflag, a.rinv) : chol_blocked(M, p, mlo, vw, &cflag, a.rinv);
    if (ok) break;
    if (!shifted) {
      if (pol == 1) break;   // no shift: the breakdown ends the call
      need_shift = true;
      continue;
    }
    if (pol != 0) break;     // the fixed shift, or a no-shift first pass, failed
    if (esc >= a.max_escalations) break;
    ++esc;
    sigma = fmax(10.0 * sigma, 2.0 * ufl);
  }
  if (!ok) {
    if (tid == 0) {
      c->status = 2;  // SQR_BREAKDOWN
      c->chol_attempts = prev_att + attempts;
      c->orth_fro = err;
      c->done = 1;
      publish(a, c);
    }
    return;
  }
  if (a.stage == 2) {
    // the R update, C_J and R~ follow in trmm_pass and cj_pass
    if (tid == 0) {
      c->passes = pass;
      c->gram32 = 0;
      if (pass <= 16) c->sigma[pass - 1] = sigma;
      c->chol_attempts = prev_att + attempts;
      c->orth_fro = err;
      publish(a, c);
    }
    return;
  }
  wg_sync(lo);
  // 6. B <- B + B~ R_old, then R <- R~ R_old (Algorithm 2; Algorithm 1).
  //    At phase 0 (R_old = I, B_old = 0) both are copies.
  //    Fixed trip counts for p <= 16 (one row of B per thread, the row of
  //    B~ in registers; stores along columns of R coalesce).
  if (outb && q > 0) {
    // R_old for bacc_pass (the identity at phase 0)
    for (int e = tid; e < pp; e += kSmallThreads) {
      const int i = e / p, j = e % p;
      a.rold[e] = ph0 ? (i == j ? 1.0 : 0.0) : Ro[e];
    }
  }
  if (ph0) {
    if (a.mode == 1 && !outb)
      for (int e = tid; e < qp; e += kSmallThreads) {
        const int i = e / p, j = e % p;
        R[i + (int64_t)(q + j) * ldr] = Bt[e];
      }
    for (int e = tid; e < pp; e += kSmallThreads) {
      const int i = e % p, j = e / p;
      R[roff + i + (int64_t)j * ldr] = (i <= j) ? M[(int64_t)i * p + j] : 0.0;
    }
  } else if (a.mode == 1 && !outb && q > 0) {
    if (p <= 16) {
      for (int i = tid; i < q; i += kSmallThreads) {
        double br[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) br[k] = (k < p) ? Bt[(int64_t)i * p + k] : 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          if (j < p) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k <= j; ++k) s += br[k] * Ro[(int64_t)k * p + j];
            R[i + (int64_t)(q + j) * ldr] = Bo[(int64_t)i * p + j] + s;
          }
        }
      }
    } else {
      for (int e = tid; e < qp; e += kSmallThreads) {
        const int i = e / p, j = e % p;
        double s = 0.0;
#pragma unroll 4
        for (int k = 0; k <= j; ++k) s += Bt[(int64_t)i * p + k] * Ro[(int64_t)k * p + j];
        R[i + (int64_t)(q + j) * ldr] = Bo[e] + s;
      }
    }
  }
  if (ph0) {
  } else if (p <= 16) {
    for (int e = tid; e < pp; e += kSmallThreads) {
      const int i = e / p, j = e % p;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k >= i && k <= j) s += M[(int64_t)i * p + k] * Ro[(int64_t)k * p + j];
      R[roff + i + (int64_t)j * ldr] = (i <= j) ? s : 0.0;
    }
  } else {
    // 16x16 tiles (I <= J) of the product of two upper triangular matrices
    // on MFMA, one tile per wave at a time: the wave forms the transposed
    // tile, sum_K Ro_KJ^T M_IK^T, with the strictly lower part of M (which
    // holds no factor entries) masked to zero.
    const int wv = tid >> 6, ln = tid & 63, x = ln & 15, g = ln >> 4;
    const int nbk = (p + 15) >> 4;
    for (int t = wv; t < nbk * (nbk + 1) / 2; t += kSmallWaves) {
      int J = 0;
      while ((J + 1) * (J + 2) / 2 <= t) ++J;
      const int I = t - J * (J + 1) / 2;
      const int ii = 16 * I + x, jj = 16 * J + x;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
      for (int K0 = I; K0 <= J; K0 += 4) {   // operands of four K blocks in flight
        double av[16], bv[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int kk = 16 * K0 + 4 * e + g;   // e = 4 (K - K0) + s4
          const bool in = K0 + (e >> 2) <= J && kk < p;
          av[e] = (in && jj < p && kk <= jj) ? Ro[(int64_t)kk * p + jj] : 0.0;
          bv[e] = (in && ii < p && kk >= ii) ? M[(int64_t)ii * p + kk] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) acc = mfma(av[e], bv[e], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * J + g + 4 * r;
        if (ii < p && j < p) R[roff + ii + (int64_t)j * ldr] = (ii <= j) ? acc[r] : 0.0;
      }
    }
    for (int e = tid; e < pp; e += kSmallThreads) {   // tiles below the diagonal
      const int i = e % p, j = e / p;
      if ((i >> 4) > (j >> 4)) R[roff + i + (int64_t)j * ldr] = 0.0;
    }
  }
  // 7. Operands of the next pass.  D_J, the inverse of the diagonal block J
  //    of R~ (identity beyond p), was stored with the factorisation (wave 0,
  //    global memory); the C_J below read it from LDS when it fits.
  wg_sync(false);
  if (a.nblk <= kLdsDBlocks)
    for (int e = tid; e < a.nblk * 256; e += kSmallThreads) vw[e] = a.rinv[e];
  wg_sync(a.nblk <= kLdsDBlocks);
  //    C_J = -[B~[:, J]; 0 (padding rows q..q16-1); R~[0:16J, J]] D_J, so the
  //    streaming kernel forms Y_J = W_J D_J + [Q_in, Y_<J] C_J directly.
  //    One row of C_J per thread: the row of the source in registers, D_J
  //    read as broadcasts.
  //    fullE: superblocks of kSuper columns, C_J = -R~[s0:16J, J] D_J with
  //    s0 the first column of J's superblock (the earlier superblocks are
  //    subtracted by proj_pass with R~ itself), each superblock's C_J from
  //    its own region of bneg.
  for (int J = 0; J < a.nblk; ++J) {
    const int b0 = 16 * J, pb = min(16, p - b0);
    const int s0 = fullE ? (b0 / kSuper) * kSuper : 0;
    const int Jl = J - s0 / 16;
    const int rows = q16 + b0 - s0;
    const double* D = (a.nblk <= kLdsDBlocks) ? vw + J * 256 : a.rinv + J * 256;
    double* bn = a.bneg + (int64_t)(s0 / kSuper) * kSuperBneg +
                 16 * ((int64_t)Jl * q16 + 8 * (int64_t)Jl * (Jl - 1));
    for (int kk = tid; kk < rows; kk += kSmallThreads) {
      double src[16];
      const bool real = kk < qe || kk >= q16;
      const double* sr = (kk < qe) ? Bt + (int64_t)kk * p + b0
                                  : (real ? M + (int64_t)(s0 + kk - q16) * p + b0 : Bt);
#pragma unroll
      for (int t = 0; t < 16; ++t) src[t] = (real && t < pb) ? sr[t] : 0.0;
#pragma unroll
      for (int cc = 0; cc < 16; cc += 2) {
        double v0 = 0.0, v1 = 0.0;
#pragma unroll
        for (int t = 0; t <= cc + 1; ++t) {
          if (t <= cc) v0 -= src[t] * D[t * 16 + cc];
          v1 -= src[t] * D[t * 16 + cc + 1];
        }
        double2 o;
        o.x = (cc < pb) ? v0 : 0.0;
        o.y = (cc + 1 < pb) ? v1 : 0.0;
        *reinterpret_cast<double2*>(bn + (int64_t)kk * 16 + cc) = o;
      }
    }
  }
  if (fullE) {
    // R~ for proj_pass (row-major, zero below the diagonal)
    for (int64_t e = tid; e < pp; e += kSmallThreads) {
      const int64_t i = e / p, j = e - i * p;
      a.rt[e] = (i <= j) ? M[e] : 0.0;
    }
  }
  if (tid == 0) {
    c->passes = pass;
    c->gram32 = (cur32 && shifted) ? 1 : 0;   // FP32 Gramians end after an unshifted pass
    if (pass <= 16) c->sigma[pass - 1] = sigma;
    c->chol_attempts = prev_att + attempts;
    c->orth_fro = err;
    publish(a, c);
  }
}

__global__ __launch_bounds__(kSmallThreads) void small_step(SmallArgs a) { small_step_body(a); }
// One workgroup per call of the batch.
__global__ __launch_bounds__(kSmallThreads) void small_step_batch(BatchTable<SmallArgs> t) {
  small_step_body(t.args[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// Blocks wider than kMaxSCols: the p x p work of a pass on many workgroups.
// small_step (stage 1) decides the stop test and the shift of the first
// factorisation; mfill_pass forms X + sigma I and copies R_old; the upper
// Cholesky factor is formed in bands of kBand rows (chol_diag: the diagonal
// block by one workgroup, as small_step factors a block; chol_panel: the
// band's rows right of it by forward substitution, one column per thread;
// chol_trail: the trailing 16x16 blocks on MFMA), a breakdown stops the later
// bands; small_step (stage 2) takes further attempts itself if needed; then
// trmm_pass forms R <- R~ R_old and cj_pass the C_J and R~ of the next pass.
// ---------------------------------------------------------------------------
constexpr int kBand = 64;

// X = G - B~^T B~ (both triangles, from the upper tiles of the reduced
// Gramian) in 32 x 32 tiles, and the tile's sum of squares of X - I (lanes,
// then waves in order) into errpart[tile].
__global__ __launch_bounds__(kThreads) void xfill_pass(BigArgs a) {
  __shared__ double L[32][33];
  __shared__ double red[kWaves];
  if (a.phase > 0 && a.ctrl->done) return;
  const int p = a.p;
  const int64_t pitch = (p + 15) & ~15;
  const int tp = (p + 31) / 32;
  const int ti = (int)blockIdx.x / tp, tj = (int)blockIdx.x % tp;
  const int lo = min(ti, tj), hi = max(ti, tj);
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8
  for (int r = ly; r < 32; r += 8) {
    const int i = 32 * lo + r, j = 32 * hi + lx;
    L[r][lx] = (i < p && j < p) ? a.E[(int64_t)i * pitch + j] : 0.0;
  }
  __syncthreads();
  double part = 0.0;
  for (int r = ly; r < 32; r += 8) {
    const int i = 32 * ti + r, j = 32 * tj + lx;
    if (i >= p || j >= p) continue;
    double g;
    if (ti < tj) g = L[r][lx];
    else if (ti > tj) g = L[lx][r];
    else g = L[min(r, lx)][max(r, lx)];
    const double xv = g - (a.btb ? a.btb[(int64_t)i * p + j] : 0.0);
    a.X[(int64_t)i * p + j] = xv;
    const double d = xv - (i == j ? 1.0 : 0.0);
    part += d * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += red[w];
    a.errpart[blockIdx.x] = s;
  }
}

// M = X + sigma I and rold = R_old (row-major; the identity at phase 0),
// 32 x 32 tiles (R_old is read along its columns and written along rows).
__global__ __launch_bounds__(kThreads) void mfill_pass(BigArgs a) {
  __shared__ double tile[32][33];
  const Ctrl* c = a.ctrl;
  if (c->done) return;
  const int p = a.p;
  const int tp = (p + 31) / 32;
  const int ti = (int)blockIdx.x / tp, tj = (int)blockIdx.x % tp;
  const double sigma = c->att_sigma;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8
  for (int r = ly; r < 32; r += 8) {
    const int i = 32 * ti + r, j = 32 * tj + lx;
    if (i < p && j < p) a.M[(int64_t)i * p + j] = a.X[(int64_t)i * p + j] + (i == j ? sigma : 0.0);
  }
  // R_old[i][j] = R[q + i + (q + j) ldr]: read with i along the lanes
  for (int r = ly; r < 32; r += 8) {
    const int j = 32 * tj + r, i = 32 * ti + lx;
    double v = 0.0;
    if (i < p && j < p) v = (a.phase == 0) ? (i == j ? 1.0 : 0.0) : a.R[(int64_t)(a.q + i) + (int64_t)(a.q + j) * a.ldr];
    tile[r][lx] = v;
  }
  __syncthreads();
  for (int r = ly; r < 32; r += 8) {
    const int i = 32 * ti + r, j = 32 * tj + lx;
    if (i < p && j < p) a.rold[(int64_t)i * p + j] = tile[lx][r];
  }
}

// The diagonal block of band k0 (its upper part, as the earlier bands left
// it) factored in LDS by one workgroup; the inverses of its 16x16 diagonal
// blocks go to rinv.  A breakdown sets ctrl->chol_fail.
__global__ __launch_bounds__(kSmallThreads) void chol_diag(BigArgs a) {
  __shared__ double L[kBand * kBand];
  __shared__ double blk[256];
  __shared__ int flag;
  Ctrl* c = a.ctrl;
  if (c->done || c->chol_fail) return;
  const int p = a.p, k0 = a.k0, w = min(kBand, p - k0);
  for (int e = threadIdx.x; e < w * w; e += kSmallThreads) {
    const int i = e / w, j = e - i * w;
    L[e] = a.M[(int64_t)(k0 + i) * p + k0 + j];
  }
  __syncthreads();
  const bool ok = chol_blocked(L, w, true, blk, &flag, a.rinv + 256 * (k0 / 16));
  if (!ok) {
    if (threadIdx.x == 0) c->chol_fail = 1;
    return;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < w * w; e += kSmallThreads) {
    const int i = e / w, j = e - i * w;
    if (i <= j) a.M[(int64_t)(k0 + i) * p + k0 + j] = L[e];
  }
}

// Rows k0 .. k0 + w - 1 right of the diagonal block: R_K,>K = R_KK^{-T}
// M_K,>K, one column per thread (the order of operations of small_step's
// blocked factorisation).
__global__ __launch_bounds__(kSmallThreads) void chol_panel(BigArgs a) {
  __shared__ double Rk[kBand * kBand];
  const Ctrl* c = a.ctrl;
  if (c->done || c->chol_fail) return;
  const int p = a.p, k0 = a.k0, w = min(kBand, p - k0);
  for (int e = threadIdx.x; e < w * w; e += kSmallThreads) {
    const int i = e / w, j = e - i * w;
    Rk[e] = a.M[(int64_t)(k0 + i) * p + k0 + j];
  }
  __syncthreads();
  const int col = k0 + w + (int)blockIdx.x * kSmallThreads + (int)threadIdx.x;
  if (col >= p) return;
  double xc[kBand];
#pragma unroll
  for (int i = 0; i < kBand; ++i) xc[i] = (i < w) ? a.M[(int64_t)(k0 + i) * p + col] : 0.0;
#pragma unroll
  for (int i = 0; i < kBand; ++i) {
    if (i < w) {
      double s = xc[i];
#pragma unroll
      for (int k = 0; k < i; ++k) s -= Rk[k * w + i] * xc[k];
      xc[i] = s / Rk[i * w + i];
    }
  }
#pragma unroll
  for (int i = 0; i < kBand; ++i)
    if (i < w) a.M[(int64_t)(k0 + i) * p + col] = xc[i];
}

// Trailing 16x16 blocks (I <= J) right of and below band k0:
// M_IJ -= R_K,I^T R_K,J over the band's rows, one block per wave.
__global__ __launch_bounds__(kThreads) void chol_trail(BigArgs a) {
  const Ctrl* c = a.ctrl;
  if (c->done || c->chol_fail) return;
  const int p = a.p, k0 = a.k0, w = min(kBand, p - k0), k1 = k0 + w;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  const int T = (p - k1 + 15) >> 4;
  const int64_t t = (int64_t)blockIdx.x * kWaves + wave;
  if (t >= (int64_t)T * (T + 1) / 2) return;
  int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)J * (J + 1) / 2 > t) --J;
  while ((int64_t)(J + 1) * (J + 2) / 2 <= t) ++J;
  const int I = (int)(t - (int64_t)J * (J + 1) / 2);
  const int ci = k1 + 16 * I + x, cj = k1 + 16 * J + x;
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = k1 + 16 * I + g + 4 * r;
    acc[r] = (row < p && cj < p) ? a.M[(int64_t)row * p + cj] : 0.0;
  }
  for (int s = 0; s < w; s += 4) {
    const int k = k0 + s + g;
    const bool kin = s + g < w;
    const double av = (kin && ci < p) ? -a.M[(int64_t)k * p + ci] : 0.0;
    const double bv = (kin && cj < p) ? a.M[(int64_t)k * p + cj] : 0.0;
    acc = mfma(av, bv, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = k1 + 16 * I + g + 4 * r;
    if (row < p && cj < p) a.M[(int64_t)row * p + cj] = acc[r];
  }
}

// R[q:q+p, q:q+p] <- R~ R_old (upper times upper; zero below the diagonal),
// one 16x16 block per wave.  The block of R~ in a row of blocks is turned
// through a wave-private LDS tile so that both operands are read along rows.
__global__ __launch_bounds__(kThreads) void trmm_pass(BigArgs a) {
  __shared__ double trs[kWaves][16 * 17];
  const Ctrl* c = a.ctrl;
  if (c->done) return;
  const int p = a.p, P = (p + 15) >> 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  const int64_t t = (int64_t)blockIdx.x * kWaves + wave;
  if (t >= (int64_t)P * P) return;
  const int I = (int)(t / P), J = (int)(t % P);   // block row I (of R~), column J
  double* Rb = a.R + a.q + (int64_t)a.q * a.ldr;
  double* tr = trs[wave];
  if (I > J) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + x, col = 16 * J + g + 4 * r;
      if (row < p && col < p) Rb[row + (int64_t)col * a.ldr] = 0.0;
    }
    return;
  }
  // D'[i][j] = newR[16 I + j][16 J + i]: A[i][k] = R_old[k][16 J + i],
  // B[k][j] = R~[16 I + j][k]; lane (x, g) register r holds row 16 I + x,
  // column 16 J + g + 4r
  d4 acc = d4{0.0, 0.0, 0.0, 0.0};
  for (int K = I; K <= J; ++K) {
    // R~ block (I, K) into LDS, masked to the upper triangle: tr[row][col]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + g + 4 * r, col = 16 * K + x;
      tr[(g + 4 * r) * 17 + x] = (row < p && col < p && col >= row) ? a.M[(int64_t)row * p + col] : 0.0;
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 16 * K + 4 * s + g;
      const int col = 16 * J + x;
      const double av = (k < p && col < p && k <= col) ? a.rold[(int64_t)k * p + col] : 0.0;
      const double bv = tr[x * 17 + 4 * s + g];
      acc = mfma(av, bv, acc);
    }
    wave_lds_sync();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * I + x, col = 16 * J + g + 4 * r;
    if (row < p && col < p) Rb[row + (int64_t)col * a.ldr] = (row <= col) ? acc[r] : 0.0;
  }
}

// Per 16-column block J (one workgroup): C_J = -R~[s0:16J, J] D_J within
// J's superblock (s0 its first column), as small_step forms it, and the
// columns of J of R~ (row-major, zero below the diagonal) for proj_pass.
__global__ __launch_bounds__(kSmallThreads) void cj_pass(BigArgs a) {
  __shared__ double D[256];
  const Ctrl* c = a.ctrl;
  if (c->done) return;
  const int p = a.p, J = blockIdx.x;
  const int b0 = 16 * J, pb = min(16, p - b0);
  const int s0 = (b0 / kSuper) * kSuper, Jl = J - s0 / 16;
  for (int e = threadIdx.x; e < 256; e += kSmallThreads) D[e] = a.rinv[256 * J + e];
  __syncthreads();
  double* bn = a.bneg + (int64_t)(s0 / kSuper) * kSuperBneg + 128 * (int64_t)Jl * (Jl - 1);
  for (int kk = threadIdx.x; kk < b0 - s0; kk += kSmallThreads) {
    double src[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) src[t] = (t < pb) ? a.M[(int64_t)(s0 + kk) * p + b0 + t] : 0.0;
#pragma unroll
    for (int cc = 0; cc < 16; cc += 2) {
      double v0 = 0.0, v1 = 0.0;
#pragma unroll
      for (int t = 0; t <= cc + 1; ++t) {
        if (t <= cc) v0 -= src[t] * D[t * 16 + cc];
        v1 -= src[t] * D[t * 16 + cc + 1];
      }
      double2 o;
      o.x = (cc < pb) ? v0 : 0.0;
      o.y = (cc + 1 < pb) ? v1 : 0.0;
      *reinterpret_cast<double2*>(bn + (int64_t)kk * 16 + cc) = o;
    }
  }
  for (int i = threadIdx.x; i < p; i += kSmallThreads) {
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (t < pb) a.rt[(int64_t)i * p + b0 + t] = (i <= b0 + t) ? a.M[(int64_t)i * p + b0 + t] : 0.0;
  }
}

}  // namespace sqr
