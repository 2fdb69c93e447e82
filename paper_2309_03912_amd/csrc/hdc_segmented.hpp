// Segmented transform_reduce: out[j] = sum over [off[j], off[j+1]) of f(x[i])
// for many uneven segments in one batch, without host synchronisation.
//
// Work decomposition (all on the device):
//   * small segments (length <= small_seg) are packed `spw` per wavefront,
//     64/spw lanes per segment, by fixed segment-index groups;
//   * every other segment is cut into pieces of `chunk` elements; a segment
//     of one piece writes its result directly, a longer one writes one
//     partial per piece, folded afterwards in piece order.
// The plan builds two piece lists (full pieces, then the short last pieces)
// without atomics: a count pass folds per-block totals, one block scans them,
// and a write pass places every entry at its block base plus its prefix
// within the block -- three short launches whose list order is fixed.  The
// persistent pass walks full pieces, short pieces, then small-segment
// groups, round-robin over its wavefronts (equal-cost items first keeps the
// static split balanced), prefetching the next item's descriptor and offsets
// while the current one streams.  Every result is computed over a fixed
// element range in a fixed order, so the output is reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"
#include "hdc_scan.hpp"

namespace hdc {

struct SegPiece {
  int32_t seg;
  int32_t k;  // piece index within the segment
};

// Totals of the plan: list lengths and partial slots handed out.
struct SegCounters {
  uint32_t full;      // entries of the full-piece list
  uint32_t part;      // entries of the short-piece list
  uint32_t partials;  // partial slots handed out to multi-piece segments
  uint32_t longs;     // entries of the multi-piece segment list
  __host__ __device__ static SegCounters zero() { return {0u, 0u, 0u, 0u}; }
  __host__ __device__ static SegCounters merge(SegCounters a, SegCounters b) {
    return {a.full + b.full, a.part + b.part, a.partials + b.partials, a.longs + b.longs};
  }
};

struct SegPlan {
  SegCounters* cnt;
  SegCounters* block_tot;   // per plan block: its totals, then its exclusive base
  SegPiece* full_list;   // capacity cap_full
  SegPiece* part_list;   // capacity cap_part
  int32_t* long_base;    // per segment: first partial slot (multi-piece only)
  int32_t* long_list;    // capacity cap_part (one per multi-piece segment)
  void* partials;        // capacity cap_partials fold states
  int64_t cap_full, cap_part, cap_partials;
  int64_t chunk;
  int64_t small_seg;
  int32_t spw;           // small segments per wavefront (power of two, <= 64)
};

constexpr int kPlanBlock = 256;

// What segment j contributes to the plan.
struct SegShape {
  int64_t L, pieces, nfull;
  bool big;
  SegCounters want;
};

__device__ __forceinline__ SegShape seg_shape(const int64_t* __restrict__ off, int64_t S, const SegPlan& p,
                                              int64_t j) {
  SegShape r{};
  if (j < S) r.L = off[j + 1] - off[j];
  r.big = j < S && r.L > p.small_seg;
  r.pieces = r.big ? (r.L + p.chunk - 1) / p.chunk : 0;
  r.nfull = r.pieces > 1 ? r.L / p.chunk : 0;
  r.want.full = (uint32_t)r.nfull;
  r.want.part = r.big && (r.pieces == 1 || r.L % p.chunk != 0) ? 1u : 0u;
  r.want.partials = r.pieces > 1 ? (uint32_t)r.pieces : 0u;
  r.want.longs = r.pieces > 1 ? 1u : 0u;
  return r;
}

// Plan pass 1: per-block totals.
static __global__ __launch_bounds__(kPlanBlock) void seg_count_kernel(const int64_t* __restrict__ off, int64_t S,
                                                                      SegPlan p) {
  __shared__ SegCounters lds[kMaxWaves];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const SegShape sh = seg_shape(off, S, p, j);
  SegCounters total;
  (void)block_exclusive_scan_acc(sh.want, lds, &total);
  if (threadIdx.x == 0) p.block_tot[blockIdx.x] = total;
}

// Plan pass 2 (one block): exclusive scan of the block totals in place, and
// the grand totals into p.cnt.
static __global__ __launch_bounds__(1024) void seg_count_scan_kernel(int64_t nblocks, SegPlan p) {
  __shared__ SegCounters lds[kMaxWaves];
  SegCounters carry = SegCounters::zero();
  for (int64_t base = 0; base < nblocks; base += blockDim.x) {
    const int64_t b = base + threadIdx.x;
    const SegCounters v = b < nblocks ? p.block_tot[b] : SegCounters::zero();
    SegCounters total;
    const SegCounters before = block_exclusive_scan_acc(v, lds, &total);
    if (b < nblocks) p.block_tot[b] = SegCounters::merge(carry, before);
    carry = SegCounters::merge(carry, total);
  }
  if (threadIdx.x == 0) *p.cnt = carry;
}

// Plan pass 3: every segment writes its entries at its block's base plus its
// prefix within the block.  A segment writes its first kOwnPieces full-piece
// entries itself; the block writes the rest of every longer one together.
constexpr int64_t kOwnPieces = 16;

static __global__ __launch_bounds__(kPlanBlock) void seg_write_kernel(const int64_t* __restrict__ off, int64_t S,
                                                                      SegPlan p) {
  __shared__ SegCounters lds[kMaxWaves];
  __shared__ int nbig;
  __shared__ int64_t big_j[kPlanBlock], big_f0[kPlanBlock], big_n[kPlanBlock];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const SegShape sh = seg_shape(off, S, p, j);
  SegCounters total;
  const SegCounters pre = SegCounters::merge(p.block_tot[blockIdx.x],
                                             block_exclusive_scan_acc(sh.want, lds, &total));
  if (threadIdx.x == 0) nbig = 0;
  __syncthreads();
  if (sh.big) {
    if (sh.pieces > 1) {
      const int64_t slot0 = pre.partials, li = pre.longs;
      p.long_base[j] = slot0 + sh.pieces <= p.cap_partials ? (int32_t)slot0 : -1;
      if (li < p.cap_part) p.long_list[li] = (int32_t)j;
    }
    const int64_t f0 = pre.full;
    const int64_t own = sh.nfull < kOwnPieces ? sh.nfull : kOwnPieces;
    for (int64_t k = 0; k < own; ++k)
      if (f0 + k < p.cap_full) p.full_list[f0 + k] = SegPiece{(int32_t)j, (int32_t)k};
    if (sh.nfull > kOwnPieces) {
      const int q = atomicAdd(&nbig, 1);
      big_j[q] = j;
      big_f0[q] = f0;
      big_n[q] = sh.nfull;
    }
    if (sh.want.part && (int64_t)pre.part < p.cap_part)
      p.part_list[pre.part] = SegPiece{(int32_t)j, (int32_t)sh.nfull};
  }
  __syncthreads();
  for (int q = 0; q < nbig; ++q)  // every entry's content is fixed, whatever q a segment drew
    for (int64_t k = kOwnPieces + threadIdx.x; k < big_n[q]; k += blockDim.x)
      if (big_f0[q] + k < p.cap_full) p.full_list[big_f0[q] + k] = SegPiece{(int32_t)big_j[q], (int32_t)k};
}

// True when the plan's lists exceed the workspace's capacity.  The plan then
// drops the entries past the end, and the persistent pass instead folds
// every segment whole with one wavefront (slower; the summation order, and
// so the last bits of a floating-point result, differ from the planned pass).
__device__ __forceinline__ bool seg_overflow(const SegPlan& p) {
  return (int64_t)p.cnt->full > p.cap_full || (int64_t)p.cnt->partials > p.cap_partials ||
         (int64_t)p.cnt->part > p.cap_part || (int64_t)p.cnt->longs > p.cap_part;
}

// Final value of a fold state as stored in `out`.
template <class Acc>
__device__ __forceinline__ void store_result(void* out, int64_t j, const Acc& a) {
  if constexpr (std::is_same_v<Acc, PlainAcc>)
    static_cast<float*>(out)[j] = a.s;
  else if constexpr (std::is_same_v<Acc, CompAcc>)
    static_cast<double*>(out)[j] = __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
  else
    static_cast<int64_t*>(out)[j] = (int64_t)a.s;
}

// Fold items get(0), ..., get(m - 1) with one wavefront: lane l folds items
// l, l + 64, ... in order, then the lanes meet in wave_reduce.  Every lane
// must be active; every lane returns the total.  A round has 16 loads per
// lane in flight, all issued unconditionally (past m a lane reads item m - 1
// again and does not fold it): loads on a lane-dependent condition made each
// round wait for its loads one at a time, and a segment spanning 16,000
// tiles took ~60 us to combine.
template <class V, class Op, class Get>
__device__ __forceinline__ V wave_fold_items(Get get, int64_t m, int lane, Op op, V zero) {
  constexpr int kRound = 16;
  V acc = zero;
  for (int64_t base = 0; base < m; base += kRound * 64) {
    V v[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      const int64_t k = base + u * 64 + lane;
      v[u] = get(k < m ? k : m - 1);
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u)
      if (base + u * 64 + lane < m) acc = op(acc, v[u]);
  }
  return wave_reduce(acc, op);
}

// The fp64 value of a compensated pair (s alone when s is not finite).
__device__ __forceinline__ double comp_value(const CompAcc& q) {
  return __builtin_isfinite(q.s) ? (double)q.s + (double)q.c : (double)q.s;
}

// Fold x[s, e) with one wavefront; every lane returns the total.
template <class F, class S, class Acc, int U>
__device__ __forceinline__ Acc wave_fold_range(const F& f, const elem_t<S>* __restrict__ x, int64_t s, int64_t e,
                                               int lane) {
  constexpr bool kInt = std::is_same_v<S, I32>;
  constexpr int KV = S::kVec;
  constexpr int N = U * KV;
  Acc acc[KV];
#pragma unroll
  for (int k = 0; k < KV; ++k) acc[k] = Acc::zero();
  const int64_t es = sizeof(elem_t<S>);
  const int64_t mis = (int64_t)((uintptr_t)(x + s) % 16);
  int64_t head = mis ? (16 - mis) / es : 0;
  if (head > e - s) head = e - s;
  const int64_t b0 = s + head;
  const int64_t nvec = (e - b0) / KV;
  const int64_t t0 = b0 + nvec * KV;
  if (lane < head) fold_elem<F, S>(acc[0], f, x[s + lane], x[s + lane]);
  if (lane < e - t0) fold_elem<F, S>(acc[1 % KV], f, x[t0 + lane], x[t0 + lane]);
  const elem_t<S>* xv = x + b0;
  // Full strides take the unguarded branch (all U loads in flight at once).
  auto step = [&](int64_t v0, auto full_c) {
    constexpr bool kFull = decltype(full_c)::value;
    Vec<S> a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = v0 + u * 64 + lane;
      if (kFull || vi < nvec)
        a[u] = load16<S>(xv + vi * KV);
      else
        a[u] = Vec<S>{};
    }
    elem_t<S> v[N];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < KV; ++k) v[u * KV + k] = a[u].e[k];
    auto ok = [&](int i) { return kFull || v0 + (i / KV) * 64 + lane < nvec; };
    if constexpr (!kInt) {
      float t[N];
#pragma unroll
      for (int i = 0; i < N; ++i) t[i] = S::widen(v[i]);
      eval_batch(f, t);
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (ok(i)) acc[i % KV].add(t[i]);
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (ok(i)) fold_elem<F, S>(acc[i % KV], f, v[i], v[i]);
    }
  };
  int64_t v0 = 0;
  for (; v0 + 64 * U <= nvec; v0 += 64 * U) step(v0, std::true_type{});
  if (v0 < nvec) step(v0, std::false_type{});
  Acc t = acc[0];
#pragma unroll
  for (int k = 1; k < KV; ++k) t = Acc::merge(t, acc[k]);
  return wave_reduce(t, MergeOp<Acc>{});
}

// The persistent pass: every wavefront walks items w, w + W, w + 2W, ...
// (wavefront-uniform indices, so descriptors and offsets are scalar loads).
template <class F, class S, class Acc, int U>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void seg_items_kernel(F f, const elem_t<S>* __restrict__ x,
                                                         const int64_t* __restrict__ off, int64_t S_, SegPlan p,
                                                         void* out) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * wpb + (threadIdx.x >> 6)));
  const int64_t W = (int64_t)gridDim.x * wpb;
  const int64_t cf = p.cnt->full, cp = p.cnt->part;
  if (seg_overflow(p)) {
    // The work lists did not fit the workspace (offsets[S] above the total
    // it was sized for): every segment is folded whole by one wavefront.
    for (int64_t j = w; j < S_; j += W) {
      const Acc r = wave_fold_range<F, S, Acc, U>(f, x, off[j], off[j + 1], lane);
      if (lane == 0) store_result<Acc>(out, j, r);
    }
    return;
  }
  const int64_t nfull = cf < p.cap_full ? cf : p.cap_full;
  const int64_t npart = cp < p.cap_part ? cp : p.cap_part;
  const int64_t npieces = nfull + npart;
  const int64_t ngroups = (S_ + p.spw - 1) / p.spw;
  Acc* partials = static_cast<Acc*>(p.partials);
  auto piece_at = [&](int64_t i) -> SegPiece { return i < nfull ? p.full_list[i] : p.part_list[i - nfull]; };
  auto valid = [&](const SegPiece& pc) { return pc.seg >= 0 && pc.seg < S_; };

  // Pieces, software-pipelined: the descriptor two items ahead and the
  // offsets one item ahead are loaded before the current item streams.
  int64_t i = w;
  SegPiece cur{-1, 0}, nxt{-1, 0};
  int64_t clo = 0, chi = 0;
  if (i < npieces) {
    cur = piece_at(i);
    if (valid(cur)) {
      clo = off[cur.seg];
      chi = off[cur.seg + 1];
    }
  }
  if (i + W < npieces) nxt = piece_at(i + W);
  for (; i < npieces; i += W) {
    int64_t nlo = 0, nhi = 0;
    SegPiece nn{-1, 0};
    if (i + W < npieces && valid(nxt)) {
      nlo = off[nxt.seg];
      nhi = off[nxt.seg + 1];
    }
    if (i + 2 * W < npieces) nn = piece_at(i + 2 * W);
    if (valid(cur)) {
      const int64_t j = cur.seg;
      const int64_t s = clo + (int64_t)cur.k * p.chunk;
      const int64_t e = chi < s + p.chunk ? chi : s + p.chunk;
      const Acc r = wave_fold_range<F, S, Acc, U>(f, x, s, e, lane);
      if (lane == 0) {
        if (chi - clo <= p.chunk) {
          store_result<Acc>(out, j, r);
        } else {
          const int64_t base = p.long_base[j];
          if (base >= 0 && base + cur.k < p.cap_partials) partials[base + cur.k] = r;
        }
      }
    }
    cur = nxt;
    clo = nlo;
    chi = nhi;
    nxt = nn;
  }

  // Small-segment groups: spw consecutive segments, 64/spw lanes each.
  const int64_t g0 = i - npieces;
  for (int64_t g = g0; g < ngroups; g += W) {
    const int lps = 64 / p.spw;
    const int sub = lane / lps, li = lane % lps;
    const int64_t j = g * p.spw + sub;
    Acc a = Acc::zero();
    bool mine = false;
    if (j < S_) {
      const int64_t lo = off[j], hi = off[j + 1];
      mine = hi - lo <= p.small_seg;
      if (mine) {
        constexpr int B = 4;
        for (int64_t e0 = lo + li; e0 < hi; e0 += B * lps) {
          elem_t<S> v[B];
#pragma unroll
          for (int b = 0; b < B; ++b) v[b] = e0 + b * lps < hi ? x[e0 + b * lps] : elem_t<S>{};
          if constexpr (!std::is_same_v<S, I32>) {
            float t[B];
#pragma unroll
            for (int b = 0; b < B; ++b) t[b] = S::widen(v[b]);
            eval_batch(f, t);
#pragma unroll
            for (int b = 0; b < B; ++b)
              if (e0 + b * lps < hi) a.add(t[b]);
          } else {
#pragma unroll
            for (int b = 0; b < B; ++b)
              if (e0 + b * lps < hi) fold_elem<F, S>(a, f, v[b], v[b]);
          }
        }
      }
    }
    // Reduce within each group of lps lanes (fixed butterfly order).
    for (int d = 1; d < lps; d <<= 1) {
      Acc o;
      constexpr int W32 = sizeof(Acc) / 4;
      int wv[W32];
      __builtin_memcpy(wv, &a, sizeof(Acc));
#pragma unroll
      for (int q = 0; q < W32; ++q) wv[q] = __shfl_xor(wv[q], d, 64);
      __builtin_memcpy(&o, wv, sizeof(Acc));
      a = (li & d) ? Acc::merge(o, a) : Acc::merge(a, o);
    }
    if (mine && li == 0) store_result<Acc>(out, j, a);
  }
}

// Fold the partials of every multi-piece segment in piece order.
template <class Acc>
__global__ __launch_bounds__(256) void seg_combine_kernel(const int64_t* __restrict__ off, int64_t S_, SegPlan p,
                                                          void* out) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t W = (int64_t)gridDim.x * wpb;
  if (seg_overflow(p)) return;  // the persistent pass folded every segment whole
  const int64_t cl = p.cnt->longs;
  const int64_t nlong = cl < p.cap_part ? cl : p.cap_part;
  const Acc* partials = static_cast<const Acc*>(p.partials);
  for (int64_t i = w; i < nlong; i += W) {
    const int64_t j = p.long_list[i];
    if (j < 0 || j >= S_) continue;
    const int64_t L = off[j + 1] - off[j];
    const int64_t np = (L + p.chunk - 1) / p.chunk;
    const int64_t base = p.long_base[j];
    const int64_t m = base >= 0 ? (base + np <= p.cap_partials ? np : p.cap_partials - base) : 0;
    if constexpr (std::is_same_v<Acc, CompAcc>) {
      // fp64 final combine of the compensated pairs
      const double d = wave_fold_items<double>([&](int64_t k) { return comp_value(partials[base + k]); }, m, lane,
                                               AddF64{}, 0.0);
      if (lane == 0) static_cast<double*>(out)[j] = d;
    } else {
      const Acc a = wave_fold_items<Acc>([&](int64_t k) { return partials[base + k]; }, m, lane, MergeOp<Acc>{},
                                         Acc::zero());
      if (lane == 0) store_result<Acc>(out, j, a);
    }
  }
}

// ===========================================================================
// Tiled schedule.  The element range [off[0], off[S]) is cut into fixed
// tiles of `tile_vecs` 16-byte vectors, independent of the segments, and
// every wavefront streams whole tiles (w, w + W, ...) exactly as the plain
// reduction streams its share: U vectors per lane per step, all loads of a
// step in flight together.  The segment boundaries inside a tile come from
// the offsets, 64 at a time in one vector register; each step first adds its
// terms to the lanes' fold states, and only when a boundary falls inside the
// step does the wavefront split the step's terms at it, reduce the part that
// ends there (wave_reduce) and store it.  A segment that starts and ends
// inside one tile is written to `out` directly.  Otherwise each tile writes
// its part of that segment to one of two slots (`first`: the segment was open
// when the tile started; `last`: it started in the tile and runs past its
// end), and a second small launch folds, in tile order, the parts of every
// segment that spans tiles (and writes 0 for empty segments).  No plan is
// built, and the work of every wavefront is the same number of vectors.
// The unaligned head of the range belongs to the first tile, its tail to the
// last one.  Everything is a fold of fixed values in a fixed order, so the
// results are reproducible bit for bit.
// ===========================================================================

struct SegTiles {
  void* first;        // per tile: its part of the segment open at its start
  void* last;         // per tile: its part of a segment starting in it and running past its end
  int64_t cap;        // tiles the workspace holds
  int64_t tile_vecs;  // 16-byte vectors per tile
};

// Geometry of the streamed range, from off[0] and off[S] (read on the device).
struct TileGeom {
  int64_t lo;          // off[0]: position 0 of the range
  int64_t n;           // off[S] - off[0]
  int64_t head;        // elements before the first 16-byte boundary
  int64_t nvec;        // whole vectors after the head
  int64_t tail_start;  // first element after the vectors
  int64_t ntiles;
};

template <class S>
__device__ __forceinline__ TileGeom tile_geom(const elem_t<S>* x, const int64_t* off, int64_t S_,
                                              int64_t tile_vecs) {
  TileGeom g{};
  g.lo = off[0];
  const int64_t hi = off[S_];
  g.n = hi > g.lo ? hi - g.lo : 0;
  const int64_t es = sizeof(elem_t<S>);
  const int64_t mis = (int64_t)((uintptr_t)(x + g.lo) % 16);
  int64_t head = mis ? (16 - mis) / es : 0;
  if (head > g.n) head = g.n;
  g.head = head;
  g.nvec = (g.n - head) / S::kVec;
  g.tail_start = head + g.nvec * S::kVec;
  g.ntiles = g.n == 0 ? 0 : (g.nvec + tile_vecs - 1) / tile_vecs;
  if (g.n > 0 && g.ntiles == 0) g.ntiles = 1;
  return g;
}

// The tile holding position p (relative to off[0]).
template <class S>
__host__ __device__ __forceinline__ int64_t tile_of(const TileGeom& g, int64_t tile_vecs, int64_t p) {
  if (p < g.head) return 0;
  const int64_t t = (p - g.head) / (tile_vecs * S::kVec);
  return t < g.ntiles - 1 ? t : g.ntiles - 1;
}

// The terms of one step of the tiled pass.  A Horner polynomial runs its
// degree as a loop bound: each round reads its coefficient from the callable
// by index (one scalar load), so no coefficient occupies a scalar register
// across the kernel and a step costs d rounds of K fmas.  A switch into a
// straight chain at the degree (the small-batch form of eval_batch) was
// compiled into predicated stages that each re-set the K accumulators, ~64
// extra moves per step at degree 8.  The fma sequence is eval_batch's: the
// same bits.
template <class F, int K>
__device__ __forceinline__ void step_terms(const F& f, float (&t)[K]) {
  if constexpr (std::is_same_v<F, Horner>) {
    const int d = f.degree;
    const float top = f.c[d];
    float acc[K];
#pragma unroll
    for (int i = 0; i < K; ++i) acc[i] = top;
#pragma unroll 1
    for (int k = d - 1; k >= 0; --k) {
      const float ck = f.c[k];
#pragma unroll
      for (int i = 0; i < K; ++i) acc[i] = __builtin_fmaf(acc[i], t[i], ck);
    }
#pragma unroll
    for (int i = 0; i < K; ++i) t[i] = acc[i];
  } else {
    eval_batch<F, K, true>(f, t);
  }
}

// Search for the segment holding absolute position p (the last j with
// off[j] <= p), one round at a time so that the rounds can overlap other
// work: a round probes 64 evenly spaced offsets and narrows the range to one
// gap between probes; the final round loads the (at most) 64 offsets of the
// range, which become the boundary batch.  For 100,000 segments: three
// rounds.  The probes are absolute offsets, so the first round needs no
// target yet (begin, then aim) and can go out before off[0] is known.
struct SegFinder {
  int64_t p;
  int32_t a, n;     // off[a] <= p; the answer is in [a, a + n)
  int32_t step;     // spacing of the round in flight (1: the final round)
  int64_t probe;    // this lane's probe of the round in flight; INT64_MAX if none

  __device__ void issue(const int64_t* off, int32_t S, int lane) {
    step = n > 64 ? (n + 63) / 64 : 1;
    const int64_t idx = (int64_t)a + (int64_t)lane * step;
    const bool ok = step == 1 ? idx <= S : idx < (int64_t)a + n;
    probe = ok ? off[idx] : INT64_MAX;
  }
  __device__ void begin(const int64_t* off, int32_t S, int lane) {
    a = 0;
    n = S + 1;
    issue(off, S, lane);
  }
  __device__ void aim(int64_t p_) { p = p_; }
  __device__ void start(const int64_t* off, int32_t S, int64_t p_, int lane) {
    aim(p_);
    begin(off, S, lane);
  }
  __device__ bool final_round() const { return step == 1; }
  // Consume a non-final round and issue the next one.
  __device__ void next(const int64_t* off, int32_t S, int lane) {
    const int cnt = __builtin_popcountll(__builtin_amdgcn_ballot_w64(probe <= p));  // a prefix of the lanes
    const int32_t na = a + (cnt - 1) * step;
    n = a + n - na < step ? a + n - na : step;
    a = na;
    issue(off, S, lane);
  }
};

template <class F, class S, class Acc, int U>
struct TileWave {
  static constexpr int KV = S::kVec;
  static constexpr int K = U * KV;  // elements per lane per step
  static constexpr bool kInt = std::is_same_v<S, I32>;
  using Term = std::conditional_t<kInt, uint64_t, float>;

  const F& f;
  const elem_t<S>* x;  // x + off[0]
  const int64_t* off;
  int64_t lo;          // off[0]
  int32_t S_;
  SegTiles st;
  void* out;
  int lane;
  int32_t tile;
  int64_t base;     // position (relative to off[0]) of the tile's first element
  int32_t len;      // elements of the tile
  // wavefront-uniform state of the current segment; positions are relative to `base`
  int32_t j;        // the segment holding the next position
  int32_t nb;       // its end (off[j + 1] - off[0] - base), clamped to len + 1
  bool started;     // it starts inside this tile
  int32_t bbase;    // offsets[bbase + l] are in lane l of `bnd`
  int64_t bnd;      // a batch of 64 offsets (relative to off[0]); past off[S]: INT64_MAX
  Acc acc;

  __device__ void load_batch(int32_t b) {
    bbase = b;
    const int64_t i = (int64_t)b + lane;
    bnd = i <= S_ ? off[i] - lo : INT64_MAX;
  }
  // off[i] - off[0] - base, clamped to len + 1: from the batch when it
  // holds offset i, else read on its own (a uniform load)
  __device__ int32_t bound(int32_t i) {
    int64_t v;
    if (i - bbase < 64)
      v = read_lane(bnd, i - bbase);
    else
      v = i <= S_ ? off[i] - lo : INT64_MAX;
    v -= base;
    return v <= len ? (int32_t)v : len + 1;
  }
  // Before a step: a batch more than half used is reloaded from the next
  // segment end on, so the boundaries of a step read their offsets from it.
  __device__ void refill() {
    if (j + 1 - bbase >= 32) load_batch(j + 1);
  }

  // The segment holding tile position 0 (the last j with off[j] - off[0] <=
  // base), from a finder started for `base`: its remaining rounds run here.
  __device__ void locate(SegFinder& fd) {
    while (!fd.final_round()) fd.next(off, S_, lane);
    bbase = fd.a;
    bnd = fd.probe == INT64_MAX ? INT64_MAX : fd.probe - lo;
    const int cnt = __builtin_popcountll(__builtin_amdgcn_ballot_w64(lane < fd.n && bnd <= base));
    j = fd.a + cnt - 1;
    started = read_lane(bnd, j - bbase) >= base;
    nb = bound(j + 1);
  }

  // Store the fold of a segment part that ends inside this tile.
  __device__ void finish(const Acc& total) {
    if (lane == 0 && j < S_) {
      if (started)
        store_result<Acc>(out, j, total);
      else
        static_cast<Acc*>(st.first)[tile] = total;
    }
  }
  // Leave segment j at its end nb: the next non-empty segment starts there.
  __device__ void advance() {
    const int32_t b = nb;
    do {
      ++j;
      nb = bound(j + 1);
    } while (nb == b);
    started = true;
  }

  // Add a step's terms.  Term k sits at tile position ps + lp + dk(k), with
  // lp this lane's offset and dk(k) a constant, and exists iff kFull or
  // ok(k); every position of the step lies in [ps, pe).  A bound on the
  // position is a uniform bound on lp, so the step keeps one per-lane value
  // instead of K.
  template <bool kFull, class Dk, class Ok>
  __device__ void step(const Term (&t)[K], int32_t lp, Dk dk, Ok ok, int32_t ps, int32_t pe) {
    if (nb >= pe) {  // no boundary inside the step (uniform)
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (kFull || ok(k)) acc.add(t[k]);
      return;
    }
    int32_t prev = 0;  // terms before ps + prev are already folded
    while (nb < pe) {
      const int32_t end = nb - ps;
#pragma unroll
      for (int k = 0; k < K; ++k)
        acc.add((kFull || ok(k)) && lp >= prev - dk(k) && lp < end - dk(k) ? t[k] : Term{});
      finish(wave_reduce(acc, MergeOp<Acc>{}));
      acc = Acc::zero();
      prev = end;
      advance();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) acc.add((kFull || ok(k)) && lp >= prev - dk(k) ? t[k] : Term{});
  }

  __device__ void terms(const elem_t<S> (&v)[K], Term (&t)[K]) {
    if constexpr (kInt) {
#pragma unroll
      for (int k = 0; k < K; ++k) t[k] = f.term(v[k]);
    } else {
      float w[K];
#pragma unroll
      for (int k = 0; k < K; ++k) w[k] = S::widen(v[k]);
      step_terms<F, K>(f, w);
#pragma unroll
      for (int k = 0; k < K; ++k) t[k] = w[k];
    }
  }

  // A step of single elements: lane l takes tile position p0 + l if below p1.
  __device__ void scalar_step(int32_t p0, int32_t p1) {
    const bool mine = p0 + lane < p1;
    elem_t<S> v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = k == 0 && mine ? x[base + p0 + lane] : elem_t<S>{};
    Term t[K];
    terms(v, t);
    step<false>(t, lane, [](int) { return 0; }, [&](int k) { return k == 0 && mine; }, p0, p1);
  }

  // Tile position 0 of tile t, relative to off[0].
  __device__ static int64_t tile_base(const TileGeom& g, int64_t tile_vecs, int64_t t) {
    return t == 0 ? 0 : g.head + t * tile_vecs * KV;
  }

  // `fd` holds a search started for this tile (have == true) or nothing; on
  // return it holds one started for tile `next` (next >= 0), whose rounds ran
  // between this tile's steps.
  __device__ void run(const TileGeom& g, SegFinder& fd, bool have, int64_t next) {
    const int64_t vb = (int64_t)tile * st.tile_vecs;
    const int64_t ve = vb + st.tile_vecs < g.nvec ? vb + st.tile_vecs : g.nvec;
    const bool first_tile = tile == 0, last_tile = tile == g.ntiles - 1;
    base = first_tile ? 0 : g.head + vb * KV;
    const int64_t end = last_tile ? g.n : g.head + ve * KV;
    len = (int32_t)(end - base);
    const int32_t vpos = (int32_t)(g.head + vb * KV - base);  // tile position of vector vb
    const elem_t<S>* xv = x + g.head + vb * KV;             // vector vb
    const int32_t nvt = (int32_t)(ve - vb);                 // vectors of the tile
    // Two steps of loads in flight: step s + 1's loads go out before step s
    // is folded.
    Vec<S> a[U], nx[U];
    // The loads of a step go through a raw buffer resource (stride 0, word 3
    // 0x00020000: 32-bit data format, no swizzle) based at the step's first
    // vector and ending at the tile's last one.  The hardware checks each
    // lane's byte offset against that range and returns zeros past it, with
    // no memory access (the partial step masks those terms out).  The lane
    // offsets stay fixed; only the base, in scalar registers, moves from step
    // to step, so no vector register is written before a load but the
    // load's own.  Cache policy 2: non-temporal.
    const int32_t lane_off = lane * 16;
    auto issue = [&](Vec<S>(&d)[U], int32_t v0) {
      const int32_t left = v0 < nvt ? (nvt - v0) * 16 : 0;
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc((void*)(xv + (int64_t)v0 * KV), (short)0, left, 0x00020000);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off + u * 1024, 0, 2);
        __builtin_memcpy(&d[u], &w, 16);
      }
    };
    // The first step's loads go out before the search for the segment
    // holding the tile's first element finishes (three dependent rounds of
    // offsets, most of them already run during the previous tile).
    if (nvt > 0) issue(a, 0);
    if (!have) fd.begin(off, S_, lane);
    fd.aim(lo + base);
    locate(fd);
    if (next >= 0) fd.start(off, S_, lo + tile_base(g, st.tile_vecs, next), lane);
    bool searching = next >= 0;
    acc = Acc::zero();

    if (first_tile && g.head > 0) scalar_step(0, (int32_t)g.head);
    // Fold the step at vector v0 from buffer d.
    auto fold = [&](const Vec<S>(&d)[U], int32_t v0) {
      refill();
      elem_t<S> v[K];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < KV; ++e) v[u * KV + e] = d[u].e[e];
      Term t[K];
      terms(v, t);
      // term (u, e) is element e of vector v0 + 64 u + lane: step position
      // lane * KV + (64 u KV + e)
      auto dk = [](int k) { return (k / KV) * 64 * KV + k % KV; };
      const int32_t ps = vpos + v0 * KV;
      if (v0 + 64 * U <= nvt) {
        step<true>(t, lane * KV, dk, [](int) { return true; }, ps, ps + 64 * U * KV);
      } else {
        const int32_t nv = nvt - v0;
        step<false>(t, lane * KV, dk, [&](int k) { return lane < nv - (k / KV) * 64; }, ps, ps + nv * KV);
      }
      if (searching) {  // one round of the next tile's search per step
        if (fd.final_round())
          searching = false;
        else
          fd.next(off, S_, lane);
      }
    };
    // Steps in pairs, the two buffers taking turns, so that no buffer is
    // copied (a copy would wait for the loads in flight).
    // Every pair the loop starts has both steps (an odd last step follows
    // it), so the loads of each buffer are always folded before the buffer
    // is loaded again.  The loads for the step after the pair go out
    // unconditionally (past the tile's end they return zeros and are never
    // folded): a load issued on one path only makes the compiler's wait for
    // the other buffer count it as absent, so the next fold would wait for
    // every load in flight.
    constexpr int32_t kStep = 64 * U;
    int32_t v0 = 0;
    for (; v0 + kStep < nvt; v0 += 2 * kStep) {
      issue(nx, v0 + kStep);
      fold(a, v0);
      issue(a, v0 + 2 * kStep);
      fold(nx, v0 + kStep);
    }
    if (v0 < nvt) fold(a, v0);
    if (last_tile && g.tail_start < g.n) scalar_step((int32_t)(g.tail_start - base), len);

    // The segment open at the tile's end: it ends exactly there, or runs on.
    const Acc total = wave_reduce(acc, MergeOp<Acc>{});
    if (nb == len) {
      finish(total);
    } else if (lane == 0) {
      if (started)
        static_cast<Acc*>(st.last)[tile] = total;
      else
        static_cast<Acc*>(st.first)[tile] = total;
    }
  }
};

template <class F, class S, class Acc, int U>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void seg_tiles_kernel(F f, const elem_t<S>* __restrict__ x,
                                                         const int64_t* __restrict__ off, int64_t S_, SegTiles st,
                                                         void* out) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * wpb + (threadIdx.x >> 6)));
  const int64_t W = (int64_t)gridDim.x * wpb;
  // The first round of the first tile's search goes out with the loads of
  // the tile geometry (it needs no position yet).
  SegFinder fd{};
  fd.begin(off, (int32_t)S_, lane);
  const TileGeom g = tile_geom<S>(x, off, S_, st.tile_vecs);
  if (g.ntiles > st.cap) {
    // More tiles than the workspace holds: every segment is folded whole by one wavefront.
    for (int64_t j = w; j < S_; j += W) {
      const Acc r = wave_fold_range<F, S, Acc, U>(f, x, off[j], off[j + 1], lane);
      if (lane == 0) store_result<Acc>(out, j, r);
    }
    return;
  }
  bool have = true;
  for (int64_t t = w; t < g.ntiles; t += W) {
    TileWave<F, S, Acc, U> tw{f, x + g.lo, off, g.lo, (int32_t)S_, st, out, lane, (int32_t)t};
    const int64_t next = t + W < g.ntiles ? t + W : -1;
    tw.run(g, fd, have, next);
    have = next >= 0;
  }
}

// Segments that span tiles: their parts folded in tile order (the part of
// the tile where the segment starts, then every later tile's `first` part);
// empty segments: 0.  Each lane takes one segment; a segment spanning more
// than kLaneTiles tiles is folded by the whole wavefront (wave_fold_items).
constexpr int64_t kLaneTiles = 16;

template <class S, class Acc>
__global__ __launch_bounds__(256) void seg_tiles_combine_kernel(const elem_t<S>* __restrict__ x,
                                                                const int64_t* __restrict__ off, int64_t S_,
                                                                SegTiles st, void* out) {
  const TileGeom g = tile_geom<S>(x, off, S_, st.tile_vecs);
  if (g.ntiles > st.cap) return;  // the tile pass folded every segment whole
  const Acc* first = static_cast<const Acc*>(st.first);
  const Acc* last = static_cast<const Acc*>(st.last);
  constexpr bool kComp = std::is_same_v<Acc, CompAcc>;
  // part k of a segment whose first tile is ts
  auto part = [&](int64_t ts, int64_t k) { return k == 0 ? last[ts] : first[ts + k]; };
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j0 = wave * 64; j0 < S_; j0 += nwaves * 64) {
    const int64_t j = j0 + lane;
    int64_t ts = 0, te = 0;
    if (j < S_) {
      const int64_t s = off[j] - g.lo, e = off[j + 1] - g.lo;
      if (e <= s) {
        store_result<Acc>(out, j, Acc::zero());
      } else {
        ts = tile_of<S>(g, st.tile_vecs, s);
        te = tile_of<S>(g, st.tile_vecs, e - 1);
      }
    }
    const bool wide = te - ts > kLaneTiles;
    if (te > ts && !wide) {  // a few tiles: this lane folds them in order
      if constexpr (kComp) {
        double d = comp_value(part(ts, 0));
        for (int64_t k = 1; k <= te - ts; ++k) d += comp_value(part(ts, k));
        static_cast<double*>(out)[j] = d;
      } else {
        Acc a = part(ts, 0);
        for (int64_t k = 1; k <= te - ts; ++k) a = Acc::merge(a, part(ts, k));
        store_result<Acc>(out, j, a);
      }
    }
    for (uint64_t mask = __builtin_amdgcn_ballot_w64(wide); mask; mask &= mask - 1) {  // uniform
      const int b = __builtin_ctzll(mask);
      const int64_t bts = read_lane(ts, b), m = read_lane(te, b) - bts + 1;
      if constexpr (kComp) {
        const double d = wave_fold_items<double>([&](int64_t k) { return comp_value(part(bts, k)); }, m, lane,
                                                 AddF64{}, 0.0);
        if (lane == 0) static_cast<double*>(out)[j0 + b] = d;
      } else {
        const Acc a = wave_fold_items<Acc>([&](int64_t k) { return part(bts, k); }, m, lane, MergeOp<Acc>{},
                                           Acc::zero());
        if (lane == 0) store_result<Acc>(out, j0 + b, a);
      }
    }
  }
}

}  // namespace hdc
