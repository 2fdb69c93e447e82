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
// prefix within the block.
static __global__ __launch_bounds__(kPlanBlock) void seg_write_kernel(const int64_t* __restrict__ off, int64_t S,
                                                                      SegPlan p) {
  __shared__ SegCounters lds[kMaxWaves];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const SegShape sh = seg_shape(off, S, p, j);
  SegCounters total;
  const SegCounters pre = SegCounters::merge(p.block_tot[blockIdx.x],
                                             block_exclusive_scan_acc(sh.want, lds, &total));
  if (!sh.big) return;
  if (sh.pieces > 1) {
    const int64_t slot0 = pre.partials, li = pre.longs;
    p.long_base[j] = slot0 + sh.pieces <= p.cap_partials ? (int32_t)slot0 : -1;
    if (li < p.cap_part) p.long_list[li] = (int32_t)j;
  }
  const int64_t f0 = pre.full;
  for (int64_t k = 0; k < sh.nfull; ++k)
    if (f0 + k < p.cap_full) p.full_list[f0 + k] = SegPiece{(int32_t)j, (int32_t)k};
  if (sh.want.part && (int64_t)pre.part < p.cap_part) p.part_list[pre.part] = SegPiece{(int32_t)j, (int32_t)sh.nfull};
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
    if constexpr (std::is_same_v<Acc, CompAcc>) {
      // fp64 final combine of the compensated pairs
      double d = 0.0;
      if (base >= 0)
        for (int64_t k = lane; k < np; k += 64)
          if (base + k < p.cap_partials) {
            const CompAcc q = partials[base + k];
            d += __builtin_isfinite(q.s) ? (double)q.s + (double)q.c : (double)q.s;
          }
      d = wave_reduce(d, AddF64{});
      if (lane == 0) static_cast<double*>(out)[j] = d;
    } else {
      Acc a = Acc::zero();
      if (base >= 0)
        for (int64_t k = lane; k < np; k += 64)
          if (base + k < p.cap_partials) a = Acc::merge(a, partials[base + k]);
      a = wave_reduce(a, MergeOp<Acc>{});
      if (lane == 0) store_result<Acc>(out, j, a);
    }
  }
}

}  // namespace hdc
