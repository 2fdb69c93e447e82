// Segmented transform_reduce: out[j] = sum over [off[j], off[j+1]) of f(x[i])
// for many uneven segments in one batch, without host synchronisation.
//
// Work decomposition (all on the device):
//   * small segments (length <= small_seg) are packed `spw` per wavefront,
//     64/spw lanes per segment, by fixed segment-index groups;
//   * every other segment is cut into pieces of `chunk` elements; a segment
//     of one piece writes its result directly, a longer one writes one
//     partial per piece, folded afterwards in piece order.
// The plan pass builds two piece lists (full pieces, then the short last
// pieces) with block-aggregated atomics.  The persistent pass walks full
// pieces, short pieces, then small-segment groups, round-robin over its
// wavefronts: equal-cost items first keeps the static split balanced.
// Where an item lands in a list depends on atomic order, but every result
// is computed over a fixed element range in a fixed order, so the output is
// reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"

namespace hdc {

struct SegPiece {
  int32_t seg;
  int32_t k;  // piece index within the segment
};

// Counters at the head of the segmented workspace.
struct SegCounters {
  uint32_t full;      // entries of the full-piece list
  uint32_t part;      // entries of the short-piece list
  uint32_t partials;  // partial slots handed out to multi-piece segments
  uint32_t longs;     // entries of the multi-piece segment list
};

struct SegPlan {
  SegCounters* cnt;
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

static __global__ void seg_reset_kernel(SegCounters* c) {
  if (threadIdx.x == 0) *c = SegCounters{0, 0, 0, 0};
}

// Exclusive prefix sum over a block of the 32-bit values `v`; returns the
// thread's prefix and writes the block total to *total (all threads).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    const uint32_t w = lds[i];
    if (i < wid) before += w;
    all += w;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// One thread per segment.
static __global__ __launch_bounds__(256) void seg_plan_kernel(const int64_t* __restrict__ off, int64_t S, SegPlan p) {
  __shared__ uint32_t lds[kMaxWaves];
  __shared__ uint32_t bases[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t L = 0;
  if (j < S) L = off[j + 1] - off[j];
  const bool big = j < S && L > p.small_seg;
  const int64_t pieces = big ? (L + p.chunk - 1) / p.chunk : 0;
  const int64_t nfull = pieces > 1 ? L / p.chunk : 0;
  const uint32_t want_full = (uint32_t)nfull;
  const uint32_t want_part = big && (pieces == 1 || L % p.chunk != 0) ? 1u : 0u;
  const uint32_t want_slots = pieces > 1 ? (uint32_t)pieces : 0u;
  const uint32_t want_long = pieces > 1 ? 1u : 0u;

  uint32_t tot_full, tot_part, tot_slots, tot_long;
  const uint32_t pre_full = block_exclusive_scan(want_full, lds, &tot_full);
  const uint32_t pre_part = block_exclusive_scan(want_part, lds, &tot_part);
  const uint32_t pre_slots = block_exclusive_scan(want_slots, lds, &tot_slots);
  const uint32_t pre_long = block_exclusive_scan(want_long, lds, &tot_long);
  if (threadIdx.x == 0) {
    bases[0] = tot_full ? atomicAdd(&p.cnt->full, tot_full) : 0;
    bases[1] = tot_part ? atomicAdd(&p.cnt->part, tot_part) : 0;
    bases[2] = tot_slots ? atomicAdd(&p.cnt->partials, tot_slots) : 0;
    bases[3] = tot_long ? atomicAdd(&p.cnt->longs, tot_long) : 0;
  }
  __syncthreads();
  if (!big) return;
  const int64_t slot0 = (int64_t)bases[2] + pre_slots;
  if (pieces > 1) {
    const int64_t li = (int64_t)bases[3] + pre_long;
    p.long_base[j] = slot0 + pieces <= p.cap_partials ? (int32_t)slot0 : -1;
    if (li < p.cap_part) p.long_list[li] = (int32_t)j;
  }
  const int64_t f0 = (int64_t)bases[0] + pre_full;
  for (int64_t k = 0; k < nfull; ++k)
    if (f0 + k < p.cap_full) p.full_list[f0 + k] = SegPiece{(int32_t)j, (int32_t)k};
  if (want_part) {
    const int64_t q = (int64_t)bases[1] + pre_part;
    if (q < p.cap_part) p.part_list[q] = SegPiece{(int32_t)j, (int32_t)nfull};
  }
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
template <class F, class S, class Acc, int U>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void seg_items_kernel(F f, const elem_t<S>* __restrict__ x,
                                                         const int64_t* __restrict__ off, int64_t S_, SegPlan p,
                                                         void* out) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t W = (int64_t)gridDim.x * wpb;
  const int64_t cf = p.cnt->full, cp = p.cnt->part;
  const int64_t nfull = cf < p.cap_full ? cf : p.cap_full;
  const int64_t npart = cp < p.cap_part ? cp : p.cap_part;
  const int64_t ngroups = (S_ + p.spw - 1) / p.spw;
  const int64_t nitems = nfull + npart + ngroups;
  Acc* partials = static_cast<Acc*>(p.partials);

  for (int64_t i = w; i < nitems; i += W) {
    if (i < nfull + npart) {
      const SegPiece pc = i < nfull ? p.full_list[i] : p.part_list[i - nfull];
      const int64_t j = pc.seg;
      if (j < 0 || j >= S_) continue;
      const int64_t lo = off[j], hi = off[j + 1];
      const int64_t s = lo + (int64_t)pc.k * p.chunk;
      const int64_t e = min(hi, s + p.chunk);
      const Acc r = wave_fold_range<F, S, Acc, U>(f, x, s, e, lane);
      if (lane == 0) {
        if (hi - lo <= p.chunk) {
          store_result<Acc>(out, j, r);
        } else {
          const int64_t base = p.long_base[j];
          if (base >= 0 && base + pc.k < p.cap_partials) partials[base + pc.k] = r;
        }
      }
    } else {
      // A group of spw consecutive segments; 64/spw lanes per segment.
      const int64_t g = i - nfull - npart;
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
}

// Fold the partials of every multi-piece segment in piece order.
template <class Acc>
__global__ __launch_bounds__(256) void seg_combine_kernel(const int64_t* __restrict__ off, int64_t S_, SegPlan p,
                                                          void* out) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t W = (int64_t)gridDim.x * wpb;
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
