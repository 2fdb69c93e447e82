// Prefix sums of f(x): y[i] = fold of f(x[0..i]) (inclusive) or f(x[0..i-1])
// (exclusive), over tiles of T = blockDim * kScanE elements.
//
// Layout of a tile: wavefront w owns the 64 * kScanE contiguous elements
// starting at w * 64 * kScanE, as Q = kScanE / V chunks of 64 * V elements
// (V = elements per 16-byte vector).  In chunk q, lane l owns the V elements
// at q * 64 V + l V: every load and store of a wavefront covers one
// contiguous 1-KiB span.  The fold order inside a tile is fixed: a lane folds
// its V terms in order, a wavefront scans the lane totals of each chunk and
// chains its chunks, the block scans the wavefront totals in wave order.
//
// Two schedules share that tile step:
//  * three passes, no inter-block waiting -- A: every tile is folded to its
//    sum; B: one block scans the tile sums into tile offsets; C: every tile
//    is scanned again and its offset added (x is read twice);
//  * one pass, tiles handed out in launch order: every tile publishes one
//    node of a binary indexed tree over the tile totals and folds its carry
//    from at most log2(tiles) nodes of earlier tiles (x is read once).
// Both are reproducible bit for bit: pass B always folds in one fixed order,
// and every tree node and carry is a fold in a fixed order of fixed values,
// whichever tile the timing lets finish first.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"

namespace hdc {

constexpr int kScanE = 16;  // elements per thread per tile

template <class T>
__device__ __forceinline__ T shfl_up_words(T v, int d) {
  constexpr int W = sizeof(T) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __shfl_up(w[i], d, 64);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Exclusive scan of fold states over a block (thread order).  Returns the
// thread's exclusive prefix; *total receives the block total (all threads).
// `lds` holds kMaxWaves states.
template <class Acc>
__device__ __forceinline__ Acc block_exclusive_scan_acc(Acc v, Acc* lds, Acc* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  Acc incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Acc t = shfl_up_words(incl, d);
    if (lane >= d) incl = Acc::merge(t, incl);
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  Acc before = Acc::zero(), all = Acc::zero();
  for (int i = 0; i < nw; ++i) {
    const Acc w = lds[i];
    if (i < wid) before = Acc::merge(before, w);
    all = Acc::merge(all, w);
  }
  __syncthreads();
  *total = all;
  // exclusive within the wave: the inclusive value of the previous lane
  Acc ex = shfl_up_words(incl, 1);
  if (lane == 0) ex = Acc::zero();
  return Acc::merge(before, ex);
}

template <class Acc>
struct ScanOut;
template <>
struct ScanOut<PlainAcc> {
  using T = float;
  __device__ static T value(const PlainAcc& a) { return a.s; }
};
template <>
struct ScanOut<CompAcc> {
  using T = double;
  __device__ static T value(const CompAcc& a) {
    return __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
  }
};
template <>
struct ScanOut<IntAcc> {
  using T = int64_t;
  __device__ static T value(const IntAcc& a) { return (int64_t)a.s; }
};

// One wavefront's part of a tile: loading, terms, the fold states of the
// fixed order above, and the outputs.
template <class F, class S, class Acc>
struct ScanWave {
  static constexpr int V = S::kVec;
  static constexpr int Q = kScanE / V;
  using OutT = typename ScanOut<Acc>::T;

  int64_t wbase;  // first element of this wavefront's part
  int lane;
  int64_t n;
  elem_t<S> v[kScanE];             // chunk q, element e at v[q V + e]
  [[maybe_unused]] float t[kScanE];  // the terms (floats)
  Acc ex[Q];                       // exclusive prefix of this lane within chunk q
  Acc wc[Q];                       // fold of chunks 0..q-1 of this wavefront
  Acc wave_total;

  __device__ int64_t index(int q, int e) const { return wbase + (int64_t)q * 64 * V + (int64_t)lane * V + e; }

  template <bool kAligned>
  __device__ void load(const elem_t<S>* x) {
    if (kAligned && wbase + 64 * kScanE <= n) {
      Vec<S> a[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) a[q] = load16<S>(x + index(q, 0));
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) v[q * V + e] = a[q].e[e];
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int64_t i = index(q, e);
          v[q * V + e] = i < n ? x[i] : elem_t<S>{};
        }
    }
  }

  // Terms, lane totals per chunk, the wavefront scans and the chunk chain.
  __device__ void fold(const F& f) {
    Acc tot[Q];
    if constexpr (!std::is_same_v<S, I32>) {
#pragma unroll
      for (int k = 0; k < kScanE; ++k) t[k] = S::widen(v[k]);
      eval_batch(f, t);  // once: the terms serve the totals and the outputs
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        tot[q] = Acc::zero();
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (index(q, e) < n) tot[q].add(t[q * V + e]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        tot[q] = Acc::zero();
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (index(q, e) < n) fold_elem<F, S>(tot[q], f, v[q * V + e], v[q * V + e]);
      }
    }
    Acc run = Acc::zero();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Acc incl = tot[q];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const Acc u = shfl_up_words(incl, d);
        if (lane >= d) incl = Acc::merge(u, incl);
      }
      Acc e = shfl_up_words(incl, 1);
      if (lane == 0) e = Acc::zero();
      ex[q] = e;
      wc[q] = run;
      run = Acc::merge(run, read_lane(incl, 63));
    }
    wave_total = run;
  }

  // Outputs of this lane, starting from the fold of everything before this
  // wavefront's part, stored chunk by chunk.  Chunk q's V outputs of a lane
  // are contiguous: V * sizeof(OutT) bytes as 16-byte stores (non-temporal
  // when a lane's run is exactly 16 bytes, so a wavefront's store covers whole
  // lines; cached otherwise, so the cache merges the interleaved runs of a
  // chunk into whole lines).
  template <bool kOutAligned>
  __device__ void emit(const F& f, const Acc& before, int exclusive, OutT* y) const {
    constexpr int PER = 16 / sizeof(OutT);
    const bool full = kOutAligned && wbase + 64 * kScanE <= n;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Acc a = Acc::merge(Acc::merge(before, wc[q]), ex[q]);
      OutT o[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const OutT prev = ScanOut<Acc>::value(a);
        if (index(q, e) < n) {
          if constexpr (!std::is_same_v<S, I32>)
            a.add(t[q * V + e]);
          else
            fold_elem<F, S>(a, f, v[q * V + e], v[q * V + e]);
        }
        o[e] = exclusive ? prev : ScanOut<Acc>::value(a);
      }
      if (full) {
#pragma unroll
        for (int h = 0; h < V / PER; ++h) {
          u32x4 w;
          __builtin_memcpy(&w, &o[h * PER], 16);
          u32x4* p = reinterpret_cast<u32x4*>(y + index(q, h * PER));
          if constexpr (V == PER)
            __builtin_nontemporal_store(w, p);
          else
            *p = w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (index(q, e) < n) y[index(q, e)] = o[e];
      }
    }
  }
};

// Exclusive fold of the wavefront totals of a block in wave order; *total
// receives the block total.  `lds` holds kMaxWaves states.
template <class Acc>
__device__ __forceinline__ Acc block_wave_prefix(const Acc& wave_total, Acc* lds, Acc* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) lds[wid] = wave_total;
  __syncthreads();
  Acc before = Acc::zero(), all = Acc::zero();
  for (int i = 0; i < nw; ++i) {
    const Acc w = lds[i];
    if (i < wid) before = Acc::merge(before, w);
    all = Acc::merge(all, w);
  }
  __syncthreads();
  *total = all;
  return before;
}

template <class F, class S, class Acc>
__device__ __forceinline__ ScanWave<F, S, Acc> scan_wave_at(int64_t tile, int64_t n) {
  ScanWave<F, S, Acc> w;
  w.lane = threadIdx.x & 63;
  w.wbase = tile * (int64_t)blockDim.x * kScanE + (int64_t)(threadIdx.x >> 6) * 64 * kScanE;
  w.n = n;
  return w;
}

// Pass A: the sum of every tile.
template <class F, class S, class Acc, bool kAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_tile_sums_kernel(F f, const elem_t<S>* x, int64_t n, Acc* sums) {
  __shared__ Acc lds[kMaxWaves];
  auto w = scan_wave_at<F, S, Acc>(blockIdx.x, n);
  w.template load<kAligned>(x);
  w.fold(f);
  Acc total;
  (void)block_wave_prefix(w.wave_total, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass B: exclusive scan of the G tile sums, in rounds of blockDim * kScanE;
// a thread folds kScanE consecutive sums (all loaded first), then the block
// scans the thread totals.
template <class Acc>
__global__ __launch_bounds__(1024) void scan_offsets_kernel(const Acc* sums, int64_t G, Acc* offsets) {
  __shared__ Acc lds[kMaxWaves];
  const int lane = threadIdx.x & 63;
  const int64_t R = (int64_t)blockDim.x * kScanE;
  Acc carry = Acc::zero();
  for (int64_t base = 0; base < G; base += R) {
    const int64_t j0 = base + (int64_t)threadIdx.x * kScanE;
    Acc in[kScanE];
#pragma unroll
    for (int k = 0; k < kScanE; ++k) in[k] = j0 + k < G ? sums[j0 + k] : Acc::zero();
    Acc own[kScanE];
    Acc a = Acc::zero();
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      own[k] = a;  // exclusive within the thread
      a = Acc::merge(a, in[k]);
    }
    Acc incl = a;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const Acc u = shfl_up_words(incl, d);
      if (lane >= d) incl = Acc::merge(u, incl);
    }
    Acc ex = shfl_up_words(incl, 1);
    if (lane == 0) ex = Acc::zero();
    Acc total;
    const Acc before = block_wave_prefix(read_lane(incl, 63), lds, &total);
    const Acc start = Acc::merge(Acc::merge(carry, before), ex);
#pragma unroll
    for (int k = 0; k < kScanE; ++k)
      if (j0 + k < G) offsets[j0 + k] = Acc::merge(start, own[k]);
    carry = Acc::merge(carry, total);
  }
}

// Pass C: scan every tile again and add its offset.
template <class F, class S, class Acc, bool kAligned, bool kOutAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_tiles_kernel(F f, const elem_t<S>* x, int64_t n, const Acc* offsets,
                                                          typename ScanOut<Acc>::T* y, int exclusive) {
  __shared__ Acc lds[kMaxWaves];
  auto w = scan_wave_at<F, S, Acc>(blockIdx.x, n);
  w.template load<kAligned>(x);
  w.fold(f);
  Acc total;
  const Acc before = block_wave_prefix(w.wave_total, lds, &total);
  w.template emit<kOutAligned>(f, Acc::merge(offsets[blockIdx.x], before), exclusive, y);
}

// ---------------------------------------------------------------------------
// Single pass with decoupled look-back
// ---------------------------------------------------------------------------

// The carry between tiles: fp64 for the float folds (so a chain of up to
// 2^31 tile sums adds no error that matters at fp32), the exact int64 for
// integers.  `of` turns a tile total into a carry, `to` a carry into the
// fold state a tile continues from.
template <class Acc>
struct ScanCarry;
template <>
struct ScanCarry<PlainAcc> {
  using T = double;
  __device__ static T of(const PlainAcc& a) { return (double)a.s; }
  __device__ static PlainAcc to(T c) { return {(float)c}; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static uint64_t bits(T c) { return __builtin_bit_cast(uint64_t, c); }
  __device__ static T from(uint64_t b) { return __builtin_bit_cast(double, b); }
};
template <>
struct ScanCarry<CompAcc> {
  using T = double;
  __device__ static T of(const CompAcc& a) {
    return __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
  }
  __device__ static CompAcc to(T c) {
    const float s = (float)c;
    return {s, __builtin_isfinite(s) ? (float)(c - (double)s) : 0.0f};
  }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static uint64_t bits(T c) { return __builtin_bit_cast(uint64_t, c); }
  __device__ static T from(uint64_t b) { return __builtin_bit_cast(double, b); }
};
template <>
struct ScanCarry<IntAcc> {
  using T = uint64_t;
  __device__ static T of(const IntAcc& a) { return a.s; }
  __device__ static IntAcc to(T c) { return {c}; }
  __device__ static T add(T a, T b) { return a + b; }
  __device__ static uint64_t bits(T c) { return c; }
  __device__ static T from(uint64_t b) { return b; }
};

// Look-back state in the workspace: one tree node per tile.  Every 64-bit
// value is published as two 64-bit words, each holding one 32-bit half below
// a ready flag (bit 32), so each word is written and read by one
// single-copy-atomic access and no fence orders a value against a separate
// flag.  All words start at zero (scan_lb_clear_kernel runs first on the
// same stream).
struct ScanLB {
  uint32_t* ticket;  // next tile to hand out
  uint32_t* status;  // nonzero: a wait gave up (the result is invalid)
  uint64_t* node;    // 2 words per tile
};

constexpr uint32_t kLookbackSpinLimit = 1u << 16;  // polls before giving up

static __global__ __launch_bounds__(256) void scan_lb_clear_kernel(uint64_t* w, int64_t nwords) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0;
}

__device__ __forceinline__ void lb_publish(uint64_t* w, uint64_t v) {
  __hip_atomic_store(w, (uint64_t(1) << 32) | (v & 0xffffffffu), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, (uint64_t(1) << 32) | (v >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool lb_read(const uint64_t* w, uint64_t* v) {
  const uint64_t lo = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t hi = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *v = (lo & 0xffffffffu) | (hi << 32);
  return (lo >> 32) != 0 && (hi >> 32) != 0;
}

__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// The carry between tiles as a binary indexed (Fenwick) tree over tile
// positions i = t + 1.  With L = lowbit(i), tile t publishes
//   node[t] = fold of tiles (i - L, i - 1]  =  (children, left to right) + A_t,
// whose children are the nodes of tiles t - 2^m, m = log2 L - 1 .. 0.  Its
// exclusive carry, the fold of tiles 0 .. t - 1, is the left fold of the
// nodes on the query path of i - L (increasing) followed by the children.
// Every term is a node of an earlier tile, at most 31 of them for 2^31
// tiles, so one lane polls each; the folds are short and in a fixed order,
// which makes every carry a fixed function of the tile totals: the result
// does not depend on which tile finished first, and no tile folds more than
// log2 of the tile count values.  Tiles take their index from a ticket in
// launch order, so every node waited on belongs to a resident or finished
// tile and the waits end; the poll count is still bounded, and a give-up
// marks the status word (the carry is then invalid, but the node is still
// published so that no other tile waits for it).
// Run by one whole wavefront; lane 0 publishes node[t].
template <class C>
__device__ typename C::T scan_tree_carry(const ScanLB& lb, int64_t t, typename C::T own) {
  const int lane = threadIdx.x & 63;
  const uint64_t i = (uint64_t)t + 1;
  const uint64_t L = i & (~i + 1);
  const int s = __builtin_ctzll(L);             // children
  const uint64_t base = i - L;                  // query position
  const int r = __builtin_popcountll(base);     // query nodes
  int64_t dep = -1;                             // this lane's node: entry `lane`
  if (lane < r) {
    uint64_t p = base;
    for (int k = 0; k < r - 1 - lane; ++k) p &= p - 1;  // clear the lowest set bits
    dep = (int64_t)p - 1;
  } else if (lane < r + s) {
    dep = t - ((int64_t)1 << (s - 1 - (lane - r)));
  }
  bool ready = dep < 0;
  uint64_t val = 0;
  bool published = false, all = false;
  const bool is_child = lane >= r && lane < r + s;
  for (uint32_t polls = 0;; ++polls) {
    if (!ready) ready = lb_read(lb.node + 2 * dep, &val);
    if (!published && __builtin_amdgcn_ballot_w64(is_child && !ready) == 0) {
      typename C::T x = own;
      if (s > 0) {
        x = C::from(read_lane_u64(val, r));
        for (int e = r + 1; e < r + s; ++e) x = C::add(x, C::from(read_lane_u64(val, e)));
        x = C::add(x, own);
      }
      if (lane == 0) lb_publish(lb.node + 2 * t, C::bits(x));
      published = true;
    }
    all = __builtin_amdgcn_ballot_w64(!ready) == 0;
    if (all || polls >= kLookbackSpinLimit) break;
    __builtin_amdgcn_s_sleep(1);
  }
  if (!all) {  // gave up: keep the others moving, flag the result
    if (lane == 0) {
      if (!published) lb_publish(lb.node + 2 * t, C::bits(own));
      __hip_atomic_store(lb.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return C::from(0);
  }
  typename C::T carry = C::from(0);
  if (r + s > 0) {
    carry = C::from(read_lane_u64(val, 0));
    for (int e = 1; e < r + s; ++e) carry = C::add(carry, C::from(read_lane_u64(val, e)));
  }
  return carry;
}

// One tile per block; the tile index comes from the ticket, not blockIdx.
template <class F, class S, class Acc, bool kAligned, bool kOutAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_onepass_kernel(F f, const elem_t<S>* x, int64_t n, ScanLB lb,
                                                            typename ScanOut<Acc>::T* y, int exclusive) {
  using C = ScanCarry<Acc>;
  __shared__ Acc lds[kMaxWaves];
  __shared__ int64_t tile_sh;
  __shared__ typename C::T carry_sh;
  if (threadIdx.x == 0) tile_sh = (int64_t)atomicAdd(lb.ticket, 1u);
  __syncthreads();
  const int64_t tile = tile_sh;
  auto w = scan_wave_at<F, S, Acc>(tile, n);
  w.template load<kAligned>(x);
  w.fold(f);
  Acc total;
  const Acc before = block_wave_prefix(w.wave_total, lds, &total);
  if (threadIdx.x < 64) {
    const typename C::T carry = scan_tree_carry<C>(lb, tile, C::of(total));
    if (threadIdx.x == 0) carry_sh = carry;
  }
  __syncthreads();
  w.template emit<kOutAligned>(f, Acc::merge(C::to(carry_sh), before), exclusive, y);
}

}  // namespace hdc
