// Prefix sums of f(x): y[i] = fold of f(x[0..i]) (inclusive) or f(x[0..i-1])
// (exclusive).  Three passes, no inter-block waiting:
//   A: every tile of T = blockDim * kScanE elements is folded to its sum;
//   B: one block scans the tile sums into tile offsets (exclusive);
//   C: every tile is scanned again and its offset added.
// Thread t of a tile owns the kScanE contiguous elements [t E, t E + E): it
// folds them in order, the block combines the per-thread totals with an
// exclusive scan, so pass A and pass C fold each tile identically and the
// result is reproducible bit for bit.
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

// Load the kScanE elements thread t owns in tile `tile` (zero past n).
template <class S, bool kAligned>
__device__ __forceinline__ void scan_load(const elem_t<S>* x, int64_t n, int64_t i0, elem_t<S> (&v)[kScanE]) {
  if (kAligned && i0 + kScanE <= n) {
    constexpr int NV = kScanE / S::kVec;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const Vec<S> a = load16_cached<S>(x + i0 + q * S::kVec);  // a lane reads 64 contiguous bytes
#pragma unroll
      for (int k = 0; k < S::kVec; ++k) v[q * S::kVec + k] = a.e[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanE; ++k) v[k] = i0 + k < n ? x[i0 + k] : elem_t<S>{};
  }
}

// Terms of the owned elements, folded in order into a per-element running
// state; returns the thread total.  With kKeep the running states are kept.
template <class F, class S, class Acc, bool kKeep>
__device__ __forceinline__ Acc scan_thread(const F& f, const elem_t<S> (&v)[kScanE], int64_t i0, int64_t n,
                                           Acc (&run)[kScanE]) {
  Acc a = Acc::zero();
  if constexpr (!std::is_same_v<S, I32>) {
    float t[kScanE];
#pragma unroll
    for (int k = 0; k < kScanE; ++k) t[k] = S::widen(v[k]);
    eval_batch(f, t);
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      if (i0 + k < n) a.add(t[k]);
      if constexpr (kKeep) run[k] = a;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      if (i0 + k < n) fold_elem<F, S>(a, f, v[k], v[k]);
      if constexpr (kKeep) run[k] = a;
    }
  }
  return a;
}

// Pass A: the sum of every tile.
template <class F, class S, class Acc, bool kAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_tile_sums_kernel(F f, const elem_t<S>* x, int64_t n, Acc* sums) {
  __shared__ Acc lds[kMaxWaves];
  const int64_t T = (int64_t)blockDim.x * kScanE;
  const int64_t i0 = (int64_t)blockIdx.x * T + (int64_t)threadIdx.x * kScanE;
  elem_t<S> v[kScanE];
  scan_load<S, kAligned>(x, n, i0, v);
  Acc run[kScanE];
  const Acc mine = scan_thread<F, S, Acc, false>(f, v, i0, n, run);
  Acc total;
  (void)block_exclusive_scan_acc(mine, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass B: exclusive scan of the G tile sums, in rounds of blockDim * kScanE.
template <class Acc>
__global__ __launch_bounds__(1024) void scan_offsets_kernel(const Acc* sums, int64_t G, Acc* offsets) {
  __shared__ Acc lds[kMaxWaves];
  const int64_t R = (int64_t)blockDim.x * kScanE;
  Acc carry = Acc::zero();
  for (int64_t base = 0; base < G; base += R) {
    const int64_t j0 = base + (int64_t)threadIdx.x * kScanE;
    Acc own[kScanE];
    Acc a = Acc::zero();
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      own[k] = a;  // exclusive within the thread
      if (j0 + k < G) a = Acc::merge(a, sums[j0 + k]);
    }
    Acc total;
    const Acc before = block_exclusive_scan_acc(a, lds, &total);
    const Acc start = Acc::merge(carry, before);
#pragma unroll
    for (int k = 0; k < kScanE; ++k)
      if (j0 + k < G) offsets[j0 + k] = Acc::merge(start, own[k]);
    carry = Acc::merge(carry, total);
  }
}

// Pass C: scan every tile and add its offset.  Each thread restarts from its
// offset (tile offset + the totals of the threads before it) and adds its
// terms in order; the outputs go out as 16-byte stores.  The stores of one
// wavefront are 64 or 128 bytes apart, so they use the cache (which merges
// them into whole lines) rather than the non-temporal path.
template <class F, class S, class Acc, bool kAligned, bool kOutAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_tiles_kernel(F f, const elem_t<S>* x, int64_t n, const Acc* offsets,
                                                          typename ScanOut<Acc>::T* y, int exclusive) {
  using OutT = typename ScanOut<Acc>::T;
  __shared__ Acc lds[kMaxWaves];
  const int64_t T = (int64_t)blockDim.x * kScanE;
  const int64_t i0 = (int64_t)blockIdx.x * T + (int64_t)threadIdx.x * kScanE;
  elem_t<S> v[kScanE];
  scan_load<S, kAligned>(x, n, i0, v);
  OutT o[kScanE];
  if constexpr (!std::is_same_v<S, I32>) {
    float t[kScanE];
#pragma unroll
    for (int k = 0; k < kScanE; ++k) t[k] = S::widen(v[k]);
    eval_batch(f, t);  // once: the terms serve the thread total and the outputs
    Acc mine = Acc::zero();
#pragma unroll
    for (int k = 0; k < kScanE; ++k)
      if (i0 + k < n) mine.add(t[k]);
    Acc total;
    const Acc before = block_exclusive_scan_acc(mine, lds, &total);
    Acc a = Acc::merge(offsets[blockIdx.x], before);
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      const OutT prev = ScanOut<Acc>::value(a);
      if (i0 + k < n) a.add(t[k]);
      o[k] = exclusive ? prev : ScanOut<Acc>::value(a);
    }
  } else {
    Acc unused[kScanE];
    const Acc mine = scan_thread<F, S, Acc, false>(f, v, i0, n, unused);
    Acc total;
    const Acc before = block_exclusive_scan_acc(mine, lds, &total);
    Acc a = Acc::merge(offsets[blockIdx.x], before);
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      const OutT prev = ScanOut<Acc>::value(a);
      if (i0 + k < n) fold_elem<F, S>(a, f, v[k], v[k]);
      o[k] = exclusive ? prev : ScanOut<Acc>::value(a);
    }
  }
  if (kOutAligned && i0 + kScanE <= n) {
    constexpr int PER = 16 / sizeof(OutT);
#pragma unroll
    for (int q = 0; q < kScanE / PER; ++q) {
      u32x4 w;
      __builtin_memcpy(&w, &o[q * PER], 16);
      *reinterpret_cast<u32x4*>(y + i0 + q * PER) = w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanE; ++k)
      if (i0 + k < n) y[i0 + k] = o[k];
  }
}

}  // namespace hdc
