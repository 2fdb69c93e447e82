// Grouped batch: many independent map + reduce calls of one class (same
// storage type, callables and fold) in one grouped launch and one combine
// launch.  The call table is a by-value kernel argument (no host-to-device
// copy, so the pair of launches can be recorded into a graph as is).
//
// Every call is cut into chunks of `chunk_vecs` 16-byte vectors; the global
// chunk index space is the concatenation of all calls' chunks.  A block takes
// chunks grid-stride, finds the call owning the chunk from the prefix table,
// maps and folds it, and writes one partial per chunk.  The combine launch
// folds each call's partials in chunk order, so results depend only on the
// data and the chunk size: bit-reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"

namespace hdc {

constexpr int kBatchMax = 32;  // calls per grouped launch (keeps the table ~2.3 KB)

struct BatchCall {
  const void* x;
  void* y;  // nullptr: no map for this call
  void* out;
  Range r;  // vector-mode walk of x (x and y share their 16-byte alignment)
};

struct BatchTable {
  int32_t count;
  int64_t chunk_vecs;                 // 16-byte vectors per chunk
  int64_t prefix[kBatchMax + 1];      // first global chunk of each call
  BatchCall call[kBatchMax];
};

template <class FM, class F, class S, class Acc, int U>
  requires device_callable<F> && device_callable<FM>
__global__ __launch_bounds__(1024) void batch_kernel(FM fm, F f, BatchTable t, Acc* partials) {
  __shared__ Acc lds[kMaxWaves];
  const int64_t B = blockDim.x;
  const int64_t tid = threadIdx.x;
  constexpr int KV = S::kVec;
  constexpr int N = U * KV;
  const int64_t total = t.prefix[t.count];
  for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
    int i = 0;
    while (i + 1 < t.count && t.prefix[i + 1] <= c) ++i;  // uniform: the owning call
    const BatchCall& call = t.call[i];
    const elem_t<S>* x = static_cast<const elem_t<S>*>(call.x);
    elem_t<S>* y = static_cast<elem_t<S>*>(call.y);
    const Range& r = call.r;
    const int64_t lc = c - t.prefix[i];
    Acc acc[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k) acc[k] = Acc::zero();
    const elem_t<S>* xv = x + r.head;
    const int64_t vend = (lc + 1) * t.chunk_vecs < r.nvec ? (lc + 1) * t.chunk_vecs : r.nvec;
    // Int32 calls (a quarter-rate multiply per element) load and store
    // through raw buffer resources based at the step and ending at the
    // chunk's last vector (word 3 0x00020000: 32-bit data format, no swizzle;
    // cache policy 2: non-temporal): fixed lane offsets instead of 64-bit
    // address arithmetic per access; past the end, loads return zeros (the
    // mask leaves them out) and stores are dropped.
    constexpr bool kBuf = std::is_same_v<S, I32>;
    auto step = [&](int64_t v0, auto full_c) {
      constexpr bool kFull = decltype(full_c)::value;
      const int64_t base = v0 + tid;
      const int32_t bytes = kBuf ? (int32_t)((vend - v0 < B * U ? vend - v0 : B * U) * 16) : 0;
      Vec<S> a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (kBuf) {
          const __amdgpu_buffer_rsrc_t rx =
              __builtin_amdgcn_make_buffer_rsrc((void*)(xv + v0 * KV), (short)0, bytes, 0x00020000);
          const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rx, (uint32_t)(tid + u * B) * 16u, 0, 2);
          __builtin_memcpy(&a[u], &w, 16);
        } else if (kFull || base + u * B < vend) {
          a[u] = load16<S>(xv + (base + u * B) * KV);
        } else {
          a[u] = Vec<S>{};
        }
      }
      elem_t<S> v[N];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < KV; ++k) v[u * KV + k] = a[u].e[k];
      auto ok = [&](int q) { return kFull || base + (q / KV) * B < vend; };
      if constexpr (!std::is_same_v<S, I32>) {
        float tv[N];
#pragma unroll
        for (int q = 0; q < N; ++q) tv[q] = S::widen(v[q]);
        eval_batch(f, tv);
#pragma unroll
        for (int q = 0; q < N; ++q)
          if (ok(q)) acc[q % KV].add(tv[q]);
      } else {
#pragma unroll
        for (int q = 0; q < N; ++q)
          if (ok(q)) fold_elem<F, S>(acc[q % KV], f, v[q], v[q]);
      }
      if (y) {
        elem_t<S> o[N];
        map_batch<FM, S>(fm, v, o);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if constexpr (kBuf) {
            const __amdgpu_buffer_rsrc_t ry =
                __builtin_amdgcn_make_buffer_rsrc((void*)(y + r.head + v0 * KV), (short)0, bytes, 0x00020000);
            u32x4 w;
            __builtin_memcpy(&w, &o[u * KV], 16);
            __builtin_amdgcn_raw_buffer_store_b128(w, ry, (uint32_t)(tid + u * B) * 16u, 0, 2);
          } else if (kFull || base + u * B < vend) {
            Vec<S> ov;
#pragma unroll
            for (int k = 0; k < KV; ++k) ov.e[k] = o[u * KV + k];
            store16_nt<S>(y + r.head + (base + u * B) * KV, ov);
          }
        }
      }
    };
    int64_t v0 = lc * t.chunk_vecs;
    for (; v0 + B * U <= vend; v0 += B * U) step(v0, std::true_type{});
    if (v0 < vend) step(v0, std::false_type{});
    if (lc == 0) {  // the first chunk also takes the unaligned head and tail
      if (tid < r.head) {
        fold_elem<F, S>(acc[0], f, x[tid], x[tid]);
        if (y) y[tid] = map_elem<FM, S>(fm, x[tid]);
      }
      if (tid < r.tail) {
        const int64_t e = r.tail_start + tid;
        fold_elem<F, S>(acc[1 % KV], f, x[e], x[e]);
        if (y) y[e] = map_elem<FM, S>(fm, x[e]);
      }
    }
    Acc tt = acc[0];
#pragma unroll
    for (int k = 1; k < KV; ++k) tt = Acc::merge(tt, acc[k]);
    tt = block_reduce(tt, MergeOp<Acc>{}, lds);
    if (tid == 0) partials[c] = tt;
  }
}

// One block per call folds that call's chunk partials: thread-strided in
// chunk order, then the fixed block reduction.
template <class Acc>
__global__ __launch_bounds__(256) void batch_combine_kernel(BatchTable t, const Acc* partials) {
  const int c = blockIdx.x;
  const int64_t lo = t.prefix[c], hi = t.prefix[c + 1];
  void* out = t.call[c].out;
  if constexpr (std::is_same_v<Acc, CompAcc>) {
    __shared__ double lds[kMaxWaves];
    double d = 0.0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
      const CompAcc q = partials[k];
      d += __builtin_isfinite(q.s) ? (double)q.s + (double)q.c : (double)q.s;
    }
    d = block_reduce(d, AddF64{}, lds);
    if (threadIdx.x == 0) *static_cast<double*>(out) = d;
  } else {
    __shared__ Acc lds[kMaxWaves];
    Acc a = Acc::zero();
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) a = Acc::merge(a, partials[k]);
    a = block_reduce(a, MergeOp<Acc>{}, lds);
    if (threadIdx.x == 0) {
      if constexpr (std::is_same_v<Acc, PlainAcc>)
        *static_cast<float*>(out) = a.s;
      else
        *static_cast<int64_t*>(out) = (int64_t)a.s;
    }
  }
}

}  // namespace hdc
