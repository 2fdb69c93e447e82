// Kernels of the map / reduce path.  Every kernel takes its callable by value
// and calls it once per element (section 2.4, listing
// lst_solution_ifdef_cudaarch: a kernel template over the callable type);
// each is constrained to device-capable callables (section 2.7, "SFINAE 1*",
// in its C++20 `requires` form), so a host-only callable fails to compile.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"

namespace hdc {

// How an array of n elements is walked.  Vector mode: `head` leading
// elements up to the first 16-byte boundary, `nvec` aligned 16-byte vectors,
// then `tail` trailing elements starting at `tail_start`.  Scalar mode (used
// when two operands disagree in alignment): all n elements one by one.
struct Range {
  int64_t n;
  int64_t head;
  int64_t nvec;
  int64_t tail_start;
  int64_t tail;
};

template <class S>
using elem_t = typename S::T;

// ---------------------------------------------------------------------------
// Element operations
// ---------------------------------------------------------------------------

template <class F, class S>
__host__ __device__ __forceinline__ elem_t<S> map_elem(const F& f, elem_t<S> x) {
  if constexpr (std::is_same_v<S, I32>)
    return f.map(x);
  else if constexpr (std::is_same_v<F, Identity>)
    return x;  // bit copy, NaN payloads included
  else
    return S::narrow(f(S::widen(x)));
}

template <class F, class S, class Acc>
__host__ __device__ __forceinline__ void fold_elem(Acc& a, const F& f, elem_t<S> x, elem_t<S> z) {
  if constexpr (std::is_same_v<S, I32>) {
    a.add(f.term(x));
  } else if constexpr (F::binary) {
    if constexpr (std::is_same_v<Acc, CompAcc>)
      a.template add_product<!std::is_same_v<S, F32>>(S::widen(x), S::widen(z));  // 16-bit products are exact in fp32
    else
      a.add_product(S::widen(x), S::widen(z));
  } else {
    a.add(f(S::widen(x)));
  }
}

// Evaluate a floating-point callable on a batch of widened values in place.
// Horner runs coefficient-outermost so that each coefficient (a uniform
// value) feeds N independent fma chains; each element still sees exactly the
// fma sequence of Horner::operator(), so results are bit-identical to it.
template <class F, int N>
__host__ __device__ __forceinline__ void eval_batch(const F& f, float (&t)[N]) {
  if constexpr (std::is_same_v<F, Horner>) {
    // Every coefficient index is a constant in both forms below, so the
    // coefficients stay in scalar registers instead of being fetched once
    // per step.  Large batches unroll over the largest degree with a uniform
    // guard per step; small batches (where the guards' saved conditions would
    // crowd the scalar registers) enter a straight chain at their degree.
    float acc[N];
    if constexpr (N >= 8) {
      float top = f.c[0];
#pragma unroll
      for (int k = 1; k <= kMaxDegree; ++k) top = k == f.degree ? f.c[k] : top;
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = top;
#pragma unroll
      for (int k = kMaxDegree - 1; k >= 0; --k) {
        if (k < f.degree) {
          const float ck = f.c[k];
#pragma unroll
          for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(acc[i], t[i], ck);
        }
      }
    } else {
      auto start = [&](int d) {
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = f.c[d];
      };
      auto step = [&](int k) {
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = __builtin_fmaf(acc[i], t[i], f.c[k]);
      };
      switch (f.degree) {
        case 16: start(16); goto s15;
        case 15: start(15); goto s14;
        case 14: start(14); goto s13;
        case 13: start(13); goto s12;
        case 12: start(12); goto s11;
        case 11: start(11); goto s10;
        case 10: start(10); goto s9;
        case 9: start(9); goto s8;
        case 8: start(8); goto s7;
        case 7: start(7); goto s6;
        case 6: start(6); goto s5;
        case 5: start(5); goto s4;
        case 4: start(4); goto s3;
        case 3: start(3); goto s2;
        case 2: start(2); goto s1;
        case 1: start(1); goto s0;
        default: start(0); goto done;
      }
    s15: step(15);
    s14: step(14);
    s13: step(13);
    s12: step(12);
    s11: step(11);
    s10: step(10);
    s9: step(9);
    s8: step(8);
    s7: step(7);
    s6: step(6);
    s5: step(5);
    s4: step(4);
    s3: step(3);
    s2: step(2);
    s1: step(1);
    s0: step(0);
    done:;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = acc[i];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = f(t[i]);
  }
}

// Map a batch of storage values: widen, evaluate, narrow (bit copy for
// Identity, integer map for int32 storage).
template <class F, class S, int N>
__host__ __device__ __forceinline__ void map_batch(const F& f, const elem_t<S> (&in)[N], elem_t<S> (&out)[N]) {
  if constexpr (std::is_same_v<S, I32> || std::is_same_v<F, Identity>) {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = map_elem<F, S>(f, in[i]);
  } else {
    float t[N];
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = S::widen(in[i]);
    eval_batch(f, t);
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = S::narrow(t[i]);
  }
}

template <class Acc>
struct MergeOp {
  __device__ Acc operator()(Acc a, Acc b) const { return Acc::merge(a, b); }
};

// ---------------------------------------------------------------------------
// map: y[i] = f(x[i])
// ---------------------------------------------------------------------------

template <class F, class S, int U, bool kVector>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void map_kernel(F f, const elem_t<S>* x, elem_t<S>* y, Range r) {
  const int64_t B = blockDim.x;
  const int64_t tid = threadIdx.x;
  if constexpr (kVector) {
    const elem_t<S>* xv = x + r.head;
    elem_t<S>* yv = y + r.head;
    const int64_t nchunk = (r.nvec + B * U - 1) / (B * U);
    // Full chunks take the unguarded branch, so all U loads of a lane are
    // issued back to back; only the last chunk checks bounds per vector.
    auto step = [&](int64_t base, auto full_c) {
      constexpr bool kFull = decltype(full_c)::value;
      Vec<S> a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kFull || base + u * B < r.nvec)
          a[u] = load16<S>(xv + (base + u * B) * S::kVec);
        else
          a[u] = Vec<S>{};
      }
      elem_t<S> in[U * S::kVec], out[U * S::kVec];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < S::kVec; ++k) in[u * S::kVec + k] = a[u].e[k];
      map_batch<F, S>(f, in, out);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kFull || base + u * B < r.nvec) {
          Vec<S> o;
#pragma unroll
          for (int k = 0; k < S::kVec; ++k) o.e[k] = out[u * S::kVec + k];
          store16_nt<S>(yv + (base + u * B) * S::kVec, o);
        }
      }
    };
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
      const int64_t base = c * B * U + tid;
      if (c * B * U + B * U <= r.nvec)
        step(base, std::true_type{});
      else
        step(base, std::false_type{});
    }
    // Unaligned head and tail: the last block's first threads.
    if (blockIdx.x == gridDim.x - 1) {
      if (tid < r.head) y[tid] = map_elem<F, S>(f, x[tid]);
      if (tid < r.tail) y[r.tail_start + tid] = map_elem<F, S>(f, x[r.tail_start + tid]);
    }
  } else {
    const int64_t stride = (int64_t)gridDim.x * B;
    for (int64_t i = blockIdx.x * B + tid; i < r.n; i += stride * U) {
      elem_t<S> v[U], o[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = (i + u * stride < r.n) ? x[i + u * stride] : elem_t<S>{};
      map_batch<F, S>(f, v, o);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i + u * stride < r.n) y[i + u * stride] = o[u];
    }
  }
}

// ---------------------------------------------------------------------------
// transform_reduce pass 1: every block folds its share into one partial.
// Each lane keeps kVec independent fold states (one per vector component);
// they are merged in component order, then across the wavefront (DPP), then
// across wavefronts (LDS) in wave order.  The block-to-data mapping depends
// only on (n, block, unroll, grid), so the partials are reproducible.
// With kMap, the same pass also writes y[i] = fm(x[i]) (fused map + reduce).
// ---------------------------------------------------------------------------

template <class F, class S, class Acc, int U, bool kVector, class FM = Identity, bool kMap = false>
  requires device_callable<F> && device_callable<FM>
__global__ __launch_bounds__(1024) void reduce_kernel(F f, const elem_t<S>* x, const elem_t<S>* z, Range r,
                                                      Acc* partials, FM fm = FM{}, elem_t<S>* y = nullptr) {
  __shared__ Acc lds[kMaxWaves];
  const int64_t B = blockDim.x;
  const int64_t tid = threadIdx.x;
  constexpr bool kInt = std::is_same_v<S, I32>;
  constexpr bool kBatch = !kInt && !F::binary;  // unary float callables run as one batch
  // Independent fold states per lane.  The exact state is 32 bytes, and
  // eight of them (one per fp16 of a vector) overflow the register file, so
  // it keeps two; each fp64 chain then takes at most kFlush * N / 2 <= 256
  // terms between flushes, far inside the exact state's 2^13.
  constexpr int K = std::is_same_v<Acc, ExactAcc> ? 2 : (kVector ? S::kVec : U);
  constexpr int N = kVector ? U * S::kVec : U;  // elements per lane per step
  // Two-level fold: `acc` takes the terms of at most kFlush steps, then is
  // merged into `outer`.  A plain fp32 chain then never grows longer than
  // kFlush * U terms plus one term per kFlush steps, whatever the grid size,
  // which keeps its rounding error far below the tolerance.
  constexpr int kFlush = 8;
  // A step adds at most ceil(N / K) terms to a chain; the head or tail adds one.
  static_assert(!std::is_same_v<Acc, ExactAcc> || kFlush * ((N + K - 1) / K) + 1 <= (1 << 13),
                "an exact fp64 chain must stay within 2^13 terms between flushes");
  Acc acc[K], outer[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = outer[k] = Acc::zero();
  int since_flush = 0;
  auto maybe_flush = [&]() {
    if (++since_flush == kFlush) {
      since_flush = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        outer[k] = Acc::merge(outer[k], acc[k]);
        acc[k] = Acc::zero();
      }
    }
  };

  // Fold N loaded elements; `ok(i)` tells whether element slot i is real.
  auto fold_step = [&](const elem_t<S>(&v)[N], const elem_t<S>(&w)[N], auto ok) {
    if constexpr (kBatch) {
      float t[N];
#pragma unroll
      for (int i = 0; i < N; ++i) t[i] = S::widen(v[i]);
      eval_batch(f, t);
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (ok(i)) acc[i % K].add(t[i]);
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (ok(i)) fold_elem<F, S>(acc[i % K], f, v[i], w[i]);
    }
  };

  if constexpr (kVector) {
    const elem_t<S>* xv = x + r.head;
    const elem_t<S>* zv = F::binary ? z + r.head : nullptr;
    const int64_t nchunk = (r.nvec + B * U - 1) / (B * U);
    auto step = [&](int64_t base, auto full_c) {
      constexpr bool kFull = decltype(full_c)::value;
      Vec<S> a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kFull || base + u * B < r.nvec) {
          a[u] = load16<S>(xv + (base + u * B) * S::kVec);
          if constexpr (F::binary) b[u] = load16<S>(zv + (base + u * B) * S::kVec);
        } else {
          a[u] = Vec<S>{};
          b[u] = Vec<S>{};
        }
      }
      elem_t<S> v[N], w[N];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int k = 0; k < S::kVec; ++k) {
          v[u * S::kVec + k] = a[u].e[k];
          w[u * S::kVec + k] = F::binary ? b[u].e[k] : a[u].e[k];
        }
      }
      fold_step(v, w, [&](int i) { return kFull || base + (i / S::kVec) * B < r.nvec; });
      if constexpr (kMap) {
        elem_t<S> o[N];
        map_batch<FM, S>(fm, v, o);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (kFull || base + u * B < r.nvec) {
            Vec<S> ov;
#pragma unroll
            for (int k = 0; k < S::kVec; ++k) ov.e[k] = o[u * S::kVec + k];
            store16_nt<S>(y + r.head + (base + u * B) * S::kVec, ov);
          }
        }
      }
    };
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
      const int64_t base = c * B * U + tid;
      if (c * B * U + B * U <= r.nvec)
        step(base, std::true_type{});
      else
        step(base, std::false_type{});
      if constexpr (std::is_same_v<Acc, PlainAcc> || std::is_same_v<Acc, ExactAcc>) maybe_flush();
    }
    if (blockIdx.x == gridDim.x - 1) {
      if (tid < r.head) {
        fold_elem<F, S>(acc[0], f, x[tid], F::binary ? z[tid] : x[tid]);
        if constexpr (kMap) y[tid] = map_elem<FM, S>(fm, x[tid]);
      }
      if (tid < r.tail) {
        const int64_t i = r.tail_start + tid;
        fold_elem<F, S>(acc[1 % K], f, x[i], F::binary ? z[i] : x[i]);
        if constexpr (kMap) y[i] = map_elem<FM, S>(fm, x[i]);
      }
    }
  } else {
    const int64_t stride = (int64_t)gridDim.x * B;
    for (int64_t i = blockIdx.x * B + tid; i < r.n; i += stride * U) {
      elem_t<S> v[N], w[N];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = i + u * stride < r.n;
        v[u] = ok ? x[i + u * stride] : elem_t<S>{};
        if constexpr (F::binary) w[u] = ok ? z[i + u * stride] : elem_t<S>{};
        else w[u] = v[u];
      }
      fold_step(v, w, [&](int u) { return i + u * stride < r.n; });
      if constexpr (std::is_same_v<Acc, PlainAcc> || std::is_same_v<Acc, ExactAcc>) maybe_flush();
      if constexpr (kMap) {
        elem_t<S> o[N];
        map_batch<FM, S>(fm, v, o);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (i + u * stride < r.n) y[i + u * stride] = o[u];
      }
    }
  }

#pragma unroll
  for (int k = 0; k < K; ++k) outer[k] = Acc::merge(outer[k], acc[k]);
  Acc t = outer[0];
#pragma unroll
  for (int k = 1; k < K; ++k) t = Acc::merge(t, outer[k]);
  t = block_reduce(t, MergeOp<Acc>{}, lds);
  if (tid == 0) partials[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// transform_reduce pass 2: one block folds the G partials in index order
// (thread-strided, then the fixed block reduction) and writes the result.
//   PlainAcc -> float (fp32 sum); CompAcc -> double (fp64 sum of s + c, or of
//   s alone when s is not finite: TwoSum of an infinity yields NaN in c);
//   ExactAcc -> double (the exact 128-bit total rounded once);
//   IntAcc -> int64 (wrapping).
// ---------------------------------------------------------------------------

struct AddF32 { __device__ float operator()(float a, float b) const { return a + b; } };
struct AddF64 { __device__ double operator()(double a, double b) const { return a + b; } };
struct AddU64 { __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; } };

template <class Acc>
__global__ __launch_bounds__(256) void reduce_final_kernel(const Acc* partials, int G, void* out) {
  const int tid = threadIdx.x;
  if constexpr (std::is_same_v<Acc, PlainAcc>) {
    __shared__ float lds[kMaxWaves];
    float s = 0.0f;
    for (int i = tid; i < G; i += blockDim.x) s += partials[i].s;
    s = block_reduce(s, AddF32{}, lds);
    if (tid == 0) *static_cast<float*>(out) = s;
  } else if constexpr (std::is_same_v<Acc, CompAcc>) {
    __shared__ double lds[kMaxWaves];
    double s = 0.0;
    for (int i = tid; i < G; i += blockDim.x) {
      const CompAcc p = partials[i];
      s += __builtin_isfinite(p.s) ? (double)p.s + (double)p.c : (double)p.s;
    }
    s = block_reduce(s, AddF64{}, lds);
    if (tid == 0) *static_cast<double*>(out) = s;
  } else if constexpr (std::is_same_v<Acc, ExactAcc>) {
    __shared__ ExactAcc lds[kMaxWaves];
    ExactAcc s = ExactAcc::zero();
    for (int i = tid; i < G; i += blockDim.x) s = ExactAcc::merge(s, partials[i]);
    s = block_reduce(s, MergeOp<ExactAcc>{}, lds);
    if (tid == 0) *static_cast<double*>(out) = s.value();
  } else {
    __shared__ uint64_t lds[kMaxWaves];
    uint64_t s = 0;
    for (int i = tid; i < G; i += blockDim.x) s += partials[i].s;
    s = block_reduce(s, AddU64{}, lds);
    if (tid == 0) *static_cast<int64_t*>(out) = (int64_t)s;
  }
}

}  // namespace hdc
