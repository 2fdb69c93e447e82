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
// kChain selects the straight chain for any batch size (kernels whose other
// scalar state leaves no room for the guards' saved conditions).
template <class F, int N, bool kChain = (N < 8)>
__host__ __device__ __forceinline__ void eval_batch(const F& f, float (&t)[N]) {
  if constexpr (std::is_same_v<F, Horner>) {
    // Every coefficient index is a constant in both forms below, so the
    // coefficients stay in scalar registers instead of being fetched once
    // per step.  Large batches unroll over the largest degree with a uniform
    // guard per step; small batches (where the guards' saved conditions would
    // crowd the scalar registers) enter a straight chain at their degree.
    float acc[N];
    if constexpr (!kChain) {
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
    if constexpr (std::is_same_v<F, IntAffine>) {
      // The int32 affine map spends a quarter-rate 32-bit multiply per
      // element, and the 64-bit address arithmetic of global loads and
      // stores (two instructions per access) then costs it ~2% of its time:
      // its loads and stores go through raw buffer resources based at the
      // chunk and ending at its last vector (accesses past it are dropped),
      // so the lane offsets stay fixed and only the bases move, in scalar
      // registers.  (The other maps measured 1-2% slower this way.)
      const int64_t cv = B * U;  // vectors per chunk
      uint32_t vo[U];
#pragma unroll
      for (int u = 0; u < U; ++u) vo[u] = (uint32_t)(tid + u * B) * 16u;
      for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const int64_t v0 = c * cv;
        const int32_t bytes = (int32_t)((r.nvec - v0 < cv ? r.nvec - v0 : cv) * 16);
        // word 3 0x00020000: 32-bit data format, no swizzle; cache policy 2: non-temporal
        const __amdgpu_buffer_rsrc_t rx =
            __builtin_amdgcn_make_buffer_rsrc((void*)(xv + v0 * S::kVec), (short)0, bytes, 0x00020000);
        const __amdgpu_buffer_rsrc_t ry =
            __builtin_amdgcn_make_buffer_rsrc((void*)(yv + v0 * S::kVec), (short)0, bytes, 0x00020000);
        Vec<S> a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rx, vo[u], 0, 2);
          __builtin_memcpy(&a[u], &w, 16);
        }
        elem_t<S> in[U * S::kVec], out[U * S::kVec];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int k = 0; k < S::kVec; ++k) in[u * S::kVec + k] = a[u].e[k];
        map_batch<F, S>(f, in, out);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          u32x4 w;
          __builtin_memcpy(&w, &out[u * S::kVec], 16);
          __builtin_amdgcn_raw_buffer_store_b128(w, ry, vo[u], 0, 2);
        }
      }
    } else {
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
// Final fold of the per-block partials, in an order that does not depend on
// the block that runs it: 256 virtual threads, virtual thread v folding
// partials v, v + 256, v + 512, ... in index order; each virtual wavefront
// of 64 is reduced by wave_reduce and the four wavefront totals are folded
// in wavefront order.  A 256-thread block runs one virtual wavefront per
// wavefront; a smaller block runs several per wavefront.  The result is
// written to `out`:
//   PlainAcc -> float (fp32 sum); CompAcc -> double (fp64 sum of s + c, or of
//   s alone when s is not finite: TwoSum of an infinity yields NaN in c);
//   ExactAcc -> double (the exact 128-bit total rounded once);
//   IntAcc -> int64 (wrapping).
// ---------------------------------------------------------------------------

struct AddF32 { __device__ float operator()(float a, float b) const { return a + b; } };
struct AddF64 { __device__ double operator()(double a, double b) const { return a + b; } };
struct AddU64 { __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; } };

template <class Acc> struct FinalFold;
template <> struct FinalFold<PlainAcc> {
  using V = float;
  using Op = AddF32;
  __device__ static V term(const PlainAcc& p) { return p.s; }
  __device__ static V invalid() { return __builtin_nanf(""); }
  __device__ static void write(void* out, V v) { *static_cast<float*>(out) = v; }
};
template <> struct FinalFold<CompAcc> {
  using V = double;
  using Op = AddF64;
  __device__ static V invalid() { return __builtin_nan(""); }
  __device__ static V term(const CompAcc& p) {
    return __builtin_isfinite(p.s) ? (double)p.s + (double)p.c : (double)p.s;
  }
  __device__ static void write(void* out, V v) { *static_cast<double*>(out) = v; }
};
template <> struct FinalFold<IntAcc> {
  using V = uint64_t;
  using Op = AddU64;
  __device__ static V term(const IntAcc& p) { return p.s; }
  __device__ static V invalid() { return (uint64_t)INT64_MIN; }
  __device__ static void write(void* out, V v) { *static_cast<int64_t*>(out) = (int64_t)v; }
};
template <> struct FinalFold<ExactAcc> {
  using V = ExactAcc;
  using Op = MergeOp<ExactAcc>;
  __device__ static V term(const ExactAcc& p) { return p; }
  __device__ static V invalid() {
    ExactAcc a = ExactAcc::zero();
    a.nf = __builtin_nanf("");
    return a;
  }
  __device__ static void write(void* out, const V& v) { *static_cast<double*>(out) = v.value(); }
};

constexpr int kFoldThreads = 256;

// Every thread of the block must call this (it synchronises the block);
// `lds` holds kFoldThreads / 64 values; get(i) returns partial i.
template <class Acc, class Get>
__device__ __forceinline__ void fold_partials(Get get, int G, void* out, typename FinalFold<Acc>::V* lds) {
  using FF = FinalFold<Acc>;
  using V = typename FF::V;
  const typename FF::Op op{};
  constexpr int kVW = kFoldThreads / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int vw = wid; vw < kVW; vw += nw) {
    V s{};
    if constexpr (std::is_same_v<Acc, ExactAcc>) s = ExactAcc::zero();
    for (int i = vw * 64 + lane; i < G; i += kFoldThreads) s = op(s, FF::term(get(i)));
    const V w = wave_reduce(s, op);
    if (lane == 0) lds[vw] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    V r = lds[0];
#pragma unroll
    for (int i = 1; i < kVW; ++i) r = op(r, lds[i]);
    FF::write(out, r);
  }
}

// ---------------------------------------------------------------------------
// One-launch fold.  A 64-bit ticket holds (epoch << 32 | arrivals).  Every
// block publishes its partial as sizeof(Acc) / 4 words of 64 bits, each
// (epoch << 32 | one 32-bit word of the fold state), by single-copy-atomic
// stores, then counts itself on the ticket.  The block that arrives last
// reads every word until it carries the launch's epoch (so no fence orders a
// value against a separate flag), folds the partials, and moves the ticket
// to the next epoch with 0 arrivals.  A word keeps its tag until rewritten,
// so a stale word could only pass for a fresh one after 2^32 launches on the
// same workspace.
// ---------------------------------------------------------------------------

template <class Acc>
constexpr int kAccWords = (int)(sizeof(Acc) / 4);

template <class Acc>
__device__ __forceinline__ void publish_partial(uint64_t* slots, int64_t i, const Acc& a, uint32_t epoch) {
  uint32_t w[kAccWords<Acc>];
  __builtin_memcpy(w, &a, sizeof(Acc));
#pragma unroll
  for (int k = 0; k < kAccWords<Acc>; ++k)
    __hip_atomic_store(slots + i * kAccWords<Acc> + k, ((uint64_t)epoch << 32) | w[k], __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
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
                                                      Acc* partials, uint64_t* ticket, void* out, FM fm = FM{},
                                                      elem_t<S>* y = nullptr) {
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
  if (!ticket) {
    if (tid == 0) partials[blockIdx.x] = t;
  } else {
    // One launch: the block that arrives last folds every partial (the
    // workspace holds the tagged words instead of plain partials).
    __shared__ int last;
    __shared__ uint32_t epoch_sh;
    __shared__ typename FinalFold<Acc>::V fold_lds[kFoldThreads / 64];
    uint64_t* slots = reinterpret_cast<uint64_t*>(partials);
    if (tid == 0) {
      const uint32_t epoch = (uint32_t)(__hip_atomic_load(ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32);
      publish_partial(slots, blockIdx.x, t, epoch);
      const uint64_t old = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = (uint32_t)old == gridDim.x - 1;
      epoch_sh = epoch;
    }
    __syncthreads();
    if (last) {
      // Stage every tagged word in LDS (dynamic, gridDim.x * kAccWords words):
      // eight independent loads per thread per round, a word re-read only
      // while it lacks the epoch; then fold from LDS in the fixed order.
      extern __shared__ uint32_t stage[];
      const uint32_t epoch = epoch_sh;
      const int nw = (int)gridDim.x * kAccWords<Acc>;
      bool ok = true;
      for (int base = 0; base < nw; base += 8 * (int)B) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = base + u * (int)B + (int)tid;
          v[u] = k < nw ? __hip_atomic_load(slots + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : (uint64_t)epoch << 32;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = base + u * (int)B + (int)tid;
          for (int polls = 0; (uint32_t)(v[u] >> 32) != epoch; ++polls) {
            if (polls == (1 << 20)) {
              ok = false;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
            v[u] = __hip_atomic_load(slots + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          if (k < nw) stage[k] = (uint32_t)v[u];
        }
      }
      __shared__ int all_ok;
      if (tid == 0) all_ok = 1;
      __syncthreads();
      if (!ok) all_ok = 0;
      __syncthreads();
      fold_partials<Acc>(
          [&](int i) {
            Acc a;
            __builtin_memcpy(&a, stage + (int64_t)i * kAccWords<Acc>, sizeof(Acc));
            return a;
          },
          (int)gridDim.x, out, fold_lds);
      if (tid == 0) {
        if (!all_ok) FinalFold<Acc>::write(out, FinalFold<Acc>::invalid());
        // arrivals back to 0, next epoch
        __hip_atomic_fetch_add(ticket, (1ull << 32) - gridDim.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// transform_reduce pass 2 (the two-launch form): one block of kFoldThreads
// threads folds the G partials (fold_partials) and writes the result.
// ---------------------------------------------------------------------------

template <class Acc>
__global__ __launch_bounds__(kFoldThreads) void reduce_final_kernel(const Acc* partials, int G, void* out) {
  __shared__ typename FinalFold<Acc>::V lds[kFoldThreads / 64];
  fold_partials<Acc>([&](int i) { return partials[i]; }, G, out, lds);
}

}  // namespace hdc
