// gfx950 device primitives: 16-byte vector memory access, error-free
// transformations, fold policies, wavefront (DPP) and workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hdc_functors.hpp"

namespace hdc {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16 bytes of storage S: 4 x fp32/int32 or 8 x fp16/bf16.
template <class S>
struct alignas(16) Vec {
  typename S::T e[S::kVec];
};

// Streaming 16-byte load (`p` must be 16-byte aligned).  Every byte of the
// inputs is read once, so the load is marked non-temporal: on gfx950 that
// keeps streamed lines from displacing cache contents and measured ~7.0 TB/s
// for a pure read against ~6.3 TB/s with the default cache policy.
template <class S>
__device__ __forceinline__ Vec<S> load16(const typename S::T* p) {
  u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  Vec<S> r;
  __builtin_memcpy(&r, &w, 16);
  return r;
}

// Streaming store that bypasses cache retention (written once, not re-read).
template <class S>
__device__ __forceinline__ void store16_nt(typename S::T* p, const Vec<S>& v) {
  u32x4 w;
  __builtin_memcpy(&w, &v, 16);
  __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(p));
}

// ---------------------------------------------------------------------------
// Error-free transformations (Knuth's TwoSum; the fma product split).
// ---------------------------------------------------------------------------

// s = fl(a + b) and e with a + b = s + e exactly (no branch, 6 flops).
__host__ __device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bp = s - a;
  float ap = s - bp;
  e = (a - ap) + (b - bp);
}

// ---------------------------------------------------------------------------
// Fold states.  `add` takes one term, `merge` joins two partial states, both
// in a fixed order wherever they are used, so results are reproducible.
// ---------------------------------------------------------------------------

struct PlainAcc {
  float s;
  __host__ __device__ static PlainAcc zero() { return {0.0f}; }
  __host__ __device__ void add(float t) { s += t; }
  __host__ __device__ void add_product(float x, float z) { s = __builtin_fmaf(x, z, s); }
  __host__ __device__ static PlainAcc merge(PlainAcc a, PlainAcc b) { return {a.s + b.s}; }
};

// Sum in fp32 with the rounding error of every addition captured by TwoSum
// and accumulated separately (compensated / doubled-precision summation).
struct CompAcc {
  float s, c;
  __host__ __device__ static CompAcc zero() { return {0.0f, 0.0f}; }
  __host__ __device__ void add(float t) {
    float e;
    two_sum(s, t, s, e);
    c += e;
  }
  // x*z = p + q exactly (fma computes the rounding error of the product).
  template <bool kExactProduct>
  __host__ __device__ void add_product(float x, float z) {
    float p = x * z;
    add(p);
    if constexpr (!kExactProduct) c += __builtin_fmaf(x, z, -p);
  }
  __host__ __device__ static CompAcc merge(CompAcc a, CompAcc b) {
    CompAcc r;
    float e;
    two_sum(a.s, b.s, r.s, e);
    r.c = (a.c + b.c) + e;
    return r;
  }
};

// int64 sum, wrapping mod 2^64.
struct IntAcc {
  uint64_t s;
  __host__ __device__ static IntAcc zero() { return {0}; }
  __host__ __device__ void add(uint64_t t) { s += t; }
  __host__ __device__ static IntAcc merge(IntAcc a, IntAcc b) { return {a.s + b.s}; }
};

// Exact sum of fp16 values.  Every fp16 value is an integer multiple of 2^-24
// below 2^16 in magnitude, so a chain of at most 2^13 of them summed in fp64
// never rounds (each partial sum is a multiple of 2^-24 below 2^29: 53 bits).
// `d` is such a chain; `normalize` moves it, exactly, into a 128-bit
// two's-complement integer in units of 2^-24 (lo, hi).  Infinities and NaNs
// are kept apart in `nf`, whose IEEE sum is the result whenever it is not 0.
// Callers keep every fp64 chain at most 2^13 terms long.
struct ExactAcc {
  double d;
  float nf;
  uint32_t pad;
  uint64_t lo;
  uint64_t hi;
  __host__ __device__ static ExactAcc zero() { return {0.0, 0.0f, 0u, 0u, 0u}; }
  __host__ __device__ void add(float t) { d += (double)t; }
  __host__ __device__ void normalize() {
    if (!__builtin_isfinite(d)) {
      nf += (float)d;
    } else if (d != 0.0) {
      const int64_t q = (int64_t)(d * 16777216.0);  // exact: an integer below 2^53
      const uint64_t l = lo + (uint64_t)q;
      hi += (uint64_t)(q >> 63) + (l < lo ? 1u : 0u);
      lo = l;
    }
    d = 0.0;
  }
  __host__ __device__ static ExactAcc merge(ExactAcc a, ExactAcc b) {
    a.normalize();
    b.normalize();
    ExactAcc r;
    r.d = 0.0;
    r.nf = a.nf + b.nf;
    r.pad = 0;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
    return r;
  }
  // The exact total rounded once to fp64 (nearest, ties to even).
  __host__ __device__ double value() const {
    ExactAcc t = *this;
    t.normalize();
    if (t.nf != 0.0f || t.nf != t.nf) return (double)t.nf;
    const bool neg = (int64_t)t.hi < 0;
    uint64_t ml = t.lo, mh = t.hi;
    if (neg) {  // magnitude of the two's complement
      ml = ~ml + 1;
      mh = ~mh + (ml == 0 ? 1u : 0u);
    }
    int top = -1;  // index of the highest set bit of the 128-bit magnitude
    if (mh) top = 127 - __builtin_clzll(mh);
    else if (ml) top = 63 - __builtin_clzll(ml);
    if (top < 0) return 0.0;
    double r;
    if (top < 53) {
      r = (double)ml;  // exact
    } else {
      const int sh = top - 52;  // drop the `sh` low bits, keep 53
      auto bit = [&](int i) -> uint64_t { return i >= 64 ? (mh >> (i - 64)) & 1u : (ml >> i) & 1u; };
      uint64_t m = 0;
      for (int i = top; i >= sh; --i) m = (m << 1) | bit(i);
      const uint64_t guard = bit(sh - 1);
      uint64_t sticky = 0;
      for (int i = sh - 2; i >= 0 && !sticky; --i) sticky = bit(i);
      if (guard && (sticky || (m & 1u))) m += 1;
      r = __builtin_ldexp((double)m, sh);  // m <= 2^53: exact
    }
    r = __builtin_ldexp(r, -24);
    return neg ? -r : r;
  }
};

// ---------------------------------------------------------------------------
// Wavefront reduction with DPP lane moves (wave64).
// ---------------------------------------------------------------------------

// Move every 32-bit word of `v` through one DPP lane permutation.
template <int kCtrl, class T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) % 4 == 0, "DPP moves 32-bit words");
  constexpr int W = sizeof(T) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_mov_dpp(w[i], kCtrl, 0xF, 0xF, false);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

template <class T>
__device__ __forceinline__ T read_lane(T v, int lane) {
  constexpr int W = sizeof(T) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_readlane(w[i], lane);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// DPP controls (gfx9 encoding).
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppRowRor4 = 0x124;  // rotate by 4 lanes within a row of 16
constexpr int kDppRowRor8 = 0x128;  // rotate by 8 lanes within a row of 16

// Reduce the 64 lanes of a wavefront; every lane returns the same value.
// Requires every lane of the wavefront to be active.  The dataflow is fixed,
// so the result is reproducible bit for bit.
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  v = op(v, dpp_move<kDppQuadXor1>(v));
  v = op(v, dpp_move<kDppQuadXor2>(v));
  v = op(v, dpp_move<kDppRowRor4>(v));
  v = op(v, dpp_move<kDppRowRor8>(v));  // every lane now holds its row's total
  T r0 = read_lane(v, 0), r1 = read_lane(v, 16), r2 = read_lane(v, 32), r3 = read_lane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}

constexpr int kMaxWaves = 16;  // 1024 threads

// Reduce a workgroup: wavefront totals meet in LDS and are folded in wave
// order.  Every thread returns the block total.  `lds` holds kMaxWaves values.
template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T w = wave_reduce(v, op);
  if (lane == 0) lds[wid] = w;
  __syncthreads();
  T r = lds[0];
  for (int i = 1; i < nw; ++i) r = op(r, lds[i]);
  __syncthreads();
  return r;
}

}  // namespace hdc
