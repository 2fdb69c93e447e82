// Exact sum of bfloat16 values: the real sum of the inputs, rounded once to
// fp64, whatever the summation order, tuning or grid -- bit-reproducible.
//
// Every finite bf16 value is m * 2^(E - 134) with an integer m < 2^8 and its
// biased exponent E in [0, 254] (m = 128 + the fraction for E >= 1; for
// subnormals, E = 0, m is twice the fraction).  Writing E = 32 d + r, the
// value is (m << r) * 2^(32 d - 134): an integer below 2^39 added to digit d
// (d in [0, 7]) of a fixed-point number whose digit j has the unit
// 2^(32 j - 134).  Each thread keeps its
// eight digits as fp64 accumulators in LDS (integers below 2^53, so every
// add is exact; no carries while folding) and adds each term to its digit
// by address.  Lanes, wavefronts and blocks then add digit by digit as
// int64 (integer additions: exact and order-free), and the final combine
// propagates the carries into 32-bit digits and rounds the whole number to
// nearest-even fp64 once.  Infinities and NaNs are tracked as flags with the
// IEEE outcome of their sum (NaN if a NaN or both infinities appear).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"

namespace hdc {

constexpr int kExactDigits = 10;  // units 2^-134 .. 2^154: every sum of < 2^31 bf16 values
constexpr int kExactFoldDigits = 8;  // digits that receive terms directly

// Fold state: digits (carry-save) and the non-finite flags
// (bit 0: +inf seen, bit 1: -inf seen, bit 2: NaN seen).
struct Bf16Exact {
  int64_t d[kExactDigits];
  uint32_t nf;
  uint32_t pad;
  __device__ static Bf16Exact zero() {
    Bf16Exact z;
#pragma unroll
    for (int j = 0; j < kExactDigits; ++j) z.d[j] = 0;
    z.nf = 0;
    z.pad = 0;
    return z;
  }
  __device__ static Bf16Exact merge(Bf16Exact a, const Bf16Exact& b) {
#pragma unroll
    for (int j = 0; j < kExactDigits; ++j) a.d[j] += b.d[j];
    a.nf |= b.nf;
    return a;
  }
  // Carries into the next digit: digits 0 .. 8 end in [0, 2^32), the top one
  // keeps the sign (floor division, so negative digits borrow correctly).
  __device__ void normalize() {
#pragma unroll
    for (int j = 0; j + 1 < kExactDigits; ++j) {
      const int64_t c = d[j] >> 32;  // arithmetic shift: floor(d / 2^32)
      d[j] -= c * (int64_t(1) << 32);
      d[j + 1] += c;
    }
  }
  // The exact value rounded once to fp64 (nearest, ties to even).
  __device__ double value() const {
    if ((nf & 4u) || (nf & 3u) == 3u) return __builtin_nan("");
    if (nf & 1u) return __builtin_inf();
    if (nf & 2u) return -__builtin_inf();
    Bf16Exact t = *this;
    t.normalize();
    const bool neg = t.d[kExactDigits - 1] < 0;
    uint32_t g[kExactDigits];  // magnitude, 32-bit digits
    uint64_t borrow = 1;       // two's complement negation: ~digits + 1
#pragma unroll
    for (int j = 0; j < kExactDigits; ++j) {
      const uint32_t v = (uint32_t)t.d[j];
      if (neg) {
        const uint64_t s = (uint64_t)(uint32_t)~v + borrow;
        g[j] = (uint32_t)s;
        borrow = s >> 32;
      } else {
        g[j] = v;
      }
    }
    int top = -1;  // highest set bit; bit 0 has the value 2^-134
    for (int j = kExactDigits - 1; j >= 0 && top < 0; --j)
      if (g[j]) top = 32 * j + 31 - __builtin_clz(g[j]);
    if (top < 0) return 0.0;
    auto bit = [&](int i) -> uint64_t { return (g[i >> 5] >> (i & 31)) & 1u; };
    double r;
    if (top < 53) {
      r = __builtin_ldexp((double)((uint64_t)g[0] | ((uint64_t)g[1] << 32)), -134);  // exact
    } else {
      const int sh = top - 52;  // keep bits [sh, top]
      uint64_t m = 0;
      for (int i = top; i >= sh; --i) m = (m << 1) | bit(i);
      const uint64_t guard = bit(sh - 1);
      uint64_t sticky = 0;
      for (int i = sh - 2; i >= 0 && !sticky; --i) sticky = bit(i);
      if (guard && (sticky || (m & 1u))) m += 1;  // m <= 2^53: exact as a double
      r = __builtin_ldexp((double)m, sh - 134);
    }
    return neg ? -r : r;
  }
};

// Pass 1: every block folds its grid-stride share of 16-byte vectors (8
// values; head and tail elements by the last block) into one state.  The
// decode is branch-free: a value's term m 2^(E mod 32) (an integer below
// 2^39, signed) is formed as an fp64 number (the value widened and scaled
// by 2^(134 - 32 d)), which holds it exactly, and added to the lane's fp64
// accumulator of digit E / 32 -- exact while a lane
// takes fewer than 2^14 terms, which the launch guarantees (at most 1024
// vectors per lane, kExactVecsPerLane).  The accumulators live in LDS, digit
// j of thread i at dig[j * blockDim + i], so a term goes to its own digit by
// address with one fp64 LDS add (no per-digit select over the batch); only
// the thread that owns a slot touches it.  Infinities and NaNs are added to
// a ninth slot that is never read (a select of the address, not of the
// fp64 term); their flags are taken on a separate, rare path.  A term costs
// nine vector instructions and the LDS add; the slot address is one 24-bit
// multiply-add (with a select of the term and a 64-bit address, thirteen:
// 10% slower at 2^28).  (Building the fp64 term from the bf16 bits with
// integer operations instead of the widening and ldexp measured 20% slower.)
constexpr int64_t kExactVecsPerLane = 1024;  // 8192 terms (+2 head/tail) < 2^14
constexpr int kExactMaxBlock = 512;          // 9 slots x 8 bytes x 512 threads = 36 KiB of LDS

template <int U>
__global__ __launch_bounds__(kExactMaxBlock) void exact_bf16_kernel(const uint16_t* __restrict__ x, Range r,
                                                                    Bf16Exact* partials) {
  __shared__ Bf16Exact lds[kMaxWaves];
  extern __shared__ double dig[];  // (kExactFoldDigits + 1) * blockDim
  constexpr int V = 8;
  const int64_t B = blockDim.x, tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j <= kExactFoldDigits; ++j) dig[j * B + tid] = 0.0;
  // LDS byte address of this thread's slot of digit d: own + 8 B d, one
  // 24-bit multiply-add (d is bits 12-14 of the bf16 word, the top three bits
  // of E).  Slot kExactFoldDigits is the sink for infinities and NaNs (never
  // read); a class test of the widened value picks it.
  using lds_f64 = __attribute__((address_space(3))) double;
  const uint32_t own = (uint32_t)(uintptr_t)(lds_f64*)(dig + tid), stride = 8u * (uint32_t)B;
  const uint32_t sink = own + stride * kExactFoldDigits;
  uint32_t nf = 0;
  auto fold = [&](const uint32_t (&u)[V]) {  // u: bf16 bits, 0 for no value
    bool special = false;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const uint32_t d = (u[i] >> 12) & 7u;  // E / 32
      // the value itself (bf16 is the top half of binary32; subnormals are kept),
      // scaled by 2^(134 - 32 d): the signed integer m 2^(E mod 32), exact in fp64
      const float v = __builtin_bit_cast(float, u[i] << 16);
      const bool fin = __builtin_isfinite(v);
      special = special || !fin;
      const double t = __builtin_ldexp((double)v, 134 - 32 * (int)d);
      const uint32_t at = fin ? own + d * stride : sink;
      __hip_atomic_fetch_add((lds_f64*)(uintptr_t)at, t, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (__builtin_amdgcn_ballot_w64(special) != 0) {  // rare: infinities and NaNs present
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (((u[i] >> 7) & 0xFFu) == 0xFFu) nf |= (u[i] & 0x7Fu) ? 4u : ((u[i] >> 15) ? 2u : 1u);
    }
  };
  const uint16_t* xv = x + r.head;
  const int64_t cv = B * U;  // vectors per chunk
  const int64_t nchunk = (r.nvec + cv - 1) / cv;
  // The chunk's loads go through a raw buffer resource based at the chunk
  // and ending at its last vector (word 3 0x00020000: 32-bit data format, no
  // swizzle; cache policy 2: non-temporal): lane offsets stay fixed, and a
  // load past the end returns zeros, which add nothing.
  uint32_t vo[U];
#pragma unroll
  for (int w = 0; w < U; ++w) vo[w] = (uint32_t)(tid + w * B) * 16u;
  for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const int64_t v0 = c * cv;
    const int32_t bytes = (int32_t)((r.nvec - v0 < cv ? r.nvec - v0 : cv) * 16);
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void*)(xv + v0 * V), (short)0, bytes, 0x00020000);
    u32x4 a[U];
#pragma unroll
    for (int w = 0; w < U; ++w) a[w] = __builtin_amdgcn_raw_buffer_load_b128(rx, vo[w], 0, 2);
#pragma unroll
    for (int w = 0; w < U; ++w) {
      uint32_t u[V];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        u[2 * k] = a[w][k] & 0xFFFFu;
        u[2 * k + 1] = a[w][k] >> 16;
      }
      fold(u);
    }
  }
  if (blockIdx.x == gridDim.x - 1) {  // unaligned head and the tail, one element per lane
    uint32_t u[V] = {};
    if (tid < r.head) u[0] = x[tid];
    if (tid < r.tail) u[1] = x[r.tail_start + tid];
    fold(u);
  }
  Bf16Exact s = Bf16Exact::zero();
#pragma unroll
  for (int j = 0; j < kExactFoldDigits; ++j) s.d[j] = (int64_t)dig[j * B + tid];  // integers below 2^53: exact
  s.nf = nf;
  s.normalize();  // digits in [0, 2^32) before the cross-lane sums
  s = block_reduce(s, MergeOp<Bf16Exact>{}, lds);
  if (tid == 0) partials[blockIdx.x] = s;
}

// Pass 2 (one block): digit sums over the partials, then the rounding.
static __global__ __launch_bounds__(256) void exact_bf16_final_kernel(const Bf16Exact* partials, int g, double* out) {
  __shared__ Bf16Exact lds[kMaxWaves];
  Bf16Exact s = Bf16Exact::zero();
  for (int i = threadIdx.x; i < g; i += blockDim.x) s = Bf16Exact::merge(s, partials[i]);
  s = block_reduce(s, MergeOp<Bf16Exact>{}, lds);
  if (threadIdx.x == 0) *out = s.value();
}

// ---------------------------------------------------------------------------
// Exact dot product of fp16 vectors.  The product p of two fp16 values is
// exact in fp32 (at most 22 significant bits, 2^-48 <= |p| < 2^32 unless 0)
// and is an integer multiple of 2^-48.  Split at 2^-8, p = h + l with
// h = trunc(p 2^8) 2^-8 (a multiple of 2^-8 below 2^32) and l = p - h (a
// multiple of 2^-48 below 2^-8); both steps are exact in fp32.  Each part
// spans at most 40 bits, so fp64 chains of up to 2^13 of them never round.
// Lanes flush their two chains once per grid-stride step into a 128-bit
// two's-complement integer in units of 2^-48 (h 2^8 and l 2^48 are integers
// below 2^53); the total, below 2^63 in magnitude for fewer than 2^31
// products, is rounded once to fp64.  A product with an infinite or NaN
// factor (inf * 0 is NaN) goes to the high chain only, and the non-finite
// chain values add by IEEE rules in `nf`.
// ---------------------------------------------------------------------------

struct F16DotExact {
  double dh;  // chain of high parts
  double dl;  // chain of low parts
  float nf;   // IEEE sum of the non-finite chains; 0 if none
  uint32_t pad;
  uint64_t lo, hi;  // 128-bit two's complement, units of 2^-48
  __device__ static F16DotExact zero() { return {0.0, 0.0, 0.0f, 0u, 0u, 0u}; }
  __device__ void add(float p) {
    const float h = __builtin_truncf(p * 256.0f) * 0.00390625f;
    const float l = __builtin_isfinite(p) ? p - h : 0.0f;
    dh += (double)h;
    dl += (double)l;
  }
  __device__ void add128(uint64_t low, uint64_t high) {
    const uint64_t s = lo + low;
    hi += high + (s < lo ? 1u : 0u);
    lo = s;
  }
  __device__ void flush() {
    if (!__builtin_isfinite(dh)) {
      nf += (float)dh;
    } else {
      const int64_t qh = (int64_t)(dh * 256.0);                // |.| < 2^53: exact
      const int64_t ql = (int64_t)(dl * 281474976710656.0);    // 2^48; |.| < 2^53: exact
      add128((uint64_t)ql, (uint64_t)(ql >> 63));
      add128((uint64_t)qh << 40, (uint64_t)(qh >> 24));     // qh 2^40 as 128 bits
    }
    dh = 0.0;
    dl = 0.0;
  }
  __device__ static F16DotExact merge(F16DotExact a, F16DotExact b) {
    a.flush();
    b.flush();
    a.nf += b.nf;
    a.add128(b.lo, b.hi);
    return a;
  }
  // The 128-bit integer rounded by the fp16 sum's rounding (units of 2^-24),
  // then scaled by 2^-24, which is exact for these magnitudes.
  __device__ double value() const {
    F16DotExact t = *this;
    t.flush();
    if (t.nf != 0.0f || t.nf != t.nf) return (double)t.nf;
    ExactAcc e = ExactAcc::zero();
    e.lo = t.lo;
    e.hi = t.hi;
    return __builtin_ldexp(e.value(), -24);
  }
};

__device__ __forceinline__ float f16_bits_to_f32(uint32_t u) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)u);
}

// Pass 1: every block folds its grid-stride share.  kVec: x and z share their
// offset from a 16-byte boundary, so the body is 16-byte vectors of 8 values
// (the head and the tail by the last block); otherwise every element alone.
template <int U, bool kVec>
__global__ __launch_bounds__(1024) void exact_f16_dot_kernel(const uint16_t* __restrict__ x,
                                                             const uint16_t* __restrict__ z, Range r,
                                                             F16DotExact* partials) {
  __shared__ F16DotExact lds[kMaxWaves];
  const int64_t B = blockDim.x, tid = threadIdx.x;
  F16DotExact acc = F16DotExact::zero();
  if constexpr (kVec) {
    constexpr int V = 8;
    const uint16_t* xv = x + r.head;
    const uint16_t* zv = z + r.head;
    const int64_t cv = B * U;  // vectors per chunk
    const int64_t nchunk = (r.nvec + cv - 1) / cv;
    // Loads through raw buffer resources based at the chunk and ending at its
    // last vector, as in exact_bf16_kernel: zeros past the end (a product of
    // zeros adds nothing), fixed lane offsets.
    uint32_t vo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) vo[u] = (uint32_t)(tid + u * B) * 16u;
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
      const int64_t v0 = c * cv;
      const int32_t bytes = (int32_t)((r.nvec - v0 < cv ? r.nvec - v0 : cv) * 16);
      const __amdgpu_buffer_rsrc_t rx =
          __builtin_amdgcn_make_buffer_rsrc((void*)(xv + v0 * V), (short)0, bytes, 0x00020000);
      const __amdgpu_buffer_rsrc_t rz =
          __builtin_amdgcn_make_buffer_rsrc((void*)(zv + v0 * V), (short)0, bytes, 0x00020000);
      u32x4 a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, vo[u], 0, 2);
        b[u] = __builtin_amdgcn_raw_buffer_load_b128(rz, vo[u], 0, 2);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          acc.add(f16_bits_to_f32(a[u][k]) * f16_bits_to_f32(b[u][k]));          // exact in fp32
          acc.add(f16_bits_to_f32(a[u][k] >> 16) * f16_bits_to_f32(b[u][k] >> 16));
        }
      acc.flush();  // chains of at most 8 U terms
    }
    if (blockIdx.x == gridDim.x - 1) {  // unaligned head and the tail, one element per lane
      if (tid < r.head) acc.add(f16_bits_to_f32(x[tid]) * f16_bits_to_f32(z[tid]));
      if (tid < r.tail) acc.add(f16_bits_to_f32(x[r.tail_start + tid]) * f16_bits_to_f32(z[r.tail_start + tid]));
    }
  } else {
    for (int64_t c = blockIdx.x; c * B < r.n; c += gridDim.x) {
      const int64_t i = c * B + tid;
      if (i < r.n) acc.add(f16_bits_to_f32(x[i]) * f16_bits_to_f32(z[i]));
      acc.flush();
    }
  }
  acc.flush();
  acc = block_reduce(acc, MergeOp<F16DotExact>{}, lds);
  if (tid == 0) partials[blockIdx.x] = acc;
}

static __global__ __launch_bounds__(256) void exact_f16_dot_final_kernel(const F16DotExact* partials, int g,
                                                                         double* out) {
  __shared__ F16DotExact lds[kMaxWaves];
  F16DotExact s = F16DotExact::zero();
  for (int i = threadIdx.x; i < g; i += blockDim.x) s = F16DotExact::merge(s, partials[i]);
  s = block_reduce(s, MergeOp<F16DotExact>{}, lds);
  if (threadIdx.x == 0) *out = s.value();
}

}  // namespace hdc
