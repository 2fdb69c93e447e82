// Exact sum of bfloat16 values: the real sum of the inputs, rounded once to
// fp64, whatever the summation order, tuning or grid -- bit-reproducible.
//
// Every finite bf16 value is m * 2^(q - 133) with an integer m < 2^8 and a
// position q in [0, 253] (q = E - 1 for a biased exponent E >= 1, q = 0 for
// subnormals).  Writing q = 32 d + r, the value is (m << r) * 2^(32 d - 133):
// an integer below 2^39 added to digit d (d in [0, 7]) of a fixed-point
// number whose digit j has the unit 2^(32 j - 133).  Each lane keeps its
// digits in int64 registers (carry-save: no carries while folding); a
// wavefront learns which digits its current batch touches from eight ballots
// and updates only those.  Lanes, wavefronts and blocks add digit by digit
// (integer additions: exact and order-free), and the final combine
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

constexpr int kExactDigits = 10;  // units 2^-133 .. 2^155: every sum of < 2^31 bf16 values
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
    int top = -1;  // highest set bit; bit 0 has the value 2^-133
    for (int j = kExactDigits - 1; j >= 0 && top < 0; --j)
      if (g[j]) top = 32 * j + 31 - __builtin_clz(g[j]);
    if (top < 0) return 0.0;
    auto bit = [&](int i) -> uint64_t { return (g[i >> 5] >> (i & 31)) & 1u; };
    double r;
    if (top < 53) {
      r = __builtin_ldexp((double)((uint64_t)g[0] | ((uint64_t)g[1] << 32)), -133);  // exact
    } else {
      const int sh = top - 52;  // keep bits [sh, top]
      uint64_t m = 0;
      for (int i = top; i >= sh; --i) m = (m << 1) | bit(i);
      const uint64_t guard = bit(sh - 1);
      uint64_t sticky = 0;
      for (int i = sh - 2; i >= 0 && !sticky; --i) sticky = bit(i);
      if (guard && (sticky || (m & 1u))) m += 1;  // m <= 2^53: exact as a double
      r = __builtin_ldexp((double)m, sh - 133);
    }
    return neg ? -r : r;
  }
};

// Add the bf16 value with bits u to the lane's digits `acc` (digit `dig` of
// the batch already known) -- the decode.
struct Bf16Term {
  int64_t c;    // signed digit increment
  int dig;      // digit index, -1 for zeros and non-finite values
  uint32_t nf;  // flags of a non-finite value
};

__device__ __forceinline__ Bf16Term bf16_term(uint16_t u) {
  const uint32_t E = (u >> 7) & 0xFFu, M = u & 0x7Fu;
  Bf16Term t{0, -1, 0u};
  if (E == 0xFFu) {
    t.nf = M ? 4u : ((u >> 15) ? 2u : 1u);
    return t;
  }
  const uint32_t m = E ? (M | 0x80u) : M;
  if (m == 0) return t;
  const uint32_t q = E ? E - 1 : 0;
  const int64_t c = (int64_t)m << (q & 31);
  t.c = (u >> 15) ? -c : c;
  t.dig = (int)(q >> 5);
  return t;
}

// Pass 1: every block folds its grid-stride share of 16-byte vectors (8
// values; head and tail elements by the last block) into one state.
template <int U>
__global__ __launch_bounds__(1024) void exact_bf16_kernel(const uint16_t* __restrict__ x, Range r,
                                                          Bf16Exact* partials) {
  __shared__ Bf16Exact lds[kMaxWaves];
  constexpr int V = 8;
  const int64_t B = blockDim.x, tid = threadIdx.x;
  int64_t acc[kExactFoldDigits];
#pragma unroll
  for (int j = 0; j < kExactFoldDigits; ++j) acc[j] = 0;
  uint32_t nf = 0;
  auto fold = [&](const Bf16Term (&tm)[V]) {  // one vector's eight values
    uint32_t mine = 0;  // digits this lane's values touch
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (tm[i].dig >= 0) mine |= 1u << tm[i].dig;
      nf |= tm[i].nf;
    }
#pragma unroll
    for (int j = 0; j < kExactFoldDigits; ++j) {
      if (__builtin_amdgcn_ballot_w64((mine >> j) & 1u) != 0) {  // uniform: some lane touches digit j
#pragma unroll
        for (int i = 0; i < V; ++i) acc[j] += tm[i].dig == j ? tm[i].c : 0;
      }
    }
  };
  const uint16_t* xv = x + r.head;
  const int64_t nchunk = (r.nvec + B * U - 1) / (B * U);
  for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const int64_t base = c * B * U + tid;
    u32x4 a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + u * B;
      a[u] = vi < r.nvec ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(xv + vi * V))
                         : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      Bf16Term tm[V];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t w = a[u][k];
        tm[2 * k] = bf16_term((uint16_t)w);
        tm[2 * k + 1] = bf16_term((uint16_t)(w >> 16));
      }
      fold(tm);
    }
    // Carry digits 0..6 up once per step, so that they stay far below 2^63
    // however many steps a lane takes; digit 7 only takes values >= 2^91.
#pragma unroll
    for (int j = 0; j + 1 < kExactFoldDigits; ++j) {
      const int64_t cy = acc[j] >> 32;
      acc[j] -= cy * (int64_t(1) << 32);
      acc[j + 1] += cy;
    }
  }
  if (blockIdx.x == gridDim.x - 1) {  // unaligned head and the tail, one element per lane
    Bf16Term tm[V];
#pragma unroll
    for (int i = 0; i < V; ++i) tm[i] = Bf16Term{0, -1, 0u};
    if (tid < r.head) tm[0] = bf16_term(x[tid]);
    if (tid < r.tail) tm[1] = bf16_term(x[r.tail_start + tid]);
    fold(tm);
  }
  Bf16Exact s = Bf16Exact::zero();
#pragma unroll
  for (int j = 0; j < kExactFoldDigits; ++j) s.d[j] = acc[j];
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
// Exact dot product of fp16 vectors.  A finite fp16 value is m 2^(q - 24)
// with an integer m < 2^11 and q in [0, 29], so a product is M 2^(Q - 48)
// with M = m_x m_z < 2^22 and Q = q_x + q_z in [0, 58]: the integer
// M << (Q mod 16) < 2^37 added to digit Q / 16 (0..3) of a fixed-point number
// whose digit j has the unit 2^(16 j - 48).  Lanes keep the four digits in
// int64 registers (carry-save) and carry them up once per grid-stride step;
// the total, below 2^63 in magnitude for fewer than 2^31 products, is the
// 128-bit integer sum_j d_j 2^(16 j) in units of 2^-48, rounded once to fp64.
// A product with an infinite or NaN factor is tracked as a flag with its IEEE
// value (inf * 0 is NaN), and their sum as for the bf16 sums.
// ---------------------------------------------------------------------------

constexpr int kDotDigits = 4;

struct F16DotExact {
  int64_t d[kDotDigits];
  uint32_t nf;  // bit 0: +inf, bit 1: -inf, bit 2: NaN
  uint32_t pad;
  __device__ static F16DotExact zero() { return {{0, 0, 0, 0}, 0u, 0u}; }
  __device__ static F16DotExact merge(F16DotExact a, const F16DotExact& b) {
#pragma unroll
    for (int j = 0; j < kDotDigits; ++j) a.d[j] += b.d[j];
    a.nf |= b.nf;
    return a;
  }
  // Digits 0..2 end in [0, 2^16); the top one keeps the sign (floor carries).
  __device__ void normalize() {
#pragma unroll
    for (int j = 0; j + 1 < kDotDigits; ++j) {
      const int64_t c = d[j] >> 16;
      d[j] -= c * (int64_t(1) << 16);
      d[j + 1] += c;
    }
  }
  __device__ double value() const {
    if ((nf & 4u) || (nf & 3u) == 3u) return __builtin_nan("");
    if (nf & 1u) return __builtin_inf();
    if (nf & 2u) return -__builtin_inf();
    F16DotExact t = *this;
    t.normalize();
    // The 128-bit two's-complement integer d0 + d1 2^16 + d2 2^32 + d3 2^48
    // (units of 2^-48), rounded by the fp16 sum's rounding (units of 2^-24)
    // and scaled by 2^-24, which is exact for these magnitudes.
    const uint64_t low = (uint64_t)t.d[0] | ((uint64_t)t.d[1] << 16) | ((uint64_t)t.d[2] << 32);
    ExactAcc e = ExactAcc::zero();
    e.lo = low | ((uint64_t)t.d[3] << 48);
    e.hi = (uint64_t)(t.d[3] >> 16);
    return __builtin_ldexp(e.value(), -24);
  }
};

struct DotTerm {
  int64_t c;    // signed digit increment
  int dig;      // digit, -1 for zero and non-finite products
  uint32_t nf;  // flags of a non-finite product
};

__device__ __forceinline__ DotTerm f16_dot_term(uint32_t a, uint32_t b) {
  const uint32_t Ea = (a >> 10) & 31u, Eb = (b >> 10) & 31u, Fa = a & 1023u, Fb = b & 1023u;
  DotTerm t{0, -1, 0u};
  if (Ea == 31u || Eb == 31u) {
    const bool zero_a = (a & 0x7FFFu) == 0, zero_b = (b & 0x7FFFu) == 0;
    const bool nan = (Ea == 31u && Fa) || (Eb == 31u && Fb) || zero_a || zero_b;
    t.nf = nan ? 4u : (((a ^ b) >> 15) & 1u) ? 2u : 1u;
    return t;
  }
  const uint32_t ma = Ea ? (Fa | 1024u) : Fa, mb = Eb ? (Fb | 1024u) : Fb;
  const uint32_t M = ma * mb;  // < 2^22
  if (M == 0) return t;
  const uint32_t Q = (Ea ? Ea - 1 : 0) + (Eb ? Eb - 1 : 0);
  const int64_t c = (int64_t)M << (Q & 15u);
  t.c = ((a ^ b) >> 15) & 1u ? -c : c;
  t.dig = (int)(Q >> 4);
  return t;
}

// Pass 1: every block folds its grid-stride share.  kVec: x and z share their
// offset from a 16-byte boundary, so the body is 16-byte vectors of 8 values
// (the head and the tail by the last block); otherwise every element alone.
template <int U, bool kVec>
__global__ __launch_bounds__(1024) void exact_f16_dot_kernel(const uint16_t* __restrict__ x,
                                                             const uint16_t* __restrict__ z, Range r,
                                                             F16DotExact* partials) {
  __shared__ F16DotExact lds[kMaxWaves];
  constexpr int V = kVec ? 8 : 1;
  const int64_t B = blockDim.x, tid = threadIdx.x;
  int64_t acc[kDotDigits] = {0, 0, 0, 0};
  uint32_t nf = 0;
  auto fold = [&](const DotTerm (&tm)[V]) {
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (tm[i].dig >= 0) mine |= 1u << tm[i].dig;
      nf |= tm[i].nf;
    }
#pragma unroll
    for (int j = 0; j < kDotDigits; ++j) {
      if (__builtin_amdgcn_ballot_w64((mine >> j) & 1u) != 0) {
#pragma unroll
        for (int i = 0; i < V; ++i) acc[j] += tm[i].dig == j ? tm[i].c : 0;
      }
    }
  };
  auto carry = [&]() {  // keeps every digit far below 2^63 whatever the grid
#pragma unroll
    for (int j = 0; j + 1 < kDotDigits; ++j) {
      const int64_t c = acc[j] >> 16;
      acc[j] -= c * (int64_t(1) << 16);
      acc[j + 1] += c;
    }
  };
  if constexpr (kVec) {
    const uint16_t* xv = x + r.head;
    const uint16_t* zv = z + r.head;
    const int64_t nchunk = (r.nvec + B * U - 1) / (B * U);
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
      const int64_t base = c * B * U + tid;
      u32x4 a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t vi = base + u * B;
        const bool in = vi < r.nvec;
        a[u] = in ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(xv + vi * V)) : u32x4{0u, 0u, 0u, 0u};
        b[u] = in ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(zv + vi * V)) : u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        DotTerm tm[V];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          tm[2 * k] = f16_dot_term(a[u][k] & 0xFFFFu, b[u][k] & 0xFFFFu);
          tm[2 * k + 1] = f16_dot_term(a[u][k] >> 16, b[u][k] >> 16);
        }
        fold(tm);
      }
      carry();
    }
    if (blockIdx.x == gridDim.x - 1) {  // unaligned head and the tail, one element per lane
      DotTerm tm[V];
#pragma unroll
      for (int i = 0; i < V; ++i) tm[i] = DotTerm{0, -1, 0u};
      if (tid < r.head) tm[0] = f16_dot_term(x[tid], z[tid]);
      if (tid < r.tail) tm[1] = f16_dot_term(x[r.tail_start + tid], z[r.tail_start + tid]);
      fold(tm);
    }
  } else {
    for (int64_t c = blockIdx.x; c * B < r.n; c += gridDim.x) {
      const int64_t i = c * B + tid;
      DotTerm tm[1] = {DotTerm{0, -1, 0u}};
      if (i < r.n) tm[0] = f16_dot_term(x[i], z[i]);
      fold(tm);
      carry();
    }
  }
  F16DotExact s = F16DotExact::zero();
#pragma unroll
  for (int j = 0; j < kDotDigits; ++j) s.d[j] = acc[j];
  s.nf = nf;
  s.normalize();
  s = block_reduce(s, MergeOp<F16DotExact>{}, lds);
  if (tid == 0) partials[blockIdx.x] = s;
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
