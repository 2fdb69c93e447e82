// Host-Device-Compatibility tags, the callables of the library, and the
// storage formats they read and write.
//
// The execution-space tag and its trait follow the paper: a scoped enum with
// the three spaces (section 2.7, listing lst_hst_dev_tags) and a trait that
// reads a static member `hdc` of a type, defaulting to host-only when the
// member is absent (appendix B, listing lst_hdc).  Here the trait is written
// with a C++20 concept instead of the has_xxx detector (appendix B, listing
// lst_has_make_20), and kernels constrain their callable with a `requires`
// clause (section 2.7, listing lst_requires_20): a host-only callable cannot
// instantiate a kernel, which turns every stray call into a compile error
// (the goal stated in section 2.1).
#pragma once

#include <hip/hip_runtime.h>

#include <concepts>
#include <cstdint>
#include <type_traits>

namespace hdc {

enum class HDC { Hst, Dev, HstDev };

template <class T>
concept has_hdc_member = requires {
  { T::hdc } -> std::convertible_to<HDC>;
};

template <class T>
inline constexpr HDC hdc_of = [] {
  if constexpr (has_hdc_member<T>)
    return static_cast<HDC>(T::hdc);
  else
    return HDC::Hst;
}();

// A callable may run inside a kernel iff its tag is Dev or HstDev.
template <class F>
concept device_callable = hdc_of<F> != HDC::Hst;

// A callable may run on the host iff its tag is Hst or HstDev.
template <class F>
concept host_callable = hdc_of<F> != HDC::Dev;

constexpr int kMaxDegree = 16;

// ---------------------------------------------------------------------------
// Floating-point callables: evaluated in fp32 on the exactly widened input.
// Every multiply-add is an explicit single-rounding fma (the library is built
// with contraction off, so nothing else is fused).
// ---------------------------------------------------------------------------

struct Identity {
  static constexpr HDC hdc = HDC::HstDev;
  static constexpr bool binary = false;
  __host__ __device__ float operator()(float x) const { return x; }
};

struct Affine {
  static constexpr HDC hdc = HDC::HstDev;
  static constexpr bool binary = false;
  float a, b;
  __host__ __device__ float operator()(float x) const { return __builtin_fmaf(a, x, b); }
};

// p(x) = sum_k c[k] x^k by Horner's rule, highest coefficient first.
struct Horner {
  static constexpr HDC hdc = HDC::HstDev;
  static constexpr bool binary = false;
  int degree;
  float c[kMaxDegree + 1];
  __host__ __device__ float operator()(float x) const {
    float acc = c[degree];
    for (int k = degree - 1; k >= 0; --k) acc = __builtin_fmaf(acc, x, c[k]);
    return acc;
  }
};

// Dot-product term.  The plain fold uses fma(x, z, s) directly; the
// compensated fold splits x*z exactly into p + e (see hdc_device.hpp).
struct Product {
  static constexpr HDC hdc = HDC::HstDev;
  static constexpr bool binary = true;
  __host__ __device__ float operator()(float x, float z) const { return x * z; }
};

// ---------------------------------------------------------------------------
// Integer callables (int32 storage).  map: result mod 2^32; reduce term:
// int64 value mod 2^64.  Unsigned arithmetic makes the wrap defined.
// ---------------------------------------------------------------------------

struct IntIdentity {
  static constexpr HDC hdc = HDC::HstDev;
  static constexpr bool binary = false;
  __host__ __device__ int32_t map(int32_t x) const { return x; }
  __host__ __device__ uint64_t term(int32_t x) const { return (uint64_t)(int64_t)x; }
};

struct IntAffine {
  static constexpr HDC hdc = HDC::HstDev;
  static constexpr bool binary = false;
  int64_t a, b;
  __host__ __device__ int32_t map(int32_t x) const {
    return (int32_t)((uint32_t)a * (uint32_t)x + (uint32_t)b);
  }
  __host__ __device__ uint64_t term(int32_t x) const {
    return (uint64_t)a * (uint64_t)(int64_t)x + (uint64_t)b;
  }
};

// ---------------------------------------------------------------------------
// Storage formats.  Each has a 16-byte vector of `kVec` elements, an exact
// widening to fp32 and a round-to-nearest-even narrowing from fp32.
// ---------------------------------------------------------------------------

struct F32 {
  using T = float;
  static constexpr int kVec = 4;
  __host__ __device__ static float widen(T v) { return v; }
  __host__ __device__ static T narrow(float v) { return v; }
};

struct F16 {
  using T = _Float16;
  static constexpr int kVec = 8;
  __host__ __device__ static float widen(T v) { return (float)v; }       // exact
  __host__ __device__ static T narrow(float v) { return (_Float16)v; }   // RNE
};

struct BF16 {
  using T = __bf16;
  static constexpr int kVec = 8;
  __host__ __device__ static float widen(T v) { return (float)v; }       // exact
  __host__ __device__ static T narrow(float v) { return (__bf16)v; }     // RNE
};

struct I32 {
  using T = int32_t;
  static constexpr int kVec = 4;
};

template <class S>
concept float_storage = std::is_same_v<S, F32> || std::is_same_v<S, F16> || std::is_same_v<S, BF16>;

}  // namespace hdc
