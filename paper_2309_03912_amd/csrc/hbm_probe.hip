// HBM probe: the bandwidth this GPU actually delivers to plain streaming
// kernels, as the denominator check for the library's roofline fractions.
//
// Read-only and copy kernels over 1 GiB of 16-byte vectors, each with the
// default and the non-temporal cache policy, swept over block size and grid,
// then the copy with every combination of the sc0 / sc1 / nt policy bits on
// its loads and stores at one geometry, store-side variants of the
// non-temporal copy, and the same copy on two data patterns; median of 7
// timed launches (HIP events) per point.  Prints one line per point and a JSON summary line.
// Exit status 0 on success, 1 on a HIP error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                               \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                \
    }                                                                          \
  } while (0)

template <int U, bool kNT>
__global__ __launch_bounds__(1024) void read_kernel(const u32x4* __restrict__ x, int64_t nvec, uint32_t* sink) {
  uint32_t acc = 0;
  const int64_t B = blockDim.x, stride = (int64_t)gridDim.x * B * U;
  for (int64_t base = (int64_t)blockIdx.x * B * U + threadIdx.x; base < nvec; base += stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * B;
      v[u] = i < nvec ? (kNT ? __builtin_nontemporal_load(x + i) : x[i]) : u32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;  // data-dependent store keeps the loads
}

template <int U, bool kNTLoad, bool kNTStore>
__global__ __launch_bounds__(1024) void copy_kernel(const u32x4* __restrict__ x, u32x4* __restrict__ y,
                                                    int64_t nvec) {
  const int64_t B = blockDim.x, stride = (int64_t)gridDim.x * B * U;
  for (int64_t base = (int64_t)blockIdx.x * B * U + threadIdx.x; base < nvec; base += stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * B;
      if (i < nvec) v[u] = kNTLoad ? __builtin_nontemporal_load(x + i) : x[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * B;
      if (i < nvec) {
        if (kNTStore)
          __builtin_nontemporal_store(v[u], y + i);
        else
          y[i] = v[u];
      }
    }
  }
}

// Store-side variants of the non-temporal copy (one launch moves the same
// 1 GiB): kPipe issues the next step's loads before the current step's
// stores (two steps of vectors in flight per lane); kLaneSpan gives every lane
// U consecutive vectors (a store instruction then covers 64 runs of 16 bytes,
// U * 16 bytes apart) instead of the interleaved layout where one
// instruction covers 1 KiB contiguously.
template <int U, bool kPipe, bool kLaneSpan>
__global__ __launch_bounds__(1024) void copy_variant_kernel(const u32x4* __restrict__ x, u32x4* __restrict__ y,
                                                            int64_t nvec) {
  const int64_t B = blockDim.x, stride = (int64_t)gridDim.x * B * U;
  auto idx = [&](int64_t base, int u) -> int64_t {
    if constexpr (kLaneSpan)
      return base - threadIdx.x + (int64_t)threadIdx.x * U + u;  // base is the block's step start + lane
    else
      return base + u * B;
  };
  auto load = [&](int64_t base, u32x4 (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = idx(base, u);
      if (i < nvec) v[u] = __builtin_nontemporal_load(x + i);
    }
  };
  auto store = [&](int64_t base, const u32x4 (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = idx(base, u);
      if (i < nvec) __builtin_nontemporal_store(v[u], y + i);
    }
  };
  int64_t base = (int64_t)blockIdx.x * B * U + threadIdx.x;
  if constexpr (kPipe) {
    u32x4 a[U], b[U];
    if (base < nvec) load(base, a);
    for (; base < nvec; base += 2 * stride) {
      if (base + stride < nvec) load(base + stride, b);
      store(base, a);
      if (base + stride >= nvec) break;
      if (base + 2 * stride < nvec) load(base + 2 * stride, a);
      store(base + stride, b);
    }
  } else {
    for (; base < nvec; base += stride) {
      u32x4 v[U];
      load(base, v);
      store(base, v);
    }
  }
}

// x[i] = pattern(i): 0 the index modulo 2^20 (small values: upper 12 bits of
// every word zero), 1 a 32-bit hash of the index (every bit pattern).
__global__ void fill_kernel(uint32_t* x, int64_t n, int pattern) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t v = (uint32_t)i;
    if (pattern == 0) {
      v &= (1u << 20) - 1;
    } else {
      v *= 0x9E3779B1u;
      v ^= v >> 15;
      v *= 0x85EBCA77u;
      v ^= v >> 13;
    }
    x[i] = v;
  }
}

// Copy through buffer instructions with explicit cache-policy bits (gfx950:
// 1 sc0, 2 nt, 16 sc1) on the loads and on the stores.  1 GiB fits one
// buffer descriptor; out-of-range accesses would read 0 and drop the store.
template <int U, int kLoadPolicy, int kStorePolicy>
__global__ __launch_bounds__(1024) void copy_policy_kernel(const u32x4* x, u32x4* y, int64_t nvec) {
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void*)x, 0, 0x7FFFFFFF, 0x00020000);
  const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc((void*)y, 0, 0x7FFFFFFF, 0x00020000);
  const int64_t B = blockDim.x, stride = (int64_t)gridDim.x * B * U;
  for (int64_t base = (int64_t)blockIdx.x * B * U + threadIdx.x; base < nvec; base += stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * B;
      if (i < nvec)
        v[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rx, (int)(i * 16), 0, kLoadPolicy));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * B;
      if (i < nvec) __builtin_amdgcn_raw_buffer_store_b128(v[u], ry, (int)(i * 16), 0, kStorePolicy);
    }
  }
}

template <class Launch>
static int median_ms(Launch launch, float* out) {
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  launch();
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  std::vector<float> t;
  for (int r = 0; r < 7; ++r) {
    CHECK(hipEventRecord(a));
    launch();
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    t.push_back(ms);
  }
  std::sort(t.begin(), t.end());
  *out = t[t.size() / 2];
  CHECK(hipEventDestroy(a));
  CHECK(hipEventDestroy(b));
  return 0;
}

int main() {
  const int64_t bytes = int64_t(1) << 30, nvec = bytes / 16;
  u32x4 *x = nullptr, *y = nullptr;
  uint32_t* sink = nullptr;
  CHECK(hipMalloc(&x, bytes));
  CHECK(hipMalloc(&y, bytes));
  CHECK(hipMalloc(&sink, 64));
  CHECK(hipMemset(x, 1, bytes));
  CHECK(hipMemset(y, 0, bytes));
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  const double gb = bytes / 1e6;  // GB/ms
  double best[5] = {0, 0, 0, 0, 0};  // read, read-nt, copy, copy-nt-store, copy-nt-both
  for (int block : {256, 512, 1024}) {
    for (int gm : {2, 4, 8, 16, 32}) {
      const unsigned g = (unsigned)(cus * gm);
      float t[5];
      if (median_ms([&] { read_kernel<8, false><<<g, block>>>(x, nvec, sink); }, &t[0])) return 1;
      if (median_ms([&] { read_kernel<8, true><<<g, block>>>(x, nvec, sink); }, &t[1])) return 1;
      if (median_ms([&] { copy_kernel<8, false, false><<<g, block>>>(x, y, nvec); }, &t[2])) return 1;
      if (median_ms([&] { copy_kernel<8, false, true><<<g, block>>>(x, y, nvec); }, &t[3])) return 1;
      if (median_ms([&] { copy_kernel<8, true, true><<<g, block>>>(x, y, nvec); }, &t[4])) return 1;
      const double r[5] = {gb / t[0], gb / t[1], 2 * gb / t[2], 2 * gb / t[3], 2 * gb / t[4]};
      for (int k = 0; k < 5; ++k) best[k] = std::max(best[k], r[k]);
      std::printf("block %4d grid %5u  read %.0f  read-nt %.0f  copy %.0f  copy-nt-store %.0f  copy-nt %.0f GB/s\n",
                  block, g, r[0], r[1], r[2], r[3], r[4]);
      std::fflush(stdout);
    }
  }
  // Cache-policy sweep of the copy at 1024 threads and 32 blocks per CU.
  {
    const unsigned g = (unsigned)(cus * 32);
    float t;
#define HBM_POLICY(L, S)                                                                                    \
  do {                                                                                                      \
    if (median_ms([&] { copy_policy_kernel<8, L, S><<<g, 1024>>>(x, y, nvec); }, &t)) return 1;             \
    std::printf("copy policy load %2d store %2d: %.0f GB/s\n", L, S, 2 * gb / t);                           \
    std::fflush(stdout);                                                                                    \
  } while (0)
    HBM_POLICY(2, 2);
    HBM_POLICY(2, 0);
    HBM_POLICY(2, 1);
    HBM_POLICY(2, 3);
    HBM_POLICY(2, 16);
    HBM_POLICY(2, 17);
    HBM_POLICY(2, 18);
    HBM_POLICY(0, 2);
    HBM_POLICY(3, 2);
    HBM_POLICY(18, 2);
#undef HBM_POLICY
  }
  // Store-side variants of the non-temporal copy at 1024 threads.
  double best_variant = 0;
  for (int gm : {8, 16, 32, 64}) {
    const unsigned g = (unsigned)(cus * gm);
    float t[6];
    if (median_ms([&] { copy_kernel<8, true, true><<<g, 1024>>>(x, y, nvec); }, &t[0])) return 1;
    if (median_ms([&] { copy_variant_kernel<16, false, false><<<g, 1024>>>(x, y, nvec); }, &t[1])) return 1;
    if (median_ms([&] { copy_variant_kernel<4, true, false><<<g, 1024>>>(x, y, nvec); }, &t[2])) return 1;
    if (median_ms([&] { copy_variant_kernel<8, true, false><<<g, 1024>>>(x, y, nvec); }, &t[3])) return 1;
    if (median_ms([&] { copy_variant_kernel<4, false, true><<<g, 1024>>>(x, y, nvec); }, &t[4])) return 1;
    if (median_ms([&] { copy_variant_kernel<8, false, true><<<g, 1024>>>(x, y, nvec); }, &t[5])) return 1;
    for (int k = 1; k < 6; ++k) best_variant = std::max(best_variant, 2 * gb / t[k]);
    std::printf("store variants grid %5u  copy-nt U8 %.0f  U16 %.0f  pipelined U4 %.0f  pipelined U8 %.0f  "
                "lane-span U4 %.0f  lane-span U8 %.0f GB/s\n",
                g, 2 * gb / t[0], 2 * gb / t[1], 2 * gb / t[2], 2 * gb / t[3], 2 * gb / t[4], 2 * gb / t[5]);
    std::fflush(stdout);
  }
  // The same non-temporal copy on two data patterns (the bytes moved are the same).
  double pat[2] = {0, 0};
  for (int pattern : {0, 1}) {
    fill_kernel<<<(unsigned)(cus * 16), 256>>>(reinterpret_cast<uint32_t*>(x), bytes / 4, pattern);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    float t = 0;
    if (median_ms([&] { copy_kernel<8, true, true><<<(unsigned)(cus * 32), 1024>>>(x, y, nvec); }, &t)) return 1;
    pat[pattern] = 2 * gb / t;
    std::printf("copy-nt data %s: %.0f GB/s\n", pattern == 0 ? "i mod 2^20 (small words)" : "hashed (all bits)",
                pat[pattern]);
    std::fflush(stdout);
  }
  float tm = 0;
  if (median_ms([&] { (void)hipMemcpyAsync(y, x, bytes, hipMemcpyDeviceToDevice, 0); }, &tm)) return 1;
  std::printf(
      "{\"cus\": %d, \"best_read_GBps\": %.0f, \"best_read_nt_GBps\": %.0f, \"best_copy_GBps\": %.0f, "
      "\"best_copy_nt_store_GBps\": %.0f, \"best_copy_nt_GBps\": %.0f, \"best_store_variant_GBps\": %.0f, "
      "\"copy_nt_small_words_GBps\": %.0f, \"copy_nt_hashed_words_GBps\": %.0f, \"hipMemcpy_d2d_GBps\": %.0f}\n",
      cus, best[0], best[1], best[2], best[3], best[4], best_variant, pat[0], pat[1], 2 * gb / tm);
  CHECK(hipFree(x));
  CHECK(hipFree(y));
  CHECK(hipFree(sink));
  return 0;
}
