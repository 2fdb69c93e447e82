// Host-side helpers shared by the translation units of the library: error
// reporting, tuning records, launch geometry, the functor-id -> type and
// dtype -> storage dispatch, and the per-family launchers (each family is
// compiled in its own translation unit so the build runs in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>

#include "hdc.h"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"
#include "hdc_segmented.hpp"

namespace hdc {

// Record a failure for hdc_last_error() and return `s`.
hdc_status fail(hdc_status s, const char* fmt, ...);
// Compute units of the current device (cached per device).
hdc_status compute_units(int* cus);

inline hdc_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return HDC_OK;
}

struct Tuning {
  int block = 256;
  int unroll = 4;
  int grid_mult = 8;
  int chunk = 4096;
  int small_seg = 128;
  int seg_per_wave = 8;
  // reductions: 1 = one launch (the last block folds), 2 = two launches;
  // segmented reduce: 1 = tiled schedule, 2 = planned schedule
  int passes = 2;
};


#define HDC_TRY(expr)                 \
  do {                                \
    hdc_status s_ = (expr);           \
    if (s_ != HDC_OK) return s_;      \
  } while (0)


constexpr int64_t kMaxGrid = 65536;  // upper bound on pass-1 blocks
constexpr size_t kPartialBytes = 32;  // every fold state fits 32 bytes

constexpr size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline size_t reduce_workspace_bytes() { return round_up(kMaxGrid * kPartialBytes, 256); }

constexpr int64_t kMinChunk = 1024;

// Layout of the segmented workspace for a given chunk (sections 256-byte aligned).
struct SegLayout {
  size_t cnt, block_tot, full, part, long_base, long_list, partials, bytes;
  int64_t cap_full, cap_part, cap_partials, plan_blocks;
};

// Partial slots of a grouped batch: at most total/chunk + count chunks.
constexpr size_t batch_workspace_bytes(int64_t total, int64_t count) {
  return round_up((size_t)(total / kMinChunk + count + 1) * kPartialBytes, 256);
}

// The sections for a full-piece capacity of `cap_full` entries.
constexpr SegLayout seg_layout_cap(int64_t cap_full, int64_t S) {
  SegLayout l{};
  l.cap_full = cap_full;
  l.cap_part = S > 0 ? S : 1;
  l.cap_partials = l.cap_full + l.cap_part;
  l.plan_blocks = (S + kPlanBlock - 1) / kPlanBlock;
  size_t o = 0;
  l.cnt = o;       o += round_up(sizeof(SegCounters), 256);
  l.block_tot = o; o += round_up((size_t)(l.plan_blocks + 1) * sizeof(SegCounters), 256);
  l.full = o;      o += round_up((size_t)l.cap_full * sizeof(SegPiece), 256);
  l.part = o;      o += round_up((size_t)l.cap_part * sizeof(SegPiece), 256);
  l.long_base = o; o += round_up((size_t)l.cap_part * sizeof(int32_t), 256);
  l.long_list = o; o += round_up((size_t)l.cap_part * sizeof(int32_t), 256);
  l.partials = o;  o += round_up((size_t)l.cap_partials * kPartialBytes, 256);
  l.bytes = o;
  return l;
}

// The layout for segments holding at most `total` elements, cut into pieces
// of `chunk`: at most total / chunk full pieces plus one.
constexpr SegLayout seg_layout(int64_t total, int64_t S, int64_t chunk) {
  return seg_layout_cap(total / chunk + 1, S);
}

// The largest full-piece capacity a workspace of `bytes` holds for S
// segments, or 0 when it cannot hold the layout of capacity 1.  A workspace
// of seg_layout(total, S, kMinChunk).bytes holds capacity total / chunk + 1
// for every chunk >= kMinChunk.
constexpr int64_t seg_capacity(size_t bytes, int64_t S) {
  const size_t fixed = seg_layout_cap(1, S).bytes;
  if (bytes < fixed) return 0;
  // 8 bytes of list entry + 32 of partial slot per entry; the two rounded
  // sections differ from that by less than 1024 bytes, so this starts above
  // the answer and steps down to it.
  int64_t c = 1 + (int64_t)((bytes - fixed + 1024) / (sizeof(SegPiece) + kPartialBytes));
  while (c > 1 && seg_layout_cap(c, S).bytes > bytes) --c;
  return c;
}

// Workspace of the tiled schedule for segments holding at most `total`
// elements: two arrays of one 32-byte slot per tile, tiles of at least
// kMinChunk elements (the head joins the first tile, the tail the last).
constexpr size_t seg_tiles_bytes(int64_t total) {
  return 2 * round_up((size_t)(total / kMinChunk + 2) * kPartialBytes, 256);
}

// Workspace of a segmented reduce for either schedule.
constexpr size_t seg_workspace_bytes(int64_t total, int64_t S) {
  const size_t a = seg_layout(total, S, kMinChunk).bytes, b = seg_tiles_bytes(total);
  return a > b ? a : b;
}

// The largest segment total that `bytes` serves at every chunk length (what
// the size bucket of a segmented call is taken from).
constexpr int64_t seg_total_bound(size_t bytes, int64_t S) {
  const int64_t c = seg_capacity(bytes, S);
  return c > 0 ? c * kMinChunk - 1 : 0;
}


template <class Body>
hdc_status with_float_fn(const hdc_functor& f, Body&& body) {
  switch (f.id) {
    case HDC_FN_IDENTITY: return body(Identity{});
    case HDC_FN_AFFINE: return body(Affine{f.a, f.b});
    case HDC_FN_HORNER: {
      Horner h{};
      h.degree = f.degree;
      for (int k = 0; k <= f.degree; ++k) h.c[k] = f.coef[k];
      return body(h);
    }
    case HDC_FN_PRODUCT: return body(Product{});
  }
  return fail(HDC_ERR_INVALID_ARGUMENT, "unknown functor id %d", f.id);
}

template <class Body>
hdc_status with_int_fn(const hdc_functor& f, Body&& body) {
  switch (f.id) {
    case HDC_FN_IDENTITY: return body(IntIdentity{});
    case HDC_FN_AFFINE: return body(IntAffine{f.ia, f.ib});
  }
  return fail(HDC_ERR_UNSUPPORTED, "functor %d is not provided for int32", f.id);
}

template <class Body>
hdc_status with_float_storage(hdc_dtype dt, Body&& body) {
  switch (dt) {
    case HDC_F32: return body(F32{});
    case HDC_F16: return body(F16{});
    case HDC_BF16: return body(BF16{});
    default: return fail(HDC_ERR_UNSUPPORTED, "dtype %d is not floating-point storage", (int)dt);
  }
}


template <class S>
inline Range make_range(const void* x, int64_t n, bool vector) {
  Range r{n, 0, 0, 0, 0};
  if (!vector) return r;
  const int64_t es = sizeof(typename S::T);
  const int64_t mis = (int64_t)((uintptr_t)x % 16);
  int64_t head = mis ? (16 - mis) / es : 0;
  if (head > n) head = n;
  r.head = head;
  r.nvec = (n - head) / S::kVec;
  r.tail_start = head + r.nvec * S::kVec;
  r.tail = n - r.tail_start;
  return r;
}

inline int64_t grid_for(int64_t units, int64_t per_block, int cus, const Tuning& t) {
  int64_t g = (units + per_block - 1) / per_block;
  int64_t cap = (int64_t)cus * t.grid_mult;
  if (cap > kMaxGrid) cap = kMaxGrid;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return g;
}


// Chunk length (in 16-byte vectors) of a grouped batch: the tuning's element
// count rounded up to a whole number of block steps, and never fewer than
// kMinChunk elements, so a call of n elements has at most n / kMinChunk + 1
// chunks (the bound batch_workspace_bytes is sized for).
constexpr int64_t batch_chunk_vecs(const Tuning& t, int kvec) {
  const int64_t step = (int64_t)t.block * t.unroll;
  const int64_t min_vecs = (kMinChunk + kvec - 1) / kvec;
  int64_t v = t.chunk / kvec;
  if (v < min_vecs) v = min_vecs;
  return (v + step - 1) / step * step;
}


// Per-family launchers (one translation unit each).
hdc_status run_map(const hdc_functor& f, hdc_dtype dt, const void* x, void* y, int64_t n, const Tuning& t,
                   hipStream_t st);
// `ticket`: NULL for the two-launch form, else a counter for the one-launch
// form (see launch_reduce).
hdc_status run_reduce(const hdc_functor& f, hdc_dtype dt, const void* x, const void* z, int64_t n, hdc_accum acc,
                      void* out, void* ws, uint64_t* ticket, const Tuning& t, hipStream_t st);
// Fused map + reduce, one translation unit per storage type.
hdc_status run_map_reduce_f32(const hdc_functor& fm, const hdc_functor& f, const void* x, void* y, int64_t n,
                              hdc_accum acc, void* out, void* ws, uint64_t* ticket, const Tuning& t,
                              hipStream_t st);
hdc_status run_map_reduce_f16(const hdc_functor& fm, const hdc_functor& f, const void* x, void* y, int64_t n,
                              hdc_accum acc, void* out, void* ws, uint64_t* ticket, const Tuning& t,
                              hipStream_t st);
hdc_status run_map_reduce_bf16(const hdc_functor& fm, const hdc_functor& f, const void* x, void* y, int64_t n,
                               hdc_accum acc, void* out, void* ws, uint64_t* ticket, const Tuning& t,
                               hipStream_t st);
hdc_status run_map_reduce_i32(const hdc_functor& fm, const hdc_functor& f, const void* x, void* y, int64_t n,
                              hdc_accum acc, void* out, void* ws, uint64_t* ticket, const Tuning& t,
                              hipStream_t st);
// `ws_bytes`: the workspace's size, which sets the work-list capacity.
hdc_status run_segmented(const hdc_functor& f, hdc_dtype dt, const void* x, const int64_t* off, int64_t nseg,
                         hdc_accum acc, void* out, void* ws, size_t ws_bytes, const Tuning& t, hipStream_t st);
// `ws_bytes` is the workspace's capacity; a group whose chunk partials do not
// fit is refused (HDC_ERR_WORKSPACE) before anything is launched.
hdc_status run_batch(const hdc_functor* fm, const hdc_functor& g, hdc_dtype dt, hdc_accum acc,
                     const hdc_batch_call* calls, const int32_t* idx, int cnt, void* ws, size_t ws_bytes,
                     const Tuning& t, hipStream_t st);

hdc_status run_scan(const hdc_functor& f, hdc_dtype dt, const void* x, void* y, int64_t n, hdc_accum acc,
                    int exclusive, void* ws, const Tuning& t, hipStream_t st);
hdc_status run_segmented_scan(const hdc_functor& f, hdc_dtype dt, const void* x, const int64_t* off,
                              int64_t nseg, void* y, int64_t n, hdc_accum acc, int exclusive, void* ws,
                              const Tuning& t, hipStream_t st);
// Workspace of a scan (also segmented), for tiles of at least 64 * 16
// elements: a 256-byte header (the status word at byte 4), then the larger
// of the three-pass need (tile sums and offsets, at most 16 bytes each per
// tile) and the single-pass need (at most 3 words of 8 bytes per tile).
constexpr size_t scan_workspace_bytes(int64_t n) {
  const int64_t G = n / 1024 + 1;
  return 256 + 2 * round_up((size_t)G * 24, 256);
}

// The host side (hdc_host_map / hdc_host_transform_reduce).
hdc_status run_host_map(const hdc_functor& f, hdc_dtype dt, const void* x, void* y, int64_t n, int32_t nthreads);
hdc_status run_host_reduce(const hdc_functor& f, hdc_dtype dt, const void* x, const void* z, int64_t n,
                           hdc_accum acc, void* out, int32_t nthreads);

}  // namespace hdc
