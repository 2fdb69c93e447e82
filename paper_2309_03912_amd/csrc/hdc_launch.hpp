// Launch templates of the kernel families: grid geometry and kernel-instance
// choice (unroll) for one concrete (callable, storage, fold) combination.
#pragma once

#include <type_traits>

#include "hdc_batch.hpp"
#include "hdc_exact.hpp"
#include "hdc_host.hpp"
#include "hdc_scan.hpp"

namespace hdc {

template <class F, class S>
hdc_status launch_map(const F& f, const void* x, void* y, int64_t n, const Tuning& t, hipStream_t st) {
  using T = typename S::T;
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  const bool vec = ((uintptr_t)x % 16) == ((uintptr_t)y % 16);
  Range r = make_range<S>(x, n, vec);
  const int64_t units = vec ? r.nvec : n;
  const int64_t g = grid_for(units, (int64_t)t.block * t.unroll, cus, t);
  auto go = [&](auto U) {
    constexpr int kU = decltype(U)::value;
    if (vec)
      map_kernel<F, S, kU, true><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(f, (const T*)x, (T*)y, r);
    else
      map_kernel<F, S, kU, false><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(f, (const T*)x, (T*)y, r);
  };
  switch (t.unroll) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  return check_launch("map kernel launch");
}

template <class Acc>
hdc_status launch_final(const Acc* partials, int64_t g, void* out, hipStream_t st) {
  reduce_final_kernel<Acc><<<dim3(1), dim3(kFoldThreads), 0, st>>>(partials, (int)g, out);
  return check_launch("final combine launch");
}

// `ticket`: a 64-bit counter (epoch, arrivals) with 0 arrivals that no other
// work uses until this call completes; with it the reduction is one launch
// (its last block folds the partials), without it (NULL) two launches.  Both
// fold in the same order, so they give the same bits.
template <class F, class S, class Acc, class FM = Identity, bool kMap = false>
hdc_status launch_reduce(const F& f, const void* x, const void* z, int64_t n, void* out, void* ws,
                         uint64_t* ticket, const Tuning& t, hipStream_t st, const FM& fm = FM{},
                         void* y = nullptr) {
  using T = typename S::T;
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  bool vec = true;
  if (F::binary && ((uintptr_t)x % 16) != ((uintptr_t)z % 16)) vec = false;
  if (kMap && ((uintptr_t)x % 16) != ((uintptr_t)y % 16)) vec = false;
  Range r = make_range<S>(x, n, vec);
  const int64_t units = vec ? r.nvec : n;
  const int64_t g = grid_for(units, (int64_t)t.block * t.unroll, cus, t);
  Acc* partials = static_cast<Acc*>(ws);
  // The one-launch form keeps 8 bytes per 32-bit word of every partial in
  // the workspace and stages the words in LDS (at most kMaxStageBytes); a
  // larger grid takes two launches.
  constexpr size_t kMaxStageBytes = 32768;
  const size_t stage = (size_t)g * kAccWords<Acc> * 4;
  if (ticket && (2 * stage > reduce_workspace_bytes() || stage > kMaxStageBytes)) ticket = nullptr;
  const size_t dyn = ticket ? stage : 0;
  auto go = [&](auto U) {
    constexpr int kU = decltype(U)::value;
    if (vec)
      reduce_kernel<F, S, Acc, kU, true, FM, kMap><<<dim3((unsigned)g), dim3(t.block), dyn, st>>>(
          f, (const T*)x, (const T*)z, r, partials, ticket, out, fm, (T*)y);
    else
      reduce_kernel<F, S, Acc, kU, false, FM, kMap><<<dim3((unsigned)g), dim3(t.block), dyn, st>>>(
          f, (const T*)x, (const T*)z, r, partials, ticket, out, fm, (T*)y);
  };
  switch (t.unroll) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  HDC_TRY(check_launch("reduce kernel launch"));
  if (ticket) return HDC_OK;
  return launch_final<Acc>(partials, g, out, st);
}


// Exact bf16 sum: pass 1 over t.block threads (at most kExactMaxBlock: the
// digit accumulators take 64 bytes of LDS per thread) x t.unroll vectors per
// step (1, 2 or 4), at most 4096 blocks (their 88-byte partials fit the
// reduce workspace), then the one-block final combine and rounding.
inline hdc_status launch_exact_bf16(const void* x, int64_t n, void* out, void* ws, const Tuning& tuned,
                                    hipStream_t st) {
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  Tuning t = tuned;
  if (t.block > kExactMaxBlock) t.block = kExactMaxBlock;
  const Range r = make_range<BF16>(x, n, true);
  const int u = t.unroll >= 4 ? 4 : t.unroll;
  int64_t g = grid_for(r.nvec, (int64_t)t.block * u, cus, t);
  if (g > 4096) g = 4096;
  // Enough lanes that none takes more than kExactVecsPerLane vectors (its
  // fp64 accumulators stay exact), within the partials the workspace holds.
  const int64_t lanes_needed = (r.nvec + kExactVecsPerLane - 1) / kExactVecsPerLane;
  const int64_t g_min = (lanes_needed + t.block - 1) / t.block;
  constexpr int64_t kMaxExactGrid = (int64_t)(kMaxGrid * kPartialBytes / sizeof(Bf16Exact));
  if (g_min > kMaxExactGrid)
    return fail(HDC_ERR_UNSUPPORTED, "n = %lld is too large for an exact bf16 sum at block %d", (long long)n, t.block);
  if (g < g_min) g = g_min;
  Bf16Exact* partials = static_cast<Bf16Exact*>(ws);
  const uint16_t* xp = static_cast<const uint16_t*>(x);
  const dim3 grid((unsigned)g), block(t.block);
  const size_t lds = sizeof(double) * (kExactFoldDigits + 1) * (size_t)t.block;
  if (u == 1)
    exact_bf16_kernel<1><<<grid, block, lds, st>>>(xp, r, partials);
  else if (u == 2)
    exact_bf16_kernel<2><<<grid, block, lds, st>>>(xp, r, partials);
  else
    exact_bf16_kernel<4><<<grid, block, lds, st>>>(xp, r, partials);
  HDC_TRY(check_launch("exact bf16 launch"));
  exact_bf16_final_kernel<<<dim3(1), dim3(256), 0, st>>>(partials, (int)g, static_cast<double*>(out));
  return check_launch("exact bf16 final launch");
}

// Exact fp16 dot product: vectors when x and z share their 16-byte offset,
// else one element at a time.
inline hdc_status launch_exact_f16_dot(const void* x, const void* z, int64_t n, void* out, void* ws,
                                       const Tuning& t, hipStream_t st) {
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  const bool vec = ((uintptr_t)x % 16) == ((uintptr_t)z % 16);
  const Range r = make_range<F16>(x, n, vec);
  const int u = !vec ? 1 : t.unroll >= 4 ? 4 : t.unroll;
  int64_t g = grid_for(vec ? r.nvec : n, (int64_t)t.block * u, cus, t);
  if (g > 4096) g = 4096;
  F16DotExact* partials = static_cast<F16DotExact*>(ws);
  const uint16_t* xp = static_cast<const uint16_t*>(x);
  const uint16_t* zp = static_cast<const uint16_t*>(z);
  const dim3 grid((unsigned)g), block(t.block);
  if (!vec)
    exact_f16_dot_kernel<1, false><<<grid, block, 0, st>>>(xp, zp, r, partials);
  else if (u == 1)
    exact_f16_dot_kernel<1, true><<<grid, block, 0, st>>>(xp, zp, r, partials);
  else if (u == 2)
    exact_f16_dot_kernel<2, true><<<grid, block, 0, st>>>(xp, zp, r, partials);
  else
    exact_f16_dot_kernel<4, true><<<grid, block, 0, st>>>(xp, zp, r, partials);
  HDC_TRY(check_launch("exact fp16 dot launch"));
  exact_f16_dot_final_kernel<<<dim3(1), dim3(256), 0, st>>>(partials, (int)g, static_cast<double*>(out));
  return check_launch("exact fp16 dot final launch");
}

// Tiled schedule of the segmented reduce (t.passes == 1): the tile pass and
// the combine of segments that span tiles.  The workspace holds two slot
// arrays (`first`, `last`) of one 32-byte fold state per tile.
template <class F, class S, class Acc>
hdc_status launch_seg_tiles(const F& f, const void* x, const int64_t* off, int64_t nseg, void* out, void* ws,
                            size_t ws_bytes, const Tuning& t, hipStream_t st) {
  using T = typename S::T;
  static_assert(sizeof(Acc) <= kPartialBytes, "a tile slot holds 32 bytes");
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  const size_t half = ws_bytes / 2 / 256 * 256;
  SegTiles tl;
  tl.first = ws;
  tl.last = static_cast<char*>(ws) + half;
  tl.cap = (int64_t)(half / kPartialBytes);
  tl.tile_vecs = t.chunk / S::kVec;
  const int64_t wpb = t.block / 64;
  int64_t g = (int64_t)cus * t.grid_mult;
  const int64_t need = (tl.cap + wpb - 1) / wpb;  // never more wavefronts than tiles fit the workspace
  if (g > need) g = need;
  if (g < 1) g = 1;
  auto go = [&](auto U) {
    constexpr int kU = decltype(U)::value;
    seg_tiles_kernel<F, S, Acc, kU><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(f, (const T*)x, off, nseg, tl, out);
  };
  switch (t.unroll) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  HDC_TRY(check_launch("segmented tile launch"));
  int64_t gc = (nseg + 255) / 256;  // one wavefront per 64 segments
  if (gc > (int64_t)cus * 8) gc = (int64_t)cus * 8;
  seg_tiles_combine_kernel<S, Acc><<<dim3((unsigned)gc), dim3(256), 0, st>>>((const T*)x, off, nseg, tl, out);
  return check_launch("segmented tile combine launch");
}

template <class F, class S, class Acc>
hdc_status launch_segmented(const F& f, const void* x, const int64_t* off, int64_t nseg, void* out, void* ws,
                            size_t ws_bytes, const Tuning& t, hipStream_t st) {
  using T = typename S::T;
  if (t.passes == 1) return launch_seg_tiles<F, S, Acc>(f, x, off, nseg, out, ws, ws_bytes, t, st);
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  const int64_t cap = seg_capacity(ws_bytes, nseg);
  if (cap < 1) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes is too small for %lld segments", ws_bytes,
                           (long long)nseg);
  const SegLayout l = seg_layout_cap(cap, nseg);
  char* base = static_cast<char*>(ws);
  SegPlan p;
  p.cnt = reinterpret_cast<SegCounters*>(base + l.cnt);
  p.block_tot = reinterpret_cast<SegCounters*>(base + l.block_tot);
  p.full_list = reinterpret_cast<SegPiece*>(base + l.full);
  p.part_list = reinterpret_cast<SegPiece*>(base + l.part);
  p.long_base = reinterpret_cast<int32_t*>(base + l.long_base);
  p.long_list = reinterpret_cast<int32_t*>(base + l.long_list);
  p.partials = base + l.partials;
  p.cap_full = l.cap_full;
  p.cap_part = l.cap_part;
  p.cap_partials = l.cap_partials;
  p.chunk = t.chunk;
  p.small_seg = t.small_seg;
  p.spw = t.seg_per_wave;

  seg_count_kernel<<<dim3((unsigned)l.plan_blocks), dim3(kPlanBlock), 0, st>>>(off, nseg, p);
  HDC_TRY(check_launch("segmented count launch"));
  seg_count_scan_kernel<<<dim3(1), dim3(1024), 0, st>>>(l.plan_blocks, p);
  HDC_TRY(check_launch("segmented count-scan launch"));
  seg_write_kernel<<<dim3((unsigned)l.plan_blocks), dim3(kPlanBlock), 0, st>>>(off, nseg, p);
  HDC_TRY(check_launch("segmented plan launch"));

  // Persistent grid: enough wavefronts to fill the chip, never more than the
  // largest possible item count needs.
  const int64_t wpb = t.block / 64;
  const int64_t max_items = l.cap_full + l.cap_part + (nseg + p.spw - 1) / p.spw;
  int64_t g = (int64_t)cus * t.grid_mult;
  const int64_t need = (max_items + wpb - 1) / wpb;
  if (g > need) g = need;
  if (g < 1) g = 1;
  auto go = [&](auto U) {
    constexpr int kU = decltype(U)::value;
    seg_items_kernel<F, S, Acc, kU><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(f, (const T*)x, off, nseg, p,
                                                                                 out);
  };
  switch (t.unroll) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  HDC_TRY(check_launch("segmented item launch"));
  int64_t gc = (nseg + 3) / 4;
  if (gc > (int64_t)cus * 8) gc = (int64_t)cus * 8;
  if (gc < 1) gc = 1;
  seg_combine_kernel<Acc><<<dim3((unsigned)gc), dim3(256), 0, st>>>(off, nseg, p, out);
  return check_launch("segmented combine launch");
}

template <class FM, class F, class S, class Acc>
hdc_status launch_batch(const FM& fm, const F& f, const hdc_batch_call* calls, const int32_t* idx, int cnt,
                        void* ws, size_t ws_bytes, const Tuning& t, hipStream_t st) {
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  BatchTable tab{};
  tab.count = cnt;
  tab.chunk_vecs = batch_chunk_vecs(t, S::kVec);
  int64_t acc_chunks = 0;
  for (int q = 0; q < cnt; ++q) {
    const hdc_batch_call& c = calls[idx[q]];
    BatchCall& b = tab.call[q];
    b.x = c.x;
    b.y = c.y;
    b.out = c.out;
    b.r = make_range<S>(c.x, c.n, true);
    tab.prefix[q] = acc_chunks;
    if (c.n > 0) {
      int64_t nc = (b.r.nvec + tab.chunk_vecs - 1) / tab.chunk_vecs;
      acc_chunks += nc > 0 ? nc : 1;
    }
  }
  tab.prefix[cnt] = acc_chunks;
  if ((size_t)acc_chunks * sizeof(Acc) > ws_bytes)
    return fail(HDC_ERR_WORKSPACE, "the batch needs %lld chunk partials (%zu bytes) but the workspace holds %zu bytes",
                (long long)acc_chunks, (size_t)acc_chunks * sizeof(Acc), ws_bytes);
  Acc* partials = static_cast<Acc*>(ws);
  if (acc_chunks > 0) {
    int64_t g = (int64_t)cus * t.grid_mult;
    if (g > acc_chunks) g = acc_chunks;
    auto go = [&](auto U) {
      constexpr int kU = decltype(U)::value;
      batch_kernel<FM, F, S, Acc, kU><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(fm, f, tab, partials);
    };
    switch (t.unroll) {
      case 1: go(std::integral_constant<int, 1>{}); break;
      case 2: go(std::integral_constant<int, 2>{}); break;
      case 4: go(std::integral_constant<int, 4>{}); break;
      default: go(std::integral_constant<int, 8>{}); break;
    }
    HDC_TRY(check_launch("batch launch"));
  }
  batch_combine_kernel<Acc><<<dim3((unsigned)cnt), dim3(256), 0, st>>>(tab, partials);
  return check_launch("batch combine launch");
}

// Scan: t.unroll == 1 selects the three-pass schedule, any other value the
// single pass.  `seg` carries the segment offsets of a segmented scan (Acc a
// SegAcc), else nothing.  Workspace (scan_workspace_bytes):
//   three passes: 256-byte header (status) | tile sums | tile offsets, one
//                 fold state per tile each;
//   single pass:  256-byte header (ticket, status) | the tree nodes
//                 (tree_nodes(G), level by level), kWords 8-byte words each.
template <class F, class S, class Acc>
hdc_status launch_scan(const F& f, const void* x, void* y, int64_t n, int exclusive, SegSpec seg, void* ws,
                       const Tuning& t, hipStream_t st) {
  using T = typename S::T;
  using OutT = typename ScanOut<Acc>::T;
  static_assert(sizeof(Acc) <= 24, "scan_workspace_bytes holds 24 bytes per tile and array");
  const int64_t tile = (int64_t)t.block * kScanE;
  const int64_t G = (n + tile - 1) / tile;
  if (G * t.block > (int64_t)UINT32_MAX) return fail(HDC_ERR_UNSUPPORTED, "n = %lld is too large for one scan", (long long)n);
  const bool xa = (uintptr_t)x % 16 == 0, ya = (uintptr_t)y % 16 == 0;
  const T* xp = static_cast<const T*>(x);
  OutT* yp = static_cast<OutT*>(y);
  const dim3 grid((unsigned)G), block(t.block);
  if (t.unroll != 1) {
    uint64_t* w = static_cast<uint64_t*>(ws);
    const int64_t nwords = 32 + (int64_t)ScanCarry<Acc>::kWords * tree_nodes(G);
    const ScanLB lb{static_cast<uint32_t*>(ws), static_cast<uint32_t*>(ws) + 1, w + 32};
    const int64_t cb = (nwords + 255) / 256;
    scan_lb_clear_kernel<<<dim3((unsigned)(cb < 1024 ? cb : 1024)), dim3(256), 0, st>>>(w, nwords);
    HDC_TRY(check_launch("scan look-back clear launch"));
    if (xa && ya)
      scan_onepass_kernel<F, S, Acc, true, true><<<grid, block, 0, st>>>(f, xp, n, seg, lb, yp, exclusive);
    else if (xa)
      scan_onepass_kernel<F, S, Acc, true, false><<<grid, block, 0, st>>>(f, xp, n, seg, lb, yp, exclusive);
    else if (ya)
      scan_onepass_kernel<F, S, Acc, false, true><<<grid, block, 0, st>>>(f, xp, n, seg, lb, yp, exclusive);
    else
      scan_onepass_kernel<F, S, Acc, false, false><<<grid, block, 0, st>>>(f, xp, n, seg, lb, yp, exclusive);
    return check_launch("scan single-pass launch");
  }
  // three passes: the same 256-byte header (its status word cleared by the
  // offsets pass), then the tile sums and the tile offsets
  Acc* sums = reinterpret_cast<Acc*>(static_cast<char*>(ws) + 256);
  Acc* offsets = reinterpret_cast<Acc*>(static_cast<char*>(ws) + 256 + round_up((size_t)G * sizeof(Acc), 256));
  if (xa)
    scan_tile_sums_kernel<F, S, Acc, true><<<grid, block, 0, st>>>(f, xp, n, seg, sums);
  else
    scan_tile_sums_kernel<F, S, Acc, false><<<grid, block, 0, st>>>(f, xp, n, seg, sums);
  HDC_TRY(check_launch("scan tile-sum launch"));
  scan_offsets_kernel<Acc><<<dim3(1), dim3(1024), 0, st>>>(sums, G, offsets, static_cast<uint32_t*>(ws) + 1);
  HDC_TRY(check_launch("scan offset launch"));
  if (xa && ya)
    scan_tiles_kernel<F, S, Acc, true, true><<<grid, block, 0, st>>>(f, xp, n, seg, offsets, yp, exclusive);
  else if (xa)
    scan_tiles_kernel<F, S, Acc, true, false><<<grid, block, 0, st>>>(f, xp, n, seg, offsets, yp, exclusive);
  else if (ya)
    scan_tiles_kernel<F, S, Acc, false, true><<<grid, block, 0, st>>>(f, xp, n, seg, offsets, yp, exclusive);
  else
    scan_tiles_kernel<F, S, Acc, false, false><<<grid, block, 0, st>>>(f, xp, n, seg, offsets, yp, exclusive);
  return check_launch("scan tile launch");
}

}  // namespace hdc
