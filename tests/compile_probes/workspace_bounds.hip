// Compile probe: workspace bounds of the grouped batch and the segmented
// reduce.  The chunk length of a grouped batch, for every tuning the
// library accepts, is a whole number of block steps of at least kMinChunk
// elements, and the chunk partials of any set of calls fit the workspace
// hdc_workspace_size(HDC_OP_BATCH, ...) provides.  Checked at compile time.
#include "hdc_host.hpp"

using hdc::batch_chunk_vecs;
using hdc::batch_workspace_bytes;
using hdc::kMinChunk;
using hdc::kPartialBytes;

// Chunks of one call of n elements (vector walk from a 16-byte boundary,
// the head peeled: at most n / kvec vectors), as the launcher counts them.
consteval int64_t chunks_of(int64_t n, int64_t cv, int kvec) {
  if (n == 0) return 0;
  const int64_t nvec = n / kvec;
  const int64_t c = (nvec + cv - 1) / cv;
  return c > 0 ? c : 1;
}

consteval bool every_tuning_fits() {
  for (int kvec : {4, 8}) {                      // 4-byte and 2-byte storage
    for (int block = 64; block <= 1024; block += 64) {
      for (int unroll : {1, 2, 4, 8}) {
        for (int chunk = 1024; chunk <= 65536; chunk *= 2) {
          hdc::Tuning t{};
          t.block = block;
          t.unroll = unroll;
          t.chunk = chunk;
          const int64_t cv = batch_chunk_vecs(t, kvec);
          if (cv % ((int64_t)block * unroll) != 0) return false;  // whole block steps
          if (cv * kvec < kMinChunk) return false;                // at least kMinChunk elements
          // sizes near chunk boundaries, single calls and a batch of 32
          for (int64_t base = 1; base <= (int64_t(1) << 34); base = base * 5 / 3 + 1) {
            for (int64_t d = -1; d <= 1; ++d) {
              const int64_t n = (base / (cv * kvec)) * (cv * kvec) + d;
              if (n < 0) continue;
              if ((size_t)chunks_of(n, cv, kvec) * kPartialBytes > batch_workspace_bytes(n, 1)) return false;
              if ((size_t)(32 * chunks_of(n, cv, kvec)) * kPartialBytes > batch_workspace_bytes(32 * n, 32))
                return false;
            }
          }
        }
      }
    }
  }
  return true;
}
static_assert(every_tuning_fits());

// The earlier rounding (down to whole block steps) gave 768-element chunks at
// block 192, unroll 1, 4-byte storage: below kMinChunk.
static_assert([] {
  hdc::Tuning t{};
  t.block = 192;
  t.unroll = 1;
  t.chunk = 1024;
  return batch_chunk_vecs(t, 4) * 4 >= kMinChunk;
}());

// The segmented work lists: a workspace of seg_layout(total, S, kMinChunk)
// bytes -- what hdc_workspace_size returns -- holds the full-piece capacity
// total / chunk + 1 at every chunk length, and the capacity read back from
// any size never needs more bytes than that size.
consteval bool segmented_capacity_holds() {
  for (int64_t S = 1; S <= 10000000; S = S * 7 / 2 + 1) {
    for (int64_t total = 0; total <= (int64_t(1) << 34); total = total * 5 / 3 + 977) {
      const size_t b = hdc::seg_layout(total, S, kMinChunk).bytes;
      const int64_t cap = hdc::seg_capacity(b, S);
      for (int64_t chunk = kMinChunk; chunk <= 65536; chunk *= 2)
        if (cap < total / chunk + 1) return false;
      if (hdc::seg_layout_cap(cap, S).bytes > b) return false;
      if (hdc::seg_total_bound(b, S) < total) return false;
      for (size_t extra : {size_t(1), size_t(255), size_t(4097)}) {
        const int64_t c2 = hdc::seg_capacity(b + extra, S);
        if (c2 < cap || hdc::seg_layout_cap(c2, S).bytes > b + extra) return false;
        if (hdc::seg_layout_cap(c2 + 1, S).bytes <= b + extra) return false;  // the largest that fits
      }
    }
  }
  return hdc::seg_capacity(hdc::seg_layout_cap(1, 100).bytes - 1, 100) == 0;
}
static_assert(segmented_capacity_holds());
