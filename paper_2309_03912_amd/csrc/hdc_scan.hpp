// Prefix sums of f(x): y[i] = fold of f(x[0..i]) (inclusive) or f(x[0..i-1])
// (exclusive), over tiles of T = blockDim * kScanE elements.
//
// Layout of a tile: wavefront w owns the 64 * kScanE contiguous elements
// starting at w * 64 * kScanE, as Q = kScanE / V chunks of 64 * V elements
// (V = elements per 16-byte vector).  In chunk q, lane l owns the V elements
// at q * 64 V + l V: every load of a wavefront covers one contiguous 1-KiB
// span, and so does every store when a lane's outputs of a chunk take 16
// bytes, or 32 (through an LDS stage).  The fold order inside a tile is fixed: a lane folds
// its V terms in order, a wavefront scans the lane totals of each chunk and
// chains its chunks, the block scans the wavefront totals in wave order.
//
// Two schedules share that tile step:
//  * three passes, no inter-block waiting -- A: every tile is folded to its
//    sum; B: one block scans the tile sums into tile offsets; C: every tile
//    is scanned again and its offset added (x is read twice);
//  * one pass, tiles handed out in launch order: every tile publishes its
//    total as a leaf of a radix-64 tree (and the last tile of a group the
//    group's node) and folds its carry from at most 63 nodes per level of
//    earlier tiles (x is read once).
// Both are reproducible bit for bit: pass B always folds in one fixed order,
// and every tree node and carry is a fold in a fixed order of fixed values,
// whichever tile the timing lets finish first.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hdc_device.hpp"
#include "hdc_functors.hpp"
#include "hdc_kernels.hpp"

namespace hdc {

constexpr int kScanE = 16;  // elements per thread per tile

template <class T>
__device__ __forceinline__ T shfl_up_words(T v, int d) {
  constexpr int W = sizeof(T) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __shfl_up(w[i], d, 64);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Move every 32-bit word of `v` through one DPP control; lanes outside
// kRowMask, or without a source lane, keep their own value.
template <int kCtrl, int kRowMask, class T>
__device__ __forceinline__ T dpp_words(T v) {
  constexpr int W = sizeof(T) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_update_dpp(w[i], w[i], kCtrl, kRowMask, 0xF, false);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Inclusive scan over the lanes of a wavefront in lane order (merge(lower,
// higher)), with DPP moves only: row_shr 1, 2, 4, 8 inside rows of 16
// lanes, then row_bcast:15 (rows 1 and 3 take the end of the row before) and
// row_bcast:31 (rows 2 and 3 take lane 31).  kRows16: only row 0 matters.
template <class Acc, bool kRows16 = false>
__device__ __forceinline__ Acc wave_incl_scan(Acc v) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  {
    const Acc u = dpp_words<0x111, 0xF>(v);
    if (r >= 1) v = Acc::merge(u, v);
  }
  {
    const Acc u = dpp_words<0x112, 0xF>(v);
    if (r >= 2) v = Acc::merge(u, v);
  }
  {
    const Acc u = dpp_words<0x114, 0xF>(v);
    if (r >= 4) v = Acc::merge(u, v);
  }
  {
    const Acc u = dpp_words<0x118, 0xF>(v);
    if (r >= 8) v = Acc::merge(u, v);
  }
  if constexpr (!kRows16) {
    {
      const Acc u = dpp_words<0x142, 0xA>(v);
      if (lane & 16) v = Acc::merge(u, v);
    }
    {
      const Acc u = dpp_words<0x143, 0xC>(v);
      if (lane >= 32) v = Acc::merge(u, v);
    }
  }
  return v;
}

// The value of the lane below (wave_shr:1); lane 0 gets `first`.
template <class Acc>
__device__ __forceinline__ Acc wave_shift_up1(Acc v, const Acc& first) {
  const Acc u = dpp_words<0x138, 0xF>(v);
  return (threadIdx.x & 63) == 0 ? first : u;
}

// Exclusive scan of fold states over a block (thread order).  Returns the
// thread's exclusive prefix; *total receives the block total (all threads).
// `lds` holds kMaxWaves states.
template <class Acc>
__device__ __forceinline__ Acc block_exclusive_scan_acc(Acc v, Acc* lds, Acc* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  Acc incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const Acc t = shfl_up_words(incl, d);
    if (lane >= d) incl = Acc::merge(t, incl);
  }
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  Acc before = Acc::zero(), all = Acc::zero();
  for (int i = 0; i < nw; ++i) {
    const Acc w = lds[i];
    if (i < wid) before = Acc::merge(before, w);
    all = Acc::merge(all, w);
  }
  __syncthreads();
  *total = all;
  // exclusive within the wave: the inclusive value of the previous lane
  Acc ex = shfl_up_words(incl, 1);
  if (lane == 0) ex = Acc::zero();
  return Acc::merge(before, ex);
}

template <class Acc>
struct ScanOut;
template <>
struct ScanOut<PlainAcc> {
  using T = float;
  __device__ static T value(const PlainAcc& a) { return a.s; }
};
template <>
struct ScanOut<CompAcc> {
  using T = double;
  __device__ static T value(const CompAcc& a) {
    return __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
  }
};
template <>
struct ScanOut<IntAcc> {
  using T = int64_t;
  __device__ static T value(const IntAcc& a) { return (int64_t)a.s; }
};

// Fold state of a segmented scan: the state of the open segment and whether
// a segment starts inside the span it covers.  merge(x, y) = y when y holds a
// segment start, else x + y: associative, so every schedule above applies.
template <class Acc>
struct SegAcc {
  Acc a;
  uint32_t f;
  __device__ static SegAcc zero() { return {Acc::zero(), 0u}; }
  __device__ static SegAcc merge(SegAcc x, SegAcc y) { return y.f ? y : SegAcc{Acc::merge(x.a, y.a), x.f}; }
  template <class T>
  __device__ void add(T t) {
    a.add(t);
  }
};
template <class Acc>
struct ScanOut<SegAcc<Acc>> {
  using T = typename ScanOut<Acc>::T;
  __device__ static T value(const SegAcc<Acc>& s) { return ScanOut<Acc>::value(s.a); }
};

template <class Acc>
struct IsSeg : std::false_type {};
template <class Acc>
struct IsSeg<SegAcc<Acc>> : std::true_type {};

// Segment boundaries of a segmented scan: the CSR offsets (m = S + 1 of them).
struct SegSpec {
  const int64_t* off;
  int64_t m;
};

// One wavefront's part of a tile: loading, terms, the fold states of the
// fixed order above, and the outputs.  For a segmented scan (Acc a SegAcc)
// each lane takes the segment-start bits of its elements from the tile's
// bitmap (tile_heads) into `hmask`; outputs are written only inside
// [off[0], off[S]).
template <class F, class S, class Acc>
struct ScanWave {
  static constexpr int V = S::kVec;
  static constexpr int Q = kScanE / V;
  static constexpr bool kSeg = IsSeg<Acc>::value;
  using OutT = typename ScanOut<Acc>::T;

  int64_t wbase;  // first element of this wavefront's part
  int lane;
  int64_t n;
  elem_t<S> v[kScanE];             // chunk q, element e at v[q V + e]
  [[maybe_unused]] float t[kScanE];  // the terms (floats)
  Acc ex[Q];                       // exclusive prefix of this lane within chunk q
  Acc wc[Q];                       // fold of chunks 0..q-1 of this wavefront
  Acc wave_total;
  uint32_t hmask;                  // segmented: bit q V + e set if element (q, e) starts a segment
  int64_t out_lo, out_hi;          // segmented: outputs are written in [out_lo, out_hi)

  __device__ int64_t index(int q, int e) const { return wbase + (int64_t)q * 64 * V + (int64_t)lane * V + e; }

  template <bool kAligned>
  __device__ void load(const elem_t<S>* x, const SegSpec& seg) {
    if (kAligned && wbase + 64 * kScanE <= n) {
      // a raw buffer resource over this wavefront's part (word 3 0x00020000:
      // 32-bit data format, no swizzle; cache policy 2: non-temporal), so the
      // lane offsets stay fixed instead of 64-bit address arithmetic per load
      const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(x + wbase), (short)0, (int)(64 * kScanE * sizeof(elem_t<S>)), 0x00020000);
      Vec<S> a[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rx, (uint32_t)(q * 64 + lane) * 16u, 0, 2);
        __builtin_memcpy(&a[q], &w, 16);
      }
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) v[q * V + e] = a[q].e[e];
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int64_t i = index(q, e);
          v[q * V + e] = i < n ? x[i] : elem_t<S>{};
        }
    }
    if constexpr (kSeg) {
      out_lo = seg.off[0];
      out_hi = seg.off[seg.m - 1];
    }
  }

  // This lane's segment-start bits from the tile bitmap (bit p: tile
  // position p starts a segment).  A lane's V elements of a chunk are V
  // consecutive bits inside one 32-bit word.
  __device__ void take_heads(const uint32_t* bits, int64_t tile_start) {
    hmask = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t p = index(q, 0) - tile_start;
      hmask |= ((bits[p >> 5] >> (p & 31)) & ((1u << V) - 1u)) << (q * V);
    }
  }

  // The lane state that emit needs, as 32-bit words: the terms (float
  // storage) or the elements (int32), the chunk prefixes and the heads.
  static constexpr int kStashWords =
      kScanE + Q * (int)(sizeof(Acc) / 4) + (kSeg ? 1 : 0);
  // Park that state in LDS (word c of lane l at s[c * 64 + l]) and take it
  // back: a wavefront that runs the carry's polls between the two holds none
  // of it in registers meanwhile.
  __device__ void stash(uint32_t* s) const {
    int c = 0;
    auto put = [&](const auto& v) {
      uint32_t w[sizeof(v) / 4];
      __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
      for (int i = 0; i < (int)(sizeof(v) / 4); ++i) s[(c + i) * 64 + lane] = w[i];
      c += (int)(sizeof(v) / 4);
    };
    if constexpr (std::is_same_v<S, I32>)
      put(v);
    else
      put(t);
    put(ex);
    if constexpr (kSeg) put(hmask);
  }
  __device__ void unstash(const uint32_t* s) {
    int c = 0;
    auto get = [&](auto& v) {
      uint32_t w[sizeof(v) / 4];
#pragma unroll
      for (int i = 0; i < (int)(sizeof(v) / 4); ++i) w[i] = s[(c + i) * 64 + lane];
      __builtin_memcpy(&v, w, sizeof(v));
      c += (int)(sizeof(v) / 4);
    };
    if constexpr (std::is_same_v<S, I32>)
      get(v);
    else
      get(t);
    get(ex);
    if constexpr (kSeg) get(hmask);
  }

  __device__ bool is_head(int q, int e) const {
    if constexpr (kSeg)
      return (hmask >> (q * V + e)) & 1u;
    else
      return false;
  }

  // Fold element (q, e) into a; a segment start first resets it.
  __device__ void accum(Acc& a, const F& f, int q, int e) const {
    if constexpr (kSeg) {
      if (is_head(q, e)) {
        a = Acc::zero();
        a.f = 1u;
      }
      if constexpr (!std::is_same_v<S, I32>)
        a.add(t[q * V + e]);
      else
        fold_elem<F, S>(a.a, f, v[q * V + e], v[q * V + e]);
    } else {
      if constexpr (!std::is_same_v<S, I32>)
        a.add(t[q * V + e]);
      else
        fold_elem<F, S>(a, f, v[q * V + e], v[q * V + e]);
    }
  }

  // Terms, lane totals per chunk, the wavefront scans and the chunk chain.
  __device__ void fold(const F& f) {
    Acc tot[Q];
    if constexpr (!std::is_same_v<S, I32>) {
#pragma unroll
      for (int k = 0; k < kScanE; ++k) t[k] = S::widen(v[k]);
      eval_batch(f, t);  // once: the terms serve the totals and the outputs
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      tot[q] = Acc::zero();
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (index(q, e) < n) accum(tot[q], f, q, e);
    }
    Acc run = Acc::zero();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const Acc incl = wave_incl_scan(tot[q]);
      ex[q] = wave_shift_up1(incl, Acc::zero());
      wc[q] = run;
      run = Acc::merge(run, read_lane(incl, 63));
    }
    wave_total = run;
  }

  // Outputs of this lane, starting from the fold of everything before this
  // wavefront's part, stored chunk by chunk.  Chunk q's V outputs of a lane
  // are contiguous: V * sizeof(OutT) bytes as 16-byte stores (non-temporal
  // when a lane's run is exactly 16 bytes, so a wavefront's store covers whole
  // lines; cached otherwise, so the cache merges the interleaved runs of a
  // chunk into whole lines).
  // With 32 output bytes per lane and chunk (V = 2 PER), a whole chunk goes
  // through the wavefront's 2 KiB `stage` (LDS): each lane writes its 32
  // bytes, then takes the 16-byte pieces at lanes l and 64 + l of the
  // chunk's output, so that each non-temporal store instruction of the
  // wavefront covers one contiguous KiB.
  template <bool kOutAligned>
  __device__ void emit(const F& f, const Acc& before, int exclusive, OutT* y, u32x4* stage) const {
    constexpr int PER = 16 / sizeof(OutT);
    bool full = kOutAligned && wbase + 64 * kScanE <= n;
    if constexpr (kSeg) full = full && wbase >= out_lo && wbase + 64 * kScanE <= out_hi;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Acc a = Acc::merge(Acc::merge(before, wc[q]), ex[q]);
      OutT o[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const OutT prev = is_head(q, e) ? OutT{} : ScanOut<Acc>::value(a);
        if (index(q, e) < n) accum(a, f, q, e);
        o[e] = exclusive ? prev : ScanOut<Acc>::value(a);
      }
      if (full) {
        if constexpr (V == 2 * PER) {
          u32x4 w0, w1;
          __builtin_memcpy(&w0, &o[0], 16);
          __builtin_memcpy(&w1, &o[PER], 16);
          stage[2 * lane] = w0;
          stage[2 * lane + 1] = w1;
          __builtin_amdgcn_wave_barrier();
          const u32x4 r0 = stage[lane], r1 = stage[64 + lane];
          __builtin_amdgcn_wave_barrier();  // the next chunk's writes come after these reads
          u32x4* p = reinterpret_cast<u32x4*>(y + index(q, 0) - (int64_t)lane * V);  // the chunk's start
          __builtin_nontemporal_store(r0, p + lane);
          __builtin_nontemporal_store(r1, p + 64 + lane);
        } else {
#pragma unroll
          for (int h = 0; h < V / PER; ++h) {
            u32x4 w;
            __builtin_memcpy(&w, &o[h * PER], 16);
            u32x4* p = reinterpret_cast<u32x4*>(y + index(q, h * PER));
            if constexpr (V == PER)
              __builtin_nontemporal_store(w, p);
            else
              *p = w;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int64_t i = index(q, e);
          bool keep = i < n;
          if constexpr (kSeg) keep = keep && i >= out_lo && i < out_hi;
          if (keep) y[i] = o[e];
        }
      }
    }
  }
};

// Exclusive fold of the wavefront totals of a block in wave order; *total
// receives the block total.  Every wavefront loads the (at most 16) totals
// into its first lanes and scans them with fixed DPP moves, so the
// results are wavefront-uniform (scalar registers) and the fold costs the
// tile no vector registers beyond the moves.  `lds` holds kMaxWaves
// states.
template <class Acc>
__device__ __forceinline__ Acc block_wave_prefix(const Acc& wave_total, Acc* lds, Acc* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) lds[wid] = wave_total;
  __syncthreads();
  const Acc v = wave_incl_scan<Acc, true>(lane < nw ? lds[lane] : Acc::zero());  // nw <= 16: row 0
  *total = read_lane(v, nw - 1);
  const Acc prev = read_lane(v, wid > 0 ? wid - 1 : 0);
  __syncthreads();
  return wid > 0 ? prev : Acc::zero();
}

template <class F, class S, class Acc>
__device__ __forceinline__ ScanWave<F, S, Acc> scan_wave_at(int64_t tile, int64_t n) {
  ScanWave<F, S, Acc> w;
  w.lane = threadIdx.x & 63;
  w.wbase = tile * (int64_t)blockDim.x * kScanE + (int64_t)(threadIdx.x >> 6) * 64 * kScanE;
  w.n = n;
  return w;
}

// Segment starts of the tile [t0, t0 + len) as a bitmap in LDS (len / 32
// words; bit p: position t0 + p starts a segment), built by the whole block
// in two dependent rounds of offset reads: one probe per thread at evenly
// spaced offsets (issued before the tile's elements are loaded, see
// heads_probe) narrows the first boundary at or after t0 to one gap between
// probes; then every thread takes one offset per round from the start of
// that gap until they pass the tile.  Then each wavefront takes its lanes'
// bits (ScanWave::take_heads).  Empty segments repeat a boundary, which sets
// the same bit again.
constexpr int kTileWords = 1024 * kScanE / 32;  // bitmap words of the largest tile

// 16-byte vectors of output staging per block: 2 KiB per wavefront when a
// lane's outputs of a chunk are 32 bytes, none otherwise.
template <class S, class Acc>
constexpr int kStageVecs =
    S::kVec * sizeof(typename ScanOut<Acc>::T) == 32 ? kMaxWaves * 128 : 1;

// This thread's probe for the first round: offset (tid + 1) step - 1 of the
// m offsets (clamped to the last one), step = ceil(m / blockDim).  With m no
// larger than the block there is no probe (step 0) and the search starts at
// offset 0.
struct HeadProbe {
  int64_t step;
  int64_t v;
};

__device__ __forceinline__ HeadProbe heads_probe(const SegSpec& seg) {
  HeadProbe p{0, 0};
  const int64_t nt = blockDim.x;
  if (seg.m > nt) {
    p.step = (seg.m + nt - 1) / nt;
    int64_t idx = ((int64_t)threadIdx.x + 1) * p.step - 1;
    if (idx > seg.m - 1) idx = seg.m - 1;
    p.v = seg.off[idx];
  }
  return p;
}

// `wfirst` (LDS, kMaxWaves words): per wavefront, its first thread whose
// probe is at or after t0.
template <class W>
__device__ void tile_heads(W& w, const SegSpec& seg, const HeadProbe& pr, int64_t t0, int64_t len, uint32_t* bits,
                           uint32_t* wfirst) {
  const int tid = threadIdx.x, nt = blockDim.x, nw = nt >> 6;
  for (int64_t i = tid; i < len / 32; i += nt) bits[i] = 0;
  if (pr.step > 0) {  // uniform
    const uint64_t ge = __builtin_amdgcn_ballot_w64(pr.v >= t0);
    if ((tid & 63) == 0) wfirst[tid >> 6] = ge ? (uint32_t)(tid + __builtin_ctzll(ge)) : 0xFFFFFFFFu;
  }
  __syncthreads();
  // The first boundary at or after t0 is past probe f - 1 and at most probe
  // f (f: the first thread whose probe is >= t0), i.e. in [f step, (f+1) step).
  // No such probe: every offset is below t0 (the last probe reads the last).
  int64_t lo = 0;
  if (pr.step > 0) {
    uint32_t f = 0xFFFFFFFFu;
    for (int k = 0; k < nw; ++k) f = wfirst[k] < f ? wfirst[k] : f;
    lo = f == 0xFFFFFFFFu ? seg.m : (int64_t)f * pr.step;
  }
  const int64_t t1 = t0 + len;
  for (int64_t j = lo + tid; j < seg.m; j += nt) {
    const int64_t b = seg.off[j];
    if (b >= t1) break;  // the offsets do not decrease: later ones are past the tile too
    if (b >= t0) atomicOr(&bits[(b - t0) >> 5], 1u << ((b - t0) & 31));
  }
  __syncthreads();
  w.take_heads(bits, t0);
}

// Pass A: the sum of every tile.
template <class F, class S, class Acc, bool kAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_tile_sums_kernel(F f, const elem_t<S>* x, int64_t n, SegSpec seg,
                                                              Acc* sums) {
  __shared__ Acc lds[kMaxWaves];
  __shared__ uint32_t heads_sh[IsSeg<Acc>::value ? kTileWords : 1];
  __shared__ uint32_t wfirst_sh[kMaxWaves];
  auto w = scan_wave_at<F, S, Acc>(blockIdx.x, n);
  HeadProbe pr{0, 0};
  if constexpr (IsSeg<Acc>::value) pr = heads_probe(seg);
  w.template load<kAligned>(x, seg);
  if constexpr (IsSeg<Acc>::value)
    tile_heads(w, seg, pr, (int64_t)blockIdx.x * blockDim.x * kScanE, (int64_t)blockDim.x * kScanE, heads_sh,
               wfirst_sh);
  w.fold(f);
  Acc total;
  (void)block_wave_prefix(w.wave_total, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass B: exclusive scan of the G tile sums, in rounds of blockDim * kScanE;
// a thread folds kScanE consecutive sums (all loaded first), then the block
// scans the thread totals.
template <class Acc>
__global__ __launch_bounds__(1024) void scan_offsets_kernel(const Acc* sums, int64_t G, Acc* offsets,
                                                            uint32_t* status) {
  __shared__ Acc lds[kMaxWaves];
  if (threadIdx.x == 0) *status = 0;  // this schedule never waits, so it never gives up
  const int lane = threadIdx.x & 63;
  const int64_t R = (int64_t)blockDim.x * kScanE;
  Acc carry = Acc::zero();
  for (int64_t base = 0; base < G; base += R) {
    const int64_t j0 = base + (int64_t)threadIdx.x * kScanE;
    Acc in[kScanE];
#pragma unroll
    for (int k = 0; k < kScanE; ++k) in[k] = j0 + k < G ? sums[j0 + k] : Acc::zero();
    Acc own[kScanE];
    Acc a = Acc::zero();
#pragma unroll
    for (int k = 0; k < kScanE; ++k) {
      own[k] = a;  // exclusive within the thread
      a = Acc::merge(a, in[k]);
    }
    Acc incl = a;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const Acc u = shfl_up_words(incl, d);
      if (lane >= d) incl = Acc::merge(u, incl);
    }
    Acc ex = shfl_up_words(incl, 1);
    if (lane == 0) ex = Acc::zero();
    Acc total;
    const Acc before = block_wave_prefix(read_lane(incl, 63), lds, &total);
    const Acc start = Acc::merge(Acc::merge(carry, before), ex);
#pragma unroll
    for (int k = 0; k < kScanE; ++k)
      if (j0 + k < G) offsets[j0 + k] = Acc::merge(start, own[k]);
    carry = Acc::merge(carry, total);
  }
}

// Pass C: scan every tile again and add its offset.
template <class F, class S, class Acc, bool kAligned, bool kOutAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) void scan_tiles_kernel(F f, const elem_t<S>* x, int64_t n, SegSpec seg,
                                                          const Acc* offsets, typename ScanOut<Acc>::T* y,
                                                          int exclusive) {
  __shared__ Acc lds[kMaxWaves];
  __shared__ uint32_t heads_sh[IsSeg<Acc>::value ? kTileWords : 1];
  __shared__ uint32_t wfirst_sh[kMaxWaves];
  __shared__ u32x4 stage_sh[kStageVecs<S, Acc>];
  auto w = scan_wave_at<F, S, Acc>(blockIdx.x, n);
  HeadProbe pr{0, 0};
  if constexpr (IsSeg<Acc>::value) pr = heads_probe(seg);
  w.template load<kAligned>(x, seg);
  if constexpr (IsSeg<Acc>::value)
    tile_heads(w, seg, pr, (int64_t)blockIdx.x * blockDim.x * kScanE, (int64_t)blockDim.x * kScanE, heads_sh,
               wfirst_sh);
  w.fold(f);
  Acc total;
  const Acc before = block_wave_prefix(w.wave_total, lds, &total);
  w.template emit<kOutAligned>(f, Acc::merge(offsets[blockIdx.x], before), exclusive, y,
                               stage_sh + (threadIdx.x >> 6) * 128);
}

// ---------------------------------------------------------------------------
// Single pass with a tree of tile totals
// ---------------------------------------------------------------------------

// The carry between tiles: fp64 for the float folds (so a chain of up to
// 2^31 tile sums adds no error that matters at fp32), the exact int64 for
// integers; a segmented scan's carry adds the segment-start flag.  `of`
// turns a tile total into a carry, `to` a carry into the fold state a tile
// continues from; `pack` / `unpack` give its kWords 32-bit words.
template <class Acc>
struct ScanCarry;

template <class T>
struct Carry64 {  // a 64-bit carry as two words
  static constexpr int kWords = 2;
  __device__ static void pack(T c, uint32_t (&w)[2]) {
    const uint64_t b = __builtin_bit_cast(uint64_t, c);
    w[0] = (uint32_t)b;
    w[1] = (uint32_t)(b >> 32);
  }
  __device__ static T unpack(const uint32_t* w) {
    return __builtin_bit_cast(T, (uint64_t)w[0] | ((uint64_t)w[1] << 32));
  }
};

template <>
struct ScanCarry<PlainAcc> : Carry64<double> {
  using T = double;
  __device__ static T zero() { return 0.0; }
  __device__ static T of(const PlainAcc& a) { return (double)a.s; }
  __device__ static PlainAcc to(T c) { return {(float)c}; }
  __device__ static T add(T a, T b) { return a + b; }
};
template <>
struct ScanCarry<CompAcc> : Carry64<double> {
  using T = double;
  __device__ static T zero() { return 0.0; }
  __device__ static T of(const CompAcc& a) {
    return __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
  }
  __device__ static CompAcc to(T c) {
    const float s = (float)c;
    return {s, __builtin_isfinite(s) ? (float)(c - (double)s) : 0.0f};
  }
  __device__ static T add(T a, T b) { return a + b; }
};
template <>
struct ScanCarry<IntAcc> : Carry64<uint64_t> {
  using T = uint64_t;
  __device__ static T zero() { return 0; }
  __device__ static T of(const IntAcc& a) { return a.s; }
  __device__ static IntAcc to(T c) { return {c}; }
  __device__ static T add(T a, T b) { return a + b; }
};
template <class Acc>
struct ScanCarry<SegAcc<Acc>> {
  using B = ScanCarry<Acc>;
  struct T {
    typename B::T v;
    uint32_t f;
  };
  static constexpr int kWords = 3;
  __device__ static T zero() { return {B::zero(), 0u}; }
  __device__ static T of(const SegAcc<Acc>& s) { return {B::of(s.a), s.f}; }
  __device__ static SegAcc<Acc> to(T c) { return {B::to(c.v), c.f}; }
  __device__ static T add(T x, T y) { return y.f ? y : T{B::add(x.v, y.v), x.f}; }
  __device__ static void pack(T c, uint32_t (&w)[3]) {
    uint32_t h[2];
    B::pack(c.v, h);
    w[0] = h[0];
    w[1] = h[1];
    w[2] = c.f;
  }
  __device__ static T unpack(const uint32_t* w) { return {B::unpack(w), w[2]}; }
};

// Look-back state in the workspace: the tree nodes (tree_nodes(tiles) of
// them, level by level), kWords 64-bit words each.  Every word holds one 32-bit part of the value below a
// ready flag (bit 32), so it is written and read by one single-copy-atomic
// access and no fence orders a value against a separate flag.  All words
// start at zero (scan_lb_clear_kernel runs first on the same stream).
struct ScanLB {
  uint32_t* ticket;  // next tile to hand out
  uint32_t* status;  // nonzero: a wait gave up (the result is invalid)
  uint64_t* node;    // level 0 (one node per tile), then levels 1, 2, ...
};

constexpr uint32_t kLookbackSpinLimit = 1u << 16;  // polls before giving up

static __global__ __launch_bounds__(256) void scan_lb_clear_kernel(uint64_t* w, int64_t nwords) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0;
}

template <int W>
__device__ __forceinline__ void lb_publish(uint64_t* node, const uint32_t (&v)[W]) {
#pragma unroll
  for (int k = 0; k < W; ++k)
    __hip_atomic_store(node + k, (uint64_t(1) << 32) | v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__device__ __forceinline__ bool lb_read(const uint64_t* node, uint32_t (&v)[W]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const uint64_t w = __hip_atomic_load(node + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v[k] = (uint32_t)w;
    ok = ok && (w >> 32) != 0;
  }
  return ok;
}

// The carry between tiles as a tree of radix 64 over the tile totals.  A
// level-0 node is one tile's total; the level-(k+1) node j is the fold of the
// level-k nodes 64 j .. 64 j + 63, i.e. of tiles [64^(k+1) j, 64^(k+1) (j+1)).
// With t written in base 64 as digits t_k, the exclusive carry of tile t is,
// for k = K-1 down to 0, the fold of the level-k nodes 64 (t >> 6(k+1)) + e,
// e < t_k: at most 63 nodes per level, which cover [0, t) left to right, so
// lane e of one wavefront polls node e of every level at once.  Tile t
// publishes its level-0 node before it waits; when t is the last tile of a
// level-(k+1) group (digits 0..k all 63) it also publishes that group's node,
// = (the 63 level-k terms of its own carry) + its own level-k node, as soon
// as those terms are in.  A node thus waits for at most k + 1 rounds of polls
// (K = 3 levels cover 262144 tiles), against log2(tiles) rounds of a binary
// tree.  Every node and carry is a fold in a fixed order (an ordered
// wavefront scan) of fixed values: the result does not depend on which tile
// finished first.  Tiles take their index from a ticket in launch order, so
// every node waited on belongs to a resident or finished tile and the waits
// end; the poll count is still bounded, and a give-up marks the status word
// (the carry is then invalid, but every node this tile owes is published so
// that no other tile waits for it).
constexpr int kTreeLevels = 5;  // 64^5 = 2^30 tiles; a launch has fewer than 2^26

__host__ __device__ constexpr int tree_levels(int64_t tiles) {
  int K = 1;
  while (K < kTreeLevels && ((int64_t)1 << (6 * K)) < tiles) ++K;
  return K;
}

// Nodes of all levels for `tiles` tiles (level k holds ceil(tiles / 64^k)).
__host__ __device__ constexpr int64_t tree_nodes(int64_t tiles) {
  int64_t sum = 0, cnt = tiles;
  for (int k = 0; k < tree_levels(tiles); ++k) {
    sum += cnt;
    cnt = (cnt + 63) >> 6;
  }
  return sum;
}

// Ordered fold of the values of lanes 0 .. m-1 (m >= 1, uniform), in lane
// order, returned in every lane.  Lane l's value is in words
// slot[i * 64 + l], i < kWords (LDS).
template <class C>
struct CarryFold {  // a carry with the merge interface of the scans
  typename C::T t;
  __device__ static CarryFold merge(const CarryFold& a, const CarryFold& b) { return {C::add(a.t, b.t)}; }
};

template <class C>
__device__ __forceinline__ typename C::T wave_ordered_fold(const uint32_t* slot, int m) {
  constexpr int W = C::kWords;
  const int lane = threadIdx.x & 63;
  uint32_t w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = slot[k * 64 + lane];
  const CarryFold<C> x = wave_incl_scan(CarryFold<C>{C::unpack(w)});  // lanes >= m never reach lane m - 1
  return read_lane(x, m - 1).t;
}

// Run by one whole wavefront; lane 0 publishes.  `tiles` is the grid size;
// `slots` (LDS, kTreeLevels * kWords * 64 words) keeps the polled values.
template <class C>
__device__ typename C::T scan_tree_carry(const ScanLB& lb, int64_t t, int64_t tiles, typename C::T own,
                                         uint32_t* slots) {
  constexpr int W = C::kWords;
  using T = typename C::T;
  const int lane = threadIdx.x & 63;
  const int K = tree_levels(tiles);
  // Level k starts at word start(k); node j of level k is at start(k) + W j.
  auto start = [&](int k) {
    int64_t off = 0, cnt = tiles;
    for (int j = 0; j < k; ++j) {
      off += (int64_t)W * cnt;
      cnt = (cnt + 63) >> 6;
    }
    return off;
  };
  auto digit = [&](int k) { return (int)((t >> (6 * k)) & 63); };
  auto publish = [&](int k, T x) {
    uint32_t w[W];
    C::pack(x, w);
    if (lane == 0) lb_publish<W>(lb.node + start(k) + (int64_t)W * (t >> (6 * k)), w);
  };
  publish(0, own);
  int P = 0;  // group nodes this tile owes: levels 1 .. P
  while (P < K - 1 && digit(P) == 63) ++P;
  uint32_t pend = 0;  // bit k: this lane still waits for its level-k node
  for (int k = 0; k < K; ++k)
    if (lane < digit(k)) pend |= 1u << k;
  T up = own;  // this tile's node at level `pub`
  int pub = 0;
  bool all = false;
  for (uint32_t polls = 0;; ++polls) {
    // Levels in groups of kBatch: the reads of a group are all issued before
    // any of them is examined, so a poll of K <= kBatch levels costs one round
    // trip (two-word carries; three-word carries take one level at a time to
    // spare registers).
    constexpr int kBatch = W == 2 ? 3 : 1;
    for (int k0 = 0; k0 < K; k0 += kBatch) {
      uint64_t got[kBatch][W];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int k = k0 + b;
        if (k < K && ((pend >> k) & 1u)) {
          const int64_t j = ((t >> (6 * (k + 1))) << 6) + lane;
#pragma unroll
          for (int i = 0; i < W; ++i)
            got[b][i] = __hip_atomic_load(lb.node + start(k) + (int64_t)W * j + i, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        }
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int k = k0 + b;
        if (k < K && ((pend >> k) & 1u)) {
          bool ok = true;
#pragma unroll
          for (int i = 0; i < W; ++i) ok = ok && (got[b][i] >> 32) != 0;
          if (ok) {
#pragma unroll
            for (int i = 0; i < W; ++i) slots[(k * W + i) * 64 + lane] = (uint32_t)got[b][i];
            pend &= ~(1u << k);
          }
        }
      }
    }
    for (; pub < P; ++pub) {
      if (__builtin_amdgcn_ballot_w64((pend >> pub) & 1u) != 0) break;
      up = C::add(wave_ordered_fold<C>(slots + pub * W * 64, 63), up);
      publish(pub + 1, up);
    }
    all = __builtin_amdgcn_ballot_w64(pend != 0) == 0;
    if (all || polls >= kLookbackSpinLimit) break;
    __builtin_amdgcn_s_sleep(1);
  }
  if (!all) {  // gave up: keep the others moving, flag the result
    for (; pub < P; ++pub) publish(pub + 1, own);
    if (lane == 0) __hip_atomic_store(lb.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return C::zero();
  }
  T carry = C::zero();
  bool any = false;
  for (int k = K - 1; k >= 0; --k) {
    const int m = digit(k);
    if (m == 0) continue;
    const T f = wave_ordered_fold<C>(slots + k * W * 64, m);
    carry = any ? C::add(carry, f) : f;
    any = true;
  }
  return carry;
}

// One tile per block; the tile index comes from the ticket, not blockIdx.
// Waves per SIMD the single-pass kernel is compiled for (1: the compiler's
// choice).  The plain segmented scan needs a few VGPRs over 64; holding it to
// 64 (two 1024-thread blocks per CU) spills 32 bytes per lane and still runs
// 18% faster.  The int64 scans would spill ~100 bytes per lane and slow down.
template <class Acc>
struct OnepassWaves : std::integral_constant<int, 1> {};
template <>
struct OnepassWaves<SegAcc<PlainAcc>> : std::integral_constant<int, 8> {};

template <class F, class S, class Acc, bool kAligned, bool kOutAligned>
  requires device_callable<F>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(OnepassWaves<Acc>::value))) void
scan_onepass_kernel(F f, const elem_t<S>* x, int64_t n, SegSpec seg,
                                                            ScanLB lb, typename ScanOut<Acc>::T* y, int exclusive) {
  using C = ScanCarry<Acc>;
  __shared__ Acc lds[kMaxWaves];
  __shared__ int64_t tile_sh;
  __shared__ typename C::T carry_sh;
  __shared__ uint32_t slots[kTreeLevels * C::kWords * 64];
  __shared__ uint32_t heads_sh[IsSeg<Acc>::value ? kTileWords : 1];
  __shared__ uint32_t wfirst_sh[kMaxWaves];
  __shared__ u32x4 stage_sh[kStageVecs<S, Acc>];
  __shared__ uint32_t park_sh[IsSeg<Acc>::value ? ScanWave<F, S, Acc>::kStashWords * 64 : 1];
  // The probes of the segment-start search do not depend on the tile: they
  // go out with the ticket.
  HeadProbe pr{0, 0};
  if constexpr (IsSeg<Acc>::value) pr = heads_probe(seg);
  if (threadIdx.x == 0) tile_sh = (int64_t)atomicAdd(lb.ticket, 1u);
  __syncthreads();
  const int64_t tile = tile_sh;
  auto w = scan_wave_at<F, S, Acc>(tile, n);
  w.template load<kAligned>(x, seg);
  if constexpr (IsSeg<Acc>::value)
    tile_heads(w, seg, pr, tile * blockDim.x * kScanE, (int64_t)blockDim.x * kScanE, heads_sh, wfirst_sh);
  w.fold(f);
  Acc total;
  const Acc before = block_wave_prefix(w.wave_total, lds, &total);
  if (threadIdx.x < 64) {
    // Segmented scans park wavefront 0's lane state in LDS while it polls:
    // the polls and the lane state together needed ~70 VGPRs, over the 64
    // that two 1024-thread blocks per CU allow.
    if constexpr (IsSeg<Acc>::value) w.stash(park_sh);
    const typename C::T carry = scan_tree_carry<C>(lb, tile, (int64_t)gridDim.x, C::of(total), slots);
    if (threadIdx.x == 0) carry_sh = carry;
    if constexpr (IsSeg<Acc>::value) w.unstash(park_sh);
  }
  __syncthreads();
  w.template emit<kOutAligned>(f, Acc::merge(C::to(carry_sh), before), exclusive, y,
                               stage_sh + (threadIdx.x >> 6) * 128);
}

}  // namespace hdc
