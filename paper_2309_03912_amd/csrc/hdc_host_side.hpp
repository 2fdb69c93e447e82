// The host side of the same callables.  The paper's subject is one generic
// callable usable from host and device code, with the execution space taken
// from the callable's type (section 2.10, "SFINAE 3 with macro"; the trait of
// appendix B).  These templates run the HstDev callables of the library on
// host memory through the very element semantics the kernels use (map_elem,
// fold_elem and the fold states are __host__ __device__); they are
// constrained to host_callable types, so a device-only callable is a compile
// error here exactly as a host-only one is in a kernel.
#pragma once

#include <cstdint>
#include <thread>
#include <vector>

#include "hdc_host.hpp"

namespace hdc {

// Elements per batch of the host loops: the batch evaluation (one
// coefficient at a time over the batch) is what the host compiler vectorizes.
constexpr int kHostBatch = 16;

template <class F, class S>
  requires host_callable<F>
void host_map_range(const F& f, const elem_t<S>* x, elem_t<S>* y, int64_t lo, int64_t hi) {
  int64_t i = lo;
  for (; i + kHostBatch <= hi; i += kHostBatch) {
    elem_t<S> in[kHostBatch], out[kHostBatch];
    for (int k = 0; k < kHostBatch; ++k) in[k] = x[i + k];
    map_batch<F, S>(f, in, out);
    for (int k = 0; k < kHostBatch; ++k) y[i + k] = out[k];
  }
  for (; i < hi; ++i) y[i] = map_elem<F, S>(f, x[i]);
}

// The fold of one block [b, e) of at most kHostBlock elements: element i
// goes to state (i - b) mod 4 (four independent chains), and the states meet
// as (0 + 1) + (2 + 3).  The result is a fixed function of the block's
// elements.
constexpr int64_t kHostBlock = 4096;

template <class F, class S, class Acc>
  requires host_callable<F>
Acc host_fold_block(const F& f, const elem_t<S>* x, const elem_t<S>* z, int64_t b, int64_t e) {
  Acc part[4] = {Acc::zero(), Acc::zero(), Acc::zero(), Acc::zero()};
  int64_t i = b;
  if constexpr (!std::is_same_v<S, I32> && !F::binary) {
    for (; i + kHostBatch <= e; i += kHostBatch) {  // the same terms as fold_elem, a batch at a time
      float t[kHostBatch];
      for (int k = 0; k < kHostBatch; ++k) t[k] = S::widen(x[i + k]);
      eval_batch(f, t);
      for (int k = 0; k < kHostBatch; ++k) part[k & 3].add(t[k]);
    }
  }
  for (; i < e; ++i) fold_elem<F, S>(part[(i - b) & 3], f, x[i], F::binary ? z[i] : x[i]);
  return Acc::merge(Acc::merge(part[0], part[1]), Acc::merge(part[2], part[3]));
}

// Split [0, n) into `parts` contiguous ranges; part p is [lo(p), lo(p+1)).
inline int64_t host_part_lo(int64_t n, int parts, int p) { return n / parts * p + (p < n % parts ? p : n % parts); }

inline int host_threads(int32_t requested, int64_t n) {
  int t = requested > 0 ? requested : (int)std::thread::hardware_concurrency();
  if (t < 1) t = 1;
  const int64_t min_per_thread = 1 << 16;
  if ((int64_t)t > (n + min_per_thread - 1) / min_per_thread) t = (int)((n + min_per_thread - 1) / min_per_thread);
  return t < 1 ? 1 : t;
}

template <class Fn>
void host_parallel(int parts, Fn&& fn) {
  if (parts == 1) {
    fn(0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(parts);
  for (int p = 0; p < parts; ++p) th.emplace_back([&fn, p] { fn(p); });
  for (auto& t : th) t.join();
}

template <class F, class S>
  requires host_callable<F>
void host_map(const F& f, const void* x, void* y, int64_t n, int32_t nthreads) {
  using T = elem_t<S>;
  const int parts = host_threads(nthreads, n);
  host_parallel(parts, [&](int p) {
    host_map_range<F, S>(f, (const T*)x, (T*)y, host_part_lo(n, parts, p), host_part_lo(n, parts, p + 1));
  });
}

// The array is cut into blocks of kHostBlock elements from its start; the
// threads fold disjoint runs of whole blocks, and one thread then merges the
// block states in a fixed order (plain: a pairwise tree in fp32;
// compensated: fp64 of s + c in block order; integers: wrapping).  So the
// result does not depend on the thread count.
template <class F, class S, class Acc>
  requires host_callable<F>
void host_reduce(const F& f, const void* x, const void* z, int64_t n, void* out, int32_t nthreads) {
  using T = elem_t<S>;
  const int64_t nb = (n + kHostBlock - 1) / kHostBlock;
  std::vector<Acc> blk((size_t)nb);
  const int parts = host_threads(nthreads, n);
  host_parallel(parts, [&](int p) {
    for (int64_t k = host_part_lo(nb, parts, p); k < host_part_lo(nb, parts, p + 1); ++k) {
      const int64_t e = n < (k + 1) * kHostBlock ? n : (k + 1) * kHostBlock;
      blk[(size_t)k] = host_fold_block<F, S, Acc>(f, (const T*)x, (const T*)z, k * kHostBlock, e);
    }
  });
  if constexpr (std::is_same_v<Acc, CompAcc>) {  // the cross-block combine in fp64, as on the device
    double t = 0.0;
    for (const Acc& a : blk) t += __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
    *static_cast<double*>(out) = t;
  } else {  // pairwise in a fixed tree over the blocks: short fp32 chains for any n
    for (size_t w = blk.size(); w > 1; w = (w + 1) / 2)
      for (size_t i = 0; i < w / 2; ++i) {
        blk[i] = Acc::merge(blk[2 * i], blk[2 * i + 1]);
        if (w % 2 && i + 1 == w / 2) blk[i + 1] = blk[w - 1];  // an odd last block moves up alone
      }
    const Acc total = blk.empty() ? Acc::zero() : blk[0];
    if constexpr (std::is_same_v<Acc, PlainAcc>)
      *static_cast<float*>(out) = total.s;
    else
      *static_cast<int64_t*>(out) = (int64_t)total.s;
  }
}

}  // namespace hdc
