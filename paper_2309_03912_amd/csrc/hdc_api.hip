// Host side of the library: argument checks, the functor-id -> concrete type
// dispatch, launch geometry, workspaces, tuning, and the C ABI of hdc.h.
//
// The dispatch is the paper's "deduce the execution space from the argument
// type" (section 2.10, "SFINAE 3 with macro") moved to a runtime boundary: a
// functor id selects one concrete HstDev-tagged type, and that type selects
// one kernel instantiation, once per call on the host.  Nothing is looked up
// per element.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "hdc.h"
#include "hdc_kernels.hpp"
#include "hdc_segmented.hpp"

using namespace hdc;

namespace {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

thread_local char g_last_error[512] = "";

hdc_status fail(hdc_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return s;
}

hdc_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return HDC_OK;
}

// ---------------------------------------------------------------------------
// Tuning
// ---------------------------------------------------------------------------

struct Tuning {
  int block = 256;
  int unroll = 4;
  int grid_mult = 8;
  int chunk = 4096;
  int small_seg = 128;
  int seg_per_wave = 8;
};

constexpr int kOps = 4, kDtypes = 6, kAccs = 3, kBuckets = 4;
std::mutex g_tune_mu;
Tuning g_tune[kOps][kDtypes][kAccs][kBuckets];

// Size bucket of a call: [0, 2^16), [2^16, 2^20), [2^20, 2^24), [2^24, inf).
int bucket_of(int64_t n) {
  if (n < (int64_t(1) << 16)) return 0;
  if (n < (int64_t(1) << 20)) return 1;
  if (n < (int64_t(1) << 24)) return 2;
  return 3;
}

bool valid_class(int op, int dt, int acc, int bucket) {
  return op >= 0 && op < kOps && dt >= 0 && dt < kDtypes && acc >= 0 && acc < kAccs && bucket >= -1 &&
         bucket < kBuckets;
}
std::once_flag g_tune_once;

bool valid_tuning(const Tuning& t) {
  auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  return t.block >= 64 && t.block <= 1024 && t.block % 64 == 0 &&
         (t.unroll == 1 || t.unroll == 2 || t.unroll == 4 || t.unroll == 8) && t.grid_mult >= 1 &&
         t.grid_mult <= 64 && pow2(t.chunk) && t.chunk >= 1024 && t.chunk <= 65536 && t.small_seg >= 0 &&
         t.small_seg <= 1024 && pow2(t.seg_per_wave) && t.seg_per_wave <= 64;
}

hdc_status load_tuning_file(const char* path) {
  FILE* fp = fopen(path, "r");
  if (!fp) return HDC_OK;
  char line[256];
  int lineno = 0;
  hdc_status st = HDC_OK;
  while (fgets(line, sizeof line, fp)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    int op, dt, acc, bucket;
    Tuning t;
    if (sscanf(line, "%d %d %d %d %d %d %d %d %d %d", &op, &dt, &acc, &bucket, &t.block, &t.unroll,
               &t.grid_mult, &t.chunk, &t.small_seg, &t.seg_per_wave) != 10 ||
        !valid_class(op, dt, acc, bucket) || bucket < 0 || !valid_tuning(t)) {
      st = fail(HDC_ERR_INVALID_ARGUMENT, "tuning cache %s: bad line %d", path, lineno);
      continue;
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[op][dt][acc][bucket] = t;
  }
  fclose(fp);
  return st;
}

// The cache named by HDC_TUNE_CACHE is read once, before the first lookup.
void ensure_tuning_loaded() {
  std::call_once(g_tune_once, [] {
    const char* p = getenv("HDC_TUNE_CACHE");
    if (p && *p) load_tuning_file(p);
  });
}

Tuning tuning_for(int op, hdc_dtype dt, hdc_accum acc, int64_t n) {
  ensure_tuning_loaded();
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune[op][dt][acc][bucket_of(n)];
}

// ---------------------------------------------------------------------------
// Device facts
// ---------------------------------------------------------------------------

constexpr int kMaxDevices = 64;
int g_cus[kMaxDevices];  // 0 = not queried yet

hdc_status compute_units(int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HDC_ERR_HIP, "device index %d out of range", dev);
  if (g_cus[dev] == 0) {
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    g_cus[dev] = v;
  }
  *cus = g_cus[dev];
  return HDC_OK;
}

// ---------------------------------------------------------------------------
// Workspaces
// ---------------------------------------------------------------------------

constexpr int64_t kMaxGrid = 65536;  // upper bound on pass-1 blocks
constexpr size_t kPartialBytes = 8;  // every fold state fits 8 bytes

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t reduce_workspace_bytes() { return round_up(kMaxGrid * kPartialBytes, 256); }

constexpr int64_t kMinChunk = 1024;

// Layout of the segmented workspace for a given chunk (sections 256-byte aligned).
struct SegLayout {
  size_t cnt, full, part, long_base, long_list, partials, bytes;
  int64_t cap_full, cap_part, cap_partials;
};

SegLayout seg_layout(int64_t total, int64_t S, int64_t chunk) {
  SegLayout l{};
  l.cap_full = total / chunk + 1;
  l.cap_part = S > 0 ? S : 1;
  l.cap_partials = l.cap_full + l.cap_part;
  size_t o = 0;
  l.cnt = o;       o += round_up(sizeof(SegCounters), 256);
  l.full = o;      o += round_up((size_t)l.cap_full * sizeof(SegPiece), 256);
  l.part = o;      o += round_up((size_t)l.cap_part * sizeof(SegPiece), 256);
  l.long_base = o; o += round_up((size_t)l.cap_part * sizeof(int32_t), 256);
  l.long_list = o; o += round_up((size_t)l.cap_part * sizeof(int32_t), 256);
  l.partials = o;  o += round_up((size_t)l.cap_partials * kPartialBytes, 256);
  l.bytes = o;
  return l;
}

struct InternalWs {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, void*>, InternalWs> g_ws;

// Resolve the workspace of a call: the caller's, or the library's buffer for
// (device, stream), grown when needed and allowed.
hdc_status resolve_workspace(void* ws, size_t ws_bytes, size_t need, hipStream_t stream, void** out) {
  if (ws) {
    if (ws_bytes < need)
      return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes,
                  need);
    *out = ws;
    return HDC_OK;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> g(g_ws_mu);
  InternalWs& w = g_ws[{dev, (void*)stream}];
  if (w.bytes < need) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipStreamIsCapturing: %s", hipGetErrorString(e));
    if (cs != hipStreamCaptureStatusNone)
      return fail(HDC_ERR_WORKSPACE, "the library workspace must grow, which is impossible while the stream is "
                                     "being captured: pass a workspace");
    if (w.ptr) {
      e = hipStreamSynchronize(stream);  // the old buffer may still be in use
      if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
      (void)hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t bytes = round_up(need, 1 << 20);
    e = hipMalloc(&w.ptr, bytes);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    e = hipMemset(w.ptr, 0, bytes);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipMemset: %s", hipGetErrorString(e));
    w.bytes = bytes;
  }
  *out = w.ptr;
  return HDC_OK;
}

// ---------------------------------------------------------------------------
// Argument checks
// ---------------------------------------------------------------------------

size_t elem_size(hdc_dtype dt) {
  switch (dt) {
    case HDC_F32: case HDC_I32: return 4;
    case HDC_F16: case HDC_BF16: return 2;
    case HDC_I64: case HDC_F64: return 8;
  }
  return 0;
}

bool is_float(hdc_dtype dt) { return dt == HDC_F32 || dt == HDC_F16 || dt == HDC_BF16; }

hdc_status check_functor(const hdc_functor* f, hdc_dtype dt, bool allow_product) {
  if (!f) return fail(HDC_ERR_INVALID_ARGUMENT, "functor is NULL");
  if ((int)dt < 0 || (int)dt > (int)HDC_F64) return fail(HDC_ERR_INVALID_ARGUMENT, "unknown dtype %d", (int)dt);
  switch (f->id) {
    case HDC_FN_IDENTITY:
    case HDC_FN_AFFINE:
      if (!is_float(dt) && dt != HDC_I32) return fail(HDC_ERR_UNSUPPORTED, "dtype %d is not provided", (int)dt);
      return HDC_OK;
    case HDC_FN_HORNER:
      if (!is_float(dt)) return fail(HDC_ERR_UNSUPPORTED, "HORNER needs floating-point storage");
      if (f->degree < 0 || f->degree > HDC_MAX_DEGREE)
        return fail(HDC_ERR_INVALID_ARGUMENT, "HORNER degree %d outside 0..%d", f->degree, HDC_MAX_DEGREE);
      return HDC_OK;
    case HDC_FN_PRODUCT:
      if (!allow_product) return fail(HDC_ERR_UNSUPPORTED, "PRODUCT is a two-operand fold term only");
      if (!is_float(dt)) return fail(HDC_ERR_UNSUPPORTED, "PRODUCT needs floating-point storage");
      return HDC_OK;
    default:
      return fail(HDC_ERR_INVALID_ARGUMENT, "unknown functor id %d", f->id);
  }
}

hdc_status check_acc(hdc_dtype dt, hdc_accum acc) {
  if (acc != HDC_ACC_PLAIN && acc != HDC_ACC_COMPENSATED && acc != HDC_ACC_EXACT_INT)
    return fail(HDC_ERR_INVALID_ARGUMENT, "unknown accumulation %d", (int)acc);
  if (is_float(dt) && acc == HDC_ACC_EXACT_INT)
    return fail(HDC_ERR_UNSUPPORTED, "EXACT_INT needs int32 storage");
  if (dt == HDC_I32 && acc != HDC_ACC_EXACT_INT)
    return fail(HDC_ERR_UNSUPPORTED, "int32 storage folds with EXACT_INT only");
  return HDC_OK;
}

hdc_status check_ptr(const void* p, hdc_dtype dt, int64_t n, const char* name) {
  if (n > 0 && !p) return fail(HDC_ERR_INVALID_ARGUMENT, "%s is NULL with n = %lld", name, (long long)n);
  if (p && (uintptr_t)p % elem_size(dt) != 0)
    return fail(HDC_ERR_INVALID_ARGUMENT, "%s is not aligned to its element size", name);
  return HDC_OK;
}

#define HDC_TRY(expr)                 \
  do {                                \
    hdc_status s_ = (expr);           \
    if (s_ != HDC_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------
// Functor id -> concrete type; dtype -> storage type
// ---------------------------------------------------------------------------

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

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------

template <class S>
Range make_range(const void* x, int64_t n, bool vector) {
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

int64_t grid_for(int64_t units, int64_t per_block, int cus, const Tuning& t) {
  int64_t g = (units + per_block - 1) / per_block;
  int64_t cap = (int64_t)cus * t.grid_mult;
  if (cap > kMaxGrid) cap = kMaxGrid;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return g;
}

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
  reduce_final_kernel<Acc><<<dim3(1), dim3(256), 0, st>>>(partials, (int)g, out);
  return check_launch("final combine launch");
}

template <class F, class S, class Acc, class FM = Identity, bool kMap = false>
hdc_status launch_reduce(const F& f, const void* x, const void* z, int64_t n, void* out, void* ws,
                         const Tuning& t, hipStream_t st, const FM& fm = FM{}, void* y = nullptr) {
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
  auto go = [&](auto U) {
    constexpr int kU = decltype(U)::value;
    if (vec)
      reduce_kernel<F, S, Acc, kU, true, FM, kMap><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(
          f, (const T*)x, (const T*)z, r, partials, fm, (T*)y);
    else
      reduce_kernel<F, S, Acc, kU, false, FM, kMap><<<dim3((unsigned)g), dim3(t.block), 0, st>>>(
          f, (const T*)x, (const T*)z, r, partials, fm, (T*)y);
  };
  switch (t.unroll) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: go(std::integral_constant<int, 8>{}); break;
  }
  HDC_TRY(check_launch("reduce kernel launch"));
  return launch_final<Acc>(partials, g, out, st);
}


template <class F, class S, class Acc>
hdc_status launch_segmented(const F& f, const void* x, const int64_t* off, int64_t nseg, int64_t total, void* out,
                            void* ws, const Tuning& t, hipStream_t st) {
  using T = typename S::T;
  int cus = 0;
  HDC_TRY(compute_units(&cus));
  const SegLayout l = seg_layout(total, nseg, t.chunk);
  char* base = static_cast<char*>(ws);
  SegPlan p;
  p.cnt = reinterpret_cast<SegCounters*>(base + l.cnt);
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

  seg_reset_kernel<<<dim3(1), dim3(64), 0, st>>>(p.cnt);
  HDC_TRY(check_launch("segmented reset launch"));
  seg_plan_kernel<<<dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st>>>(off, nseg, p);
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

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

hdc_status hdc_map(const hdc_functor* f, hdc_dtype dt, const void* x, void* y, int64_t n, void* stream) {
  HDC_TRY(check_functor(f, dt, false));
  if (n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "n = %lld is negative", (long long)n);
  HDC_TRY(check_ptr(x, dt, n, "x"));
  HDC_TRY(check_ptr(y, dt, n, "y"));
  if (n == 0) return HDC_OK;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y, len = (uintptr_t)n * elem_size(dt);
  if (xb != yb && xb < yb + len && yb < xb + len)
    return fail(HDC_ERR_INVALID_ARGUMENT, "x and y overlap partially");
  const Tuning t = tuning_for(HDC_OP_MAP, dt, HDC_ACC_PLAIN, n);
  hipStream_t st = (hipStream_t)stream;
  if (dt == HDC_I32)
    return with_int_fn(*f, [&](auto fn) { return launch_map<decltype(fn), I32>(fn, x, y, n, t, st); });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(*f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary)
        return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
      else
        return launch_map<F, S>(fn, x, y, n, t, st);
    });
  });
}

static hdc_status reduce_common(const hdc_functor* f, const hdc_functor* fm, hdc_dtype dt, const void* x,
                                const void* z, void* y, int64_t n, hdc_accum acc, void* out, void* workspace,
                                size_t ws_bytes, void* stream) {
  const bool fused = fm != nullptr;
  HDC_TRY(check_functor(f, dt, !fused));
  if (fused) HDC_TRY(check_functor(fm, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "n = %lld is negative", (long long)n);
  HDC_TRY(check_ptr(x, dt, n, "x"));
  if (f->id == HDC_FN_PRODUCT) {
    if (!z && n > 0) return fail(HDC_ERR_UNSUPPORTED, "PRODUCT needs the second operand z");
    HDC_TRY(check_ptr(z, dt, n, "z"));
  }
  if (fused) {
    HDC_TRY(check_ptr(y, dt, n, "y"));
    const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y, len = (uintptr_t)n * elem_size(dt);
    if (n > 0 && xb != yb && xb < yb + len && yb < xb + len)
      return fail(HDC_ERR_INVALID_ARGUMENT, "x and y overlap partially");
    if (n > 0 && xb == yb) return fail(HDC_ERR_INVALID_ARGUMENT, "map_reduce cannot run in place");
  }
  if (!out) return fail(HDC_ERR_INVALID_ARGUMENT, "out is NULL");
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  HDC_TRY(resolve_workspace(workspace, ws_bytes, reduce_workspace_bytes(), st, &ws));
  const Tuning t = tuning_for(fused ? HDC_OP_MAP_REDUCE : HDC_OP_TRANSFORM_REDUCE, dt, acc, n);

  if (dt == HDC_I32) {
    return with_int_fn(*f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if (!fused) return launch_reduce<F, I32, IntAcc>(fn, x, z, n, out, ws, t, st);
      return with_int_fn(*fm, [&](auto mfn) {
        return launch_reduce<F, I32, IntAcc, decltype(mfn), true>(fn, x, z, n, out, ws, t, st, mfn, y);
      });
    });
  }
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(*f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      auto run = [&](auto a) -> hdc_status {
        using Acc = decltype(a);
        if (!fused) return launch_reduce<F, S, Acc>(fn, x, z, n, out, ws, t, st);
        if constexpr (F::binary) {
          return fail(HDC_ERR_UNSUPPORTED, "map_reduce folds one operand");
        } else {
          return with_float_fn(*fm, [&](auto mfn) -> hdc_status {
            using FM = decltype(mfn);
            if constexpr (FM::binary)
              return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
            else
              return launch_reduce<F, S, Acc, FM, true>(fn, x, z, n, out, ws, t, st, mfn, y);
          });
        }
      };
      if (acc == HDC_ACC_COMPENSATED) return run(CompAcc{});
      return run(PlainAcc{});
    });
  });
}

hdc_status hdc_transform_reduce(const hdc_functor* f, hdc_dtype dt, const void* x, const void* z, int64_t n,
                                hdc_accum acc, void* out, void* workspace, size_t ws_bytes, void* stream) {
  return reduce_common(f, nullptr, dt, x, z, nullptr, n, acc, out, workspace, ws_bytes, stream);
}

hdc_status hdc_map_reduce(const hdc_functor* f, const hdc_functor* g, hdc_dtype dt, const void* x, void* y,
                          int64_t n, hdc_accum acc, void* out, void* workspace, size_t ws_bytes, void* stream) {
  if (!f) return fail(HDC_ERR_INVALID_ARGUMENT, "map functor is NULL");
  return reduce_common(g, f, dt, x, nullptr, y, n, acc, out, workspace, ws_bytes, stream);
}

hdc_status hdc_segmented_reduce(const hdc_functor* f, hdc_dtype dt, const void* x, const int64_t* offsets,
                                int64_t num_segments, int64_t total, hdc_accum acc, void* out, void* workspace,
                                size_t ws_bytes, void* stream) {
  HDC_TRY(check_functor(f, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (num_segments < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "num_segments is negative");
  if (num_segments >= INT32_MAX) return fail(HDC_ERR_INVALID_ARGUMENT, "more than 2^31 - 2 segments");
  if (total < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "total is negative");
  if (total / kMinChunk >= INT32_MAX / 2) return fail(HDC_ERR_INVALID_ARGUMENT, "total is too large");
  if (num_segments == 0) return HDC_OK;
  if (!offsets) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is NULL");
  if ((uintptr_t)offsets % 8) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is not 8-byte aligned");
  HDC_TRY(check_ptr(x, dt, total, "x"));
  if (!out) return fail(HDC_ERR_INVALID_ARGUMENT, "out is NULL");
  const size_t osz = acc == HDC_ACC_PLAIN ? 4 : 8;
  if ((uintptr_t)out % osz) return fail(HDC_ERR_INVALID_ARGUMENT, "out is not aligned to its element size");
  hipStream_t st = (hipStream_t)stream;
  const Tuning t = tuning_for(HDC_OP_SEGMENTED_REDUCE, dt, acc, total);
  void* ws = nullptr;
  HDC_TRY(resolve_workspace(workspace, ws_bytes, seg_layout(total, num_segments, t.chunk).bytes, st, &ws));
  if ((uintptr_t)ws % 256) return fail(HDC_ERR_INVALID_ARGUMENT, "workspace is not 256-byte aligned");

  if (dt == HDC_I32)
    return with_int_fn(*f, [&](auto fn) {
      return launch_segmented<decltype(fn), I32, IntAcc>(fn, x, offsets, num_segments, total, out, ws, t, st);
    });
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(*f, [&](auto fn) -> hdc_status {
      using F = decltype(fn);
      if constexpr (F::binary) {
        return fail(HDC_ERR_UNSUPPORTED, "PRODUCT is not a segmented fold term");
      } else {
        if (acc == HDC_ACC_COMPENSATED)
          return launch_segmented<F, S, CompAcc>(fn, x, offsets, num_segments, total, out, ws, t, st);
        return launch_segmented<F, S, PlainAcc>(fn, x, offsets, num_segments, total, out, ws, t, st);
      }
    });
  });
}

hdc_status hdc_workspace_size(int op, hdc_dtype dt, hdc_accum acc, int64_t n, int64_t num_segments,
                              size_t* bytes) {
  if (!bytes) return fail(HDC_ERR_INVALID_ARGUMENT, "bytes is NULL");
  if (n < 0 || num_segments < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "negative size");
  (void)dt;
  (void)acc;
  switch (op) {
    case HDC_OP_MAP: *bytes = 0; return HDC_OK;
    case HDC_OP_TRANSFORM_REDUCE:
    case HDC_OP_MAP_REDUCE: *bytes = reduce_workspace_bytes(); return HDC_OK;
    case HDC_OP_SEGMENTED_REDUCE:
      if (n / kMinChunk >= INT32_MAX / 2 || num_segments >= INT32_MAX)
        return fail(HDC_ERR_INVALID_ARGUMENT, "sizes too large");
      *bytes = seg_layout(n, num_segments, kMinChunk).bytes;  // enough for every chunk setting
      return HDC_OK;
  }
  return fail(HDC_ERR_INVALID_ARGUMENT, "unknown op %d", op);
}

hdc_status hdc_validate_offsets(const int64_t* offsets, int64_t num_segments, int64_t total, void* stream) {
  if (num_segments < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "num_segments is negative");
  if (!offsets) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is NULL");
  const size_t bytes = (size_t)(num_segments + 1) * sizeof(int64_t);
  int64_t* h = (int64_t*)malloc(bytes);
  if (!h) return fail(HDC_ERR_INVALID_ARGUMENT, "host allocation of %zu bytes failed", bytes);
  hipError_t e = hipMemcpyAsync(h, offsets, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    free(h);
    return fail(HDC_ERR_HIP, "copying offsets: %s", hipGetErrorString(e));
  }
  hdc_status st = HDC_OK;
  if (h[0] < 0) st = fail(HDC_ERR_INVALID_ARGUMENT, "offsets[0] = %lld is negative", (long long)h[0]);
  for (int64_t j = 0; st == HDC_OK && j < num_segments; ++j)
    if (h[j + 1] < h[j]) st = fail(HDC_ERR_INVALID_ARGUMENT, "offsets decrease at segment %lld", (long long)j);
  if (st == HDC_OK && h[num_segments] > total)
    st = fail(HDC_ERR_INVALID_ARGUMENT, "offsets[S] = %lld exceeds total %lld", (long long)h[num_segments],
              (long long)total);
  free(h);
  return st;
}

hdc_status hdc_set_tuning(int op, hdc_dtype dt, hdc_accum acc, int bucket, const hdc_tuning* t) {
  if (!t) return fail(HDC_ERR_INVALID_ARGUMENT, "tuning is NULL");
  if (!valid_class(op, (int)dt, (int)acc, bucket)) return fail(HDC_ERR_INVALID_ARGUMENT, "no such tuning class");
  ensure_tuning_loaded();  // so that the cache cannot override this later
  std::lock_guard<std::mutex> g(g_tune_mu);
  const int lo = bucket < 0 ? 0 : bucket, hi = bucket < 0 ? kBuckets : bucket + 1;
  Tuning upd[kBuckets];
  for (int b = lo; b < hi; ++b) {
    Tuning n = g_tune[op][dt][acc][b];
    if (t->block) n.block = t->block;
    if (t->unroll) n.unroll = t->unroll;
    if (t->grid_mult) n.grid_mult = t->grid_mult;
    if (t->chunk) n.chunk = t->chunk;
    if (t->small_seg) n.small_seg = t->small_seg;
    if (t->seg_per_wave) n.seg_per_wave = t->seg_per_wave;
    if (!valid_tuning(n)) return fail(HDC_ERR_INVALID_ARGUMENT, "tuning values out of range");
    upd[b] = n;
  }
  for (int b = lo; b < hi; ++b) g_tune[op][dt][acc][b] = upd[b];
  return HDC_OK;
}

hdc_status hdc_get_tuning(int op, hdc_dtype dt, hdc_accum acc, int bucket, hdc_tuning* t) {
  if (!t) return fail(HDC_ERR_INVALID_ARGUMENT, "tuning is NULL");
  if (!valid_class(op, (int)dt, (int)acc, bucket) || bucket < 0)
    return fail(HDC_ERR_INVALID_ARGUMENT, "no such tuning class");
  ensure_tuning_loaded();
  std::lock_guard<std::mutex> g(g_tune_mu);
  const Tuning& c = g_tune[op][dt][acc][bucket];
  t->block = c.block;
  t->unroll = c.unroll;
  t->grid_mult = c.grid_mult;
  t->chunk = c.chunk;
  t->small_seg = c.small_seg;
  t->seg_per_wave = c.seg_per_wave;
  return HDC_OK;
}

hdc_status hdc_tuning_bucket(int64_t n, int32_t* bucket) {
  if (!bucket || n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "bad arguments");
  *bucket = bucket_of(n);
  return HDC_OK;
}

hdc_status hdc_load_tuning(const char* path) {
  if (!path) path = getenv("HDC_TUNE_CACHE");
  if (!path || !*path) return HDC_OK;
  return load_tuning_file(path);
}

const char* hdc_status_string(hdc_status s) {
  switch (s) {
    case HDC_OK: return "HDC_OK";
    case HDC_ERR_INVALID_ARGUMENT: return "HDC_ERR_INVALID_ARGUMENT";
    case HDC_ERR_UNSUPPORTED: return "HDC_ERR_UNSUPPORTED";
    case HDC_ERR_WORKSPACE: return "HDC_ERR_WORKSPACE";
    case HDC_ERR_HIP: return "HDC_ERR_HIP";
  }
  return "unknown hdc_status";
}

const char* hdc_last_error(void) { return g_last_error; }

int32_t hdc_version(void) { return 100; }

}  // extern "C"
