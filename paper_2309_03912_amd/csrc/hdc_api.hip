// Host side of the library: the C ABI of hdc.h, argument checks, workspaces
// and tuning.  The functor-id -> concrete type dispatch and the launches live
// in the per-family translation units (hdc_run_*.hip).
//
// The dispatch is the paper's "deduce the execution space from the argument
// type" (section 2.10, "SFINAE 3 with macro") moved to a runtime boundary: a
// functor id selects one concrete HstDev-tagged type, and that type selects
// one kernel instantiation, once per call on the host.  Nothing is looked up
// per element.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <unordered_map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hdc.h"
#include "hdc_batch.hpp"
#include "hdc_host.hpp"

namespace hdc {

// ---------------------------------------------------------------------------
// Errors and device facts (shared with the launcher translation units)
// ---------------------------------------------------------------------------

namespace {
thread_local char g_last_error[512] = "";
}  // namespace

hdc_status fail(hdc_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return s;
}

namespace {
constexpr int kMaxDevices = 64;
// Compute units per device; 0 = not queried yet.  Concurrent first calls may
// both query and store the same value, so the accesses are atomic.
std::atomic<int> g_cus[kMaxDevices];
}  // namespace

hdc_status compute_units(int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HDC_ERR_HIP, "device index %d out of range", dev);
  int v = g_cus[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    g_cus[dev].store(v, std::memory_order_relaxed);
  }
  *cus = v;
  return HDC_OK;
}

}  // namespace hdc

using namespace hdc;

namespace {

// ---------------------------------------------------------------------------
// Tuning
// ---------------------------------------------------------------------------

constexpr int kOps = 7, kDtypes = 6, kAccs = 4, kBuckets = 4;
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
         t.small_seg <= 1024 && pow2(t.seg_per_wave) && t.seg_per_wave <= 64 && (t.passes == 1 || t.passes == 2);
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
    Tuning t;  // a line without the last field (passes) keeps its default
    const int got = sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d", &op, &dt, &acc, &bucket, &t.block, &t.unroll,
                           &t.grid_mult, &t.chunk, &t.small_seg, &t.seg_per_wave, &t.passes);
    if ((got != 10 && got != 11) || !valid_class(op, dt, acc, bucket) || bucket < 0 || !valid_tuning(t)) {
      st = fail(HDC_ERR_INVALID_ARGUMENT, "tuning cache %s: bad line %d", path, lineno);
      continue;
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[op][dt][acc][bucket] = t;
  }
  fclose(fp);
  return st;
}

// HDC_LOG set to anything but "0": one line per dispatch decision on stderr.
bool log_on() {
  static const bool on = [] {
    const char* p = getenv("HDC_LOG");
    return p && *p && strcmp(p, "0") != 0;
  }();
  return on;
}

void log_line(const char* fmt, ...) {
  if (!log_on()) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  va_list ap;
  va_start(ap, fmt);
  fputs("hdc: ", stderr);
  vfprintf(stderr, fmt, ap);
  fputc('\n', stderr);
  va_end(ap);
}

const char* dtype_name(hdc_dtype dt) {
  switch (dt) {
    case HDC_F32: return "f32";
    case HDC_F16: return "f16";
    case HDC_BF16: return "bf16";
    case HDC_I32: return "i32";
    default: return "?";
  }
}

const char* acc_name(hdc_accum acc) {
  switch (acc) {
    case HDC_ACC_PLAIN: return "plain";
    case HDC_ACC_COMPENSATED: return "compensated";
    case HDC_ACC_EXACT_INT: return "exact_int";
    case HDC_ACC_EXACT: return "exact";
    default: return "?";
  }
}

// The decision of one call: operation, types, size and its bucket, the
// tuning taken, the schedule it selects and where the workspace came from.
void log_dispatch(const char* op, hdc_dtype dt, hdc_accum acc, int64_t n, const Tuning& t, const char* schedule,
                  const char* ws_from) {
  if (!log_on()) return;
  log_line("%s dtype=%s acc=%s n=%lld bucket=%d block=%d unroll=%d grid_mult=%d chunk=%d small_seg=%d "
           "seg_per_wave=%d passes=%d schedule=%s workspace=%s",
           op, dtype_name(dt), acc_name(acc), (long long)n, bucket_of(n), t.block, t.unroll, t.grid_mult, t.chunk,
           t.small_seg, t.seg_per_wave, t.passes, schedule, ws_from);
}

// HDC_TUNE=0: no tuning cache is read at start-up (HDC_TUNE_CACHE is
// ignored); the built-in defaults apply until a caller loads or sets tuning
// explicitly.
bool tune_cache_on() {
  const char* p = getenv("HDC_TUNE");
  return !(p && strcmp(p, "0") == 0);
}

// Defaults are set, and the cache named by HDC_TUNE_CACHE read, once: before
// the first lookup and before any explicit load or set, so neither can be
// overwritten by the defaults afterwards.
void ensure_tuning_loaded() {
  std::call_once(g_tune_once, [] {
    // defaults that differ from the struct's: scans use 1024-thread tiles
    // (16384 elements), so one block scans the tile sums of 2^28 elements
    for (auto& per_dt : g_tune[HDC_OP_SCAN])
      for (auto& per_acc : per_dt)
        for (Tuning& t : per_acc) t.block = 1024;
    // grouped batches fold chunks of 32768 elements (one partial per chunk)
    for (auto& per_dt : g_tune[HDC_OP_BATCH])
      for (auto& per_acc : per_dt)
        for (Tuning& t : per_acc) t.chunk = 32768;
    const char* p = getenv("HDC_TUNE_CACHE");
    if (p && *p) {
      if (!tune_cache_on()) {
        log_line("HDC_TUNE=0: tuning cache %s not read, built-in defaults", p);
      } else {
        const hdc_status r = load_tuning_file(p);
        log_line("tuning cache %s read at start-up: %s", p, hdc_status_string(r));
      }
    }
  });
}

Tuning tuning_for(int op, hdc_dtype dt, hdc_accum acc, int64_t n) {
  ensure_tuning_loaded();
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune[op][dt][acc][bucket_of(n)];
}

// ---------------------------------------------------------------------------
// Workspaces
// ---------------------------------------------------------------------------

struct InternalWs {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, void*>, InternalWs> g_ws;
// Buffers replaced by a larger one are kept until the process ends: work
// already enqueued (possibly by another host thread on the same stream) may
// still use them.  Growth at least doubles, so this at most doubles the total.
std::vector<void*> g_ws_retired;

// Resolve the workspace of a call: the caller's, or the library's buffer for
// (device, stream), grown when needed and allowed.
hdc_status resolve_workspace(void* ws, size_t ws_bytes, size_t need, hipStream_t stream, void** out) {
  if (ws) {
    if ((uintptr_t)ws % 256 != 0) return fail(HDC_ERR_INVALID_ARGUMENT, "workspace is not 256-byte aligned");
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
    size_t bytes = round_up(need > 2 * w.bytes ? need : 2 * w.bytes, 1 << 20);
    void* fresh = nullptr;
    e = hipMalloc(&fresh, bytes);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    if (w.ptr) g_ws_retired.push_back(w.ptr);
    w.ptr = fresh;
    w.bytes = bytes;
  }
  *out = w.ptr;
  return HDC_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free transform_reduce
// ---------------------------------------------------------------------------

// The pass-1 partials of hdc_transform_reduce_noalloc: one 32-byte fold
// state per block, for the most blocks any call launches (kMaxGrid).  Each
// device holds its own copy from module load until the process ends.  In
// host code `scratch` names a host-side shadow, never the device memory:
// the kernels get the device address that hipGetSymbolAddress returns.
constexpr size_t kScratchBytes = size_t(2) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, null until set up

// The device address of the current device's `scratch`, looked up once per
// device with that device current.
hdc_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HDC_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HDC_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HDC_OK;
}

// ---------------------------------------------------------------------------
// Tickets of the one-launch reductions
// ---------------------------------------------------------------------------

// A one-launch reduction counts its finished blocks on a ticket (a launch
// epoch and an arrival count) whose count must be 0 when the kernel starts;
// the block that arrives last folds the partials and moves the ticket to the
// next epoch with a count of 0.  The tickets are library-owned device memory
// (an object of static storage, so zero-initialized when the code object is
// loaded), one per workspace buffer: calls that share a workspace are ordered
// on one stream, so they never use one ticket at the same time, while calls
// on different workspaces never share one.  Once every slot of a device is
// taken, calls with new workspace buffers use the two-launch form.
constexpr int kTicketSlots = 1 << 16;
static __device__ uint64_t tickets[kTicketSlots];

struct TicketTable {
  uint64_t* base = nullptr;  // device address of `tickets` on this device
  std::unordered_map<const void*, int> slot;
};
std::mutex g_ticket_mu;
TicketTable g_ticket_tables[kMaxDevices];

// The ticket of workspace buffer `ws` on the current device, or NULL when
// no slot is left.
hdc_status ticket_for(const void* ws, uint64_t** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HDC_ERR_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> g(g_ticket_mu);
  TicketTable& tt = g_ticket_tables[dev];
  if (!tt.base) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(tickets));
    if (e != hipSuccess || !p) return fail(HDC_ERR_HIP, "hipGetSymbolAddress(tickets): %s", hipGetErrorString(e));
    tt.base = static_cast<uint64_t*>(p);
  }
  auto it = tt.slot.find(ws);
  if (it == tt.slot.end()) {
    if (tt.slot.size() >= (size_t)kTicketSlots) return HDC_OK;
    it = tt.slot.emplace(ws, (int)tt.slot.size()).first;
  }
  *out = tt.base + it->second;
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
  if (acc != HDC_ACC_PLAIN && acc != HDC_ACC_COMPENSATED && acc != HDC_ACC_EXACT_INT && acc != HDC_ACC_EXACT)
    return fail(HDC_ERR_INVALID_ARGUMENT, "unknown accumulation %d", (int)acc);
  if (acc == HDC_ACC_EXACT && dt != HDC_F16 && dt != HDC_BF16)
    return fail(HDC_ERR_UNSUPPORTED, "EXACT needs fp16 or bf16 storage");
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
  log_dispatch("map", dt, HDC_ACC_PLAIN, n, t,
               ((uintptr_t)x % 16) == ((uintptr_t)y % 16) ? "16-byte vectors" : "scalar (x, y misaligned)", "none");
  hipStream_t st = (hipStream_t)stream;
  return run_map(*f, dt, x, y, n, t, st);
}

// `noalloc`: the partials go to the library's scratch array (workspace and
// ws_bytes are ignored).
static hdc_status reduce_common(const hdc_functor* f, const hdc_functor* fm, hdc_dtype dt, const void* x,
                                const void* z, void* y, int64_t n, hdc_accum acc, void* out, void* workspace,
                                size_t ws_bytes, void* stream, bool noalloc = false) {
  const bool fused = fm != nullptr;
  HDC_TRY(check_functor(f, dt, !fused));
  if (fused) HDC_TRY(check_functor(fm, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (acc == HDC_ACC_EXACT && f->id != HDC_FN_IDENTITY && !(f->id == HDC_FN_PRODUCT && dt == HDC_F16 && !fused))
    return fail(HDC_ERR_UNSUPPORTED, "EXACT folds IDENTITY (fp16, bf16) and PRODUCT (fp16) only");
  if (acc == HDC_ACC_EXACT && f->id == HDC_FN_PRODUCT && n >= (int64_t(1) << 31))
    return fail(HDC_ERR_UNSUPPORTED, "EXACT dot products take fewer than 2^31 terms");
  if (acc == HDC_ACC_EXACT && fused && dt != HDC_F16)
    return fail(HDC_ERR_UNSUPPORTED, "EXACT map_reduce is provided for fp16 storage");
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
  if (noalloc) {
    if (reduce_workspace_bytes() > kScratchBytes)
      return fail(HDC_ERR_WORKSPACE, "the call needs %zu bytes of partials; the scratch array holds %zu",
                  reduce_workspace_bytes(), kScratchBytes);
    HDC_TRY(scratch_address(&ws));
  } else {
    HDC_TRY(resolve_workspace(workspace, ws_bytes, reduce_workspace_bytes(), st, &ws));
  }
  const int op = fused ? HDC_OP_MAP_REDUCE : f->id == HDC_FN_PRODUCT ? HDC_OP_DOT : HDC_OP_TRANSFORM_REDUCE;
  const Tuning t = tuning_for(op, dt, acc, n);
  uint64_t* ticket = nullptr;
  if (t.passes == 1) HDC_TRY(ticket_for(ws, &ticket));
  if (log_on()) {
    const bool own = acc == HDC_ACC_EXACT && !fused && (f->id == HDC_FN_PRODUCT || dt == HDC_BF16);
    log_dispatch(fused ? "map_reduce" : f->id == HDC_FN_PRODUCT ? "dot" : "transform_reduce", dt, acc, n, t,
                 own ? "exact kernel and its final fold (two launches)"
                     : t.passes == 1 ? "one launch (the last block folds the partials)" : "two launches",
                 noalloc ? "static scratch" : workspace ? "caller" : "library");
  }

  if (!fused) return run_reduce(*f, dt, x, z, n, acc, out, ws, ticket, t, st);
  switch (dt) {
    case HDC_F32: return run_map_reduce_f32(*fm, *f, x, y, n, acc, out, ws, ticket, t, st);
    case HDC_F16: return run_map_reduce_f16(*fm, *f, x, y, n, acc, out, ws, ticket, t, st);
    case HDC_BF16: return run_map_reduce_bf16(*fm, *f, x, y, n, acc, out, ws, ticket, t, st);
    case HDC_I32: return run_map_reduce_i32(*fm, *f, x, y, n, acc, out, ws, ticket, t, st);
    default: return fail(HDC_ERR_UNSUPPORTED, "dtype %d is not provided", (int)dt);
  }
}

hdc_status hdc_transform_reduce(const hdc_functor* f, hdc_dtype dt, const void* x, const void* z, int64_t n,
                                hdc_accum acc, void* out, void* workspace, size_t ws_bytes, void* stream) {
  return reduce_common(f, nullptr, dt, x, z, nullptr, n, acc, out, workspace, ws_bytes, stream);
}

hdc_status hdc_transform_reduce_noalloc(const hdc_functor* f, hdc_dtype dt, const void* x, const void* z,
                                        int64_t n, hdc_accum acc, void* out, void* stream) {
  return reduce_common(f, nullptr, dt, x, z, nullptr, n, acc, out, nullptr, 0, stream, true);
}

hdc_status hdc_map_reduce(const hdc_functor* f, const hdc_functor* g, hdc_dtype dt, const void* x, void* y,
                          int64_t n, hdc_accum acc, void* out, void* workspace, size_t ws_bytes, void* stream) {
  if (!f) return fail(HDC_ERR_INVALID_ARGUMENT, "map functor is NULL");
  return reduce_common(g, f, dt, x, nullptr, y, n, acc, out, workspace, ws_bytes, stream);
}

hdc_status hdc_segmented_reduce(const hdc_functor* f, hdc_dtype dt, const void* x, const int64_t* offsets,
                                int64_t num_segments, hdc_accum acc, void* out, void* workspace, size_t ws_bytes,
                                void* stream) {
  HDC_TRY(check_functor(f, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (acc == HDC_ACC_EXACT) return fail(HDC_ERR_UNSUPPORTED, "EXACT is provided for transform_reduce and map_reduce");
  if (num_segments < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "num_segments is negative");
  if (num_segments >= INT32_MAX) return fail(HDC_ERR_INVALID_ARGUMENT, "more than 2^31 - 2 segments");
  if (num_segments == 0) return HDC_OK;
  if (!offsets) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is NULL");
  if ((uintptr_t)offsets % 8) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is not 8-byte aligned");
  HDC_TRY(check_ptr(x, dt, 0, "x"));
  if (!out) return fail(HDC_ERR_INVALID_ARGUMENT, "out is NULL");
  const size_t osz = acc == HDC_ACC_PLAIN ? 4 : 8;
  if ((uintptr_t)out % osz) return fail(HDC_ERR_INVALID_ARGUMENT, "out is not aligned to its element size");
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  size_t cap_bytes = 0;
  int64_t total_bound = 0;  // the size bucket's element count
  if (workspace) {
    if ((uintptr_t)workspace % 256) return fail(HDC_ERR_INVALID_ARGUMENT, "workspace is not 256-byte aligned");
    if (seg_capacity(ws_bytes, num_segments) < 1)
      return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes %lld segments need",
                  ws_bytes, seg_layout_cap(1, num_segments).bytes, (long long)num_segments);
    ws = workspace;
    cap_bytes = ws_bytes;
    total_bound = seg_total_bound(ws_bytes, num_segments);
  } else {
    // The library's buffer is sized from offsets[S], read from the device.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipStreamIsCapturing: %s", hipGetErrorString(e));
    if (cs != hipStreamCaptureStatusNone)
      return fail(HDC_ERR_WORKSPACE, "a segmented reduce under graph capture needs a workspace");
    int64_t total = 0;
    e = hipMemcpyAsync(&total, offsets + num_segments, sizeof total, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "reading offsets[S]: %s", hipGetErrorString(e));
    if (total < 0 || total / kMinChunk >= INT32_MAX / 2)
      return fail(HDC_ERR_INVALID_ARGUMENT, "offsets[S] = %lld is out of range", (long long)total);
    cap_bytes = seg_workspace_bytes(total, num_segments);
    HDC_TRY(resolve_workspace(nullptr, 0, cap_bytes, st, &ws));
    total_bound = total;
  }
  const Tuning t = tuning_for(HDC_OP_SEGMENTED_REDUCE, dt, acc, total_bound);
  log_dispatch("segmented_reduce", dt, acc, total_bound, t, t.passes == 1 ? "tiled" : "planned",
               workspace ? "caller" : "library");
  return run_segmented(*f, dt, x, offsets, num_segments, acc, out, ws, cap_bytes, t, st);
}

hdc_status hdc_batch_map_reduce(const hdc_functor* f, const hdc_functor* g, hdc_dtype dt, hdc_accum acc,
                                const hdc_batch_call* calls, int32_t count, void* workspace, size_t ws_bytes,
                                void* stream) {
  if (f) HDC_TRY(check_functor(f, dt, false));
  HDC_TRY(check_functor(g, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (acc == HDC_ACC_EXACT) return fail(HDC_ERR_UNSUPPORTED, "EXACT is provided for transform_reduce and map_reduce");
  if (count < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "count is negative");
  if (count == 0) return HDC_OK;
  if (!calls) return fail(HDC_ERR_INVALID_ARGUMENT, "calls is NULL");
  int64_t total = 0;
  const size_t es = elem_size(dt), osz = acc == HDC_ACC_PLAIN ? 4 : 8;
  for (int32_t i = 0; i < count; ++i) {
    const hdc_batch_call& c = calls[i];
    if (c.n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "call %d: n is negative", i);
    HDC_TRY(check_ptr(c.x, dt, c.n, "x"));
    if (!c.out || (uintptr_t)c.out % osz) return fail(HDC_ERR_INVALID_ARGUMENT, "call %d: bad out pointer", i);
    if (f && c.y) {
      HDC_TRY(check_ptr(c.y, dt, c.n, "y"));
      const uintptr_t xb = (uintptr_t)c.x, yb = (uintptr_t)c.y, len = (uintptr_t)c.n * es;
      if (c.n > 0 && xb < yb + len && yb < xb + len)
        return fail(HDC_ERR_INVALID_ARGUMENT, "call %d: x and y overlap", i);
    }
    total += c.n;
  }
  hipStream_t st = (hipStream_t)stream;
  const Tuning t = tuning_for(HDC_OP_BATCH, dt, acc, total / count);
  void* ws = nullptr;
  size_t need = batch_workspace_bytes(total, count);
  if (need < reduce_workspace_bytes()) need = reduce_workspace_bytes();  // calls run one by one reuse it
  HDC_TRY(resolve_workspace(workspace, ws_bytes, need, st, &ws));
  const size_t cap = workspace ? ws_bytes : need;  // the library's buffer holds at least `need`
  log_dispatch("batch_map_reduce", dt, acc, total / count, t, f ? "grouped map + reduce" : "grouped reduce",
               workspace ? "caller" : "library");

  // Calls whose x and y disagree in 16-byte alignment run one by one; the
  // rest go in groups of up to kBatchMax calls.
  int32_t grp[kBatchMax];
  int ng = 0;
  char* wsb = static_cast<char*>(ws);  // groups run in stream order and share it
  auto flush = [&]() -> hdc_status {
    if (ng == 0) return HDC_OK;
    const hdc_status r = run_batch(f, *g, dt, acc, calls, grp, ng, wsb, cap, t, st);
    ng = 0;
    return r;
  };
  for (int32_t i = 0; i < count; ++i) {
    const hdc_batch_call& c = calls[i];
    const bool vec = !(f && c.y) || ((uintptr_t)c.x % 16) == ((uintptr_t)c.y % 16);
    if (!vec) {
      if (f && c.y)
        HDC_TRY(hdc_map_reduce(f, g, dt, c.x, c.y, c.n, acc, c.out, ws, need, stream));
      continue;
    }
    grp[ng++] = i;
    if (ng == kBatchMax) HDC_TRY(flush());
  }
  return flush();
}


hdc_status hdc_host_map(const hdc_functor* f, hdc_dtype dt, const void* x, void* y, int64_t n, int32_t nthreads) {
  HDC_TRY(check_functor(f, dt, false));
  if (n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "n = %lld is negative", (long long)n);
  if (nthreads < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "nthreads is negative");
  HDC_TRY(check_ptr(x, dt, n, "x"));
  HDC_TRY(check_ptr(y, dt, n, "y"));
  if (n == 0) return HDC_OK;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y, len = (uintptr_t)n * elem_size(dt);
  if (xb != yb && xb < yb + len && yb < xb + len)
    return fail(HDC_ERR_INVALID_ARGUMENT, "x and y overlap partially");
  log_line("host_map dtype=%s n=%lld threads=%d (0: every core)", dtype_name(dt), (long long)n, (int)nthreads);
  return run_host_map(*f, dt, x, y, n, nthreads);
}

hdc_status hdc_host_transform_reduce(const hdc_functor* f, hdc_dtype dt, const void* x, const void* z, int64_t n,
                                     hdc_accum acc, void* out, int32_t nthreads) {
  HDC_TRY(check_functor(f, dt, true));
  HDC_TRY(check_acc(dt, acc));
  if (acc == HDC_ACC_EXACT) return fail(HDC_ERR_UNSUPPORTED, "EXACT is provided on the device only");
  if (n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "n = %lld is negative", (long long)n);
  if (nthreads < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "nthreads is negative");
  HDC_TRY(check_ptr(x, dt, n, "x"));
  if (f->id == HDC_FN_PRODUCT) {
    if (!z && n > 0) return fail(HDC_ERR_UNSUPPORTED, "PRODUCT needs the second operand z");
    HDC_TRY(check_ptr(z, dt, n, "z"));
  }
  if (!out) return fail(HDC_ERR_INVALID_ARGUMENT, "out is NULL");
  log_line("host_transform_reduce dtype=%s acc=%s n=%lld threads=%d (0: every core)", dtype_name(dt), acc_name(acc),
           (long long)n, (int)nthreads);
  return run_host_reduce(*f, dt, x, z, n, acc, out, nthreads);
}


hdc_status hdc_scan(const hdc_functor* f, hdc_dtype dt, const void* x, void* y, int64_t n, hdc_accum acc,
                    int32_t exclusive, void* workspace, size_t ws_bytes, void* stream) {
  HDC_TRY(check_functor(f, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (acc == HDC_ACC_EXACT) return fail(HDC_ERR_UNSUPPORTED, "EXACT is provided for transform_reduce and map_reduce");
  if (n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "n = %lld is negative", (long long)n);
  if (exclusive != 0 && exclusive != 1) return fail(HDC_ERR_INVALID_ARGUMENT, "exclusive must be 0 or 1");
  HDC_TRY(check_ptr(x, dt, n, "x"));
  const size_t osz = acc == HDC_ACC_PLAIN ? 4 : 8;
  if (n > 0 && !y) return fail(HDC_ERR_INVALID_ARGUMENT, "y is NULL");
  if (y && (uintptr_t)y % osz) return fail(HDC_ERR_INVALID_ARGUMENT, "y is not aligned to its element size");
  if (n == 0) return HDC_OK;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y;
  if (xb < yb + (uintptr_t)n * osz && yb < xb + (uintptr_t)n * elem_size(dt))
    return fail(HDC_ERR_INVALID_ARGUMENT, "x and y overlap");
  hipStream_t st = (hipStream_t)stream;
  const Tuning t = tuning_for(HDC_OP_SCAN, dt, acc, n);
  void* ws = nullptr;
  HDC_TRY(resolve_workspace(workspace, ws_bytes, scan_workspace_bytes(n), st, &ws));
  log_dispatch(exclusive ? "scan (exclusive)" : "scan (inclusive)", dt, acc, n, t,
               t.unroll == 1 ? "three passes" : "one pass (tree carry)", workspace ? "caller" : "library");
  return run_scan(*f, dt, x, y, n, acc, exclusive, ws, t, st);
}

hdc_status hdc_segmented_scan(const hdc_functor* f, hdc_dtype dt, const void* x, const int64_t* offsets,
                              int64_t num_segments, int64_t total, void* y, hdc_accum acc, int32_t exclusive,
                              void* workspace, size_t ws_bytes, void* stream) {
  HDC_TRY(check_functor(f, dt, false));
  HDC_TRY(check_acc(dt, acc));
  if (acc == HDC_ACC_EXACT) return fail(HDC_ERR_UNSUPPORTED, "EXACT is provided for transform_reduce and map_reduce");
  if (num_segments < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "num_segments is negative");
  if (total < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "total is negative");
  if (exclusive != 0 && exclusive != 1) return fail(HDC_ERR_INVALID_ARGUMENT, "exclusive must be 0 or 1");
  if (num_segments == 0 || total == 0) return HDC_OK;
  if (!offsets) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is NULL");
  if ((uintptr_t)offsets % 8) return fail(HDC_ERR_INVALID_ARGUMENT, "offsets is not 8-byte aligned");
  HDC_TRY(check_ptr(x, dt, total, "x"));
  const size_t osz = acc == HDC_ACC_PLAIN ? 4 : 8;
  if (!y) return fail(HDC_ERR_INVALID_ARGUMENT, "y is NULL");
  if ((uintptr_t)y % osz) return fail(HDC_ERR_INVALID_ARGUMENT, "y is not aligned to its element size");
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y;
  if (xb < yb + (uintptr_t)total * osz && yb < xb + (uintptr_t)total * elem_size(dt))
    return fail(HDC_ERR_INVALID_ARGUMENT, "x and y overlap");
  hipStream_t st = (hipStream_t)stream;
  const Tuning t = tuning_for(HDC_OP_SCAN, dt, acc, total);
  void* ws = nullptr;
  HDC_TRY(resolve_workspace(workspace, ws_bytes, scan_workspace_bytes(total), st, &ws));
  log_dispatch(exclusive ? "segmented_scan (exclusive)" : "segmented_scan (inclusive)", dt, acc, total, t,
               t.unroll == 1 ? "three passes" : "one pass (tree carry)", workspace ? "caller" : "library");
  return run_segmented_scan(*f, dt, x, offsets, num_segments, y, total, acc, exclusive, ws, t, st);
}

hdc_status hdc_scan_status(const void* workspace, int32_t* status, void* stream) {
  if (!status) return fail(HDC_ERR_INVALID_ARGUMENT, "status is NULL");
  hipStream_t st = (hipStream_t)stream;
  const void* ws = workspace;
  if (!ws) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HDC_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto it = g_ws.find({dev, (void*)stream});
    if (it == g_ws.end() || !it->second.ptr)
      return fail(HDC_ERR_INVALID_ARGUMENT, "no library workspace exists for this device and stream");
    ws = it->second.ptr;
  }
  if ((uintptr_t)ws % 256) return fail(HDC_ERR_INVALID_ARGUMENT, "workspace is not 256-byte aligned");
  const hipError_t e = hipMemcpyAsync(status, static_cast<const char*>(ws) + 4, sizeof(int32_t), hipMemcpyDefault, st);
  if (e != hipSuccess) return fail(HDC_ERR_HIP, "copying the scan status: %s", hipGetErrorString(e));
  return HDC_OK;
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
    case HDC_OP_DOT:
    case HDC_OP_MAP_REDUCE: *bytes = reduce_workspace_bytes(); return HDC_OK;
    case HDC_OP_SCAN:
      *bytes = scan_workspace_bytes(n);
      return HDC_OK;
    case HDC_OP_BATCH:
      *bytes = batch_workspace_bytes(n, num_segments);
      if (*bytes < reduce_workspace_bytes()) *bytes = reduce_workspace_bytes();  // calls run one by one reuse it
      return HDC_OK;
    case HDC_OP_SEGMENTED_REDUCE:
      if (n / kMinChunk >= INT32_MAX / 2 || num_segments >= INT32_MAX)
        return fail(HDC_ERR_INVALID_ARGUMENT, "sizes too large");
      *bytes = seg_workspace_bytes(n, num_segments);  // enough for every schedule and chunk setting
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
    if (t->passes) n.passes = t->passes;
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
  t->passes = c.passes;
  return HDC_OK;
}

hdc_status hdc_tuning_bucket(int64_t n, int32_t* bucket) {
  if (!bucket || n < 0) return fail(HDC_ERR_INVALID_ARGUMENT, "bad arguments");
  *bucket = bucket_of(n);
  return HDC_OK;
}

hdc_status hdc_load_tuning(const char* path) {
  ensure_tuning_loaded();
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
