/*
 * hdc.h -- C ABI of the MI355X (gfx950) generic map / reduce library.
 *
 * The operation: one generic callable applied element by element over a
 * device array (map), and the results folded into a sum (transform_reduce,
 * dot, segmented reduce).  The paper's kernels take a callable *by value* and
 * invoke it in every device thread (section 2.4, listing
 * lst_solution_ifdef_cudaarch; section 2.6, listing
 * lst_solution_exp_constexpr_la); which overload runs is decided at compile
 * time from the callable's type through the Host-Device-Compatibility tag
 * (section 2.7, listing lst_hst_dev_tags; section 2.10 "SFINAE 3 with macro";
 * appendix B, listing lst_hdc).  A C ABI cannot carry templates, so the
 * callable crosses this boundary as a closed set of functor ids plus their
 * parameters (hdc_functor); inside the library every id is a concrete C++
 * type tagged HstDev whose call is fully inlined into its kernel -- there is
 * no per-element indirect call.
 *
 * Conventions shared by every entry point:
 *  - Pointers named x, y, z, out, offsets, workspace are DEVICE pointers owned
 *    by the caller; the library never frees them and keeps no reference after
 *    the call returns (a captured graph references them for its lifetime).
 *  - `stream` is a hipStream_t passed as void*; NULL means the legacy default
 *    stream.  Work is stream-ordered and asynchronous: results are valid after
 *    the caller synchronises the stream.
 *  - Element pointers must be aligned to their element size; any further
 *    alignment is handled inside (unaligned heads and tails are peeled).
 *  - Every argument check runs on the host BEFORE anything is enqueued, so a
 *    call that returns an error has written nothing.  Errors are reported by
 *    the return code (HDC_OK == 0 is success, as the paper's error-code
 *    convention in section 1.2, "Cuda error checking"); a thread-local text
 *    explaining the last failure is available from hdc_last_error().
 *  - Device faults are sticky and surface at the caller's next
 *    synchronisation (section 2.4, variant "no sensible implementation").
 *  - Calls from several host threads are safe.  Calls that share one
 *    workspace buffer must be ordered on one stream.  A caller's workspace
 *    must be 256-byte aligned (HDC_ERR_INVALID_ARGUMENT otherwise).
 */
#ifndef HDC_H
#define HDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enums are 32-bit integers on both sides.  In C++ they get that fixed
 * underlying type, so a caller's out-of-range value is still a value of the
 * enum that the argument checks can reject (without it, merely loading such
 * a value would be undefined). */
#ifdef __cplusplus
#define HDC_ENUM(name) enum name : int32_t
#else
#define HDC_ENUM(name) enum name
#endif

typedef HDC_ENUM(hdc_status) {
  HDC_OK = 0,
  HDC_ERR_INVALID_ARGUMENT = 1, /* null pointer, negative size, bad alignment */
  HDC_ERR_UNSUPPORTED = 2,      /* functor / dtype / accumulation not provided */
  HDC_ERR_WORKSPACE = 3,        /* workspace too small, or growth while capturing */
  HDC_ERR_HIP = 4               /* a HIP runtime call or kernel launch failed */
} hdc_status;

typedef HDC_ENUM(hdc_dtype) {
  HDC_F32 = 0,  /* IEEE binary32 */
  HDC_F16 = 1,  /* IEEE binary16 */
  HDC_BF16 = 2, /* bfloat16 (upper half of binary32) */
  HDC_I32 = 3,  /* two's-complement int32 */
  HDC_I64 = 4,  /* declared for completeness; no operation accepts it yet */
  HDC_F64 = 5   /* declared for completeness; no operation accepts it yet */
} hdc_dtype;

typedef HDC_ENUM(hdc_fn) {
  HDC_FN_IDENTITY = 0, /* f(x) = x */
  HDC_FN_AFFINE = 1,   /* floats: f(x) = fma(a, x, b) in fp32 (one rounding);
                          int32: f(x) = ia*x + ib with two's-complement wrap
                          (map: mod 2^32; reduce terms: mod 2^64) */
  HDC_FN_HORNER = 2,   /* f(x) = sum_{k<=degree} coef[k] x^k, evaluated as
                          acc = coef[degree]; acc = fma(acc, x, coef[k]),
                          k = degree-1 .. 0, in fp32 (floats only) */
  HDC_FN_PRODUCT = 3   /* dot-product term x[i]*z[i]; transform_reduce only */
} hdc_fn;

typedef HDC_ENUM(hdc_accum) {
  HDC_ACC_PLAIN = 0,       /* floats: fp32 partial sums; `out` is one float */
  HDC_ACC_COMPENSATED = 1, /* floats: fp32 TwoSum-compensated partials, fp64
                              final cross-block combine; `out` is one double */
  HDC_ACC_EXACT_INT = 2,   /* int32: int64 sums wrapping mod 2^64; `out` is
                              one int64 */
  HDC_ACC_EXACT = 3        /* the exact real sum rounded once to fp64
                              (nearest-even); `out` is one double.
                              Independent of order and tuning:
                              bit-reproducible.  IDENTITY folds of fp16 or
                              bf16 storage (transform_reduce; map_reduce for
                              fp16) and PRODUCT folds (dot products) of fp16
                              storage with n < 2^31; bf16 sums take any n
                              below 2^33 (a larger n may return
                              HDC_ERR_UNSUPPORTED).  A non-finite term
                              makes the result its IEEE sum of the
                              non-finite terms (inf * 0 is NaN). */
} hdc_accum;

typedef HDC_ENUM(hdc_op) {
  HDC_OP_MAP = 0,
  HDC_OP_TRANSFORM_REDUCE = 1,
  HDC_OP_SEGMENTED_REDUCE = 2,
  HDC_OP_MAP_REDUCE = 3,
  HDC_OP_BATCH = 4,
  HDC_OP_SCAN = 5,
  HDC_OP_DOT = 6 /* tuning class of transform_reduce with PRODUCT (dot products,
                    two operands per element); its workspace is that of
                    HDC_OP_TRANSFORM_REDUCE */
} hdc_op;

#define HDC_MAX_DEGREE 16

/* The callable.  Fields not used by `id` are ignored. */
typedef struct hdc_functor {
  int32_t id;                    /* hdc_fn */
  int32_t degree;                /* HORNER: 0 .. HDC_MAX_DEGREE */
  float a, b;                    /* AFFINE on floating-point storage */
  float coef[HDC_MAX_DEGREE + 1]; /* HORNER: coef[k] multiplies x^k */
  int64_t ia, ib;                /* AFFINE on int32 storage */
} hdc_functor;

/*
 * y[i] = f(x[i]) for 0 <= i < n, written in x's storage type.
 *   The operation is the paper's kernel that takes a callable by value and
 *   applies it once per element in every device thread (section 2.4, listing
 *   lst_solution_ifdef_cudaarch; one callable for both sides, section 2.6,
 *   listing lst_solution_exp_constexpr_la); `f` is that callable, chosen from
 *   the closed set of hdc_fn (section 2.10: the type decides the overload).
 *   Floats: f evaluated in fp32 on the exactly widened input; fp16 / bf16
 *   results are rounded to nearest-even.  IDENTITY copies bits.
 *   Supported: IDENTITY, AFFINE on F32/F16/BF16/I32; HORNER on F32/F16/BF16.
 *   x, y: device arrays of n elements, caller-owned.  x == y (in place) is
 *   allowed; partial overlap is rejected.  n == 0 is a no-op.  Errors:
 *   HDC_ERR_INVALID_ARGUMENT (NULL with n > 0, misaligned element, n < 0,
 *   overlap), HDC_ERR_UNSUPPORTED (functor / dtype pair not provided).
 *   Bytes moved: 2 n sizeof(element).
 */
hdc_status hdc_map(const hdc_functor* f, hdc_dtype dt, const void* x, void* y,
                   int64_t n, void* stream);

/*
 * out = sum_i f(x[i])  (PRODUCT: sum_i x[i] * z[i], z of the same dtype).
 *   The callable applied per element as in hdc_map (section 2.4, listing
 *   lst_solution_ifdef_cudaarch), its results folded into one sum.
 *   acc PLAIN or COMPENSATED for F32/F16/BF16, EXACT_INT for I32 (IDENTITY
 *   or AFFINE).  n == 0 writes 0.  The summation order is fixed by (n, the
 *   tuning in force): results are bit-reproducible run to run, but a
 *   different tuning may change the last bits of a floating-point result.
 *   x, z: device arrays of n elements; out: one device float (PLAIN), double
 *   (COMPENSATED, EXACT) or int64 (EXACT_INT), all caller-owned.
 *   workspace: device scratch of at least hdc_workspace_size(...) bytes, or
 *   NULL to use a library-owned buffer (per device and stream, grown outside
 *   graph capture only).  Errors: HDC_ERR_INVALID_ARGUMENT (NULL or
 *   misaligned pointers, n < 0), HDC_ERR_UNSUPPORTED (functor / dtype /
 *   accumulation not provided), HDC_ERR_WORKSPACE (workspace too small, or
 *   the library buffer would have to grow under capture).
 *   Bytes moved: n sizeof(element) (x2 for PRODUCT).
 */
hdc_status hdc_transform_reduce(const hdc_functor* f, hdc_dtype dt,
                                const void* x, const void* z, int64_t n,
                                hdc_accum acc, void* out, void* workspace,
                                size_t ws_bytes, void* stream);

/*
 * hdc_transform_reduce without a workspace and without any allocation, for
 * callers that cannot allocate device memory: code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.
 *   Arguments, results and errors are those of hdc_transform_reduce (the same
 *   kernels, tuning and summation order, so the same bits), minus workspace
 *   and ws_bytes: the per-block partials go to a scratch array of 2 MiB
 *   compiled into the library, one copy per device, held from the first
 *   call on that device until the process ends.  The scratch holds the
 *   partials of the most blocks any call launches, so every n that
 *   hdc_transform_reduce accepts fits; a call that needed more would fail
 *   with HDC_ERR_WORKSPACE before enqueuing anything.  The call never runs
 *   hipMalloc, hipFree or an allocating library routine; the first call on
 *   a device looks up the scratch array's device address (no allocation).
 *   Every call on one device shares that device's scratch: calls that may
 *   overlap in time on one device (different streams, or graphs replayed
 *   concurrently) race and give wrong results.  Order them on one stream.
 *   The scratch keeps the last call's partials; nothing in it needs to start
 *   at zero (each call writes every partial it reads).
 */
hdc_status hdc_transform_reduce_noalloc(const hdc_functor* f, hdc_dtype dt,
                                        const void* x, const void* z,
                                        int64_t n, hdc_accum acc, void* out,
                                        void* stream);

/*
 * out[j] = sum_{offsets[j] <= i < offsets[j+1]} f(x[i]) for 0 <= j < S.
 *   The per-element callable as in hdc_transform_reduce (section 2.4,
 *   listing lst_solution_ifdef_cudaarch), folded separately over each of
 *   many uneven segments in one batch.
 *   x: device array of at least offsets[S] elements.
 *   offsets: device int64 array of S+1 entries, non-decreasing, offsets[0] >= 0
 *   (a precondition, not checked per call: checking it would need a device
 *   round trip; hdc_validate_offsets checks it synchronously).
 *   out: S floats (PLAIN), doubles (COMPENSATED) or int64 (EXACT_INT).
 *   Empty segments give 0.  No host synchronisation (with a workspace).
 *   Two schedules, chosen by the tuning's `passes`: tiled (1) streams fixed
 *   tiles of the element range and folds the segments that span tiles in a
 *   second launch; planned (2) builds work lists in three small launches,
 *   runs one persistent pass over them and a combine launch.  Both give
 *   reproducible bits for a fixed tuning.
 *   IDENTITY, AFFINE, HORNER as for transform_reduce (no PRODUCT).
 *   workspace: at least hdc_workspace_size(HDC_OP_SEGMENTED_REDUCE, dt, acc,
 *   total, S) bytes for a total >= offsets[S]; its size sets the capacity
 *   of the work lists.  If the segments need more than ws_bytes holds
 *   (offsets[S] above the total it was sized for), the call still returns
 *   the correct sums, folding every segment whole with one wavefront
 *   (slower, and the last bits of a floating-point sum may differ); the
 *   tiled schedule does the same when the workspace holds fewer tile slots
 *   than the range has tiles.  The size bucket of the tuning is that of the
 *   largest total ws_bytes serves.
 *   NULL: the library's buffer, sized from offsets[S], which the call then
 *   reads from the device (a synchronous 8-byte copy on `stream`; refused
 *   with HDC_ERR_WORKSPACE under graph capture).
 *   Errors: HDC_ERR_INVALID_ARGUMENT (S < 0 or >= 2^31 - 1, NULL or
 *   misaligned offsets / out, misaligned x or workspace),
 *   HDC_ERR_UNSUPPORTED (functor / dtype / accumulation not provided),
 *   HDC_ERR_WORKSPACE (ws_bytes below the bound for S segments).
 */
hdc_status hdc_segmented_reduce(const hdc_functor* f, hdc_dtype dt,
                                const void* x, const int64_t* offsets,
                                int64_t num_segments, hdc_accum acc,
                                void* out, void* workspace, size_t ws_bytes,
                                void* stream);

/*
 * Fused map + transform_reduce: y[i] = f(x[i]) as hdc_map, and
 * out = the fold of g over x as hdc_transform_reduce(g, ...), reading x once.
 *   Bytes moved: 2 n sizeof(element) instead of 3.
 */
hdc_status hdc_map_reduce(const hdc_functor* f, const hdc_functor* g,
                          hdc_dtype dt, const void* x, void* y, int64_t n,
                          hdc_accum acc, void* out, void* workspace,
                          size_t ws_bytes, void* stream);

/*
 * Prefix sums: y[i] = the fold of f over x[0..i] (exclusive = 1: over
 * x[0..i-1], so y[0] = 0).  acc PLAIN (y: float), COMPENSATED (y: double)
 * for F32/F16/BF16, EXACT_INT (y: int64, wrapping) for I32; IDENTITY,
 * AFFINE, HORNER.  x and y must not overlap.  Workspace:
 * hdc_workspace_size(HDC_OP_SCAN, dt, acc, n, 0, ...); calls sharing it must
 * be ordered on one stream.  Two schedules, chosen by the tuning's `unroll`:
 *  - any value but 1 (the default): one pass.  Tiles are handed out in
 *    launch order.  Each tile publishes its total as a leaf of a radix-64
 *    tree (the last tile of a group also the group's node), and folds its
 *    carry from at most 63 nodes per tree level, in a fixed order.  The carry between tiles is
 *    fp64 for floats and int64 for integers.  x is read once.  A small
 *    clear kernel runs first on the same stream.  Every wait is bounded:
 *    if one gives up, the call's output is invalid and hdc_scan_status
 *    reports it.  Tiles start in order, so a give-up is not expected.
 *  - 1: three passes (tile sums, tile offsets, tile scans) with no waiting
 *    between blocks.  x is read twice.
 * Results are bit-reproducible for a fixed tuning.
 */
hdc_status hdc_scan(const hdc_functor* f, hdc_dtype dt, const void* x,
                    void* y, int64_t n, hdc_accum acc, int32_t exclusive,
                    void* workspace, size_t ws_bytes, void* stream);

/*
 * Segmented prefix sums: for every segment j and every i in
 * [offsets[j], offsets[j+1]), y[i] = the fold of f over x[offsets[j]..i]
 * (exclusive = 1: over x[offsets[j]..i-1], so a segment's first output is 0).
 * The prefix restarts at every segment start.  x and y hold `total` elements.
 * offsets is a DEVICE array of num_segments + 1 non-decreasing entries with
 * offsets[num_segments] <= total; this is a precondition and is not checked.
 * Only positions inside a segment are written.  dtype, functor and
 * accumulation as hdc_scan; tuning class HDC_OP_SCAN.  One pass or three, as
 * hdc_scan; every wavefront finds the segment starts in its part of a tile
 * from the offsets (a 64-way search, then the next 64 boundaries at a time).
 * Bytes moved: as hdc_scan, plus the offsets once.  Workspace:
 * hdc_workspace_size(HDC_OP_SCAN, dt, acc, total, 0, ...).
 * num_segments == 0 or total == 0 writes nothing.
 */
hdc_status hdc_segmented_scan(const hdc_functor* f, hdc_dtype dt, const void* x,
                              const int64_t* offsets, int64_t num_segments,
                              int64_t total, void* y, hdc_accum acc,
                              int32_t exclusive, void* workspace,
                              size_t ws_bytes, void* stream);

/*
 * Status of the last hdc_scan or hdc_segmented_scan that ran with this
 * workspace (NULL: the library's buffer of the current device and
 * `stream`): copies one int32 into *status, stream-ordered and
 * asynchronous (a device pointer, or pinned host memory read after the
 * stream is synchronised).  0: the scan's output is valid; nonzero: a wait
 * of the single-pass schedule for an earlier tile gave up and that output
 * is invalid (run it again).  Calls that launch nothing (n == 0) leave the
 * word as it was.  Errors: HDC_ERR_INVALID_ARGUMENT (status NULL, no
 * library buffer for this stream, misaligned workspace), HDC_ERR_HIP.
 */
hdc_status hdc_scan_status(const void* workspace, int32_t* status,
                           void* stream);

/* One call of a grouped batch (device pointers). */
typedef struct hdc_batch_call {
  const void* x;
  void* y;        /* map output, or NULL: this call only folds */
  int64_t n;
  void* out;      /* one float / double / int64, as the accumulation says */
} hdc_batch_call;

/*
 * Many independent calls of one class -- same dtype, map callable f, fold
 * callable g and accumulation -- in one grouped launch plus one combine
 * launch per 32 calls: y = f(x) (when f and the call's y are non-NULL) and
 * *out = the fold of g over x, each call exactly as hdc_map_reduce /
 * hdc_transform_reduce define it.  `calls` is a HOST array read during this
 * call (the table is passed to the kernels by value, so the launches can be
 * recorded into a graph).  A call whose x and y differ in 16-byte alignment
 * runs on its own.  Workspace: hdc_workspace_size(HDC_OP_BATCH, dt, acc,
 * sum of n, count, ...).  Reduction results depend on the tuning of
 * HDC_OP_BATCH (chunk length), not on the batch composition.
 */
hdc_status hdc_batch_map_reduce(const hdc_functor* f, const hdc_functor* g,
                                hdc_dtype dt, hdc_accum acc,
                                const hdc_batch_call* calls, int32_t count,
                                void* workspace, size_t ws_bytes,
                                void* stream);

/*
 * The host side of the same callables (the paper's one-callable-two-sides
 * idea, section 2.10 and appendix B): x, y, z and out are HOST pointers, the
 * call is synchronous and runs on `nthreads` host threads (0: all hardware
 * threads).  Element semantics are those of hdc_map / hdc_transform_reduce
 * (the same C++ code evaluates them); reductions fold contiguous per-thread
 * ranges and merge them in thread order, so their last bits depend on
 * nthreads.  These are separate entry points: the device entry points never
 * run on the host.
 */
hdc_status hdc_host_map(const hdc_functor* f, hdc_dtype dt, const void* x,
                        void* y, int64_t n, int32_t nthreads);
hdc_status hdc_host_transform_reduce(const hdc_functor* f, hdc_dtype dt,
                                     const void* x, const void* z, int64_t n,
                                     hdc_accum acc, void* out,
                                     int32_t nthreads);

/* Bytes of workspace `op` needs for these sizes (0 for HDC_OP_MAP).  For
 * HDC_OP_SEGMENTED_REDUCE, n is `total` and num_segments is S; for
 * HDC_OP_BATCH, n is the sum of the calls' n and num_segments the count. */
hdc_status hdc_workspace_size(int op, hdc_dtype dt, hdc_accum acc, int64_t n,
                              int64_t num_segments, size_t* bytes);

/* Synchronous check of a CSR offsets array (device pointer): returns HDC_OK
 * when it is non-decreasing with offsets[0] >= 0 and offsets[S] <= total.
 * For tests and debugging; it copies the array to the host. */
hdc_status hdc_validate_offsets(const int64_t* offsets, int64_t num_segments,
                                int64_t total, void* stream);

/* Tuning of one class of calls: (op, dtype, accumulation, size bucket).
 * Buckets split n (the element count; for the segmented op, the total) at
 * 2^16, 2^20 and 2^24 into buckets 0..3.  block: threads per block (64..1024,
 * multiple of 64); unroll: 16-byte vectors per lane per step (1, 2, 4 or 8);
 * grid_mult: blocks per compute unit (1..64); chunk: elements per work item
 * of the segmented pass (power of two, 1024..65536); small_seg: segments at
 * most this long are packed several per wavefront (0..1024); seg_per_wave:
 * how many small segments share one wavefront (power of two, 1..64, each
 * served by 64/seg_per_wave lanes).  For HDC_OP_SCAN, block sets the tile
 * (block * 16 elements) and unroll 1 selects the three-pass schedule.
 * passes, 1 or 2 (default 2).  HDC_OP_TRANSFORM_REDUCE, HDC_OP_DOT,
 * HDC_OP_MAP_REDUCE: 1 folds the per-block partials in the same launch, in
 * the block that arrives last on a ticket (library-owned device memory, one
 * per workspace buffer), if the grid's partials fit its LDS stage (32 KiB),
 * else in a second launch; 2 always folds them in a second launch.  Both
 * fold in the same order, so `passes` does not change any result bit.  (A
 * one-launch fold whose wait for a partial gave up -- not expected -- writes
 * NaN, or INT64_MIN for int64 sums.)  The exact bf16 sum and the exact fp16
 * dot always use two launches.  HDC_OP_SEGMENTED_REDUCE: 1 selects the tiled
 * schedule (fixed tiles of `chunk` elements, no plan), 2 the planned one
 * (pieces of `chunk`, packed small segments).  Tuning changes
 * the summation order, so the last bits of a floating-point sum may change;
 * results stay within the stated tolerance. */
typedef struct hdc_tuning {
  int32_t block;
  int32_t unroll;
  int32_t grid_mult;
  int32_t chunk;
  int32_t small_seg;
  int32_t seg_per_wave;
  int32_t passes;
} hdc_tuning;

/* Set the class (bucket -1: every bucket); fields set to 0 keep their value.
 * Nothing changes if any resulting value is out of range. */
hdc_status hdc_set_tuning(int op, hdc_dtype dt, hdc_accum acc, int bucket,
                          const hdc_tuning* t);
hdc_status hdc_get_tuning(int op, hdc_dtype dt, hdc_accum acc, int bucket,
                          hdc_tuning* t);
/* The size bucket a call of n elements falls in. */
hdc_status hdc_tuning_bucket(int64_t n, int32_t* bucket);
/* Load a tuning cache written by the autotuner: one line per class,
 * "op dtype acc bucket block unroll grid_mult chunk small_seg seg_per_wave
 * [passes]" (passes may be left out: 2), '#' starts a
 * comment line.  NULL reads the path in the HDC_TUNE_CACHE environment
 * variable (which is also read once, before the first call, unless the
 * environment sets HDC_TUNE=0: then no cache is read at start-up and the
 * built-in defaults apply until a caller loads or sets tuning explicitly).
 * A missing file is not an error; a malformed line is reported and skipped.
 *
 * Environment: HDC_LOG set to anything but "0" prints one line per call on
 * stderr with the dispatch decision: operation, storage and fold types, the
 * element count and its size bucket, the tuning fields taken, the schedule
 * they select (one or two launches; tiled or planned segmented schedule;
 * one or three scan passes; vector or scalar map) and where the workspace
 * came from (the caller's, the library's buffer, the static scratch array). */
hdc_status hdc_load_tuning(const char* path);

const char* hdc_status_string(hdc_status s);
/* Thread-local explanation of the last non-OK status on this thread. */
const char* hdc_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t hdc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HDC_H */
