"""Python binding of the MI355X generic map / reduce library (include/hdc.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libhdc.so.  PyTorch supplies device memory and the current stream.
There is no fallback: if the library is not built, or a tensor is not on a
GPU, the call raises.

Callables are plain dicts (or the helpers below):
    identity()                      {"fn": "identity"}
    affine(a, b)                    {"fn": "affine", "a": a, "b": b}
    horner([c0, ..., cd])           {"fn": "horner", "coef": [...]}
    product()                       {"fn": "product"}     (dot-product term)
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# HDC_LIBRARY names another build of the same sources (the sanitized host-only
# build used by the CPU sanitizer test); there is no fallback either way.
LIB_PATH = os.environ.get("HDC_LIBRARY") or os.path.join(HERE, "libhdc.so")
# Tuning cache written by the autotuner for gfx950; loaded with the library
# unless HDC_TUNE_CACHE names another one (which the library reads itself) or
# HDC_TUNE=0 asks for the built-in defaults.
TUNING_CACHE = os.path.join(HERE, "tuning_gfx950.txt")

# C enums (hdc.h)
OK, ERR_INVALID_ARGUMENT, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP = range(5)
F32, F16, BF16, I32, I64, F64 = range(6)
FN_IDENTITY, FN_AFFINE, FN_HORNER, FN_PRODUCT = range(4)
ACC_PLAIN, ACC_COMPENSATED, ACC_EXACT_INT, ACC_EXACT = range(4)
OP_MAP, OP_TRANSFORM_REDUCE, OP_SEGMENTED_REDUCE, OP_MAP_REDUCE, OP_BATCH, OP_SCAN, OP_DOT = range(7)
MAX_DEGREE = 16

DTYPE = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16, torch.int32: I32}
ACC = {"plain": ACC_PLAIN, "compensated": ACC_COMPENSATED, "exact_int": ACC_EXACT_INT, "exact": ACC_EXACT}
OUT_DTYPE = {ACC_PLAIN: torch.float32, ACC_COMPENSATED: torch.float64, ACC_EXACT_INT: torch.int64,
             ACC_EXACT: torch.float64}
FN = {"identity": FN_IDENTITY, "affine": FN_AFFINE, "horner": FN_HORNER, "product": FN_PRODUCT}

# Every symbol include/hdc.h declares.
EXPORTS = [
    "hdc_map", "hdc_transform_reduce", "hdc_transform_reduce_noalloc", "hdc_segmented_reduce", "hdc_map_reduce",
    "hdc_batch_map_reduce", "hdc_host_map", "hdc_host_transform_reduce", "hdc_scan", "hdc_segmented_scan", "hdc_scan_status",
    "hdc_workspace_size", "hdc_validate_offsets", "hdc_set_tuning", "hdc_get_tuning",
    "hdc_load_tuning", "hdc_tuning_bucket", "hdc_status_string", "hdc_last_error", "hdc_version",
]


class Functor(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("a", ctypes.c_float), ("b", ctypes.c_float),
                ("coef", ctypes.c_float * (MAX_DEGREE + 1)),
                ("ia", ctypes.c_int64), ("ib", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("grid_mult", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("small_seg", ctypes.c_int32), ("seg_per_wave", ctypes.c_int32),
                ("passes", ctypes.c_int32)]


class BatchCall(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n", ctypes.c_int64), ("out", ctypes.c_void_p)]


class HdcError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")


_STATUS_NAMES = {OK: "HDC_OK", ERR_INVALID_ARGUMENT: "HDC_ERR_INVALID_ARGUMENT",
                 ERR_UNSUPPORTED: "HDC_ERR_UNSUPPORTED", ERR_WORKSPACE: "HDC_ERR_WORKSPACE",
                 ERR_HIP: "HDC_ERR_HIP"}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2309_03912_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, vp, i64, i32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        st = ctypes.c_int
        L.hdc_map.argtypes = [P(Functor), i32, vp, vp, i64, vp]
        L.hdc_transform_reduce.argtypes = [P(Functor), i32, vp, vp, i64, i32, vp, vp, ctypes.c_size_t, vp]
        L.hdc_transform_reduce_noalloc.argtypes = [P(Functor), i32, vp, vp, i64, i32, vp, vp]
        L.hdc_segmented_reduce.argtypes = [P(Functor), i32, vp, vp, i64, i32, vp, vp, ctypes.c_size_t, vp]
        L.hdc_map_reduce.argtypes = [P(Functor), P(Functor), i32, vp, vp, i64, i32, vp, vp, ctypes.c_size_t, vp]
        L.hdc_batch_map_reduce.argtypes = [P(Functor), P(Functor), i32, i32, P(BatchCall), ctypes.c_int32, vp,
                                           ctypes.c_size_t, vp]
        L.hdc_host_map.argtypes = [P(Functor), i32, vp, vp, i64, ctypes.c_int32]
        L.hdc_host_transform_reduce.argtypes = [P(Functor), i32, vp, vp, i64, i32, vp, ctypes.c_int32]
        L.hdc_scan.argtypes = [P(Functor), i32, vp, vp, i64, i32, ctypes.c_int32, vp, ctypes.c_size_t, vp]
        L.hdc_segmented_scan.argtypes = [P(Functor), i32, vp, vp, i64, i64, vp, i32, ctypes.c_int32, vp,
                                         ctypes.c_size_t, vp]
        L.hdc_scan_status.argtypes = [vp, vp, vp]
        L.hdc_workspace_size.argtypes = [i32, i32, i32, i64, i64, P(ctypes.c_size_t)]
        L.hdc_validate_offsets.argtypes = [vp, i64, i64, vp]
        L.hdc_set_tuning.argtypes = [i32, i32, i32, i32, P(Tuning)]
        L.hdc_get_tuning.argtypes = [i32, i32, i32, i32, P(Tuning)]
        L.hdc_tuning_bucket.argtypes = [i64, P(ctypes.c_int32)]
        L.hdc_load_tuning.argtypes = [ctypes.c_char_p]
        for name in ["hdc_map", "hdc_transform_reduce", "hdc_transform_reduce_noalloc", "hdc_segmented_reduce",
                     "hdc_map_reduce", "hdc_batch_map_reduce", "hdc_host_map", "hdc_host_transform_reduce", "hdc_scan",
                     "hdc_segmented_scan", "hdc_scan_status", "hdc_workspace_size", "hdc_validate_offsets",
                     "hdc_set_tuning", "hdc_get_tuning", "hdc_load_tuning", "hdc_tuning_bucket"]:
            getattr(L, name).restype = st
        L.hdc_status_string.argtypes = [st]
        L.hdc_status_string.restype = ctypes.c_char_p
        L.hdc_last_error.argtypes = []
        L.hdc_last_error.restype = ctypes.c_char_p
        L.hdc_version.argtypes = []
        L.hdc_version.restype = ctypes.c_int32
        _lib = L
        if (not os.environ.get("HDC_TUNE_CACHE") and os.environ.get("HDC_TUNE", "1") != "0"
                and os.path.exists(TUNING_CACHE)):
            _check(L.hdc_load_tuning(TUNING_CACHE.encode()))
    return _lib


def _check(status: int) -> None:
    if status != OK:
        raise HdcError(status, lib().hdc_last_error().decode())


# ---------------------------------------------------------------------------
# Callables
# ---------------------------------------------------------------------------

def identity() -> dict:
    return {"fn": "identity"}


def affine(a, b) -> dict:
    return {"fn": "affine", "a": a, "b": b}


def horner(coef) -> dict:
    return {"fn": "horner", "coef": list(coef)}


def product() -> dict:
    return {"fn": "product"}


def make_functor(spec) -> Functor:
    if isinstance(spec, Functor):
        return spec
    f = Functor()
    f.id = FN[spec["fn"]]
    if spec["fn"] == "affine":
        a, b = spec["a"], spec["b"]
        f.a, f.b = float(a), float(b)
        if isinstance(a, int) and isinstance(b, int):
            f.ia, f.ib = a, b
    elif spec["fn"] == "horner":
        c = list(spec["coef"])
        if not 1 <= len(c) <= MAX_DEGREE + 1:
            raise ValueError(f"horner needs 1..{MAX_DEGREE + 1} coefficients")
        f.degree = len(c) - 1
        for k, v in enumerate(c):
            f.coef[k] = float(v)
    return f


# ---------------------------------------------------------------------------
# Marshalling helpers
# ---------------------------------------------------------------------------

def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _gpu_tensor(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _dtype(t: torch.Tensor) -> int:
    if t.dtype not in DTYPE:
        raise ValueError(f"unsupported dtype {t.dtype}")
    return DTYPE[t.dtype]


def _acc(acc) -> int:
    return ACC[acc] if isinstance(acc, str) else int(acc)


_workspaces: dict = {}


def workspace_size(op: int, dtype: int, acc: int, n: int, num_segments: int = 0) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().hdc_workspace_size(op, dtype, acc, n, num_segments, ctypes.byref(b)))
    return b.value


def workspace(device, op: int, dtype: int, acc: int, n: int, num_segments: int = 0) -> torch.Tensor:
    """A cached device workspace for the current stream of ``device``, large enough for the call."""
    need = workspace_size(op, dtype, acc, n, num_segments)
    stream = torch.cuda.current_stream(device).cuda_stream
    key = (torch.device(device).index, stream)
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < need:
        # zero-filled on first allocation; every kernel leaves it reusable
        ws = torch.zeros(max(need, 256), dtype=torch.uint8, device=device)
        _workspaces[key] = ws
    return ws


# ---------------------------------------------------------------------------
# Operations
# ---------------------------------------------------------------------------

def map(x: torch.Tensor, fn, out: torch.Tensor | None = None) -> torch.Tensor:
    """y[i] = fn(x[i]) in x's dtype (``out`` may be ``x`` for in place)."""
    x = _gpu_tensor(x, "x")
    y = torch.empty_like(x) if out is None else _gpu_tensor(out, "out")
    if y.dtype != x.dtype or y.numel() != x.numel():
        raise ValueError("out must match x in dtype and size")
    f = make_functor(fn)
    _check(lib().hdc_map(ctypes.byref(f), _dtype(x), x.data_ptr(), y.data_ptr(), x.numel(), _stream(x)))
    return y


def transform_reduce(x: torch.Tensor, fn, acc="plain", z: torch.Tensor | None = None,
                     out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """sum_i fn(x[i]) (or sum_i x[i]*z[i] for product()) as a 0-d device tensor:
    float32 (plain), float64 (compensated, exact) or int64 (exact_int)."""
    x = _gpu_tensor(x, "x")
    a = _acc(acc)
    dt = _dtype(x)
    zp = None
    if z is not None:
        z = _gpu_tensor(z, "z")
        if z.dtype != x.dtype or z.numel() != x.numel():
            raise ValueError("z must match x in dtype and size")
        zp = z.data_ptr()
    r = torch.empty((), dtype=OUT_DTYPE[a], device=x.device) if out is None else out
    if ws is None:
        ws = workspace(x.device, OP_TRANSFORM_REDUCE, dt, a, x.numel())
    f = make_functor(fn)
    _check(lib().hdc_transform_reduce(ctypes.byref(f), dt, x.data_ptr(), zp, x.numel(), a, r.data_ptr(),
                                      ws.data_ptr(), ws.numel(), _stream(x)))
    return r


def transform_reduce_noalloc(x: torch.Tensor, fn, acc="plain", z: torch.Tensor | None = None,
                             out: torch.Tensor | None = None) -> torch.Tensor:
    """transform_reduce through hdc_transform_reduce_noalloc: no workspace, the partials go to
    the library's per-device scratch array.  Pass ``out`` to keep the call free of allocations."""
    x = _gpu_tensor(x, "x")
    a = _acc(acc)
    dt = _dtype(x)
    zp = None
    if z is not None:
        z = _gpu_tensor(z, "z")
        if z.dtype != x.dtype or z.numel() != x.numel():
            raise ValueError("z must match x in dtype and size")
        zp = z.data_ptr()
    r = torch.empty((), dtype=OUT_DTYPE[a], device=x.device) if out is None else out
    f = make_functor(fn)
    _check(lib().hdc_transform_reduce_noalloc(ctypes.byref(f), dt, x.data_ptr(), zp, x.numel(), a, r.data_ptr(),
                                              _stream(x)))
    return r


def map_reduce(x: torch.Tensor, map_fn, reduce_fn, acc="plain", out: torch.Tensor | None = None,
               result: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Fused: y = map(x, map_fn) and r = transform_reduce(x, reduce_fn, acc), reading x once."""
    x = _gpu_tensor(x, "x")
    a = _acc(acc)
    dt = _dtype(x)
    y = torch.empty_like(x) if out is None else _gpu_tensor(out, "out")
    r = torch.empty((), dtype=OUT_DTYPE[a], device=x.device) if result is None else result
    if ws is None:
        ws = workspace(x.device, OP_MAP_REDUCE, dt, a, x.numel())
    f, g = make_functor(map_fn), make_functor(reduce_fn)
    _check(lib().hdc_map_reduce(ctypes.byref(f), ctypes.byref(g), dt, x.data_ptr(), y.data_ptr(), x.numel(), a,
                                r.data_ptr(), ws.data_ptr(), ws.numel(), _stream(x)))
    return y, r


def segmented_reduce(x: torch.Tensor, offsets: torch.Tensor, fn, acc="plain",
                     out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """out[j] = sum_{offsets[j] <= i < offsets[j+1]} fn(x[i]) for every segment j
    (offsets[S] <= x.numel(); the default workspace is sized for x.numel())."""
    x = _gpu_tensor(x, "x")
    offsets = _gpu_tensor(offsets, "offsets")
    if offsets.dtype != torch.int64:
        raise ValueError("offsets must be int64")
    a = _acc(acc)
    dt = _dtype(x)
    S = offsets.numel() - 1
    if S < 0:
        raise ValueError("offsets needs at least one entry")
    r = torch.empty(S, dtype=OUT_DTYPE[a], device=x.device) if out is None else out
    if ws is None:
        ws = workspace(x.device, OP_SEGMENTED_REDUCE, dt, a, x.numel(), S)
    f = make_functor(fn)
    _check(lib().hdc_segmented_reduce(ctypes.byref(f), dt, x.data_ptr(), offsets.data_ptr(), S, a,
                                      r.data_ptr(), ws.data_ptr(), ws.numel(), _stream(x)))
    return r


def batch_map_reduce(xs, map_fn, reduce_fn, acc="plain", ys=None, outs=None, ws=None):
    """Grouped form of many map_reduce calls of one class: ys[i] = map_fn(xs[i])
    (skipped when map_fn is None or ys[i] is None) and outs[i] = the fold of
    reduce_fn over xs[i].  Returns (ys, outs)."""
    if not xs:
        return [], []
    a = _acc(acc)
    dt = _dtype(xs[0])
    dev = xs[0].device
    if ys is None:
        ys = [torch.empty_like(x) for x in xs] if map_fn is not None else [None] * len(xs)
    if outs is None:
        outs = [torch.empty((), dtype=OUT_DTYPE[a], device=dev) for _ in xs]
    table = (BatchCall * len(xs))()
    for i, x in enumerate(xs):
        _gpu_tensor(x, "x")
        if _dtype(x) != dt:
            raise ValueError("all calls of a batch share one dtype")
        y = ys[i]
        table[i].x = x.data_ptr()
        table[i].y = y.data_ptr() if (y is not None and map_fn is not None) else None
        table[i].n = x.numel()
        table[i].out = outs[i].data_ptr()
    if ws is None:
        ws = workspace(dev, OP_BATCH, dt, a, sum(x.numel() for x in xs), len(xs))
    f = ctypes.byref(make_functor(map_fn)) if map_fn is not None else None
    g = make_functor(reduce_fn)
    _check(lib().hdc_batch_map_reduce(f, ctypes.byref(g), dt, a, table, len(xs), ws.data_ptr(), ws.numel(),
                                      _stream(xs[0])))
    return ys, outs


def scan_status(ws: torch.Tensor) -> int:
    """The status word of the last scan run with workspace ``ws`` (hdc_scan_status), read
    synchronously: 0 = its output is valid, nonzero = a wait gave up and the output is invalid."""
    st = torch.zeros((), dtype=torch.int32, device=ws.device)
    _check(lib().hdc_scan_status(ws.data_ptr(), st.data_ptr(), _stream(ws)))
    return int(st.item())


def _check_scan(ws: torch.Tensor, check: bool) -> None:
    # a synchronous read, skipped while the stream is being captured into a graph
    if check and not torch.cuda.is_current_stream_capturing():
        if scan_status(ws) != 0:
            raise HdcError(ERR_HIP, "a wait of the single-pass scan gave up; the output is invalid")


def scan(x: torch.Tensor, fn, acc="plain", exclusive: bool = False, out: torch.Tensor | None = None,
         ws: torch.Tensor | None = None, check: bool = True) -> torch.Tensor:
    """Prefix sums of fn(x): float32 (plain), float64 (compensated) or int64 (exact_int).
    ``check`` reads the scan's status word afterwards (a stream synchronisation) and raises
    HdcError if the single pass gave up; pass False to keep the call asynchronous and read
    ``scan_status(ws)`` later."""
    x = _gpu_tensor(x, "x")
    a = _acc(acc)
    dt = _dtype(x)
    y = torch.empty(x.numel(), dtype=OUT_DTYPE[a], device=x.device) if out is None else _gpu_tensor(out, "out")
    if ws is None:
        ws = workspace(x.device, OP_SCAN, dt, a, x.numel())
    f = make_functor(fn)
    _check(lib().hdc_scan(ctypes.byref(f), dt, x.data_ptr(), y.data_ptr(), x.numel(), a, int(exclusive),
                          ws.data_ptr(), ws.numel(), _stream(x)))
    if x.numel() > 0:
        _check_scan(ws, check)
    return y


def segmented_scan(x: torch.Tensor, offsets: torch.Tensor, fn, acc="plain", exclusive: bool = False,
                   total: int | None = None, out: torch.Tensor | None = None,
                   ws: torch.Tensor | None = None, check: bool = True) -> torch.Tensor:
    """Prefix sums of fn(x) restarting at every segment start (offsets: int64 CSR on the GPU).
    Positions outside every segment keep the contents of `out` (zeros when it is allocated here).
    ``check`` as for scan()."""
    x = _gpu_tensor(x, "x")
    offsets = _gpu_tensor(offsets, "offsets")
    if offsets.dtype != torch.int64:
        raise ValueError("offsets must be int64")
    a = _acc(acc)
    dt = _dtype(x)
    S = offsets.numel() - 1
    if S < 0:
        raise ValueError("offsets needs at least one entry")
    total = x.numel() if total is None else int(total)
    y = torch.zeros(total, dtype=OUT_DTYPE[a], device=x.device) if out is None else _gpu_tensor(out, "out")
    if ws is None:
        ws = workspace(x.device, OP_SCAN, dt, a, total)
    f = make_functor(fn)
    _check(lib().hdc_segmented_scan(ctypes.byref(f), dt, x.data_ptr(), offsets.data_ptr(), S, total,
                                    y.data_ptr(), a, int(exclusive), ws.data_ptr(), ws.numel(), _stream(x)))
    if S > 0 and total > 0:
        _check_scan(ws, check)
    return y


def _host_tensor(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cpu":
        raise ValueError(f"{name} must be a CPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def host_map(x: torch.Tensor, fn, out: torch.Tensor | None = None, threads: int = 0) -> torch.Tensor:
    """The host side of map: the same callables on CPU tensors (synchronous)."""
    x = _host_tensor(x, "x")
    y = torch.empty_like(x) if out is None else _host_tensor(out, "out")
    f = make_functor(fn)
    _check(lib().hdc_host_map(ctypes.byref(f), _dtype(x), x.data_ptr(), y.data_ptr(), x.numel(), threads))
    return y


def host_transform_reduce(x: torch.Tensor, fn, acc="plain", z: torch.Tensor | None = None,
                          threads: int = 0) -> torch.Tensor:
    """The host side of transform_reduce on CPU tensors (synchronous); 0-d CPU tensor."""
    x = _host_tensor(x, "x")
    a = _acc(acc)
    zp = _host_tensor(z, "z").data_ptr() if z is not None else None
    r = torch.empty((), dtype=OUT_DTYPE[a])
    f = make_functor(fn)
    _check(lib().hdc_host_transform_reduce(ctypes.byref(f), _dtype(x), x.data_ptr(), zp, x.numel(), a,
                                           r.data_ptr(), threads))
    return r


def validate_offsets(offsets: torch.Tensor, total: int) -> None:
    offsets = _gpu_tensor(offsets, "offsets")
    _check(lib().hdc_validate_offsets(offsets.data_ptr(), offsets.numel() - 1, total, _stream(offsets)))


BUCKETS = 4


def tuning_bucket(n: int) -> int:
    b = ctypes.c_int32(0)
    _check(lib().hdc_tuning_bucket(n, ctypes.byref(b)))
    return b.value


def set_tuning(op: int, dtype: int, acc: int, bucket: int = -1, block=0, unroll=0, grid_mult=0, chunk=0,
               small_seg=0, seg_per_wave=0, passes=0) -> None:
    """Set a tuning class; bucket -1 sets every size bucket; 0 keeps a field."""
    t = Tuning(block, unroll, grid_mult, chunk, small_seg, seg_per_wave, passes)
    _check(lib().hdc_set_tuning(op, dtype, acc, bucket, ctypes.byref(t)))


def get_tuning(op: int, dtype: int, acc: int, bucket: int = 3) -> dict:
    t = Tuning()
    _check(lib().hdc_get_tuning(op, dtype, acc, bucket, ctypes.byref(t)))
    return {"block": t.block, "unroll": t.unroll, "grid_mult": t.grid_mult, "chunk": t.chunk,
            "small_seg": t.small_seg, "seg_per_wave": t.seg_per_wave, "passes": t.passes}


def load_tuning(path: str | None = None) -> None:
    _check(lib().hdc_load_tuning(None if path is None else path.encode()))


def version() -> int:
    return lib().hdc_version()
