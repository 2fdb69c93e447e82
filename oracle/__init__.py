"""Python access to the C oracle (oracle.c): TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library: it has
its own C source, header, functor layout and binding, and it never loads the
GPU library.

Callables are described by plain dicts (test data):
    {"fn": "identity"}
    {"fn": "affine", "a": 2.5, "b": 0.5}            (floating point)
    {"fn": "affine", "a": 3, "b": -7}               (integers: wrapping)
    {"fn": "horner", "coef": [c0, c1, ..., cd]}     (p(x) = sum c_k x^k)
    {"fn": "product"}                               (dot-product term x*z)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# HDC_ORACLE_LIBRARY / HDC_ORACLE_MT_LIBRARY name other builds of the same
# sources (the sanitized ones of build_sanitized()).
LIB_PATH = os.environ.get("HDC_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]

KINDS = {"identity": 0, "affine": 1, "horner": 2, "product": 3}
DTYPES = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2, torch.int32: 3}
MAX_DEGREE = 16


class OrFn(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("degree", ctypes.c_int),
                ("a", ctypes.c_float), ("b", ctypes.c_float),
                ("coef", ctypes.c_float * (MAX_DEGREE + 1)),
                ("ia", ctypes.c_int64), ("ib", ctypes.c_int64)]


class OrResult(ctypes.Structure):
    _fields_ = [("exact", ctypes.c_double), ("seq64", ctypes.c_double),
                ("abs_sum", ctypes.c_double), ("isum", ctypes.c_int64)]


MT_LIB_PATH = os.environ.get("HDC_ORACLE_MT_LIBRARY") or os.path.join(HERE, "liboracle_mt.so")
SAN_DIR = os.path.join(HERE, "_build")


def build() -> str:
    """Compile liboracle.so and liboracle_mt.so (the same oracle on several host
    threads, for the multicore CPU baseline) with gcc (always recompiles)."""
    for src, out, extra in ((os.path.join(HERE, "oracle.c"), LIB_PATH, []),
                            (os.path.join(HERE, "oracle_mt.c"), MT_LIB_PATH, ["-lpthread"])):
        tmp = out + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, src, "-lm", *extra], check=True)
        os.replace(tmp, out)
    return LIB_PATH


def build_sanitized() -> tuple[str, str]:
    """liboracle.so and liboracle_mt.so built by clang with AddressSanitizer and
    UndefinedBehaviorSanitizer into oracle/_build/ (for the CPU sanitizer test)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    flags = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-shared-libsan"]
    outs = []
    for src, name, extra in (("oracle.c", "liboracle.so", []), ("oracle_mt.c", "liboracle_mt.so", ["-lpthread"])):
        out = os.path.join(SAN_DIR, name)
        subprocess.run(["/opt/rocm/llvm/bin/clang", *flags, "-o", out, os.path.join(HERE, src), "-lm", *extra],
                       check=True)
        outs.append(out)
    return outs[0], outs[1]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.or_decode_f16.restype = ctypes.c_double
        L.or_decode_f16.argtypes = [ctypes.c_uint16]
        L.or_decode_bf16.restype = ctypes.c_double
        L.or_decode_bf16.argtypes = [ctypes.c_uint16]
        L.or_encode_f16.restype = ctypes.c_uint16
        L.or_encode_f16.argtypes = [ctypes.c_float]
        L.or_encode_bf16.restype = ctypes.c_uint16
        L.or_encode_bf16.argtypes = [ctypes.c_float]
        L.or_term_f32.restype = ctypes.c_float
        L.or_term_f32.argtypes = [P(OrFn), ctypes.c_float]
        L.or_term_f64.restype = ctypes.c_double
        L.or_term_f64.argtypes = [P(OrFn), ctypes.c_double]
        L.or_map.restype = ctypes.c_int
        L.or_map.argtypes = [P(OrFn), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.or_reduce.restype = ctypes.c_int
        L.or_reduce.argtypes = [P(OrFn), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_int64, P(OrResult)]
        L.or_segmented.restype = ctypes.c_int
        L.or_segmented.argtypes = [P(OrFn), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int64, P(OrResult)]
        L.or_scan.restype = ctypes.c_int
        L.or_scan.argtypes = [P(OrFn), ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_exact_sum.restype = ctypes.c_double
        L.or_exact_sum.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        _lib = L
    return _lib


_mt_lib = None


def mt_lib():
    global _mt_lib
    if _mt_lib is None:
        if not os.path.exists(MT_LIB_PATH):
            build()
        L = ctypes.CDLL(MT_LIB_PATH)
        P = ctypes.POINTER
        L.or_reduce_mt.restype = ctypes.c_int
        L.or_reduce_mt.argtypes = [P(OrFn), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_int, P(OrResult)]
        L.or_map_mt.restype = ctypes.c_int
        L.or_map_mt.argtypes = [P(OrFn), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_int]
        _mt_lib = L
    return _mt_lib


def host_threads() -> int:
    """Host cores this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def make_fn(spec: dict) -> OrFn:
    f = OrFn()
    f.kind = KINDS[spec["fn"]]
    if spec["fn"] == "affine":
        if isinstance(spec["a"], int) and isinstance(spec["b"], int):
            f.ia, f.ib = spec["a"], spec["b"]
        f.a, f.b = float(spec["a"]), float(spec["b"])
    if spec["fn"] == "horner":
        c = list(spec["coef"])
        if not 1 <= len(c) <= MAX_DEGREE + 1:
            raise ValueError("degree out of range")
        f.degree = len(c) - 1
        for k, v in enumerate(c):
            f.coef[k] = v
    return f


def _host(t: torch.Tensor) -> torch.Tensor:
    t = t.detach()
    if t.device.type != "cpu":
        t = t.cpu()
    return t.contiguous()


def map(spec: dict, x: torch.Tensor) -> torch.Tensor:
    """y = f(x) element by element (CPU tensor of x's dtype)."""
    x = _host(x)
    y = torch.empty_like(x)
    f = make_fn(spec)
    if lib().or_map(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), y.data_ptr(), x.numel()) != 0:
        raise ValueError("oracle: unsupported map")
    return y


def reduce(spec: dict, x: torch.Tensor, z: torch.Tensor | None = None) -> dict:
    """Reference values of the fold of f over x (dict: exact, seq64, abs_sum, isum)."""
    x = _host(x)
    zp = None
    if z is not None:
        z = _host(z)
        assert z.dtype == x.dtype and z.numel() == x.numel()
        zp = z.data_ptr()
    f = make_fn(spec)
    r = OrResult()
    if lib().or_reduce(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), zp, x.numel(),
                       ctypes.byref(r)) != 0:
        raise ValueError("oracle: unsupported reduce")
    return {"exact": r.exact, "seq64": r.seq64, "abs_sum": r.abs_sum, "isum": r.isum}


def map_mt(spec: dict, x: torch.Tensor, threads: int | None = None) -> torch.Tensor:
    """map() on `threads` host threads (default: every core of the affinity mask)."""
    x = _host(x)
    y = torch.empty_like(x)
    f = make_fn(spec)
    if mt_lib().or_map_mt(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), y.data_ptr(), x.numel(),
                          threads or host_threads()) != 0:
        raise ValueError("oracle: unsupported map")
    return y


def reduce_mt(spec: dict, x: torch.Tensor, z: torch.Tensor | None = None, threads: int | None = None) -> dict:
    """reduce() on `threads` host threads: the same exact and integer results; seq64 is the
    in-order sum of the per-thread fp64 sums."""
    x = _host(x)
    zp = None
    if z is not None:
        z = _host(z)
        assert z.dtype == x.dtype and z.numel() == x.numel()
        zp = z.data_ptr()
    f = make_fn(spec)
    r = OrResult()
    if mt_lib().or_reduce_mt(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), zp, x.numel(),
                             threads or host_threads(), ctypes.byref(r)) != 0:
        raise ValueError("oracle: unsupported reduce")
    return {"exact": r.exact, "seq64": r.seq64, "abs_sum": r.abs_sum, "isum": r.isum}


def segmented(spec: dict, x: torch.Tensor, offsets: torch.Tensor) -> dict:
    """Per-segment reference values (numpy arrays: exact, seq64, abs_sum, isum)."""
    x = _host(x)
    off = _host(offsets).to(torch.int64)
    S = off.numel() - 1
    res = (OrResult * max(S, 1))()
    f = make_fn(spec)
    if lib().or_segmented(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), off.data_ptr(), S,
                          res) != 0:
        raise ValueError("oracle: unsupported segmented reduce")
    out = {
        "exact": np.array([res[j].exact for j in range(S)]),
        "seq64": np.array([res[j].seq64 for j in range(S)]),
        "abs_sum": np.array([res[j].abs_sum for j in range(S)]),
        "isum": np.array([res[j].isum for j in range(S)], dtype=np.int64),
    }
    return out


def scan(spec: dict, x: torch.Tensor, exclusive: bool = False) -> dict:
    """Prefix sums of f(x) (numpy arrays): exact / abs_sum for floats, isum for int32."""
    x = _host(x)
    n = x.numel()
    f = make_fn(spec)
    if x.dtype == torch.int32:
        out = np.zeros(n, dtype=np.int64)
        if lib().or_scan(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), n, int(exclusive), None, None,
                         out.ctypes.data) != 0:
            raise ValueError("oracle: unsupported scan")
        return {"isum": out}
    ex = np.zeros(n)
    ab = np.zeros(n)
    if lib().or_scan(ctypes.byref(f), DTYPES[x.dtype], x.data_ptr(), n, int(exclusive), ex.ctypes.data,
                     ab.ctypes.data, None) != 0:
        raise ValueError("oracle: unsupported scan")
    return {"exact": ex, "abs_sum": ab}


def segmented_scan(spec: dict, x: torch.Tensor, offsets: torch.Tensor, exclusive: bool = False) -> dict:
    """Prefix sums restarting at every segment start: the scan definition applied to each segment
    [offsets[j], offsets[j+1]) on its own.  Arrays over all n positions; positions outside every
    segment hold NaN (floats) or 0 (int32) and are not part of the result."""
    x = _host(x)
    off = _host(offsets).to(torch.int64)
    n = x.numel()
    f = make_fn(spec)
    es = x.element_size()
    is_int = x.dtype == torch.int32
    if is_int:
        out = np.zeros(n, dtype=np.int64)
    else:
        ex = np.full(n, np.nan)
        ab = np.full(n, np.nan)
    for j in range(off.numel() - 1):
        lo, hi = int(off[j]), int(off[j + 1])
        if hi <= lo:
            continue
        xp = x.data_ptr() + lo * es
        if is_int:
            rc = lib().or_scan(ctypes.byref(f), DTYPES[x.dtype], xp, hi - lo, int(exclusive), None, None,
                               out.ctypes.data + lo * 8)
        else:
            rc = lib().or_scan(ctypes.byref(f), DTYPES[x.dtype], xp, hi - lo, int(exclusive),
                               ex.ctypes.data + lo * 8, ab.ctypes.data + lo * 8, None)
        if rc != 0:
            raise ValueError("oracle: unsupported segmented scan")
    return {"isum": out} if is_int else {"exact": ex, "abs_sum": ab}


def exact_sum(v) -> float:
    """Exact sum of float64 values, rounded once to float64."""
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return lib().or_exact_sum(a.ctypes.data, a.size)


def term_f32(spec: dict, x: float) -> float:
    f = make_fn(spec)
    return lib().or_term_f32(ctypes.byref(f), x)


def term_f64(spec: dict, x: float) -> float:
    f = make_fn(spec)
    return lib().or_term_f64(ctypes.byref(f), x)


def encode_f16(v: float) -> int:
    return lib().or_encode_f16(v)


def encode_bf16(v: float) -> int:
    return lib().or_encode_bf16(v)


def decode_f16(h: int) -> float:
    return lib().or_decode_f16(h)


def decode_bf16(h: int) -> float:
    return lib().or_decode_bf16(h)


def time_reduce(spec: dict, x: torch.Tensor, z: torch.Tensor | None = None, repeats: int = 1):
    """Wall time (s, best of ``repeats``) of one oracle reduction on the calling thread."""
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        reduce(spec, x, z)
        best = min(best, time.perf_counter() - t0)
    return best


def time_map(spec: dict, x: torch.Tensor, repeats: int = 1):
    best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        map(spec, x)
        best = min(best, time.perf_counter() - t0)
    return best
