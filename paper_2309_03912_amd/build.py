"""Build libhdc.so (the HIP library behind include/hdc.h) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libhdc.so")
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
# (source, object name, extra defines): one translation unit per kernel family,
# the fused map + reduce family once per storage type.
UNITS = [("hdc_api.hip", "hdc_api", []),
         ("hdc_run_map.hip", "hdc_run_map", []),
         ("hdc_run_reduce.hip", "hdc_run_reduce", []),
         ("hdc_run_segmented.hip", "hdc_run_segmented", []),
         ("hdc_run_batch.hip", "hdc_run_batch", []),
         ("hdc_run_host.hip", "hdc_run_host", []),
         ("hdc_run_scan.hip", "hdc_run_scan", []),
         ("hdc_run_segscan.hip", "hdc_run_segscan", [])] + [
    ("hdc_run_map_reduce.hip", f"hdc_run_map_reduce_{t.lower()}",
     [f"-DHDC_MR_STORAGE={t}", f"-DHDC_MR_NAME=run_map_reduce_{t.lower()}"]) for t in ("F32", "F16", "BF16", "I32")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-std=c++20",
    "-O3",
    "-fPIC",
    # IEEE evaluation exactly as written: no contraction into fma (every fma is
    # explicit), no fast-math; fp32 denormals are kept (the gfx950 default).
    "-ffp-contract=off",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    # host side of the callables: hardware fma (every x86-64 host of an
    # MI355X has it) instead of a libm call per fmaf
    "-Xarch_host", "-mfma", "-Xarch_host", "-mavx2",
]


def _filter(stderr: str) -> str:
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


def _compile(unit, verbose):
    src, obj, defs = unit
    out = os.path.join(BUILD_DIR, obj + ".o")
    cmd = [HIPCC, *FLAGS, *defs, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", "-o", out,
           os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + _filter(proc.stderr))
    return out


PROBE_PATH = os.path.join(HERE, "hbm_probe")


def build_probe(verbose: bool = False) -> str:
    """Compile the standalone HBM probe (csrc/hbm_probe.hip) to paper_2309_03912_amd/hbm_probe."""
    cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++20", "-O3", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wall", "-o", PROBE_PATH + ".tmp", os.path.join(CSRC, "hbm_probe.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed on hbm_probe.hip:\n" + _filter(proc.stderr))
    os.replace(PROBE_PATH + ".tmp", PROBE_PATH)
    return PROBE_PATH


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every translation unit in parallel, link libhdc.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("link failed:\n" + _filter(proc.stderr))
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


SAN_DIR = os.path.join(BUILD_DIR, "sanitized")
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime that a sanitized build needs preloaded."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("no clang AddressSanitizer runtime found under /opt/rocm/llvm")
    return hits[-1]


def build_sanitized(verbose: bool = False) -> str:
    """Every translation unit built with AddressSanitizer and
    UndefinedBehaviorSanitizer on its host side (the device code is compiled as
    usual), linked as _build/sanitized/libhdc.so: for CPU-only tests of the
    argument checks, the workspace and tuning logic and the host backend."""
    os.makedirs(SAN_DIR, exist_ok=True)
    host_flags = ["--offload-arch=gfx950", "-std=c++20", "-O1", "-g", "-fPIC",
                  "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-Wno-unused-command-line-argument",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]

    def one(unit):
        src, obj, defs = unit
        out = os.path.join(SAN_DIR, obj + ".o")
        cmd = [HIPCC, *host_flags, *defs, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", "-o", out,
               os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        proc = subprocess.run(cmd, capture_output=True, text=True)
        if proc.returncode != 0:
            raise RuntimeError(f"sanitized host compile failed on {src}:\n" + _filter(proc.stderr))
        return out

    with ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, UNITS))
    lib = os.path.join(SAN_DIR, "libhdc.so")
    # host link of the objects (no .hip source on this line)
    link = [CLANGXX, "-shared", "-fsanitize=address,undefined", "-shared-libsan", "-o", lib, *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    proc = subprocess.run(link, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("sanitized link failed:\n" + proc.stderr)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
