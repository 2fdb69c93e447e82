"""The C-ABI boundary without a GPU: the library loads, exports every symbol the
header declares, and rejects every invalid argument on the host before
anything is enqueued (the calls below never reach the HIP runtime)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2309_03912_amd as hdc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdc.h")
FAKE = 0x10000  # a well-aligned, never dereferenced "device" address


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = hdc.lib()
    names = declared_functions()
    assert set(names) == set(hdc.EXPORTS)
    for name in names:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", hdc.LIB_PATH], capture_output=True, text=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}$", out, flags=re.M), name


def test_status_strings_and_version():
    L = hdc.lib()
    assert L.hdc_status_string(0) == b"HDC_OK"
    assert L.hdc_status_string(3) == b"HDC_ERR_WORKSPACE"
    assert hdc.version() >= 100


def fn(spec):
    return ctypes.byref(hdc.make_functor(spec))


def last():
    return hdc.lib().hdc_last_error().decode()


def test_map_rejects_bad_arguments():
    L = hdc.lib()
    ident = fn({"fn": "identity"})
    assert L.hdc_map(None, hdc.F32, FAKE, FAKE, 4, None) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_map(ident, hdc.F32, FAKE, FAKE, -1, None) == hdc.ERR_INVALID_ARGUMENT
    assert "negative" in last()
    assert L.hdc_map(ident, hdc.F32, None, FAKE, 4, None) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_map(ident, hdc.F32, FAKE, None, 4, None) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_map(ident, hdc.F32, FAKE + 2, FAKE + 64, 4, None) == hdc.ERR_INVALID_ARGUMENT  # misaligned
    assert L.hdc_map(ident, hdc.F32, FAKE, FAKE + 4, 4, None) == hdc.ERR_INVALID_ARGUMENT      # partial overlap
    assert "overlap" in last()
    assert L.hdc_map(fn({"fn": "horner", "coef": [1.0]}), hdc.I32, FAKE, FAKE + 64, 4, None) == hdc.ERR_UNSUPPORTED
    assert L.hdc_map(fn({"fn": "product"}), hdc.F32, FAKE, FAKE + 64, 4, None) == hdc.ERR_UNSUPPORTED
    assert L.hdc_map(ident, hdc.I64, FAKE, FAKE + 64, 4, None) == hdc.ERR_UNSUPPORTED
    assert L.hdc_map(ident, 17, FAKE, FAKE + 64, 4, None) == hdc.ERR_INVALID_ARGUMENT
    bad = hdc.make_functor({"fn": "horner", "coef": [1.0]})
    bad.degree = 17
    assert L.hdc_map(ctypes.byref(bad), hdc.F32, FAKE, FAKE + 64, 4, None) == hdc.ERR_INVALID_ARGUMENT
    bad.id = 9
    assert L.hdc_map(ctypes.byref(bad), hdc.F32, FAKE, FAKE + 64, 4, None) == hdc.ERR_INVALID_ARGUMENT
    # n == 0 is a no-op that needs no pointers and no device
    assert L.hdc_map(ident, hdc.F32, None, None, 0, None) == hdc.OK


def test_transform_reduce_rejects_bad_arguments():
    L = hdc.lib()
    ident = fn({"fn": "identity"})
    need = hdc.workspace_size(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, 100)
    args = lambda **k: (k.get("f", ident), k.get("dt", hdc.F32), k.get("x", FAKE), k.get("z", None),
                        k.get("n", 100), k.get("acc", hdc.ACC_PLAIN), k.get("out", FAKE),
                        k.get("ws", FAKE), k.get("wsb", need), None)
    assert L.hdc_transform_reduce(*args(n=-5)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce(*args(x=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce(*args(out=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce(*args(acc=hdc.ACC_EXACT_INT)) == hdc.ERR_UNSUPPORTED
    assert L.hdc_transform_reduce(*args(dt=hdc.I32)) == hdc.ERR_UNSUPPORTED          # int needs EXACT_INT
    assert L.hdc_transform_reduce(*args(acc=7)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce(*args(f=fn({"fn": "product"}))) == hdc.ERR_UNSUPPORTED  # no z
    assert L.hdc_transform_reduce(*args(f=fn({"fn": "product"}), z=FAKE + 1)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce(*args(dt=hdc.I32, acc=hdc.ACC_EXACT_INT,
                                        f=fn({"fn": "horner", "coef": [1.0]}))) == hdc.ERR_UNSUPPORTED
    assert L.hdc_transform_reduce(*args(acc=hdc.ACC_EXACT)) == hdc.ERR_UNSUPPORTED            # exact: 16-bit only
    assert L.hdc_transform_reduce(*args(acc=hdc.ACC_EXACT, dt=hdc.F16,
                                        f=fn({"fn": "horner", "coef": [1.0]}))) == hdc.ERR_UNSUPPORTED
    prod = fn({"fn": "product"})
    assert L.hdc_transform_reduce(*args(acc=hdc.ACC_EXACT, dt=hdc.BF16, f=prod, z=FAKE)) == hdc.ERR_UNSUPPORTED
    assert "PRODUCT (fp16)" in last()                                                   # exact dot: fp16 only
    assert L.hdc_transform_reduce(*args(acc=hdc.ACC_EXACT, dt=hdc.F16, f=prod, z=FAKE,
                                        n=1 << 31)) == hdc.ERR_UNSUPPORTED
    assert "2^31" in last()
    assert L.hdc_transform_reduce(*args(wsb=need - 1)) == hdc.ERR_WORKSPACE
    assert "smaller" in last()
    assert L.hdc_transform_reduce(*args(ws=FAKE + 8)) == hdc.ERR_INVALID_ARGUMENT
    assert "256-byte aligned" in last()


def test_transform_reduce_noalloc_rejects_bad_arguments():
    L = hdc.lib()
    ident = fn({"fn": "identity"})
    args = lambda **k: (k.get("f", ident), k.get("dt", hdc.F32), k.get("x", FAKE), k.get("z", None),
                        k.get("n", 100), k.get("acc", hdc.ACC_PLAIN), k.get("out", FAKE), None)
    assert L.hdc_transform_reduce_noalloc(*args(f=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce_noalloc(*args(n=-5)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce_noalloc(*args(x=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce_noalloc(*args(x=FAKE + 2)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce_noalloc(*args(out=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_transform_reduce_noalloc(*args(acc=hdc.ACC_EXACT_INT)) == hdc.ERR_UNSUPPORTED
    assert L.hdc_transform_reduce_noalloc(*args(f=fn({"fn": "product"}))) == hdc.ERR_UNSUPPORTED  # no z
    assert L.hdc_transform_reduce_noalloc(*args(acc=hdc.ACC_EXACT)) == hdc.ERR_UNSUPPORTED


def test_map_reduce_and_segmented_reject_bad_arguments():
    L = hdc.lib()
    ident = fn({"fn": "identity"})
    need = hdc.workspace_size(hdc.OP_MAP_REDUCE, hdc.F32, hdc.ACC_PLAIN, 100)
    assert L.hdc_map_reduce(None, ident, hdc.F32, FAKE, FAKE + 4096, 100, 0, FAKE, FAKE, need, None) \
        == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_map_reduce(ident, ident, hdc.F32, FAKE, FAKE, 100, 0, FAKE, FAKE, need, None) \
        == hdc.ERR_INVALID_ARGUMENT  # in place is not allowed for the fused form
    assert L.hdc_map_reduce(ident, fn({"fn": "product"}), hdc.F32, FAKE, FAKE + 4096, 100, 0, FAKE, FAKE, need,
                            None) == hdc.ERR_UNSUPPORTED
    sneed = hdc.workspace_size(hdc.OP_SEGMENTED_REDUCE, hdc.F32, hdc.ACC_PLAIN, 1000, 10)
    # the section 8(b) signature: (f, dt, x, offsets, S, acc, out, workspace, ws_bytes, stream)
    assert [a.__name__ for a in L.hdc_segmented_reduce.argtypes[1:]] == [
        "c_int", "c_void_p", "c_void_p", "c_long", "c_int", "c_void_p", "c_void_p", "c_ulong", "c_void_p"]
    assert L.hdc_segmented_reduce(ident, hdc.F32, FAKE, FAKE, -1, 0, FAKE, FAKE, sneed, None) \
        == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_reduce(ident, hdc.F32, FAKE, None, 10, 0, FAKE, FAKE, sneed, None) \
        == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_reduce(fn({"fn": "product"}), hdc.F32, FAKE, FAKE, 10, 0, FAKE, FAKE, sneed,
                                  None) == hdc.ERR_UNSUPPORTED
    assert L.hdc_segmented_reduce(ident, hdc.F32, FAKE, FAKE, 0, 0, FAKE, FAKE, 0, None) == hdc.OK  # S = 0
    assert L.hdc_segmented_reduce(ident, hdc.F32, FAKE, FAKE, 10, 0, None, FAKE, sneed, None) \
        == hdc.ERR_INVALID_ARGUMENT  # out NULL
    assert L.hdc_segmented_reduce(ident, hdc.F32, FAKE, FAKE, 10, 0, FAKE, FAKE + 8, sneed, None) \
        == hdc.ERR_INVALID_ARGUMENT  # workspace not 256-byte aligned
    small = hdc.workspace_size(hdc.OP_SEGMENTED_REDUCE, hdc.F32, hdc.ACC_PLAIN, 0, 10)
    assert L.hdc_segmented_reduce(ident, hdc.F32, FAKE, FAKE, 10, 0, FAKE, FAKE, small - 1, None) \
        == hdc.ERR_WORKSPACE  # below the bound for 10 segments at any total
    assert "smaller" in last()


def test_scan_status_rejects_bad_arguments():
    L = hdc.lib()
    assert L.hdc_scan_status(FAKE, None, None) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_scan_status(FAKE + 8, FAKE, None) == hdc.ERR_INVALID_ARGUMENT
    assert "256-byte aligned" in last()


def test_workspace_sizes():
    assert hdc.workspace_size(hdc.OP_MAP, hdc.F32, 0, 1 << 20) == 0
    a = hdc.workspace_size(hdc.OP_TRANSFORM_REDUCE, hdc.F32, 0, 1 << 28)
    assert hdc.workspace_size(hdc.OP_DOT, hdc.F32, 0, 1 << 28) == a
    assert 0 < a <= 1 << 22
    with pytest.raises(hdc.HdcError):
        hdc.workspace_size(99, hdc.F32, 0, 10)
    with pytest.raises(hdc.HdcError):
        hdc.workspace_size(hdc.OP_MAP, hdc.F32, 0, -1)


def test_tuning_roundtrip_and_cache(tmp_path):
    hdc.set_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, block=512, unroll=2)
    for b in range(hdc.BUCKETS):
        t = hdc.get_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, b)
        assert t["block"] == 512 and t["unroll"] == 2
    hdc.set_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, 1, block=128)
    assert hdc.get_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, 1)["block"] == 128
    before = hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, 3)
    dot = hdc.get_tuning(hdc.OP_DOT, hdc.F32, hdc.ACC_PLAIN, 3)
    hdc.set_tuning(hdc.OP_DOT, hdc.F32, hdc.ACC_PLAIN, 3, block=64 if dot["block"] != 64 else 128)
    assert hdc.get_tuning(hdc.OP_DOT, hdc.F32, hdc.ACC_PLAIN, 3)["block"] != dot["block"]
    assert hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, 3) == before  # its own class
    hdc.set_tuning(hdc.OP_DOT, hdc.F32, hdc.ACC_PLAIN, 3, **dot)
    assert hdc.get_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, 2)["block"] == 512
    assert [hdc.tuning_bucket(n) for n in (0, 65535, 65536, 1 << 20, (1 << 24) - 1, 1 << 28)] == [0, 0, 1, 2, 2, 3]
    with pytest.raises(hdc.HdcError):
        hdc.set_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, block=100)
    with pytest.raises(hdc.HdcError):
        hdc.set_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, unroll=3)
    p = tmp_path / "tune.txt"
    p.write_text("# op dtype acc bucket block unroll grid_mult chunk small_seg spw\n1 2 1 3 1024 8 4 4096 32 16\n")
    hdc.load_tuning(str(p))
    assert hdc.get_tuning(1, 2, 1, 3) == {"block": 1024, "unroll": 8, "grid_mult": 4, "chunk": 4096,
                                          "small_seg": 32, "seg_per_wave": 16, "passes": 2}
    p.write_text("1 2 1 3 1024 8 4 4096 32 16 1\n")  # with the optional passes field
    hdc.load_tuning(str(p))
    assert hdc.get_tuning(1, 2, 1, 3)["passes"] == 1
    p.write_text("1 2 1 3 1024 8 4 4096 32 16 3\n")
    with pytest.raises(hdc.HdcError):
        hdc.load_tuning(str(p))
    p.write_text("1 2 1 3 1000 8 4 4096 32 16\n")
    with pytest.raises(hdc.HdcError):
        hdc.load_tuning(str(p))
    hdc.load_tuning(str(tmp_path / "missing.txt"))  # a missing cache keeps the defaults
    hdc.set_tuning(hdc.OP_MAP, hdc.F16, hdc.ACC_PLAIN, block=256, unroll=4)
    hdc.set_tuning(1, 2, 1, block=256, unroll=4, grid_mult=8, chunk=4096, small_seg=128, seg_per_wave=8)
    hdc.set_tuning(1, 2, 1, passes=2)
    with pytest.raises(hdc.HdcError):
        hdc.set_tuning(1, 2, 1, passes=3)
    with pytest.raises(hdc.HdcError):
        hdc.set_tuning(2, 0, 0, seg_per_wave=3)
    with pytest.raises(hdc.HdcError):
        hdc.set_tuning(1, 2, 1, 4, block=256)


def _hipcc_probe(extra):
    src = os.path.join(ROOT, "tests", "compile_probes", "host_only_functor.hip")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++20", "-fsyntax-only",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2309_03912_amd", "csrc"),
           *extra, src]
    return subprocess.run(cmd, capture_output=True, text=True)


def test_host_only_callable_cannot_instantiate_a_kernel():
    bad = _hipcc_probe([])
    assert bad.returncode != 0
    assert "constraints not satisfied" in bad.stderr or "no matching" in bad.stderr
    good = _hipcc_probe(["-DPROBE_DEVICE_TAGGED"])
    assert good.returncode == 0, good.stderr


def test_scan_tree_shape_and_workspace_bound():
    """Compile-time checks of the carry tree's levels and node counts, and that its state fits the
    scan workspace for every tile size (tests/compile_probes/scan_tree.hip)."""
    src = os.path.join(ROOT, "tests", "compile_probes", "scan_tree.hip")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++20", "-fsyntax-only",
           "-fconstexpr-steps=100000000", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2309_03912_amd", "csrc"), src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_batch_and_segmented_workspace_bounds():
    """Compile-time checks, over every accepted tuning, that a grouped batch's chunks are whole block
    steps of at least 1024 elements whose partials fit the batch workspace, and that the segmented
    reduce's work-list capacity read from a workspace size covers the total that size was computed
    for (tests/compile_probes/workspace_bounds.hip)."""
    src = os.path.join(ROOT, "tests", "compile_probes", "workspace_bounds.hip")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++20", "-fsyntax-only",
           "-fconstexpr-steps=200000000", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2309_03912_amd", "csrc"), src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_segmented_scan_rejects_bad_arguments():
    L = hdc.lib()
    ident = fn({"fn": "identity"})
    need = hdc.workspace_size(hdc.OP_SCAN, hdc.F32, hdc.ACC_PLAIN, 1000)
    args = lambda **k: (k.get("f", ident), k.get("dt", hdc.F32), k.get("x", FAKE), k.get("off", FAKE + 65536),
                        k.get("S", 10), k.get("total", 1000), k.get("y", FAKE + 131072),
                        k.get("acc", hdc.ACC_PLAIN), k.get("ex", 0), k.get("ws", FAKE + 262144),
                        k.get("wsb", need), None)
    assert L.hdc_segmented_scan(*args(S=-1)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_scan(*args(total=-1)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_scan(*args(ex=2)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_scan(*args(off=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_scan(*args(off=FAKE + 4)) == hdc.ERR_INVALID_ARGUMENT    # not 8-byte aligned
    assert L.hdc_segmented_scan(*args(y=None)) == hdc.ERR_INVALID_ARGUMENT
    assert L.hdc_segmented_scan(*args(y=FAKE)) == hdc.ERR_INVALID_ARGUMENT          # overlaps x
    assert L.hdc_segmented_scan(*args(acc=hdc.ACC_EXACT_INT)) == hdc.ERR_UNSUPPORTED
    assert L.hdc_segmented_scan(*args(acc=hdc.ACC_EXACT)) == hdc.ERR_UNSUPPORTED
    assert L.hdc_segmented_scan(*args(f=fn({"fn": "product"}))) == hdc.ERR_UNSUPPORTED
    assert L.hdc_segmented_scan(*args(wsb=need - 1)) == hdc.ERR_WORKSPACE
    assert L.hdc_segmented_scan(*args(S=0)) == hdc.OK                 # nothing to do, nothing enqueued
    assert L.hdc_segmented_scan(*args(total=0)) == hdc.OK


def test_scan_rejects_bad_arguments():
    L = hdc.lib()
    ident = fn({"fn": "identity"})
    need = hdc.workspace_size(hdc.OP_SCAN, hdc.F32, hdc.ACC_PLAIN, 1000)
    assert need > 0
    call = lambda **k: L.hdc_scan(k.get("f", ident), k.get("dt", hdc.F32), k.get("x", FAKE), k.get("y", FAKE + 65536),
                                  k.get("n", 1000), k.get("acc", hdc.ACC_PLAIN), k.get("ex", 0), FAKE * 4,
                                  k.get("wsb", need), None)
    assert call(n=-1) == hdc.ERR_INVALID_ARGUMENT
    assert call(ex=2) == hdc.ERR_INVALID_ARGUMENT
    assert call(y=None) == hdc.ERR_INVALID_ARGUMENT
    assert call(y=FAKE + 100) == hdc.ERR_INVALID_ARGUMENT                   # overlaps x
    assert call(f=fn({"fn": "product"})) == hdc.ERR_UNSUPPORTED
    assert call(acc=hdc.ACC_EXACT_INT) == hdc.ERR_UNSUPPORTED
    assert call(wsb=need - 1) == hdc.ERR_WORKSPACE
    assert call(n=0, x=None, y=None) == hdc.OK
