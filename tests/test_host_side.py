"""The host side of the callables (hdc_host_map / hdc_host_transform_reduce):
the same HstDev callables and element semantics as the kernels, run by host
threads on CPU tensors.  Checked against the oracle on the CPU (no GPU)."""
import os
import subprocess

import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOR = {"fn": "horner", "coef": synth.horner_coefficients(8)}
FAFF = {"fn": "affine", "a": 2.5, "b": 0.5}
FNS = [{"fn": "identity"}, FAFF, HOR]


def bits(t):
    return t.view(torch.int16) if t.element_size() == 2 else t.view(torch.int32)


@pytest.mark.parametrize("dt", [torch.float32, torch.float16, torch.bfloat16])
def test_host_map_bit_exact(dt):
    for n in [0, 1, 17, 100003, 1 << 18]:
        x = synth.to_storage(synth.uniform_pm1_f32(n + 1, 0, n).double() * 3, dt)
        for fn in FNS:
            for threads in (1, 3):
                y = hdc.host_map(x, fn, threads=threads)
                assert torch.equal(bits(y), bits(oracle.map(fn, x))), (fn["fn"], n, threads)


def test_host_horner_every_degree():
    """Every Horner degree (the batch evaluation enters its fma chain at the degree) against the oracle."""
    for d in range(hdc.MAX_DEGREE + 1):
        g = torch.Generator().manual_seed(1000 + d)
        c = (torch.randint(-64, 65, (d + 1,), generator=g).double() / 32.0).tolist()
        if d == 3:
            c[-1] = -0.0
        fn = {"fn": "horner", "coef": c}
        for dt in (torch.float32, torch.float16):
            x = synth.to_storage(synth.uniform_pm1_f32(d + 1, 0, 4099).double(), dt)
            assert torch.equal(bits(hdc.host_map(x, fn)), bits(oracle.map(fn, x))), (d, dt)


def test_host_map_16bit_all_patterns():
    for dt in (torch.float16, torch.bfloat16):
        x = torch.arange(-32768, 32768, dtype=torch.int32).to(torch.int16).view(dt)
        x = x[torch.isfinite(x.float())].contiguous()
        y = hdc.host_map(x, FAFF)
        ref = oracle.map(FAFF, x)
        m = ~torch.isnan(ref.float())
        assert torch.equal(torch.isnan(y.float()), torch.isnan(ref.float()))
        assert torch.equal(bits(y[m]), bits(ref[m]))


def test_host_int_map_and_sum():
    x = synth.uniform_int(3, 10, 300001)
    aff = {"fn": "affine", "a": 3, "b": -7}
    assert torch.equal(hdc.host_map(x, aff), oracle.map(aff, x))
    for threads in (1, 4):
        assert hdc.host_transform_reduce(x, aff, "exact_int", threads=threads).item() == oracle.reduce(aff, x)["isum"]


@pytest.mark.parametrize("acc", ["plain", "compensated"])
@pytest.mark.parametrize("dt", [torch.float32, torch.float16, torch.bfloat16])
def test_host_reduce_within_tolerance(acc, dt):
    for n in [0, 5, 65537, 1 << 20]:
        x = synth.to_storage(synth.uniform_pm1_f32(n + 2, 0, n).double(), dt)
        for fn in FNS:
            r = hdc.host_transform_reduce(x, fn, acc, threads=4).item()
            ref = oracle.reduce(fn, x)
            assert abs(r - ref["exact"]) <= 1e-6 * ref["abs_sum"] or (ref["abs_sum"] == 0 and r == 0)
    z = synth.to_storage(synth.normal_f64(9, 1, 1 << 16), dt)
    x = synth.to_storage(synth.normal_f64(9, 2, 1 << 16), dt)
    r = hdc.host_transform_reduce(x, {"fn": "product"}, acc, z=z).item()
    ref = oracle.reduce({"fn": "product"}, x, z)
    assert abs(r - ref["exact"]) <= 1e-6 * ref["abs_sum"]


def test_host_compensated_ill_conditioned():
    v, info = synth.ill_conditioned(synth.seed_of(3), 1 << 18, torch.float16)
    r = hdc.host_transform_reduce(v, {"fn": "identity"}, "compensated", threads=1).item()
    assert abs(r - info["target"]) <= 1e-3 * abs(info["target"])


def test_host_rejects_bad_arguments():
    with pytest.raises(ValueError):
        hdc.host_map(torch.zeros(4, device="meta"), FAFF)
    with pytest.raises(hdc.HdcError):
        hdc.host_transform_reduce(torch.zeros(4), FAFF, "exact_int")
    with pytest.raises(hdc.HdcError):
        hdc.host_transform_reduce(torch.zeros(4), {"fn": "product"})


def _probe(extra):
    src = os.path.join(ROOT, "tests", "compile_probes", "host_only_functor.hip")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++20", "-fsyntax-only",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2309_03912_amd", "csrc"),
           "-DPROBE_DEVICE_TAGGED", "-DPROBE_HOST_SIDE", *extra, src]
    return subprocess.run(cmd, capture_output=True, text=True)


def test_device_only_callable_cannot_run_on_the_host():
    good = _probe([])
    assert good.returncode == 0, good.stderr
    bad = _probe(["-DPROBE_HOST_DEVONLY"])
    assert bad.returncode != 0
    assert "constraints not satisfied" in bad.stderr or "no matching" in bad.stderr


@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_host_reduce_independent_of_thread_count(acc):
    """Blocks are cut from the array start and merged in block order: the same bits for any thread count."""
    x = synth.uniform_pm1_f32(44, 0, (1 << 20) + 4099)
    fn = {"fn": "horner", "coef": synth.horner_coefficients(8)}
    ref = hdc.host_transform_reduce(x, fn, acc, threads=1).item()
    for threads in (2, 3, 7, 16):
        assert hdc.host_transform_reduce(x, fn, acc, threads=threads).item() == ref, threads
    r = oracle.reduce(fn, x)
    assert abs(ref - r["exact"]) <= 1e-6 * r["abs_sum"]
