"""GPU parity of hdc_scan (prefix sums) against the oracle, through the C ABI.

Per element: integers bit-exact; floating point within 1e-6 of the running
sum of magnitudes of the exact prefix sum (exactly 0 where it is 0)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

pytestmark = pytest.mark.gpu

FNS = {"identity": {"fn": "identity"}, "affine": {"fn": "affine", "a": 2.5, "b": 0.5},
       "horner": {"fn": "horner", "coef": synth.horner_coefficients(8)}}
SIZES = [0, 1, 15, 16, 17, 4095, 4096, 4097, 16383, 16384, 16385, 100003, (1 << 18) + 7]


def gpu():
    return torch.device("cuda", 0)


def check(got, ref, what):
    got = got.cpu().double().numpy()
    err = np.abs(got - ref["exact"])
    bad = np.where(err > 1e-6 * ref["abs_sum"])[0]
    assert bad.size == 0, f"{what}: {bad.size} bad, first {bad[:4]}"
    assert np.all(got[ref["abs_sum"] == 0] == 0.0)


@pytest.mark.parametrize("acc", ["plain", "compensated"])
@pytest.mark.parametrize("dt", [torch.float32, torch.float16, torch.bfloat16])
def test_scan_float(acc, dt):
    for n in SIZES:
        x = synth.to_storage(synth.uniform_pm1_f32(n + 3, 0, n).double(), dt)
        for name in ("identity", "horner"):
            for exclusive in (False, True):
                y = hdc.scan(x.to(gpu()), FNS[name], acc, exclusive=exclusive)
                check(y, oracle.scan(FNS[name], x, exclusive), f"{name} {dt} {acc} n={n} ex={exclusive}")


def test_scan_int_bit_exact():
    aff = {"fn": "affine", "a": 3, "b": -7}
    for n in SIZES:
        x = synth.uniform_int(n + 4, 10, n)
        for exclusive in (False, True):
            y = hdc.scan(x.to(gpu()), aff, "exact_int", exclusive=exclusive)
            assert np.array_equal(y.cpu().numpy(), oracle.scan(aff, x, exclusive)["isum"]), (n, exclusive)


def test_scan_misaligned_and_deterministic():
    n = 70001
    base = synth.uniform_pm1_f32(5, 0, n + 8)
    g = base.to(gpu())
    ref = oracle.scan(FNS["affine"], base[3:3 + n])
    out = torch.zeros(n + 8, device=gpu())
    y = hdc.scan(g[3:3 + n], FNS["affine"], "plain", out=out[1:1 + n])
    check(y, ref, "misaligned")
    assert torch.equal(out[0].cpu(), torch.tensor(0.0)) and torch.equal(out[1 + n:].cpu(), torch.zeros(7))
    a = hdc.scan(g, FNS["horner"], "compensated")
    b = hdc.scan(g, FNS["horner"], "compensated")
    assert torch.equal(a, b)


def test_scan_large_sampled():
    n = 1 << 24
    x = synth.uniform_pm1_f32(6, 0, n)
    y = hdc.scan(x.to(gpu()), FNS["horner"], "plain").cpu().double().numpy()
    for k in (0, 12345, 1 << 20, n // 2 + 17, n - 1):
        r = oracle.reduce(FNS["horner"], x[:k + 1])
        assert abs(y[k] - r["exact"]) <= 1e-6 * r["abs_sum"], k
