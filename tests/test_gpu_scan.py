"""GPU parity of hdc_scan (prefix sums) against the oracle, through the C ABI.

Per element: integers bit-exact; floating point within 1e-6 of the running
sum of magnitudes of the exact prefix sum (exactly 0 where it is 0).  Every
test runs under both schedules: the single pass with a decoupled look-back
(tuning unroll != 1, the default) and the three-pass schedule (unroll 1)."""
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


SCAN_CLASSES = [(hdc.F32, hdc.ACC_PLAIN), (hdc.F32, hdc.ACC_COMPENSATED), (hdc.F16, hdc.ACC_PLAIN),
                (hdc.F16, hdc.ACC_COMPENSATED), (hdc.BF16, hdc.ACC_PLAIN), (hdc.BF16, hdc.ACC_COMPENSATED),
                (hdc.I32, hdc.ACC_EXACT_INT)]


def gpu():
    return torch.device("cuda", 0)


def set_scan_tuning(unroll, block=0):
    for dt, acc in SCAN_CLASSES:
        hdc.set_tuning(hdc.OP_SCAN, dt, acc, -1, block=block, unroll=unroll)


@pytest.fixture(params=["single_pass", "three_pass"], autouse=True)
def schedule(request):
    saved = {(dt, acc, b): hdc.get_tuning(hdc.OP_SCAN, dt, acc, b) for dt, acc in SCAN_CLASSES for b in range(4)}
    set_scan_tuning(4 if request.param == "single_pass" else 1)
    yield request.param
    for (dt, acc, b), t in saved.items():
        hdc.set_tuning(hdc.OP_SCAN, dt, acc, b, **t)


def lookback_status(ws):
    """The scan's status word through hdc_scan_status: nonzero if a wait of the single pass gave up."""
    return hdc.scan_status(ws)


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


@pytest.mark.parametrize("block", [64, 256, 1024])
def test_scan_many_tiles_and_status(block, schedule):
    """Thousands of tiles, every output checked.  At block 64 there are 4101 tiles: the carry tree has three
    levels (groups of 64 and of 4096 tiles) and the last tile is a partial one."""
    set_scan_tuning(4 if schedule == "single_pass" else 1, block=block)
    n = 64 * 16 * 4100 + 123 if block == 64 else (1 << 22) + 5
    x = synth.uniform_pm1_f32(11, 0, n)
    ws = hdc.workspace(gpu(), hdc.OP_SCAN, hdc.F32, hdc.ACC_COMPENSATED, n)
    y = hdc.scan(x.to(gpu()), FNS["horner"], "compensated", ws=ws)
    if schedule == "single_pass":
        assert lookback_status(ws) == 0
    ref = oracle.scan(FNS["horner"], x)
    check(y, ref, f"block {block}")
    y2 = hdc.scan(x.to(gpu()), FNS["horner"], "compensated", ws=ws)
    assert torch.equal(y, y2)
    xi = synth.uniform_int(12, 10, n)
    wsi = hdc.workspace(gpu(), hdc.OP_SCAN, hdc.I32, hdc.ACC_EXACT_INT, n)
    yi = hdc.scan(xi.to(gpu()), {"fn": "affine", "a": 3, "b": -7}, "exact_int", exclusive=True, ws=wsi)
    if schedule == "single_pass":
        assert lookback_status(wsi) == 0
    assert np.array_equal(yi.cpu().numpy(), oracle.scan({"fn": "affine", "a": 3, "b": -7}, xi, True)["isum"])


def test_scan_full_size_sampled(schedule):
    """2^28 f32 Horner scan in the launch configuration the benchmark times: sampled prefixes vs the oracle,
    and the last output vs the oracle's full reduction."""
    n = 1 << 28
    x = synth.uniform_pm1_f32(synth.seed_of(2), synth.STREAM["x"], n, gpu())
    ws = hdc.workspace(gpu(), hdc.OP_SCAN, hdc.F32, hdc.ACC_PLAIN, n)
    y = hdc.scan(x, FNS["horner"], "plain", ws=ws)
    if schedule == "single_pass":
        assert lookback_status(ws) == 0
    xc = x.cpu()
    for k in (0, 16383, 16384, 1 << 24, (1 << 27) + 12345, n - 1):
        r = oracle.reduce(FNS["horner"], xc[:k + 1])
        got = y[k].item()
        assert abs(got - r["exact"]) <= 1e-6 * r["abs_sum"], (k, got, r["exact"])
    del x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("degree", [0, 1, 7, 16])
def test_scan_horner_degrees(degree, schedule):
    g = torch.Generator().manual_seed(3000 + degree)
    fn = {"fn": "horner", "coef": (torch.randint(-64, 65, (degree + 1,), generator=g).double() / 32.0).tolist()}
    x = synth.uniform_pm1_f32(degree + 30, 0, 70001)
    y = hdc.scan(x.to(gpu()), fn, "compensated")
    check(y, oracle.scan(fn, x), f"degree {degree}")
