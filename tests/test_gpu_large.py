"""GPU parity beyond 2^31 elements (the largest sizes the boundary takes): element indices,
grid-stride strides, tile counts and segment lengths all pass the int32 range.  Checked on
sampled outputs against the oracle and on closed forms of the periodic inputs x_i = i mod 16,
whose sums and prefixes are exact integers."""
import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

pytestmark = pytest.mark.gpu

N = (1 << 31) + 77


def gpu():
    return torch.device("cuda", 0)


def periodic(n, dtype):
    """x_i = i mod 16 in `dtype`, built on the device."""
    return torch.arange(16, dtype=dtype, device=gpu()).repeat(n // 16 + 1)[:n]


def prefix(m):
    """sum_{k < m} (k mod 16)"""
    return 120 * (m // 16) + (m % 16) * (m % 16 - 1) // 2


def sample_index(n, count=20000, seed=5):
    g = torch.Generator().manual_seed(seed)
    idx = torch.randint(0, n, (count,), generator=g, dtype=torch.int64)
    return torch.cat([torch.arange(0, 1000), torch.arange(n - 1000, n), idx,
                      torch.arange((1 << 31) - 64, (1 << 31) + 64)])


def test_map_beyond_2_31():
    x = synth.uniform_pm1_f32(21, 0, N, gpu())
    y = hdc.map(x, hdc.affine(2.5, 0.5))
    idx = sample_index(N)
    xs, ys = x[idx.to(gpu())].cpu(), y[idx.to(gpu())].cpu()
    ref = oracle.map({"fn": "affine", "a": 2.5, "b": 0.5}, xs)
    assert torch.equal(ys.view(torch.int32), ref.view(torch.int32))
    del x, y
    xi = periodic(N, torch.int32)
    yi = hdc.map(xi, {"fn": "affine", "a": 3, "b": -7})
    assert torch.equal(yi[idx.to(gpu())].cpu(), 3 * (idx % 16).to(torch.int32) - 7)


def test_sums_and_dot_beyond_2_31():
    xi = periodic(N, torch.int32)
    assert hdc.transform_reduce(xi, hdc.identity(), "exact_int").item() == prefix(N)
    del xi
    xf = periodic(N, torch.float32)
    exact = prefix(N)
    for acc in ("plain", "compensated"):
        r = hdc.transform_reduce(xf, hdc.identity(), acc).item()
        assert abs(r - exact) <= 1e-6 * exact, acc
    ones = torch.ones(N, dtype=torch.float32, device=gpu())
    r = hdc.transform_reduce(ones, hdc.product(), "compensated", z=xf).item()
    assert abs(r - exact) <= 1e-6 * exact
    del xf, ones
    xh = periodic(N, torch.float16)
    assert hdc.transform_reduce(xh, hdc.identity(), "exact").item() == exact
    xb = periodic(N, torch.bfloat16)
    assert hdc.transform_reduce(xb, hdc.identity(), "exact").item() == exact


def test_exact_dot_at_its_largest_n():
    n = (1 << 31) - 1
    xh = periodic(n, torch.float16)
    ones = torch.ones(n, dtype=torch.float16, device=gpu())
    assert hdc.transform_reduce(ones, hdc.product(), "exact", z=xh).item() == prefix(n)


def test_scan_beyond_2_31():
    xi = periodic(N, torch.int32)
    idx = sample_index(N)
    for unroll in (4, 1):  # single pass and three passes
        old = hdc.get_tuning(hdc.OP_SCAN, hdc.I32, hdc.ACC_EXACT_INT, 3)
        try:
            hdc.set_tuning(hdc.OP_SCAN, hdc.I32, hdc.ACC_EXACT_INT, 3, unroll=unroll)
            y = hdc.scan(xi, hdc.identity(), "exact_int")
            got = y[idx.to(gpu())].cpu()
            assert torch.equal(got, torch.tensor([prefix(int(i) + 1) for i in idx], dtype=torch.int64)), unroll
            del y
        finally:
            hdc.set_tuning(hdc.OP_SCAN, hdc.I32, hdc.ACC_EXACT_INT, 3, **old)


def test_segmented_beyond_2_31():
    """One segment longer than 2^31 among short and empty ones."""
    xi = periodic(N, torch.int32)
    cuts = [0, 5, 5, 21, (1 << 31) + 40, N - 3, N]
    off = torch.tensor(cuts, dtype=torch.int64)
    r = hdc.segmented_reduce(xi, off.to(gpu()), hdc.identity(), "exact_int").cpu().tolist()
    assert r == [prefix(b) - prefix(a) for a, b in zip(cuts[:-1], cuts[1:])]
    del xi
    xf = periodic(N, torch.float32)
    r = hdc.segmented_reduce(xf, off.to(gpu()), hdc.identity(), "compensated").cpu().tolist()
    for got, a, b in zip(r, cuts[:-1], cuts[1:]):
        e = prefix(b) - prefix(a)
        assert abs(got - e) <= 1e-6 * e, (a, b)
