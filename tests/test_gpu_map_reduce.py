"""GPU parity of hdc_map / hdc_transform_reduce / hdc_map_reduce against the
CPU oracle, through the C ABI (the Python binding only marshals arguments).

Bars: map outputs and integer sums bit-exact; floating-point sums within
1e-6 * sum|terms| of the exact sum (and exactly 0 when every term is 0).
"""
import itertools
import math

import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

pytestmark = pytest.mark.gpu

COEF8 = synth.horner_coefficients(8)
FNS = {
    "identity": {"fn": "identity"},
    "affine": {"fn": "affine", "a": 2.5, "b": 0.5},
    "horner": {"fn": "horner", "coef": COEF8},
}
INT_FNS = {"identity": {"fn": "identity"}, "affine": {"fn": "affine", "a": 3, "b": -7}}
FLOAT_DTYPES = [torch.float32, torch.float16, torch.bfloat16]
SIZES = [0, 1, 3, 7, 8, 9, 63, 64, 65, 255, 1000, 4097, 65541, (1 << 20) + 3]
TOL = 1e-6


def gpu():
    return torch.device("cuda", 0)


def make_x(n, dt, seed=1, stream=0, scale=1.0):
    if dt == torch.int32:
        return synth.uniform_int(seed, stream, n, bits=20)
    return synth.to_storage(synth.uniform_pm1_f32(seed, stream, n).double() * scale, dt)


def bits(t):
    return t.view(torch.int16) if t.element_size() == 2 else t.view(torch.int32)


def assert_close_sum(got, ref, what=""):
    exact, A = ref["exact"], ref["abs_sum"]
    if A == 0:
        assert got == 0.0, what
        return
    assert abs(got - exact) <= TOL * A, f"{what}: got {got!r} exact {exact!r} A {A!r}"


# --------------------------------------------------------------------------
# map
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dt", FLOAT_DTYPES)
@pytest.mark.parametrize("name", list(FNS))
def test_map_float_bit_exact(dt, name):
    for n in SIZES:
        x = make_x(n, dt, seed=n + 1, scale=3.0)
        y = hdc.map(x.to(gpu()), FNS[name])
        ref = oracle.map(FNS[name], x)
        assert torch.equal(bits(y.cpu()), bits(ref)), (name, dt, n)


@pytest.mark.parametrize("name", list(INT_FNS))
def test_map_int_bit_exact(name):
    for n in SIZES:
        x = make_x(n, torch.int32, seed=n + 2)
        y = hdc.map(x.to(gpu()), INT_FNS[name])
        assert torch.equal(y.cpu(), oracle.map(INT_FNS[name], x)), (name, n)
    x = torch.tensor([0, 1, -1, 2 ** 31 - 1, -2 ** 31, 123456789], dtype=torch.int32)
    assert torch.equal(hdc.map(x.to(gpu()), INT_FNS["affine"]).cpu(), oracle.map(INT_FNS["affine"], x))


MAP_SHAPES = [(64, 1), (256, 8), (1024, 64)]  # (block, blocks per compute unit)


@pytest.mark.parametrize("dt", FLOAT_DTYPES + [torch.int32])
@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_map_every_instance_bit_exact(dt, unroll):
    """Every map kernel instance the tuning can select (16-byte vectors per lane per step 1, 2, 4, 8) at
    several block and grid shapes, on sizes spanning many grid steps and a ragged tail, from an aligned
    start and from an unaligned view (peeled head): bit-equal to the oracle."""
    code = hdc.DTYPE[dt]
    saved = {b: hdc.get_tuning(hdc.OP_MAP, code, hdc.ACC_PLAIN, b) for b in range(4)}
    fns = [INT_FNS["affine"]] if dt == torch.int32 else [FNS["affine"], FNS["horner"]]
    try:
        for block, gm in MAP_SHAPES:
            hdc.set_tuning(hdc.OP_MAP, code, hdc.ACC_PLAIN, -1, block=block, unroll=unroll, grid_mult=gm)
            for n in (70001, (1 << 20) + 13):
                base = make_x(n + 3, dt, seed=block + unroll + n, scale=3.0)
                bg = base.to(gpu())
                yg = torch.empty_like(bg)
                for lo in (0, 3):
                    x = base[lo:lo + n]
                    for fn in fns:
                        ref = bits(oracle.map(fn, x))
                        # x and y at the same offset: the vector walk with a peeled head
                        y = hdc.map(bg[lo:lo + n], fn, out=yg[lo:lo + n])
                        assert torch.equal(bits(y.cpu()), ref), (block, unroll, gm, n, lo, fn)
                        if lo:  # different 16-byte offsets: the element-by-element walk
                            y = hdc.map(bg[lo:lo + n], fn)
                            assert torch.equal(bits(y.cpu()), ref), (block, unroll, gm, n, lo, fn, "scalar")
    finally:
        for b, t in saved.items():
            hdc.set_tuning(hdc.OP_MAP, code, hdc.ACC_PLAIN, b, **t)


@pytest.mark.parametrize("dt", FLOAT_DTYPES + [torch.int32])
def test_map_misaligned_views_and_in_place(dt):
    n = 100003
    fn = FNS["affine"] if dt != torch.int32 else INT_FNS["affine"]
    base = make_x(n + 16, dt, seed=5)
    ref_all = oracle.map(fn, base)
    g = base.to(gpu())
    for xo, yo in [(1, 1), (1, 3), (3, 0), (0, 5), (7, 7)]:
        out = torch.zeros(n + 16, dtype=dt, device=gpu())
        hdc.map(g[xo:xo + n], fn, out=out[yo:yo + n])
        assert torch.equal(bits(out[yo:yo + n].cpu()), bits(ref_all[xo:xo + n])), (xo, yo)
        assert torch.equal(bits(out[:yo].cpu()), bits(torch.zeros(yo, dtype=dt)))  # nothing written outside
        assert torch.equal(bits(out[yo + n:].cpu()), bits(torch.zeros(16 - yo, dtype=dt)))
    h = g.clone()
    hdc.map(h[2:2 + n], fn, out=h[2:2 + n])
    assert torch.equal(bits(h[2:2 + n].cpu()), bits(ref_all[2:2 + n]))


def test_map_special_values_f32():
    x = torch.tensor([0.0, -0.0, math.inf, -math.inf, 1e-45, -1e-45, 3.4e38, -3.4e38, 1.17549435e-38],
                     dtype=torch.float32)
    for name, fn in FNS.items():
        y = hdc.map(x.to(gpu()), fn).cpu()
        ref = oracle.map(fn, x)
        assert torch.equal(torch.isnan(y), torch.isnan(ref)), name
        m = ~torch.isnan(ref)
        assert torch.equal(bits(y[m]), bits(ref[m])), name


@pytest.mark.parametrize("dt", [torch.float16, torch.bfloat16])
def test_map_16bit_rounding_all_patterns(dt):
    # every finite 16-bit value through f(x) = 2.5 x + 0.5: exercises RNE, overflow and subnormals
    x = torch.arange(-32768, 32768, dtype=torch.int32).to(torch.int16).view(dt)
    x = x[torch.isfinite(x.float())]
    y = hdc.map(x.to(gpu()), FNS["affine"]).cpu()
    ref = oracle.map(FNS["affine"], x)
    assert torch.equal(torch.isnan(y.float()), torch.isnan(ref.float()))
    m = ~torch.isnan(ref.float())
    assert torch.equal(bits(y[m]), bits(ref[m]))


# --------------------------------------------------------------------------
# transform_reduce
# --------------------------------------------------------------------------

@pytest.mark.parametrize("acc", ["plain", "compensated"])
@pytest.mark.parametrize("dt", FLOAT_DTYPES)
@pytest.mark.parametrize("name", list(FNS))
def test_transform_reduce_float(acc, dt, name):
    for n in SIZES:
        x = make_x(n, dt, seed=n + 3)
        r = hdc.transform_reduce(x.to(gpu()), FNS[name], acc).item()
        assert_close_sum(r, oracle.reduce(FNS[name], x), f"{name} {dt} {acc} n={n}")


@pytest.mark.parametrize("acc", ["plain", "compensated"])
@pytest.mark.parametrize("dt", FLOAT_DTYPES)
def test_dot(acc, dt):
    for n in SIZES:
        x = synth.to_storage(synth.normal_f64(n + 4, 9, n), dt)
        z = synth.to_storage(synth.normal_f64(n + 4, 1, n), dt)
        r = hdc.transform_reduce(x.to(gpu()), {"fn": "product"}, acc, z=z.to(gpu())).item()
        assert_close_sum(r, oracle.reduce({"fn": "product"}, x, z), f"dot {dt} {acc} n={n}")


def test_dot_closed_form_and_misaligned_operands():
    n = 100003
    x = torch.ones(n + 8)
    z = (torch.arange(n + 8) % 16).float()
    g, h = x.to(gpu()), z.to(gpu())
    for xo, zo in [(0, 0), (1, 1), (1, 2), (3, 0)]:
        r = hdc.transform_reduce(g[xo:xo + n], {"fn": "product"}, "plain", z=h[zo:zo + n]).item()
        ref = oracle.reduce({"fn": "product"}, x[xo:xo + n], z[zo:zo + n])["exact"]
        assert r == ref, (xo, zo)  # integer-valued partial sums below 2^24 are exact in any order


@pytest.mark.parametrize("name", list(INT_FNS))
def test_int_sum_bit_exact(name):
    for n in SIZES:
        x = make_x(n, torch.int32, seed=n + 6)
        r = hdc.transform_reduce(x.to(gpu()), INT_FNS[name], "exact_int").item()
        assert r == oracle.reduce(INT_FNS[name], x)["isum"], (name, n)
    # wrap mod 2^64
    x = torch.full((4096,), 2 ** 31 - 1, dtype=torch.int32)
    fn = {"fn": "affine", "a": 1 << 40, "b": 0}
    assert hdc.transform_reduce(x.to(gpu()), fn, "exact_int").item() == oracle.reduce(fn, x)["isum"]


def test_arithmetic_series_int():
    for n in [1 << 16, (1 << 20) + 7]:
        x = torch.arange(n, dtype=torch.int32)
        assert hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact_int").item() == n * (n - 1) // 2


def test_sums_exact_in_any_order():
    # integers in [0, 15] (partial sums < 2^24) and 2^-i: exact regardless of association
    xi = synth.uniform_int(3, 0, 1 << 20, bits=4).float()
    assert hdc.transform_reduce(xi.to(gpu()), {"fn": "identity"}).item() == float(xi.double().sum())
    for n in range(1, 25):
        x = torch.tensor([2.0 ** -i for i in range(n)])
        assert hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}).item() == 2.0 - 2.0 ** (1 - n)


def test_compensated_textbook_all_orders():
    for perm in itertools.permutations([1.0, 1e8, -1e8]):
        x = torch.tensor(perm, dtype=torch.float32).to(gpu())
        assert hdc.transform_reduce(x, {"fn": "identity"}, "compensated").item() == 1.0


def test_compensated_recovers_ill_conditioned_sum():
    for dt in (torch.bfloat16, torch.float16):
        v, info = synth.ill_conditioned(synth.seed_of(3), 1 << 20, dt)
        g = v.to(gpu())
        comp = hdc.transform_reduce(g, {"fn": "identity"}, "compensated").item()
        plain = hdc.transform_reduce(g, {"fn": "identity"}, "plain").item()
        t = info["target"]
        assert abs(comp - t) <= 1e-6 * info["abs_sum"]
        assert abs(comp - t) <= 1e-2 * abs(t)          # digits survive at kappa ~ 1e8
        assert abs(plain - t) <= 1e-6 * info["abs_sum"]  # the plain sum only meets the sum|x| gate


def test_nonfinite_propagates():
    x = torch.zeros(100000)
    x[777] = math.inf
    g = x.to(gpu())
    assert hdc.transform_reduce(g, {"fn": "identity"}, "plain").item() == math.inf
    assert hdc.transform_reduce(g, {"fn": "identity"}, "compensated").item() == math.inf
    x[99999] = -math.inf
    g = x.to(gpu())
    assert math.isnan(hdc.transform_reduce(g, {"fn": "identity"}, "compensated").item())


def test_deterministic_bits():
    x = synth.to_storage(synth.normal_f64(8, 0, (1 << 22) + 11), torch.float32).to(gpu())
    for acc in ("plain", "compensated"):
        a = hdc.transform_reduce(x, FNS["horner"], acc)
        b = hdc.transform_reduce(x, FNS["horner"], acc)
        assert torch.equal(a, b)


def test_tuning_variants_stay_within_tolerance():
    n = (1 << 21) + 13
    x = make_x(n, torch.float32, seed=21)
    ref = oracle.reduce(FNS["horner"], x)
    g = x.to(gpu())
    b = hdc.tuning_bucket(n)
    old = hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, b)
    try:
        for block, unroll, gm in [(64, 1, 1), (128, 2, 3), (512, 8, 16), (1024, 4, 64), (256, 8, 2)]:
            hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, b, block=block, unroll=unroll,
                           grid_mult=gm)
            assert_close_sum(hdc.transform_reduce(g, FNS["horner"]).item(), ref, str((block, unroll, gm)))
    finally:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, b, **old)


def test_library_workspace_when_none_passed():
    x = make_x(50000, torch.float32, seed=4).to(gpu())
    r = torch.empty((), dtype=torch.float32, device=gpu())
    f = hdc.make_functor(FNS["identity"])
    import ctypes
    st = hdc.lib().hdc_transform_reduce(ctypes.byref(f), hdc.F32, x.data_ptr(), None, x.numel(), 0,
                                        r.data_ptr(), None, 0, torch.cuda.current_stream().cuda_stream)
    assert st == hdc.OK
    assert_close_sum(r.item(), oracle.reduce(FNS["identity"], x.cpu()))


# --------------------------------------------------------------------------
# fused map + reduce
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dt", FLOAT_DTYPES + [torch.int32])
def test_map_reduce_fused(dt):
    if dt == torch.int32:
        mf, rf, acc = INT_FNS["affine"], INT_FNS["identity"], "exact_int"
    else:
        mf, rf, acc = FNS["affine"], FNS["horner"], "compensated"
    for n in [0, 5, 1000, 65541, (1 << 20) + 3]:
        x = make_x(n, dt, seed=n + 8)
        y, r = hdc.map_reduce(x.to(gpu()), mf, rf, acc)
        assert torch.equal(bits(y.cpu()), bits(oracle.map(mf, x)))
        ref = oracle.reduce(rf, x)
        if dt == torch.int32:
            assert r.item() == ref["isum"]
        else:
            assert_close_sum(r.item(), ref, f"fused {dt} n={n}")


def test_smallest_grid_on_large_input_stays_within_tolerance():
    # one 64-thread block per compute unit, one vector per step: each lane
    # folds ~1000 terms, which a single fp32 chain would not keep within 1e-6
    n = 1 << 26
    x = synth.uniform_pm1_f32(33, 0, n)
    ref = oracle.reduce(FNS["horner"], x)
    g = x.to(gpu())
    b = hdc.tuning_bucket(n)
    old = hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, b)
    try:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, b, block=64, unroll=1, grid_mult=1)
        assert_close_sum(hdc.transform_reduce(g, FNS["horner"]).item(), ref, "smallest grid")
    finally:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, b, **old)


# --------------------------------------------------------------------------
# exact fp16 sums: bit-exact against the oracle, whatever the tuning
# --------------------------------------------------------------------------

def _fp16_cases():
    yield "uniform", synth.to_storage(synth.uniform_pm1_f32(51, 0, (1 << 20) + 5).double(), torch.float16)
    yield "wide", synth.to_storage(synth.normal_f64(52, 0, 300007) * torch.exp(
        3.0 * synth.normal_f64(52, 1, 300007)), torch.float16)  # subnormals to 65504
    v, _ = synth.ill_conditioned(synth.seed_of(3), 1 << 20, torch.float16)
    yield "kappa1e8", v
    yield "tiny", torch.tensor([2.0 ** -24, -2.0 ** -24, 2.0 ** -24, 65504.0, -65504.0, 1.0], dtype=torch.float16)
    for n in (0, 1, 7, 8, 9, 4097):
        yield f"n{n}", synth.to_storage(synth.uniform_pm1_f32(n + 60, 0, n).double() * 1000, torch.float16)


def test_exact_fp16_sum_is_bit_exact():
    for name, x in _fp16_cases():
        r = hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item()
        assert r == oracle.reduce({"fn": "identity"}, x)["exact"], name


def test_exact_fp16_sum_independent_of_tuning():
    x = synth.to_storage(synth.normal_f64(53, 0, (1 << 22) + 3) * 100, torch.float16)
    ref = oracle.reduce({"fn": "identity"}, x)["exact"]
    g = x.to(gpu())
    b = hdc.tuning_bucket(x.numel())
    old = hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F16, hdc.ACC_EXACT, b)
    try:
        for block, unroll, gm in [(64, 1, 1), (256, 4, 8), (1024, 8, 64), (128, 2, 3)]:
            hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F16, hdc.ACC_EXACT, b, block=block, unroll=unroll,
                           grid_mult=gm)
            assert hdc.transform_reduce(g, {"fn": "identity"}, "exact").item() == ref, (block, unroll, gm)
    finally:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F16, hdc.ACC_EXACT, b, **old)


def test_exact_fp16_nonfinite_and_fused():
    x = torch.zeros(10000, dtype=torch.float16)
    x[5] = math.inf
    assert hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item() == math.inf
    x[9000] = -math.inf
    assert math.isnan(hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item())
    x = synth.to_storage(synth.uniform_pm1_f32(54, 0, 100003).double(), torch.float16)
    y, r = hdc.map_reduce(x.to(gpu()), FNS["affine"], {"fn": "identity"}, "exact")
    assert torch.equal(bits(y.cpu()), bits(oracle.map(FNS["affine"], x)))
    assert r.item() == oracle.reduce({"fn": "identity"}, x)["exact"]


# --------------------------------------------------------------------------
# exact bf16 sums: the full bf16 range (2^-133 .. 2^128) in 32-bit digits
# --------------------------------------------------------------------------

def _bf16_cases():
    yield "normal", synth.to_storage(synth.normal_f64(61, 0, (1 << 20) + 5), torch.bfloat16)
    yield "wide", synth.to_storage(synth.normal_f64(62, 0, 300007) * torch.exp(
        15.0 * synth.normal_f64(62, 1, 300007)), torch.bfloat16)  # magnitudes over ~220 binary orders
    v, _ = synth.ill_conditioned(synth.seed_of(3), 1 << 20, torch.bfloat16)
    yield "kappa1e8", v
    big = float(torch.finfo(torch.bfloat16).max)
    sub = 2.0 ** -133
    yield "extremes", torch.tensor([big, big, -big, sub, -sub, sub, 2.0 ** -126, 1.0, -0.0, big, -big, -big,
                                    sub * 127, 3.0], dtype=torch.bfloat16)
    yield "cancel_to_subnormal", torch.tensor([big, sub, -big], dtype=torch.bfloat16)
    yield "all_max", torch.full((70001,), big, dtype=torch.bfloat16)  # sum far above any bf16
    for n in (0, 1, 7, 8, 9, 4097):
        yield f"n{n}", synth.to_storage(synth.uniform_pm1_f32(n + 70, 0, n).double() * 1e30, torch.bfloat16)


def test_exact_bf16_sum_is_bit_exact():
    for name, x in _bf16_cases():
        r = hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item()
        ref = oracle.reduce({"fn": "identity"}, x)["exact"]
        assert r == ref, (name, r, ref)
        # unaligned start: a view that begins one element in
        if x.numel() > 1:
            r1 = hdc.transform_reduce(x.to(gpu())[1:], {"fn": "identity"}, "exact").item()
            assert r1 == oracle.reduce({"fn": "identity"}, x[1:])["exact"], name


def test_exact_bf16_sum_independent_of_tuning():
    x = synth.to_storage(synth.normal_f64(63, 0, (1 << 22) + 3) * torch.exp(
        10.0 * synth.normal_f64(63, 1, (1 << 22) + 3)), torch.bfloat16)
    ref = oracle.reduce({"fn": "identity"}, x)["exact"]
    g = x.to(gpu())
    b = hdc.tuning_bucket(x.numel())
    old = hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_EXACT, b)
    try:
        for block, unroll, gm in [(64, 1, 1), (256, 4, 8), (1024, 8, 64), (128, 2, 3)]:
            hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_EXACT, b, block=block, unroll=unroll,
                           grid_mult=gm)
            assert hdc.transform_reduce(g, {"fn": "identity"}, "exact").item() == ref, (block, unroll, gm)
    finally:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_EXACT, b, **old)


def test_exact_bf16_nonfinite():
    x = torch.zeros(10000, dtype=torch.bfloat16)
    x[5] = -math.inf
    assert hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item() == -math.inf
    x[9000] = math.inf
    assert math.isnan(hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item())
    x[9000] = math.nan
    x[5] = 1.0
    assert math.isnan(hdc.transform_reduce(x.to(gpu()), {"fn": "identity"}, "exact").item())


def horner_of_degree(d, seed=0):
    """Degree-d coefficients with mixed signs and magnitudes (exact in fp32); degree 3 gets a -0.0 top."""
    g = torch.Generator().manual_seed(1000 + d + seed)
    c = ((torch.randint(-64, 65, (d + 1,), generator=g).double()) / 32.0).tolist()
    if d == 3:
        c[-1] = -0.0
    return {"fn": "horner", "coef": c}


@pytest.mark.parametrize("degree", range(hdc.MAX_DEGREE + 1))
def test_horner_every_degree(degree):
    """Every Horner degree through every batch form of the kernels: maps bit-exact, sums within tolerance."""
    fn = horner_of_degree(degree)
    for n in (4097, (1 << 16) + 3):
        x = make_x(n, torch.float32, seed=degree + 1)
        y = hdc.map(x.to(gpu()), fn)
        assert torch.equal(bits(y.cpu()), bits(oracle.map(fn, x))), (degree, n)
        ref = oracle.reduce(fn, x)
        for acc in ("plain", "compensated"):
            assert_close_sum(hdc.transform_reduce(x.to(gpu()), fn, acc).item(), ref, f"d={degree} {acc} n={n}")
        x16 = make_x(n, torch.float16, seed=degree + 2)
        y16 = hdc.map(x16.to(gpu()), fn)
        assert torch.equal(bits(y16.cpu()), bits(oracle.map(fn, x16))), (degree, n, "f16")


# --------------------------------------------------------------------------
# exact fp16 dot products: 16-bit digits over the whole product range
# --------------------------------------------------------------------------

def _fp16_dot_cases():
    n = (1 << 20) + 5
    yield "normal", (synth.to_storage(synth.normal_f64(81, 0, n), torch.float16),
                     synth.to_storage(synth.normal_f64(81, 1, n), torch.float16))
    wide = lambda s, k: synth.to_storage(synth.normal_f64(s, k, 300007) * torch.exp(
        3.0 * synth.normal_f64(s, k + 2, 300007)), torch.float16)  # subnormals to 65504
    yield "wide", (wide(82, 0), wide(82, 1))
    x, z, _ = synth.ill_conditioned_dot(synth.seed_of(3), 1 << 20, torch.float16)
    yield "kappa1e8", (x, z)
    ext = torch.tensor([65504.0, -65504.0, 2.0 ** -24, -(2.0 ** -24), 0.0, -0.0, 1.0, 3.0], dtype=torch.float16)
    yield "extremes", (ext, torch.tensor([65504.0, 65504.0, 2.0 ** -24, 2.0 ** -24, 5.0, 7.0, -1.0, 2.0 ** -14],
                                         dtype=torch.float16))
    yield "max_products", (torch.full((70001,), 65504.0, dtype=torch.float16),
                           torch.full((70001,), -65504.0, dtype=torch.float16))
    for m in (0, 1, 7, 8, 9, 4097):
        yield f"n{m}", (synth.to_storage(synth.uniform_pm1_f32(m + 90, 0, m).double() * 300, torch.float16),
                        synth.to_storage(synth.uniform_pm1_f32(m + 90, 1, m).double() * 300, torch.float16))


def test_exact_fp16_dot_is_bit_exact():
    for name, (x, z) in _fp16_dot_cases():
        gx, gz = x.to(gpu()), z.to(gpu())
        r = hdc.transform_reduce(gx, {"fn": "product"}, "exact", z=gz).item()
        ref = oracle.reduce({"fn": "product"}, x, z)["exact"]
        assert r == ref, (name, r, ref)
        if x.numel() > 2:
            # both one element in (vector body with a head), and x one in against z two in (element path)
            r1 = hdc.transform_reduce(gx[1:], {"fn": "product"}, "exact", z=gz[1:]).item()
            assert r1 == oracle.reduce({"fn": "product"}, x[1:], z[1:])["exact"], name
            r2 = hdc.transform_reduce(gx[1:-1], {"fn": "product"}, "exact", z=gz[2:]).item()
            assert r2 == oracle.reduce({"fn": "product"}, x[1:-1], z[2:])["exact"], name


def test_exact_fp16_dot_ill_conditioned_equals_target():
    x, z, info = synth.ill_conditioned_dot(synth.seed_of(3), 1 << 22, torch.float16)
    assert info["kappa"] > 1e7
    r = hdc.transform_reduce(x.to(gpu()), {"fn": "product"}, "exact", z=z.to(gpu())).item()
    assert r == info["target"]


def test_exact_fp16_dot_independent_of_tuning():
    n = (1 << 22) + 3
    x = synth.to_storage(synth.normal_f64(83, 0, n) * 50, torch.float16)
    z = synth.to_storage(synth.normal_f64(83, 1, n) * 50, torch.float16)
    ref = oracle.reduce({"fn": "product"}, x, z)["exact"]
    gx, gz = x.to(gpu()), z.to(gpu())
    b = hdc.tuning_bucket(n)
    old = hdc.get_tuning(hdc.OP_DOT, hdc.F16, hdc.ACC_EXACT, b)
    try:
        for block, unroll, gm in [(64, 1, 1), (256, 4, 8), (1024, 8, 64), (128, 2, 3)]:
            hdc.set_tuning(hdc.OP_DOT, hdc.F16, hdc.ACC_EXACT, b, block=block, unroll=unroll, grid_mult=gm)
            assert hdc.transform_reduce(gx, {"fn": "product"}, "exact", z=gz).item() == ref, (block, unroll, gm)
    finally:
        hdc.set_tuning(hdc.OP_DOT, hdc.F16, hdc.ACC_EXACT, b, **old)


def test_exact_fp16_dot_nonfinite():
    x = torch.ones(10000, dtype=torch.float16)
    z = torch.ones(10000, dtype=torch.float16)
    dot = lambda: hdc.transform_reduce(x.to(gpu()), {"fn": "product"}, "exact", z=z.to(gpu())).item()
    x[5] = math.inf
    assert dot() == math.inf
    z[5] = -2.0
    assert dot() == -math.inf
    z[5] = 0.0                      # inf * 0
    assert math.isnan(dot())
    z[5] = 1.0
    x[9000] = -math.inf             # inf + -inf
    z[9000] = 1.0
    assert math.isnan(dot())
    x[9000] = 1.0
    x[77] = math.nan
    assert math.isnan(dot())


def test_exact_bf16_sum_raises_a_small_grid():
    """With 64-thread blocks and one block per CU, 2^28 values would give a lane more than 1024
    vectors: the launch raises the grid so that every lane's fp64 digit sums stay exact."""
    n = (1 << 28) + 5
    # 3.984375 = 255 * 2^-6 is the largest term of its digit (255 << 31 units): 2^14 of them in one
    # lane's fp64 sum would round, 8192 do not
    x = torch.full((n,), 3.984375, dtype=torch.bfloat16, device=gpu())
    exact = n * 3.984375
    b = hdc.tuning_bucket(n)
    old = hdc.get_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_EXACT, b)
    try:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_EXACT, b, block=64, unroll=1, grid_mult=1)
        assert hdc.transform_reduce(x, {"fn": "identity"}, "exact").item() == exact
    finally:
        hdc.set_tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_EXACT, b, **old)
