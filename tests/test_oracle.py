"""Pins of the CPU oracle against things other than itself: library routines
with documented exact semantics (math.fsum, fractions, numpy/torch rounding),
closed forms, invariants and brute force on tiny inputs.

Each pin is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a wrong rounding rule) fails it.
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
COEF8 = synth.horner_coefficients(8)
HORNER = {"fn": "horner", "coef": COEF8}
U32 = 2.0 ** -24  # unit roundoff of fp32


def frac(pair):
    return Fraction(pair[0], pair[1])


# --------------------------------------------------------------------------
# Exact summation
# --------------------------------------------------------------------------

def _wide_values(rng, n):
    out = []
    for _ in range(n):
        kind = rng.random()
        if kind < 0.1:
            out.append(rng.choice([1, -1]) * rng.randint(1, 2 ** 52) * 2.0 ** -1074)  # subnormal
        elif kind < 0.2:
            out.append(rng.choice([1, -1]) * rng.random() * 2.0 ** 1020)
        else:
            out.append(rng.choice([1, -1]) * rng.random() * 2.0 ** rng.randint(-200, 200))
    return out


def test_exact_sum_matches_fsum_random_wide_range():
    rng = random.Random(7)
    for _ in range(300):
        v = _wide_values(rng, rng.randint(0, 64))
        assert oracle.exact_sum(v) == math.fsum(v)


def test_exact_sum_matches_fractions_with_cancellation():
    rng = random.Random(11)
    for _ in range(100):
        v = _wide_values(rng, 20)
        v = v + [-x for x in v[:10]] + [rng.random() * 2.0 ** -60]
        rng.shuffle(v)
        exact = sum((Fraction(x) for x in v), Fraction(0))
        assert oracle.exact_sum(v) == float(exact)  # Fraction -> float rounds correctly


def test_exact_sum_large_n_matches_fsum():
    x = synth.normal_f64(3, 0, 1 << 16).numpy() * np.exp2(synth.normal_f64(3, 1, 1 << 16).numpy() * 20)
    assert oracle.exact_sum(x) == math.fsum(x.tolist())


def test_exact_sum_ties_and_overflow():
    assert oracle.exact_sum([1.0, 2.0 ** -53]) == 1.0                       # tie -> even
    assert oracle.exact_sum([1.0, 2.0 ** -53, 2.0 ** -105]) == 1.0 + 2.0 ** -52  # sticky bit
    assert oracle.exact_sum([1.0 + 2.0 ** -52, 2.0 ** -53]) == 1.0 + 2.0 ** -51  # tie, odd -> up
    big = np.finfo(np.float64).max
    assert oracle.exact_sum([big, big]) == math.inf
    assert oracle.exact_sum([big, big, -big]) == big                      # exact intermediate
    assert oracle.exact_sum([-big, -big]) == -math.inf
    assert oracle.exact_sum([2.0 ** -1074, 2.0 ** -1074]) == 2.0 ** -1073
    assert oracle.exact_sum([]) == 0.0


def test_exact_sum_nonfinite():
    assert math.isnan(oracle.exact_sum([math.inf, -math.inf]))
    assert math.isnan(oracle.exact_sum([1.0, math.nan]))
    assert oracle.exact_sum([math.inf, 1e308, 1e308]) == math.inf
    assert oracle.exact_sum([-math.inf, 5.0]) == -math.inf


# --------------------------------------------------------------------------
# 16-bit formats
# --------------------------------------------------------------------------

def test_decode_f16_all_patterns_match_numpy():
    bits = np.arange(1 << 16, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = np.array([oracle.decode_f16(int(b)) for b in bits])
    both_nan = np.isnan(ref) & np.isnan(got)
    assert np.array_equal(ref[~both_nan], got[~both_nan])
    assert np.array_equal(np.isnan(ref), np.isnan(got))


def test_decode_bf16_all_patterns_match_torch():
    bits = torch.arange(1 << 16, dtype=torch.int32).to(torch.int16)
    ref = bits.view(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.decode_bf16(int(b) & 0xFFFF) for b in bits.tolist()])
    assert np.array_equal(np.isnan(ref), np.isnan(got))
    m = ~np.isnan(ref)
    assert np.array_equal(ref[m], got[m])


def _f32_probe_values():
    rng = np.random.default_rng(5)
    v = rng.integers(0, 1 << 32, 40000, dtype=np.uint64).astype(np.uint32).view(np.float32)
    # midpoints (ties) and neighbours around every positive finite fp16 value
    h = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float64)
    mids = ((h[:-1] + h[1:]) / 2).astype(np.float32)
    extra = np.array([65504, 65519.99, 65520, 65536, 1e-8, 2.0 ** -25, 2.0 ** -24 * 1.5,
                      3.0e38, 3.3895314e38, 3.4e38, 1.0, 0.0, -0.0, 2.0 ** -126, 2.0 ** -149,
                      2.0 ** -133, 2.0 ** -134, 2.0 ** -133 * 1.5], dtype=np.float32)
    allv = np.concatenate([v, mids, -mids, extra, -extra,
                           np.nextafter(mids, np.float32(np.inf)),
                           np.nextafter(mids, np.float32(0))])
    return allv[np.isfinite(allv)]


def test_encode_f16_matches_numpy_rne():
    v = _f32_probe_values()
    with np.errstate(over="ignore"):
        ref = v.astype(np.float16).view(np.uint16)
    got = np.array([oracle.encode_f16(float(x)) for x in v], dtype=np.uint16)
    assert np.array_equal(ref, got)


def test_encode_bf16_matches_torch_rne():
    v = _f32_probe_values()
    bmids = torch.arange(0, 0x7F80, dtype=torch.int32).to(torch.int16).view(torch.bfloat16).to(torch.float64)
    bm = ((bmids[:-1] + bmids[1:]) / 2).to(torch.float32).numpy()
    v = np.concatenate([v, bm, -bm])
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = np.array([oracle.encode_bf16(float(x)) for x in v], dtype=np.uint16)
    assert np.array_equal(ref, got)


def test_encode_nonfinite():
    assert oracle.encode_f16(math.inf) == 0x7C00
    assert oracle.encode_f16(-math.inf) == 0xFC00
    assert (oracle.encode_f16(math.nan) & 0x7C00) == 0x7C00 and (oracle.encode_f16(math.nan) & 0x3FF)
    assert oracle.encode_bf16(math.inf) == 0x7F80
    assert (oracle.encode_bf16(math.nan) & 0x7F80) == 0x7F80 and (oracle.encode_bf16(math.nan) & 0x7F)


# --------------------------------------------------------------------------
# Element semantics
# --------------------------------------------------------------------------

def _horner_bound(x):
    # |fl(p(x)) - p(x)| <= sum_k |c_k - 1/(k+1)| |x|^k + gamma_{2d} sum_k |c_k| |x|^k
    d = 8
    g = 2 * d * U32 / (1 - 2 * d * U32)
    coef_err = sum(abs(Fraction(c) - Fraction(1, k + 1)) * Fraction(abs(x)) ** k for k, c in enumerate(COEF8))
    return float(coef_err) + g * sum(abs(c) * abs(x) ** k for k, c in enumerate(COEF8))


@pytest.mark.parametrize("x,key", [(1.0, "p_at_1"), (-1.0, "p_at_minus_1"), (0.0, "p_at_0")])
def test_horner_closed_forms(x, key):
    exact = frac(GOLD[key]["value"])
    got = oracle.term_f32(HORNER, x)
    assert abs(Fraction(got) - exact) <= Fraction(_horner_bound(x))
    if x == 0.0:
        assert got == 1.0


def test_horner_fp64_matches_expanded_polynomial():
    # fp64 Horner against the exactly expanded sum_k c_k x^k (rational arithmetic);
    # asymmetric points catch a reversed coefficient order, odd points a sign slip.
    for x in [0.5, -0.5, 0.3, -0.7, 0.9999, 2.0, -3.0]:
        exact = sum(Fraction(c) * Fraction(x) ** k for k, c in enumerate(COEF8))
        scale = sum(abs(Fraction(c)) * abs(Fraction(x)) ** k for k, c in enumerate(COEF8))
        got = oracle.term_f64(HORNER, x)
        assert abs(Fraction(got) - exact) <= float(scale) * 16 * 2.0 ** -53
        # the fp32 evaluation agrees within the fp32 Horner bound
        got32 = oracle.term_f32(HORNER, np.float32(x).item())
        x32 = Fraction(np.float32(x).item())
        exact32 = sum(Fraction(c) * x32 ** k for k, c in enumerate(COEF8))
        assert abs(Fraction(got32) - exact32) <= Fraction(float(scale) * 17 * U32 * 1.01)


def test_horner_degree_edge_cases():
    assert oracle.term_f32({"fn": "horner", "coef": [3.25]}, 123.0) == 3.25
    # degree 16 with one non-zero top coefficient: x^16 exactly for small powers of two
    c = [0.0] * 16 + [1.0]
    assert oracle.term_f32({"fn": "horner", "coef": c}, 2.0) == 2.0 ** 16
    assert oracle.term_f32({"fn": "horner", "coef": c}, -0.5) == 2.0 ** -16


def _rn_f32(q: Fraction) -> float:
    """The binary32 value nearest to the rational q, ties to even (IEEE 754
    roundTiesToEven), with gradual underflow and overflow to infinity.
    Written from the format's definition: 24-bit significands, exponents
    -126..127, quantum 2^(max(e, -126) - 23) for 2^e <= |q| < 2^(e+1)."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    m = abs(q)
    e = m.numerator.bit_length() - m.denominator.bit_length()
    if m < Fraction(2) ** e:
        e -= 1
    assert Fraction(2) ** e <= m < Fraction(2) ** (e + 1)
    quantum = Fraction(2) ** (max(e, -126) - 23)
    scaled = m / quantum
    k = scaled.numerator // scaled.denominator
    rem = scaled - k
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and k % 2 == 1):
        k += 1
    v = k * quantum
    if v >= Fraction(2) ** 128:
        return sign * math.inf
    return sign * float(v)  # v is a binary32 value, so float() is exact


def test_rn_f32_matches_numpy_on_doubles():
    # the rounding helper itself: every double rounds to binary32 exactly as
    # numpy's (IEEE) conversion does, subnormals and overflow included
    rng = np.random.default_rng(3)
    v = rng.integers(0, 1 << 64, 20000, dtype=np.uint64).view(np.float64)
    v = v[np.isfinite(v) & (np.abs(v) < 3.5e38)]
    v = np.concatenate([v, rng.normal(size=5000) * 2.0 ** rng.integers(-160, 120, 5000),
                        np.array([2.0 ** -150, 3 * 2.0 ** -151, 2.0 ** -149 * 1.5, 3.4028235677973366e38])])
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32).astype(np.float64)
    for x, r in zip(v.tolist(), ref.tolist()):
        assert _rn_f32(Fraction(x)) == r, x


def _horner_one_rounding(coef, x):
    acc = Fraction(np.float32(coef[-1]).item())
    xf = Fraction(x)
    for c in reversed(coef[:-1]):
        acc = Fraction(_rn_f32(acc * xf + Fraction(np.float32(c).item())))
    return float(acc)


def _horner_two_roundings(coef, x):
    acc = Fraction(np.float32(coef[-1]).item())
    xf = Fraction(x)
    for c in reversed(coef[:-1]):
        acc = Fraction(_rn_f32(Fraction(_rn_f32(acc * xf)) + Fraction(np.float32(c).item())))
    return float(acc)


def test_horner_rounding_sequence_is_one_fma_per_step():
    # The fp32 Horner term is acc = c_d, then acc = RN(acc * x + c_k) for
    # k = d-1 .. 0: one rounding per step (a fused multiply-add).  Emulated
    # exactly in rational arithmetic with the rounding above, for the
    # workload's coefficients and for random coefficients of every degree
    # 0..16.  A multiply and a separate add (two roundings) differ on many of
    # these points, so that reading of the oracle would fail here.
    rng = np.random.default_rng(17)
    xs = np.concatenate([rng.uniform(-1, 1, 1500), rng.uniform(-4, 4, 300)]).astype(np.float32)
    differs = 0
    for x in xs.tolist():
        want = _horner_one_rounding(COEF8, x)
        assert oracle.term_f32(HORNER, x) == want, x
        differs += _horner_two_roundings(COEF8, x) != want
    assert differs > 100  # the test separates one rounding from two
    for d in range(0, 17):
        coef = (rng.normal(size=d + 1) * 2.0 ** rng.integers(-6, 6, d + 1)).astype(np.float32).tolist()
        spec = {"fn": "horner", "coef": coef}
        for x in rng.uniform(-1.5, 1.5, 60).astype(np.float32).tolist():
            assert oracle.term_f32(spec, x) == _horner_one_rounding(coef, x), (d, x)


def test_horner_fp64_rounding_sequence():
    # fp64 Horner (the sequential fp64 reference's terms): one rounding to
    # binary64 per step; float(Fraction) rounds correctly to nearest-even.
    rng = np.random.default_rng(19)
    for x in rng.uniform(-2, 2, 400).tolist():
        acc = Fraction(np.float32(COEF8[-1]).item())
        for c in reversed(COEF8[:-1]):
            acc = Fraction(float(acc * Fraction(x) + Fraction(np.float32(c).item())))
        assert oracle.term_f64(HORNER, x) == float(acc), x


def test_affine_map_f32_single_rounding():
    x = synth.uniform_pm1_f32(1, 0, 4096)
    x = torch.cat([x, torch.tensor([3.4e38, -3.4e38, 1e-45, 0.1, 1 / 3], dtype=torch.float32)])
    y = oracle.map({"fn": "affine", "a": 2.5, "b": 0.5}, x)
    # 2.5*x + 0.5 is exact in fp64 for these inputs; one rounding to fp32 gives the fma result
    ref = (2.5 * x.double() + 0.5).float()
    assert torch.equal(y, ref)


def test_affine_map_dyadic_inputs_are_exact():
    k = torch.arange(-4096, 4096, dtype=torch.float32)
    x = k * 2.0 ** -12
    y = oracle.map({"fn": "affine", "a": 2.5, "b": 0.5}, x)
    assert torch.equal(y.double(), 2.5 * x.double() + 0.5)


@pytest.mark.parametrize("dt", [torch.float16, torch.bfloat16])
def test_affine_map_16bit_two_roundings(dt):
    x = synth.to_storage(synth.normal_f64(2, 0, 8192) * 3, dt)
    y = oracle.map({"fn": "affine", "a": 2.5, "b": 0.5}, x)
    ref = (2.5 * x.double() + 0.5).float()       # fp32 fma value (exact product + one rounding)
    ref = torch.from_numpy(ref.numpy().astype(np.float16)) if dt == torch.float16 else ref.to(dt)
    assert torch.equal(y.view(torch.int16), ref.view(torch.int16))


def test_identity_map_copies_bits():
    for dt in (torch.float32, torch.float16, torch.bfloat16, torch.int32):
        x = torch.randint(-30000, 30000, (1000,), dtype=torch.int32).to(torch.int16 if dt in (torch.float16, torch.bfloat16) else torch.int32)
        x = x.view(dt)
        y = oracle.map({"fn": "identity"}, x)
        assert torch.equal(y.view(torch.int16 if x.element_size() == 2 else torch.int32),
                           x.view(torch.int16 if x.element_size() == 2 else torch.int32))


def test_int_affine_map_wraps():
    x = torch.tensor([0, 1, -1, 2 ** 31 - 1, -2 ** 31, 1 << 20, 123456789], dtype=torch.int32)
    y = oracle.map({"fn": "affine", "a": 3, "b": -7}, x)
    ref = (x.numpy().astype(np.int64) * 3 - 7).astype(np.int32)   # numpy astype wraps
    assert np.array_equal(y.numpy(), ref)


def test_unsupported_combinations_rejected():
    with pytest.raises(ValueError):
        oracle.map({"fn": "horner", "coef": [1.0]}, torch.zeros(4, dtype=torch.int32))
    with pytest.raises(ValueError):
        oracle.map({"fn": "product"}, torch.zeros(4))
    with pytest.raises(ValueError):
        oracle.reduce({"fn": "product"}, torch.zeros(4))


# --------------------------------------------------------------------------
# Reductions
# --------------------------------------------------------------------------

def test_sum_small_integers_exact():
    n = 1 << 20
    xi = synth.uniform_int(9, 0, n, bits=4)
    r = oracle.reduce({"fn": "identity"}, xi.float())
    assert r["exact"] == r["seq64"] == float(xi.long().sum().item())
    assert r["abs_sum"] == r["exact"]


def test_geometric_series():
    for n in range(0, 25):
        x = torch.tensor([2.0 ** -i for i in range(n)], dtype=torch.float32)
        r = oracle.reduce({"fn": "identity"}, x)
        assert r["exact"] == (2.0 - 2.0 ** (1 - n) if n else 0.0)


def test_arithmetic_series_int():
    for n in [0, 1, 2, 1000, 65537]:
        x = torch.arange(n, dtype=torch.int32)
        r = oracle.reduce({"fn": "identity"}, x)
        assert r["isum"] == n * (n - 1) // 2


def test_int_affine_sum_identity():
    x = synth.uniform_int(4, 10, 100000)
    r1 = oracle.reduce({"fn": "identity"}, x)
    r2 = oracle.reduce({"fn": "affine", "a": 3, "b": -7}, x)
    assert r2["isum"] == 3 * r1["isum"] - 7 * x.numel()


def test_int_sum_wraps_mod_2_64():
    # 2^33 copies of 2^31-1 would overflow; emulate the wrap with a = 2^40 on few elements
    x = torch.full((4096,), 2 ** 31 - 1, dtype=torch.int32)
    r = oracle.reduce({"fn": "affine", "a": 1 << 40, "b": 0}, x)
    ref = (4096 * (1 << 40) * (2 ** 31 - 1)) % (1 << 64)
    ref = ref - (1 << 64) if ref >= 1 << 63 else ref
    assert r["isum"] == ref


def test_dot_closed_form():
    for n in [0, 1, 15, 16, 17, 1000, 4099]:
        x = torch.ones(n)
        z = (torch.arange(n) % 16).float()
        r = oracle.reduce({"fn": "product"}, x, z)
        q, rem = divmod(n, 16)
        assert r["exact"] == 120 * q + rem * (rem - 1) // 2


def test_dot_is_exact_products():
    # fp32 products have <= 48 significant bits: the exact sum of a few of them
    # is the Fraction sum.
    x = synth.uniform_pm1_f32(5, 0, 64)
    z = synth.uniform_pm1_f32(5, 1, 64)
    r = oracle.reduce({"fn": "product"}, x, z)
    exact = sum(Fraction(a) * Fraction(b) for a, b in zip(x.tolist(), z.tolist()))
    assert r["exact"] == float(exact)
    # swapping the operands gives the same bits
    assert oracle.reduce({"fn": "product"}, z, x)["exact"] == r["exact"]


def test_dot_f16_exact_over_the_whole_range():
    # fp16 x fp16 products are exact in fp32 (<= 22 significant bits); over the whole
    # fp16 range (65504^2 down to 2^-48) the exact dot is the Fraction sum, rounded once.
    rng = np.random.default_rng(3)
    bits = rng.integers(0, 1 << 16, 6000, dtype=np.int64)
    bits = bits[((bits >> 10) & 31) != 31]            # finite values only
    x = torch.from_numpy(bits[:2500].astype(np.int16)).view(torch.float16)
    z = torch.from_numpy(bits[2500:5000].astype(np.int16)).view(torch.float16)
    special = torch.tensor([65504.0, -65504.0, 2.0 ** -24, -(2.0 ** -24), 0.0, -0.0, 1.0], dtype=torch.float16)
    x = torch.cat([x, special, special])
    z = torch.cat([z, special, special.flip(0)])
    r = oracle.reduce({"fn": "product"}, x, z)
    exact = sum(Fraction(a) * Fraction(b) for a, b in zip(x.double().tolist(), z.double().tolist()))
    assert r["exact"] == float(exact)
    A = float(sum(abs(Fraction(a) * Fraction(b)) for a, b in zip(x.double().tolist(), z.double().tolist())))
    assert abs(r["abs_sum"] - A) <= 1e-12 * A  # the tolerance denominator is a plain fp64 sum


def test_dot_f16_ill_conditioned_target():
    # x * z == v exactly for the ill-conditioned construction: the exact dot is its target
    x, z, info = synth.ill_conditioned_dot(7, 1 << 14, torch.float16, kappa=1e6)
    assert torch.equal(x.double() * z.double(), synth.ill_conditioned(7, 1 << 14, torch.float16, kappa=1e6)[0].double())
    assert oracle.reduce({"fn": "product"}, x, z)["exact"] == info["target"]


def test_reduce_equals_fsum_of_mapped_terms():
    x = synth.uniform_pm1_f32(1, 0, 20000)
    terms = oracle.map(HORNER, x).double().tolist()
    r = oracle.reduce(HORNER, x)
    assert r["exact"] == math.fsum(terms)
    assert r["abs_sum"] == pytest.approx(sum(abs(t) for t in terms), rel=1e-12)
    assert abs(r["seq64"] - r["exact"]) <= 1e-6 * r["abs_sum"]


def test_mean_horner_over_uniform():
    n = 1 << 20
    x = synth.uniform_pm1_f32(synth.seed_of(1), 0, n)
    r = oracle.reduce(HORNER, x)
    mean = r["exact"] / n
    assert abs(mean - float(frac(GOLD["mean_p_uniform_pm1"]["value"]))) < 5e-3


def test_compensation_textbook_case_exact():
    x = torch.tensor(GOLD["compensation_textbook"]["values"], dtype=torch.float32)
    assert oracle.reduce({"fn": "identity"}, x)["exact"] == 1.0


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_ill_conditioned_target_is_exact(dt):
    v, info = synth.ill_conditioned(synth.seed_of(3), 1 << 18, dt)
    r = oracle.reduce({"fn": "identity"}, v)
    assert r["exact"] == info["target"]
    assert info["kappa"] > 3e7
    assert r["abs_sum"] == pytest.approx(info["abs_sum"], rel=1e-12)


def test_reduce_nonfinite_propagates():
    x = torch.tensor([1.0, math.inf, 2.0])
    assert oracle.reduce({"fn": "identity"}, x)["exact"] == math.inf
    x = torch.tensor([1.0, math.inf, -math.inf])
    assert math.isnan(oracle.reduce({"fn": "identity"}, x)["exact"])


def test_empty_reduce_is_zero():
    for dt in (torch.float32, torch.float16, torch.bfloat16, torch.int32):
        r = oracle.reduce({"fn": "identity"}, torch.zeros(0, dtype=dt))
        assert r["exact"] == 0.0 and r["isum"] == 0


# --------------------------------------------------------------------------
# Segmented
# --------------------------------------------------------------------------

def test_segmented_single_segment_equals_reduce():
    x = synth.uniform_pm1_f32(2, 0, 5000)
    off = torch.tensor([0, 5000])
    s = oracle.segmented(HORNER, x, off)
    r = oracle.reduce(HORNER, x)
    assert s["exact"][0] == r["exact"] and s["abs_sum"][0] == r["abs_sum"]


def test_segmented_brute_force_and_empty():
    rng = random.Random(3)
    L = [rng.choice([0, 0, 1, 2, 3, 7, 64, 65, 300]) for _ in range(200)]
    off = torch.tensor([0] + list(np.cumsum(L)), dtype=torch.int64)
    x = synth.uniform_pm1_f32(2, 1, int(off[-1]))
    s = oracle.segmented(HORNER, x, off)
    terms = oracle.map(HORNER, x).double().tolist()
    for j in range(len(L)):
        seg = terms[off[j]:off[j + 1]]
        assert s["exact"][j] == math.fsum(seg)
        if L[j] == 0:
            assert s["exact"][j] == 0.0
    xi = synth.uniform_int(2, 2, int(off[-1]))
    si = oracle.segmented({"fn": "identity"}, xi, off)
    for j in range(len(L)):
        assert si["isum"][j] == int(xi[off[j]:off[j + 1]].long().sum())


def test_segmented_rejects_decreasing_offsets():
    with pytest.raises(ValueError):
        oracle.segmented({"fn": "identity"}, torch.zeros(10), torch.tensor([0, 5, 3, 10]))


# --------------------------------------------------------------------------
# Prefix sums
# --------------------------------------------------------------------------

def test_scan_closed_forms():
    n = 5000
    ones = torch.ones(n)
    r = oracle.scan({"fn": "identity"}, ones)
    assert np.array_equal(r["exact"], np.arange(1, n + 1))
    r = oracle.scan({"fn": "identity"}, ones, exclusive=True)
    assert np.array_equal(r["exact"], np.arange(0, n))
    xi = torch.arange(n, dtype=torch.int32)
    r = oracle.scan({"fn": "identity"}, xi)
    i = np.arange(n)
    assert np.array_equal(r["isum"], i * (i + 1) // 2)                       # arithmetic series
    r = oracle.scan({"fn": "affine", "a": 3, "b": -7}, xi, exclusive=True)
    assert np.array_equal(r["isum"], 3 * (i * (i - 1) // 2) - 7 * i)


def test_scan_matches_fsum_prefixes_and_reduce():
    x = synth.uniform_pm1_f32(4, 0, 3000)
    r = oracle.scan(HORNER, x)
    terms = oracle.map(HORNER, x).double().tolist()
    for k in (0, 1, 17, 1000, 2999):
        assert r["exact"][k] == math.fsum(terms[:k + 1])
    assert r["exact"][-1] == oracle.reduce(HORNER, x)["exact"]
    rex = oracle.scan(HORNER, x, exclusive=True)
    assert rex["exact"][0] == 0.0 and np.array_equal(rex["exact"][1:], r["exact"][:-1])
    assert np.all(np.diff(r["abs_sum"]) >= 0)


def test_segmented_scan_single_segment_equals_scan():
    x = synth.uniform_pm1_f32(6, 0, 2000)
    whole = torch.tensor([0, 2000])
    for ex in (False, True):
        a = oracle.segmented_scan(HORNER, x, whole, ex)
        b = oracle.scan(HORNER, x, ex)
        assert np.array_equal(a["exact"], b["exact"]) and np.array_equal(a["abs_sum"], b["abs_sum"])


def test_segmented_scan_brute_force():
    """Tiny segments (empty ones included, and a gap before the first): every prefix is the fsum of the
    terms from its segment's start; the last prefix of a segment equals the segmented reduce."""
    x = synth.uniform_pm1_f32(7, 0, 400)
    terms = oracle.map(HORNER, x).double().tolist()
    off = torch.tensor([5, 5, 9, 40, 41, 41, 200, 399])
    r = oracle.segmented_scan(HORNER, x, off)
    rex = oracle.segmented_scan(HORNER, x, off, exclusive=True)
    red = oracle.segmented(HORNER, x, off)
    for j in range(off.numel() - 1):
        lo, hi = int(off[j]), int(off[j + 1])
        for i in range(lo, hi):
            assert r["exact"][i] == math.fsum(terms[lo:i + 1])
            assert rex["exact"][i] == math.fsum(terms[lo:i])
        if hi > lo:
            assert r["exact"][hi - 1] == red["exact"][j]
    outside = np.r_[0:5, 399:400]
    assert np.all(np.isnan(r["exact"][outside]))
    xi = synth.uniform_int(8, 0, 400)
    ri = oracle.segmented_scan({"fn": "affine", "a": 3, "b": -7}, xi, off)["isum"]
    for j in range(off.numel() - 1):
        lo, hi = int(off[j]), int(off[j + 1])
        acc = 0
        for i in range(lo, hi):
            acc += 3 * int(xi[i]) - 7
            assert ri[i] == acc


def test_multithreaded_oracle_matches_single_thread():
    """The multicore CPU baseline joins per-thread exact accumulators without rounding: its exact and
    integer results are the single-thread oracle's bit for bit, and its maps are identical, for any
    thread count (more threads than elements included)."""
    horner = {"fn": "horner", "coef": synth.horner_coefficients(8)}
    cases = [
        ({"fn": "identity"}, synth.to_storage(synth.random_sign(11, 2, 5003) * torch.exp(4.0 * synth.normal_f64(11, 0, 5003)),
                                              torch.float32), None),
        (horner, synth.uniform_pm1_f32(12, 0, 40001), None),
        ({"fn": "product"}, synth.to_storage(synth.normal_f64(13, 0, 7777), torch.float16),
         synth.to_storage(synth.normal_f64(13, 1, 7777), torch.float16)),
        ({"fn": "identity"}, synth.to_storage(synth.normal_f64(14, 0, 999), torch.bfloat16), None),
        ({"fn": "affine", "a": 3, "b": -7}, synth.uniform_int(15, 0, 12345, bits=31), None),
    ]
    for spec, x, z in cases:
        one = oracle.reduce(spec, x, z)
        for threads in (1, 3, 8, 17, 64):
            mt = oracle.reduce_mt(spec, x, z, threads=threads)
            assert mt["exact"] == one["exact"] and mt["isum"] == one["isum"], (spec, threads)
            assert math.isclose(mt["abs_sum"], one["abs_sum"], rel_tol=1e-12)
            assert abs(mt["seq64"] - one["seq64"]) <= 1e-12 * one["abs_sum"]
            if spec["fn"] != "product":
                assert torch.equal(oracle.map_mt(spec, x, threads=threads), oracle.map(spec, x))
    assert oracle.reduce_mt({"fn": "identity"}, torch.zeros(0), threads=4)["exact"] == 0.0
    few = torch.tensor([1e30, 1.0, -1e30, 3.0, 2.0 ** -140], dtype=torch.float32)  # more threads than values
    assert oracle.reduce_mt({"fn": "identity"}, few, threads=8)["exact"] == oracle.reduce({"fn": "identity"}, few)["exact"]
