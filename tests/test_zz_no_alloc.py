"""hdc_transform_reduce_noalloc (no workspace, no allocation: the partials go
to the library's per-device scratch array) against hdc_transform_reduce with
a workspace, through the C ABI.  Same kernels and tuning, so the results must
be the same bits; each is also held to the oracle's bar (bit-exact for
integer and exact sums, 1e-6 * sum|terms| for floating-point sums).  Every
case makes two calls in a row, the second on a smaller input, so partials
left in the scratch by the first call cannot leak into the second."""
import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

pytestmark = pytest.mark.gpu

COEF8 = synth.horner_coefficients(8)
TOL = 1e-6

CASES = [
    # (name, dtype, functor, accumulation, binary)
    ("f32_horner_plain", torch.float32, {"fn": "horner", "coef": COEF8}, "plain", False),
    ("f32_affine_comp", torch.float32, {"fn": "affine", "a": 2.5, "b": 0.5}, "compensated", False),
    ("f32_dot_plain", torch.float32, {"fn": "product"}, "plain", True),
    ("bf16_sum_comp", torch.bfloat16, {"fn": "identity"}, "compensated", False),
    ("f16_dot_comp", torch.float16, {"fn": "product"}, "compensated", True),
    ("f16_sum_exact", torch.float16, {"fn": "identity"}, "exact", False),
    ("bf16_sum_exact", torch.bfloat16, {"fn": "identity"}, "exact", False),
    ("f16_dot_exact", torch.float16, {"fn": "product"}, "exact", True),
    ("i32_affine_int", torch.int32, {"fn": "affine", "a": 3, "b": -7}, "exact_int", False),
]
SIZE_PAIRS = [((1 << 22) + 5, 4097), ((1 << 20) + 3, 1), (65541, 0)]


def make(n, dt, seed, stream):
    if dt == torch.int32:
        return synth.uniform_int(seed, stream, n, bits=20)
    return synth.to_storage(synth.normal_f64(seed, stream, n), dt)


def same_bits(a, b):
    iv = torch.int64 if a.element_size() == 8 else torch.int32
    return a.cpu().reshape(1).view(iv).item() == b.cpu().reshape(1).view(iv).item()


def check_vs_oracle(got, fn, acc, x, z, what):
    ref = oracle.reduce(fn, x, z) if z is not None else oracle.reduce(fn, x)
    if acc == "exact_int":
        assert got == ref["isum"], what
    elif acc == "exact":
        assert got == ref["exact"], what
    elif ref["abs_sum"] == 0:
        assert got == 0.0, what
    else:
        assert abs(got - ref["exact"]) <= TOL * ref["abs_sum"], (what, got, ref["exact"])


@pytest.mark.parametrize("name,dt,fn,acc,binary", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_workspace_call(name, dt, fn, acc, binary):
    dev = torch.device("cuda", 0)
    for pair, (n1, n2) in enumerate(SIZE_PAIRS):
        seed = 230903930 + pair
        x_big, z_big = make(n1, dt, seed, 0), make(n1, dt, seed, 1) if binary else None
        a = hdc.ACC[acc]
        out_ref = torch.empty((), dtype=hdc.OUT_DTYPE[a], device=dev)
        out_na = torch.empty((), dtype=hdc.OUT_DTYPE[a], device=dev)
        for n in (n1, n2):  # two calls in a row, the second on a smaller input
            x = x_big[:n]
            z = z_big[:n] if binary else None
            xg = x.to(dev)
            zg = z.to(dev) if binary else None
            ws = torch.zeros(hdc.workspace_size(hdc.OP_TRANSFORM_REDUCE, hdc.DTYPE[dt], a, n), dtype=torch.uint8,
                             device=dev)
            print(f"noalloc {name} n={n}", flush=True)
            hdc.transform_reduce(xg, fn, acc, z=zg, out=out_ref, ws=ws)
            hdc.transform_reduce_noalloc(xg, fn, acc, z=zg, out=out_na)
            torch.cuda.synchronize()
            got_ref, got_na = out_ref.item(), out_na.item()
            assert same_bits(out_na, out_ref), (name, n, got_na, got_ref)
            check_vs_oracle(got_na, fn, acc, x, z, (name, n))


def test_noalloc_on_another_stream_and_n_zero():
    dev = torch.device("cuda", 0)
    x = synth.to_storage(synth.uniform_pm1_f32(230903940, 0, (1 << 21) + 7).double(), torch.float32).to(dev)
    out = torch.full((), 7.0, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        hdc.transform_reduce_noalloc(x, {"fn": "identity"}, "plain", out=out)
        r1 = out.clone()
        hdc.transform_reduce_noalloc(x[:0], {"fn": "identity"}, "plain", out=out)
        r0 = out.clone()
    s.synchronize()
    ref = oracle.reduce({"fn": "identity"}, x.cpu())
    assert abs(r1.item() - ref["exact"]) <= TOL * ref["abs_sum"]
    assert r0.item() == 0.0
