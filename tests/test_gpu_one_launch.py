"""The one-launch reduction (the block that finishes last folds the per-block
partials, counted on a ticket) against the two-launch form, through the C ABI.
Both fold the partials in the same fixed order, so for one tuning they must
give the same bits; each result is also held to the oracle's bar.  Covers
every fold state (plain, compensated, int64, exact fp16; dot; fused map +
reduce), blocks of 64..1024 threads with one to many partials, long runs of
calls on one workspace (the ticket must be back at 0 after every call),
graph replays, and calls on several workspaces in a row."""
import contextlib

import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

pytestmark = pytest.mark.gpu

COEF8 = synth.horner_coefficients(8)
HORNER = {"fn": "horner", "coef": COEF8}
TOL = 1e-6


@contextlib.contextmanager
def tuning(op, dt, acc, **kw):
    saved = {b: hdc.get_tuning(op, dt, acc, b) for b in range(hdc.BUCKETS)}
    try:
        hdc.set_tuning(op, dt, acc, -1, **kw)
        yield
    finally:
        for b, t in saved.items():
            hdc.set_tuning(op, dt, acc, b, **t)


def bits(t):
    iv = torch.int64 if t.element_size() == 8 else torch.int32 if t.element_size() == 4 else torch.int16
    return t.cpu().reshape(-1).view(iv)


def check(got, ref, acc, what):
    if acc == "exact_int":
        assert got == ref["isum"], what
    elif acc == "exact":
        assert got == ref["exact"], what
    else:
        assert abs(got - ref["exact"]) <= TOL * ref["abs_sum"], (what, got, ref["exact"])


CASES = [
    # name, op, dtype, functor, accumulation, binary
    ("f32_horner_plain", hdc.OP_TRANSFORM_REDUCE, torch.float32, HORNER, "plain", False),
    ("bf16_identity_comp", hdc.OP_TRANSFORM_REDUCE, torch.bfloat16, {"fn": "identity"}, "compensated", False),
    ("f16_horner_comp", hdc.OP_TRANSFORM_REDUCE, torch.float16, HORNER, "compensated", False),
    ("i32_affine_int", hdc.OP_TRANSFORM_REDUCE, torch.int32, {"fn": "affine", "a": 3, "b": -7}, "exact_int", False),
    ("f16_identity_exact", hdc.OP_TRANSFORM_REDUCE, torch.float16, {"fn": "identity"}, "exact", False),
    ("f32_dot_plain", hdc.OP_DOT, torch.float32, {"fn": "product"}, "plain", True),
    ("f16_dot_comp", hdc.OP_DOT, torch.float16, {"fn": "product"}, "compensated", True),
]
GEOMETRIES = [(64, 1, 1), (64, 8, 64), (128, 2, 4), (256, 4, 8), (1024, 8, 2), (1024, 1, 64)]  # block, unroll, gm


def make(n, dt, seed, stream):
    if dt == torch.int32:
        return synth.uniform_int(seed, stream, n, bits=20)
    return synth.to_storage(synth.normal_f64(seed, stream, n), dt)


@pytest.mark.parametrize("name,op,dt,fn,acc,binary", CASES, ids=[c[0] for c in CASES])
def test_one_launch_equals_two_launches(name, op, dt, fn, acc, binary):
    dev = torch.device("cuda", 0)
    code, a = hdc.DTYPE[dt], hdc.ACC[acc]
    ws = torch.zeros(hdc.workspace_size(op, code, a, 1 << 22), dtype=torch.uint8, device=dev)
    for n in (1, 1000, 65541, (1 << 21) + 13):
        x = make(n, dt, 230903950 + n, 0)
        z = make(n, dt, 230903950 + n, 1) if binary else None
        xg, zg = x.to(dev), (z.to(dev) if binary else None)
        ref = oracle.reduce(fn, x, z)
        for block, unroll, gm in GEOMETRIES:
            got = {}
            for passes in (2, 1):
                with tuning(op, code, a, block=block, unroll=unroll, grid_mult=gm, passes=passes):
                    print(f"one-launch {name} n={n} block={block} unroll={unroll} gm={gm} passes={passes}",
                          flush=True)
                    got[passes] = hdc.transform_reduce(xg, fn, acc, z=zg, ws=ws)
            torch.cuda.synchronize()
            assert torch.equal(bits(got[1]), bits(got[2])), (name, n, block, unroll, gm)
            check(got[1].item(), ref, acc, (name, n, block, unroll, gm))


@pytest.mark.parametrize("dt", [torch.float32, torch.float16, torch.int32])
def test_one_launch_fused_map_reduce(dt):
    dev = torch.device("cuda", 0)
    code = hdc.DTYPE[dt]
    if dt == torch.int32:
        fm, fr, acc = {"fn": "affine", "a": 3, "b": -7}, {"fn": "identity"}, "exact_int"
    else:
        fm, fr, acc = {"fn": "affine", "a": 2.5, "b": 0.5}, HORNER, "compensated"
    a = hdc.ACC[acc]
    n = (1 << 20) + 5
    x = make(n, dt, 230903960, 0)
    xg = x.to(dev)
    ref = oracle.reduce(fr, x)
    ymap = oracle.map(fm, x)
    got = {}
    for passes in (2, 1):
        with tuning(hdc.OP_MAP_REDUCE, code, a, block=256, unroll=2, grid_mult=4, passes=passes):
            got[passes] = hdc.map_reduce(xg, fm, fr, acc)
    torch.cuda.synchronize()
    assert torch.equal(bits(got[1][1]), bits(got[2][1]))
    assert torch.equal(bits(got[1][0]), bits(ymap))
    check(got[1][1].item(), ref, acc, dt)


def test_one_launch_many_calls_in_a_row_and_several_workspaces():
    """200 calls of changing size and grid on one workspace, interleaved with calls on two other
    workspaces: every result must match its two-launch twin, so every ticket was back at 0."""
    dev = torch.device("cuda", 0)
    sizes = [1 + (37 * k * k) % ((1 << 20) + 3) for k in range(200)]
    xs = synth.to_storage(synth.normal_f64(230903970, 0, max(sizes)), torch.float32)
    xg = xs.to(dev)
    wss = [torch.zeros(hdc.workspace_size(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, 1), dtype=torch.uint8,
                       device=dev) for _ in range(3)]
    outs = {1: torch.empty(len(sizes), dtype=torch.float32, device=dev),
            2: torch.empty(len(sizes), dtype=torch.float32, device=dev)}
    for passes in (2, 1):
        for k, n in enumerate(sizes):
            gm = (1, 2, 8, 64)[k % 4]
            with tuning(hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, block=256, unroll=2, grid_mult=gm,
                        passes=passes):
                hdc.transform_reduce(xg[:n], HORNER, "plain", out=outs[passes][k], ws=wss[k % 3])
    torch.cuda.synchronize()
    assert torch.equal(bits(outs[1]), bits(outs[2]))
    for k in (0, 1, 57, 199):
        check(outs[1][k].item(), oracle.reduce(HORNER, xs[:sizes[k]]), "plain", k)


def test_one_launch_in_a_replayed_graph():
    """A captured one-launch reduction replayed 20 times, with eager work between replays: every
    replay equals the eager result bit for bit (the ticket is reset inside the graph)."""
    dev = torch.device("cuda", 0)
    n = (1 << 22) + 3
    x = synth.to_storage(synth.normal_f64(230903980, 0, n), torch.bfloat16).to(dev)
    ws = torch.zeros(hdc.workspace_size(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_COMPENSATED, n), dtype=torch.uint8,
                     device=dev)
    out = torch.empty((), dtype=torch.float64, device=dev)
    with tuning(hdc.OP_TRANSFORM_REDUCE, hdc.BF16, hdc.ACC_COMPENSATED, passes=1):
        eager = hdc.transform_reduce(x, {"fn": "identity"}, "compensated", ws=ws).clone()
        s = torch.cuda.Stream(device=dev)
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            hdc.transform_reduce(x, {"fn": "identity"}, "compensated", out=out, ws=ws)
        torch.cuda.synchronize()
        for r in range(20):
            out.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(bits(out), bits(eager)), r
            hdc.transform_reduce(x[: n // 3], {"fn": "identity"}, "compensated", ws=ws)  # eager work between
            torch.cuda.synchronize()
