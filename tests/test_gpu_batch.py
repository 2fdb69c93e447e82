"""GPU parity of the grouped batch entry point (hdc_batch_map_reduce)."""
import pytest
import torch

import oracle
import paper_2309_03912_amd as hdc
import synth

pytestmark = pytest.mark.gpu

HOR = {"fn": "horner", "coef": synth.horner_coefficients(8)}
FAFF = {"fn": "affine", "a": 2.5, "b": 0.5}
IAFF = {"fn": "affine", "a": 3, "b": -7}
IID = {"fn": "identity"}


def gpu():
    return torch.device("cuda", 0)


def bits(t):
    return t.view(torch.int16) if t.element_size() == 2 else t.view(torch.int32)


SIZES = [0, 1, 5, 15, 16, 17, 1000, 8191, 8192, 8193, 65541, 300001, 1 << 20] + \
    synth.call_sizes(9, calls=30, lo_log2=4, hi_log2=21)


@pytest.mark.parametrize("dt,acc,mf,rf", [(torch.float16, "compensated", FAFF, HOR),
                                          (torch.bfloat16, "plain", FAFF, HOR),
                                          (torch.float32, "compensated", HOR, FAFF),
                                          (torch.int32, "exact_int", IAFF, IID)])
def test_batch_matches_oracle(dt, acc, mf, rf):
    xs_cpu = []
    for i, n in enumerate(SIZES):
        if dt == torch.int32:
            xs_cpu.append(synth.uniform_int(40 + i, 10, n))
        else:
            xs_cpu.append(synth.to_storage(synth.uniform_pm1_f32(40 + i, 0, n).double(), dt))
    # some calls are unaligned views: x and y with equal and with different misalignment
    xs, ys = [], []
    for i, x in enumerate(xs_cpu):
        off = i % 3
        big = torch.zeros(x.numel() + 8, dtype=dt, device=gpu())
        big[off:off + x.numel()] = x.to(gpu())
        xs.append(big[off:off + x.numel()])
        ybig = torch.zeros(x.numel() + 8, dtype=dt, device=gpu())
        yo = off if i % 5 else (off + 1) % 3
        ys.append(ybig[yo:yo + x.numel()])
    ys, outs = hdc.batch_map_reduce(xs, mf, rf, acc, ys=ys)
    torch.cuda.synchronize()
    for i, x in enumerate(xs_cpu):
        assert torch.equal(bits(ys[i].cpu()), bits(oracle.map(mf, x))), f"map of call {i} (n={x.numel()})"
        ref = oracle.reduce(rf, x)
        if dt == torch.int32:
            assert outs[i].item() == ref["isum"], i
        elif ref["abs_sum"] == 0:
            assert outs[i].item() == 0.0
        else:
            assert abs(outs[i].item() - ref["exact"]) <= 1e-6 * ref["abs_sum"], (i, x.numel())


def test_batch_reduce_only_and_deterministic():
    xs = [synth.to_storage(synth.uniform_pm1_f32(70 + i, 0, n).double(), torch.float16).to(gpu())
          for i, n in enumerate(SIZES)]
    _, a = hdc.batch_map_reduce(xs, None, HOR, "compensated")
    _, b = hdc.batch_map_reduce(xs, None, HOR, "compensated")
    torch.cuda.synchronize()
    for i, x in enumerate(xs):
        assert torch.equal(a[i], b[i])
        ref = oracle.reduce(HOR, x.cpu())
        assert abs(a[i].item() - ref["exact"]) <= 1e-6 * max(ref["abs_sum"], 1e-300)


def test_batch_in_graph_replays_equal_eager():
    xs = [synth.uniform_int(90 + i, 10, n).to(gpu()) for i, n in enumerate(SIZES)]
    ys = [torch.empty_like(x) for x in xs]
    outs = [torch.empty((), dtype=torch.int64, device=gpu()) for _ in xs]
    ws = torch.zeros(hdc.workspace_size(hdc.OP_BATCH, hdc.I32, hdc.ACC_EXACT_INT, sum(x.numel() for x in xs),
                                        len(xs)), dtype=torch.uint8, device=gpu())
    hdc.batch_map_reduce(xs, IAFF, IID, "exact_int", ys=ys, outs=outs, ws=ws)
    torch.cuda.synchronize()
    eager = [(y.clone(), o.clone()) for y, o in zip(ys, outs)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=torch.cuda.Stream(device=gpu())):
        hdc.batch_map_reduce(xs, IAFF, IID, "exact_int", ys=ys, outs=outs, ws=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        for y, o in zip(ys, outs):
            y.fill_(0)
            o.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (y, o), (ye, oe) in zip(zip(ys, outs), eager):
            assert torch.equal(y, ye) and torch.equal(o, oe), rep
