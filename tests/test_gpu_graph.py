"""Captured-graph batching: many map + reduce calls recorded once and replayed.

Every replay must reproduce the eager results bit for bit (the library records
no memset node and allocates nothing while a stream is capturing), with the
program's own eager work and synchronisations between the replays; results
are also checked against the oracle.
"""
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


def make_calls(sizes, seed=17):
    calls = []
    for i, n in enumerate(sizes):
        if i % 2 == 0:
            x = synth.to_storage(synth.uniform_pm1_f32(seed + i, 0, n).double(), torch.float16).to(gpu())
            calls.append(("fp16", x, torch.empty_like(x), torch.empty((), dtype=torch.float64, device=gpu())))
        else:
            x = synth.uniform_int(seed + i, 10, n).to(gpu())
            calls.append(("i32", x, torch.empty_like(x), torch.empty((), dtype=torch.int64, device=gpu())))
    return calls


def issue(calls, wss, fused, streams=None):
    main = torch.cuda.current_stream()
    if streams:
        for s in streams:
            s.wait_stream(main)
    for k, (kind, x, y, r) in enumerate(calls):
        ws = wss[k % len(wss)]
        ctx = torch.cuda.stream(streams[k % len(streams)]) if streams else torch.cuda.stream(main)
        with ctx:
            if kind == "fp16":
                if fused:
                    hdc.map_reduce(x, FAFF, HOR, "compensated", out=y, result=r, ws=ws)
                else:
                    hdc.map(x, FAFF, out=y)
                    hdc.transform_reduce(x, HOR, "compensated", out=r, ws=ws)
            else:
                if fused:
                    hdc.map_reduce(x, IAFF, IID, "exact_int", out=y, result=r, ws=ws)
                else:
                    hdc.map(x, IAFF, out=y)
                    hdc.transform_reduce(x, IID, "exact_int", out=r, ws=ws)
    if streams:
        for s in streams:
            main.wait_stream(s)


def snapshot(calls):
    return [(y.clone(), r.clone()) for _, _, y, r in calls]


def same(a, b):
    return all(torch.equal(ya.view(torch.int16) if ya.element_size() == 2 else ya,
                           yb.view(torch.int16) if yb.element_size() == 2 else yb) and torch.equal(ra, rb)
               for (ya, ra), (yb, rb) in zip(a, b))


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("branches", [1, 3])
def test_graph_replays_equal_eager(fused, branches):
    sizes = synth.call_sizes(5, calls=12, lo_log2=10, hi_log2=20)
    calls = make_calls(sizes)
    nws = max(1, branches)
    wss = [torch.zeros(hdc.workspace_size(hdc.OP_MAP_REDUCE, hdc.F16, hdc.ACC_COMPENSATED, 1 << 20),
                       dtype=torch.uint8, device=gpu()) for _ in range(nws)]
    streams = [torch.cuda.Stream(device=gpu()) for _ in range(branches)] if branches > 1 else None
    issue(calls, wss, fused, streams)
    torch.cuda.synchronize()
    eager = snapshot(calls)
    # oracle check of the eager results
    for (kind, x, _, _), (y, r) in zip(calls, eager):
        xc = x.cpu()
        if kind == "fp16":
            ref = oracle.reduce(HOR, xc)
            assert abs(r.item() - ref["exact"]) <= 1e-6 * ref["abs_sum"]
            assert torch.equal(y.cpu().view(torch.int16), oracle.map(FAFF, xc).view(torch.int16))
        else:
            assert r.item() == oracle.reduce(IID, xc)["isum"]
            assert torch.equal(y.cpu(), oracle.map(IAFF, xc))

    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(device=gpu())
    with torch.cuda.graph(g, stream=cap):
        issue(calls, wss, fused, streams)
    torch.cuda.synchronize()
    for rep in range(4):
        for _, _, y, r in calls:  # scribble over the outputs eagerly between replays
            y.fill_(0)
            r.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert same(snapshot(calls), eager), f"replay {rep} differs from eager"


def test_capture_without_workspace_is_refused():
    x = torch.ones(1 << 16, device=gpu())
    out = torch.empty((), device=gpu())
    import ctypes
    f = hdc.make_functor(IID)
    stream = torch.cuda.Stream(device=gpu())
    g = torch.cuda.CUDAGraph()
    status = []
    # a stream the library has not served before: its internal workspace would have to be created
    with torch.cuda.graph(g, stream=stream):
        status.append(hdc.lib().hdc_transform_reduce(ctypes.byref(f), hdc.F32, x.data_ptr(), None, x.numel(), 0,
                                                     out.data_ptr(), None, 0, stream.cuda_stream))
    assert status == [hdc.ERR_WORKSPACE]
