"""The seeded input generators: counter-based SplitMix64 and the workload recipes."""
import math

import torch

import synth


def test_counter_form_equals_sequential_splitmix64():
    for seed, stream in [(0, 0), (synth.seed_of(1), 0), (synth.seed_of(3), 6), (2 ** 63 + 5, 10)]:
        st = synth.stream_state(seed, stream)
        ref = synth.splitmix64_reference(st, 4096)
        got = [v & synth.MASK64 for v in synth.u64(seed, stream, 0, 4096).tolist()]
        assert got == ref


def test_slices_are_index_addressable():
    full = synth.u64(7, 3, 0, 10000)
    part = synth.u64(7, 3, 1234, 500)
    assert torch.equal(full[1234:1734], part)


def test_streams_differ():
    a = synth.u64(7, 0, 0, 1000)
    b = synth.u64(7, 1, 0, 1000)
    assert (a == b).sum() == 0


def test_uniform_pm1_exact_grid():
    x = synth.uniform_pm1_f32(1, 0, 100000)
    k = x.double() * 2 ** 23
    assert torch.equal(k, torch.round(k))
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.double().mean().item()) < 0.01


def test_uniform_int_range():
    xi = synth.uniform_int(1, 10, 100000, bits=20)
    assert xi.dtype == torch.int32 and xi.min() >= 0 and xi.max() < (1 << 20)


def test_normal_moments():
    g = synth.normal_f64(1, 9, 200000)
    assert abs(g.mean().item()) < 0.01 and abs(g.std().item() - 1) < 0.01


def test_segment_lengths_recipe():
    L = synth.segment_lengths(synth.seed_of(4))
    assert L.numel() == 100000
    assert L.max().item() == 1 << 20
    assert abs(L.sum().item() / 2 ** 27 - 1) < 0.05
    assert 50 <= (L == 0).sum().item() <= 200
    assert L.median().item() in range(240, 272)
    off = synth.offsets_from_lengths(L)
    assert off[0] == 0 and off[-1] == L.sum() and bool((off[1:] >= off[:-1]).all())


def test_call_sizes_recipe():
    n = synth.call_sizes(synth.seed_of(5))
    assert len(n) == 64 and n[0] == 1 << 10 and n[-1] == 1 << 26
    assert all(1 << 10 <= v <= 1 << 26 for v in n)


def test_fp16_storage_clamps():
    v = torch.tensor([1e6, -1e6, 65519.0, 1e-9], dtype=torch.float64)
    s = synth.to_storage(v, torch.float16)
    assert s.tolist()[:3] == [65504.0, -65504.0, 65504.0]
    assert math.isfinite(s.float().abs().max().item())


def test_horner_coefficients():
    c = synth.horner_coefficients(8)
    assert len(c) == 9 and c[0] == 1.0 and c[1] == 0.5
    assert all(float(torch.tensor(v, dtype=torch.float32)) == v for v in c)
