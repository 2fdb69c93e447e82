"""Autotuner of the library's launch parameters.

For each tuning class (op, dtype, accumulation, size bucket) it times every
candidate setting of (block, unroll, grid_mult) -- then, for the segmented op,
(chunk, small_seg, seg_per_wave), and for the reductions one or two launches
(passes) -- on a synthetic workload of that class:

  * HIP events on the launching stream, `reps` calls per measurement, median
    of `rounds` measurements; candidates are interleaved round by round so
    that clock or thermal drift hits all of them alike;
  * the best three are re-timed with twice the rounds before one is chosen;
  * every candidate's output must agree with the others: maps bit for bit,
    integer sums exactly, floating-point sums within the library tolerance
    (1e-6 of the sum of magnitudes; the tuning workloads have positive terms,
    so that is 1e-6 of the result).

The winners are written as a tuning cache (one line per class:
"op dtype acc bucket block unroll grid_mult chunk small_seg seg_per_wave passes"),
which the library reads through hdc_load_tuning / HDC_TUNE_CACHE.

    python -m paper_2309_03912_amd.autotune --out paper_2309_03912_amd/tuning_gfx950.txt
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import statistics
import sys
import time

import torch

from . import (ACC_COMPENSATED, ACC_EXACT, ACC_EXACT_INT, ACC_PLAIN, BF16, F16, F32, I32, OP_BATCH, OP_MAP,
               OP_DOT, OP_MAP_REDUCE, OP_SCAN, OP_SEGMENTED_REDUCE, OP_TRANSFORM_REDUCE, get_tuning, set_tuning,
               tuning_bucket)
from . import map as hdc_map
from . import batch_map_reduce, map_reduce, scan, scan_status, segmented_reduce, transform_reduce, workspace

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_gfx950.txt")
TORCH_DT = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16, I32: torch.int32}
FIELDS = ["block", "unroll", "grid_mult", "chunk", "small_seg", "seg_per_wave", "passes"]


def _inputs(dt, n, dev, seed=1):
    """Positive-term tuning data: U[-1, 1) for floats (p(x) > 0 there), U[0, 2^20) ints."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    if dt == I32:
        return torch.randint(0, 1 << 20, (n,), generator=g, dtype=torch.int32).to(dev)
    x = (torch.randint(0, 1 << 24, (n,), generator=g, dtype=torch.int64) - (1 << 23)).to(torch.float32)
    return (x * 2.0 ** -23).to(TORCH_DT[dt]).to(dev)


def _time(fn, reps):
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


class Case:
    """One tuning class with its workload and a runner returning the output."""

    def __init__(self, op, dt, acc, n, dev, segments=None):
        self.op, self.dt, self.acc, self.n = op, dt, acc, n
        self.bucket = tuning_bucket(n)
        self.x = _inputs(dt, n, dev)
        coef = [1.0 / (k + 1) for k in range(9)]
        self.horner = {"fn": "horner", "coef": coef}
        self.aff = {"fn": "affine", "a": 3, "b": -7} if dt == I32 else {"fn": "affine", "a": 2.5, "b": 0.5}
        self.ident = {"fn": "identity"}
        self.y = torch.empty_like(self.x)
        accname = {ACC_PLAIN: "plain", ACC_COMPENSATED: "compensated", ACC_EXACT_INT: "exact_int",
                   ACC_EXACT: "exact"}[acc]
        self.accname = accname
        if op == OP_BATCH:
            # `segments` holds the call sizes of the batch
            self.xs = [_inputs(dt, m, dev, seed=10 + i) for i, m in enumerate(segments)]
            self.ys = [torch.empty_like(v) for v in self.xs]
            self.outs = [torch.empty((), dtype={ACC_PLAIN: torch.float32, ACC_COMPENSATED: torch.float64,
                                                ACC_EXACT_INT: torch.int64}[acc], device=dev) for _ in self.xs]
            self.ws = workspace(dev, op, dt, acc, sum(segments), len(segments))
            self.bucket = tuning_bucket(n)
        elif op == OP_SCAN:
            self.ys = torch.empty(n, dtype={ACC_PLAIN: torch.float32, ACC_COMPENSATED: torch.float64,
                                            ACC_EXACT_INT: torch.int64}[acc], device=dev)
            self.ws = workspace(dev, op, dt, acc, n)
        elif op == OP_SEGMENTED_REDUCE:
            self.off = segments.to(dev)
            S = self.off.numel() - 1
            self.ws = workspace(dev, op, dt, acc, n, S)
            self.out = torch.empty(S, dtype={ACC_PLAIN: torch.float32, ACC_COMPENSATED: torch.float64,
                                             ACC_EXACT_INT: torch.int64}[acc], device=dev)
        elif op != OP_MAP:
            self.ws = workspace(dev, op, dt, acc, n)
            self.out = torch.empty((), dtype={ACC_PLAIN: torch.float32, ACC_COMPENSATED: torch.float64,
                                              ACC_EXACT_INT: torch.int64, ACC_EXACT: torch.float64}[acc],
                                   device=dev)
        if op == OP_DOT:
            self.z = _inputs(dt, n, dev, seed=2)

    def run(self):
        if self.op == OP_BATCH:
            fn = self.ident if self.dt == I32 else self.horner
            batch_map_reduce(self.xs, self.aff, fn, self.accname, ys=self.ys, outs=self.outs, ws=self.ws)
            return
        if self.op == OP_SCAN:
            fn = self.ident if self.dt == I32 else self.horner
            scan(self.x, fn, self.accname, out=self.ys, ws=self.ws, check=False)  # checked in output()
            return
        if self.op == OP_MAP:
            hdc_map(self.x, self.aff, out=self.y)
        elif self.op == OP_TRANSFORM_REDUCE:
            fn = self.ident if self.dt == I32 or self.acc == ACC_EXACT else self.horner
            transform_reduce(self.x, fn, self.accname, out=self.out, ws=self.ws)
        elif self.op == OP_DOT:
            transform_reduce(self.x, {"fn": "product"}, self.accname, z=self.z, out=self.out, ws=self.ws)
        elif self.op == OP_MAP_REDUCE:
            fn = self.ident if self.dt == I32 else self.horner
            map_reduce(self.x, self.aff, fn, self.accname, out=self.y, result=self.out, ws=self.ws)
        else:
            fn = self.ident if self.dt == I32 else self.horner
            segmented_reduce(self.x, self.off, fn, self.accname, out=self.out, ws=self.ws)

    def output(self):
        if self.op == OP_BATCH:
            return ([y.clone() for y in self.ys], [o.clone() for o in self.outs])
        if self.op == OP_SCAN:
            if scan_status(self.ws) != 0:
                raise RuntimeError(f"a single-pass scan gave up on {self.key()}: its output is invalid")
            return self.ys.clone()
        if self.op == OP_MAP:
            return self.y.clone()
        if self.op == OP_MAP_REDUCE:
            return (self.y.clone(), self.out.clone())
        return self.out.clone()

    def agrees(self, a, b):
        if self.op == OP_BATCH:
            return all(self.agrees_map(p, q) for p, q in zip(a[0], b[0])) and \
                all(self.agrees_sum(p, q) for p, q in zip(a[1], b[1]))
        if self.op == OP_SCAN:
            return self.agrees_sum(a, b)
        if self.op == OP_MAP:
            return torch.equal(a.view(torch.int16) if a.element_size() == 2 else a.view(torch.int32),
                               b.view(torch.int16) if b.element_size() == 2 else b.view(torch.int32))
        if self.op == OP_MAP_REDUCE:
            return self.agrees_map(a[0], b[0]) and self.agrees_sum(a[1], b[1])
        return self.agrees_sum(a, b)

    def agrees_map(self, a, b):
        return torch.equal(a.view(torch.int16) if a.element_size() == 2 else a.view(torch.int32),
                           b.view(torch.int16) if b.element_size() == 2 else b.view(torch.int32))

    def agrees_sum(self, a, b):
        if self.acc in (ACC_EXACT_INT, ACC_EXACT):
            return torch.equal(a, b)
        a, b = a.double(), b.double()
        return bool(((a - b).abs() <= 2e-6 * torch.maximum(a.abs(), b.abs()) + 1e-30).all())

    def key(self):
        return (self.op, self.dt, self.acc, self.bucket)


def candidates(op, quick=False):
    blocks = [256, 512, 1024] if quick else [64, 128, 256, 512, 1024]
    unrolls = [2, 4, 8] if quick else [1, 2, 4, 8]
    gms = [4, 8, 16] if quick else [2, 4, 8, 16, 32, 64]
    base = [dict(block=b, unroll=u, grid_mult=g) for b, u, g in itertools.product(blocks, unrolls, gms)]
    if op == OP_BATCH:
        return base, [dict(chunk=c) for c in [8192, 16384, 32768, 65536]]
    if op == OP_SCAN:  # tile size x schedule (unroll 1: three passes, else one pass)
        return [dict(block=b, unroll=u) for b in [256, 512, 1024] for u in [1, 4]]
    if op in (OP_TRANSFORM_REDUCE, OP_DOT, OP_MAP_REDUCE):  # geometry, then one or two launches
        return base, [dict(passes=p) for p in (1, 2)]
    if op != OP_SEGMENTED_REDUCE:
        return base
    seg = [dict(chunk=c, small_seg=s, seg_per_wave=w)
           for c, s, w in itertools.product([2048, 4096, 8192] if quick else [1024, 2048, 4096, 8192, 16384],
                                            [64, 128, 256, 512], [2, 4, 8, 16] if quick else [1, 2, 4, 8, 16, 32, 64])]
    # per schedule (tiled, planned): the geometry at the default split, then the split (tile length for
    # the tiled schedule; piece length and small-segment packing for the planned one)
    return base, seg


def tune_case(case: Case, quick=False, reps=5, rounds=3, log=print):
    op, dt, acc, b = case.key()
    if op == OP_SEGMENTED_REDUCE:
        # each schedule tuned on its own, then the two winners timed against each other
        start = get_tuning(op, dt, acc, b)
        wins = []
        for passes in (1, 2):
            set_tuning(op, dt, acc, b, **dict(start, passes=passes))
            wins.append(_tune_stages(case, quick, reps, rounds, log))
        times = {i: [] for i in range(2)}
        for _ in range(2 * rounds):
            for i, w in enumerate(wins):
                set_tuning(op, dt, acc, b, **w)
                times[i].append(_time(case.run, reps))
        best = wins[min(times, key=lambda i: statistics.median(times[i]))]
        set_tuning(op, dt, acc, b, **best)
        log(json.dumps({"class": case.key(), "schedules": [
            {"passes": w["passes"], "ms": round(statistics.median(times[i]), 5)} for i, w in enumerate(wins)],
            "best": best}))
        return best
    return _tune_stages(case, quick, reps, rounds, log)


def _tune_stages(case: Case, quick, reps, rounds, log):
    op, dt, acc, b = case.key()
    cands = candidates(op, quick)
    stages = list(cands) if isinstance(cands, tuple) else [cands]
    best = get_tuning(op, dt, acc, b)
    for stage in stages:
        trial = [dict(best, **c) for c in stage]
        if op == OP_SEGMENTED_REDUCE and best.get("passes") == 1:  # tiled: only the tile length matters
            seen, uniq = set(), []
            for c in trial:
                key = tuple(sorted((k, v) for k, v in c.items() if k not in ("small_seg", "seg_per_wave")))
                if key not in seen:
                    seen.add(key)
                    uniq.append(c)
            trial = uniq
        times = {i: [] for i in range(len(trial))}
        ref = None
        for r in range(rounds):
            order = list(range(len(trial))) if r % 2 == 0 else list(reversed(range(len(trial))))
            for i in order:
                set_tuning(op, dt, acc, b, **trial[i])
                case.run()
                if r == 0:
                    out = case.output()
                    if ref is None:
                        ref = out
                    elif not case.agrees(ref, out):
                        raise RuntimeError(f"candidate {trial[i]} disagrees with {trial[0]} on {case.key()}")
                times[i].append(_time(case.run, reps))
        med = {i: statistics.median(v) for i, v in times.items()}
        top = sorted(med, key=med.get)[:3]
        re = {i: [] for i in top}
        for r in range(2 * rounds):
            for i in top:
                set_tuning(op, dt, acc, b, **trial[i])
                re[i].append(_time(case.run, reps))
        win = min(top, key=lambda i: statistics.median(re[i]))
        best = trial[win]
        set_tuning(op, dt, acc, b, **best)
        log(json.dumps({"class": case.key(), "n": case.n, "best": best,
                        "ms": round(statistics.median(re[win]), 5),
                        "default_ms": round(med[0], 5), "candidates": len(trial)}))
    return best


def default_cases(dev, quick=False, log2n=28):
    """The classes the workloads of this project use, at their sizes."""
    import synth  # seeded generators of the workloads (segment lengths)
    n = 1 << log2n
    cases = [
        Case(OP_MAP, F32, ACC_PLAIN, n, dev),
        Case(OP_MAP, I32, ACC_PLAIN, n, dev),
        Case(OP_TRANSFORM_REDUCE, F32, ACC_PLAIN, n, dev),
        Case(OP_TRANSFORM_REDUCE, I32, ACC_EXACT_INT, n, dev),
        Case(OP_TRANSFORM_REDUCE, BF16, ACC_COMPENSATED, n, dev),
        Case(OP_TRANSFORM_REDUCE, F16, ACC_COMPENSATED, n, dev),
        Case(OP_TRANSFORM_REDUCE, F32, ACC_COMPENSATED, n, dev),
        Case(OP_TRANSFORM_REDUCE, BF16, ACC_EXACT, n, dev),
        Case(OP_TRANSFORM_REDUCE, F16, ACC_EXACT, n, dev),
        Case(OP_DOT, F32, ACC_PLAIN, n, dev),
        Case(OP_DOT, BF16, ACC_COMPENSATED, n, dev),
        Case(OP_DOT, F16, ACC_COMPENSATED, n, dev),
        Case(OP_DOT, F16, ACC_EXACT, n, dev),
    ]
    L = synth.segment_lengths(synth.seed_of(4))
    off = synth.offsets_from_lengths(L)
    cases += [Case(OP_SEGMENTED_REDUCE, F32, ACC_PLAIN, int(off[-1]), dev, off),
              Case(OP_SEGMENTED_REDUCE, F32, ACC_COMPENSATED, int(off[-1]), dev, off)]
    # the 64-call graph workload as two grouped batches (fp16 and int32 halves)
    sizes = synth.call_sizes(synth.seed_of(5))
    cases += [Case(OP_BATCH, F16, ACC_COMPENSATED, sum(sizes[0::2]) // 32, dev, sizes[0::2]),
              Case(OP_BATCH, I32, ACC_EXACT_INT, sum(sizes[1::2]) // 32, dev, sizes[1::2])]
    cases += [Case(OP_SCAN, F32, ACC_PLAIN, n, dev), Case(OP_SCAN, F32, ACC_COMPENSATED, n, dev),
              Case(OP_SCAN, I32, ACC_EXACT_INT, n, dev)]
    # batched calls: every size bucket of the fused map + reduce
    for m in ([1 << 14, 1 << 18, 1 << 22, 1 << 25] if not quick else [1 << 18, 1 << 25]):
        cases += [Case(OP_MAP_REDUCE, F16, ACC_COMPENSATED, m, dev), Case(OP_MAP_REDUCE, I32, ACC_EXACT_INT, m, dev),
                  Case(OP_MAP, F16, ACC_PLAIN, m, dev), Case(OP_TRANSFORM_REDUCE, F16, ACC_COMPENSATED, m, dev)]
    return cases


def write_cache(path, results):
    lines = ["# hdc tuning cache (gfx950): op dtype acc bucket block unroll grid_mult chunk small_seg seg_per_wave "
             "passes"]
    for (op, dt, acc, b), t in sorted(results.items()):
        lines.append(" ".join(str(v) for v in (op, dt, acc, b, *(t[f] for f in FIELDS))))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_cache(path):
    """The classes of an existing cache file, as write_cache writes them."""
    results = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(w) for w in line.split()]
            results[tuple(v[:4])] = dict(zip(FIELDS, v[4:] + [2] * (len(FIELDS) + 4 - len(v))))
    return results


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__)
    p.add_argument("--out", default=DEFAULT_CACHE)
    p.add_argument("--quick", action="store_true")
    p.add_argument("--log2n", type=int, default=28)
    p.add_argument("--ops", default="", help="comma-separated op ids to tune (default: all)")
    p.add_argument("--merge", default="", help="cache file whose other classes are kept in the output")
    a = p.parse_args(argv)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    results = read_cache(a.merge) if a.merge else {}
    ops = {int(o) for o in a.ops.split(",")} if a.ops else None
    tuned = set()
    for case in default_cases(dev, a.quick, a.log2n):
        # a class is tuned once, at the first (largest) size listed for it
        if (ops is not None and case.op not in ops) or case.key() in tuned:
            continue
        tuned.add(case.key())
        results[case.key()] = tune_case(case, a.quick, log=lambda s: print(s, flush=True))
        del case
        torch.cuda.empty_cache()
    write_cache(a.out, results)
    print(json.dumps({"written": a.out, "classes": len(results), "seconds": round(time.time() - t0, 1)}),
          flush=True)


if __name__ == "__main__":
    sys.exit(main())
