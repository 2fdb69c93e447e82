"""Benchmark of the generic map / reduce path on one MI355X.

One step = one pass of the whole plain-FP32 hot path over the bandwidth-scale
workload (n = 2^28 per array): map y = 2.5 x + 0.5; sum of the degree-8
Horner polynomial p(x); dot(x', z') with x', z' ~ N(0,1); int32 map
y = 3 x - 7; int64 sums of x and y.  `value` = algorithmic HBM bytes of the
step / time per step (GB/s).  The precision, batching and graph forms are
timed after it and reported under "forms".

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GiB = 1 << 30


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--log2n", type=int, default=28)
    p.add_argument("--no-check", action="store_true", help="skip the full-size oracle accuracy check")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-log2", type=int, default=26)
    return p.parse_args()


class OpTimer:
    """HIP events around each operation on the stream it is launched on."""

    def __init__(self, torch, names):
        self.torch = torch
        self.names = names
        self.pairs = {k: [] for k in names}

    def run(self, name, fn):
        s = self.torch.cuda.Event(enable_timing=True)
        e = self.torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        self.pairs[name].append((s, e))

    def mean_ms(self, name):
        v = [s.elapsed_time(e) for s, e in self.pairs[name]]
        return sum(v) / len(v)


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU design is described, "
                                   "not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2309_03912_amd as hdc
    import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = 1 << args.log2n
    seed = synth.seed_of(2)
    S = synth.STREAM
    coef = synth.horner_coefficients(8)
    F_AFF, F_HOR, F_DOT = hdc.affine(2.5, 0.5), hdc.horner(coef), hdc.product()
    I_AFF, I_ID = hdc.affine(3, -7), hdc.identity()

    t0 = time.time()
    x = synth.uniform_pm1_f32(seed, S["x"], n, dev)
    xn = synth.to_storage(synth.normal_f64(seed, S["xn"], n, dev), torch.float32)
    zn = synth.to_storage(synth.normal_f64(seed, S["z"], n, dev), torch.float32)
    xi = synth.uniform_int(seed, S["xi"], n, 20, dev)
    y = torch.empty_like(x)
    yi = torch.empty_like(xi)
    r_p = torch.empty((), dtype=torch.float32, device=dev)
    r_d = torch.empty((), dtype=torch.float32, device=dev)
    r_x = torch.empty((), dtype=torch.int64, device=dev)
    r_y = torch.empty((), dtype=torch.int64, device=dev)
    ws = hdc.workspace(dev, hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, n)
    torch.cuda.synchronize()
    gen_s = time.time() - t0

    ops = [
        ("map_f32_affine", 2 * 4 * n, lambda: hdc.map(x, F_AFF, out=y)),
        ("sum_f32_horner", 4 * n, lambda: hdc.transform_reduce(x, F_HOR, "plain", out=r_p, ws=ws)),
        ("dot_f32", 2 * 4 * n, lambda: hdc.transform_reduce(xn, F_DOT, "plain", z=zn, out=r_d, ws=ws)),
        ("map_i32_affine", 2 * 4 * n, lambda: hdc.map(xi, I_AFF, out=yi)),
        ("sum_i32_x_to_i64", 4 * n, lambda: hdc.transform_reduce(xi, I_ID, "exact_int", out=r_x, ws=ws)),
        ("sum_i32_y_to_i64", 4 * n, lambda: hdc.transform_reduce(yi, I_ID, "exact_int", out=r_y, ws=ws)),
    ]
    step_bytes = sum(b for _, b, _ in ops)

    def step(timer=None):
        for name, _, fn in ops:
            if timer is None:
                fn()
            else:
                timer.run(name, fn)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: exactly K steps, synchronised on both sides.
    timer = OpTimer(torch, [o[0] for o in ops])
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(timer)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    per_op = {}
    for name, b, _ in ops:
        ms = timer.mean_ms(name)
        per_op[name] = {"ms": round(ms, 5), "GBps": round(b / (ms * 1e-3) / 1e9, 1),
                        "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "bytes": b}
    dominant = max(per_op, key=lambda k: per_op[k]["ms"])
    d = per_op[dominant]
    roofline = {"bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["GBps"] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dominant,
                "bytes_per_launch": d["bytes"], "launch_ms": d["ms"]}

    out = {
        "metric": "HBM GB/s & % peak: plain FP32 vs BF16-compensated/batched at <=1e-6 rel err",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded counter-based generators, generated on the GPU)",
        "config": {"workload": "plain-fp32 bandwidth scale: n=2^%d per array; map 2.5x+0.5, sum Horner-8 p(x), "
                               "dot N(0,1), int32 map 3x-7, int64 sums" % args.log2n,
                   "n": n, "step_bytes": step_bytes},
        "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
        "per_op": per_op,
        "roofline": roofline,
        "gen_s": round(gen_s, 2),
    }

    if not args.no_check:
        import oracle
        t1 = time.time()
        torch.cuda.synchronize()
        xc, xnc, znc, xic = x.cpu(), xn.cpu(), zn.cpu(), xi.cpu()
        ref_p = oracle.reduce(F_HOR, xc)
        ref_d = oracle.reduce(F_DOT, xnc, znc)
        ref_x = oracle.reduce(I_ID, xic)
        ref_y = oracle.reduce(I_AFF, xic)
        chk = {
            "sum_f32_horner_err_over_abs": abs(r_p.item() - ref_p["exact"]) / ref_p["abs_sum"],
            "dot_f32_err_over_abs": abs(r_d.item() - ref_d["exact"]) / ref_d["abs_sum"],
            "sum_f32_horner_rel_err": abs(r_p.item() - ref_p["exact"]) / abs(ref_p["exact"]),
            "dot_f32_rel_err": abs(r_d.item() - ref_d["exact"]) / abs(ref_d["exact"]),
            "int_sums_bit_exact": r_x.item() == ref_x["isum"] and r_y.item() == ref_y["isum"],
        }
        chk["pass"] = (chk["sum_f32_horner_err_over_abs"] <= 1e-6 and chk["dot_f32_err_over_abs"] <= 1e-6
                       and chk["int_sums_bit_exact"])
        chk["check_s"] = round(time.time() - t1, 1)
        out["accuracy"] = chk

    if not args.no_cpu_baseline:
        import oracle
        m = min(n, 1 << args.cpu_sample_log2)
        xc, xnc, znc, xic = x[:m].cpu(), xn[:m].cpu(), zn[:m].cpu(), xi[:m].cpu()
        yic = yi[:m].cpu()
        t1 = time.perf_counter()
        oracle.map(F_AFF, xc)
        oracle.reduce(F_HOR, xc)
        oracle.reduce(F_DOT, xnc, znc)
        oracle.map(I_AFF, xic)
        oracle.reduce(I_ID, xic)
        oracle.reduce(I_ID, yic)
        cpu_s = time.perf_counter() - t1
        sample_bytes = step_bytes * m // n
        out["cpu_baseline"] = {"value": round(sample_bytes / cpu_s / 1e9, 3), "unit": "GB/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the six operations of one step on the first 2^{m.bit_length() - 1} "
                                         f"elements of each array ({cpu_s:.1f} s, single thread); host has "
                                         f"{host_cores()} cores: {cpu_model()}"}

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
