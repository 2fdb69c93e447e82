"""Benchmark of the generic map / reduce path on one MI355X.

`value` (the headline): one step = one pass of the plain-FP32 hot path over
the bandwidth-scale workload, n = 2^28 per array:
    map y = 2.5 x + 0.5 (f32); sum of the degree-8 Horner polynomial p(x);
    dot(x', z') with x', z' ~ N(0,1); int32 map y = 3 x - 7; int64 sums of x
    and y.
value = algorithmic HBM bytes of the step / time per step (GB/s).

"forms" reports, after the timed steps, the precision form (16-bit storage,
compensated sums, kappa ~ 1e8 sum), the batching form (100,000 lognormal
segments in one persistent pass) and the graph form (64 map+reduce calls
replayed from one captured graph), each next to its plain-FP32 comparator,
with the error against the exact (oracle) result.

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--log2n", type=int, default=28)
    p.add_argument("--no-check", action="store_true", help="skip the oracle accuracy checks")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-forms", action="store_true", help="only the headline plain-FP32 step")
    p.add_argument("--forms", default="c1,c3,c4,c5,scan,host")
    p.add_argument("--cpu-sample-log2", type=int, default=28)
    p.add_argument("--with-copy", action="store_true",
                   help="add a plain copy (identity map, f32) to each step: the reference kernel of known size "
                        "that calibrates the HBM traffic counters")
    p.add_argument("--replays", type=int, default=1000)
    p.add_argument("--no-per-call-comparator", action="store_true",
                   help="skip the segmented form's comparator of one host-issued call per segment "
                        "(100,000 launches, too many for a counter-collection run)")
    return p.parse_args()


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


def gbps(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def ev_time(torch, fn, reps=20, warm=3, groups=5, warm_s=0.25):
    """Mean ms per call of `fn` over `reps` calls issued back to back, from two HIP events on the
    current stream around each group of calls (the time each call adds to a stream of work, with no
    idle GPU between calls; a lone call on an idle GPU also waits for its own launch from the host).
    Before timing, `fn` runs `warm` times and then for at least `warm_s` seconds: an idle GPU runs
    its first fraction of a second at lower clocks, and a short kernel timed then reads up to ~20%
    slow.  Returns the median over `groups` groups."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    ts = []
    for _ in range(groups):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e) / reps)
    ts.sort()
    return ts[len(ts) // 2]


def err_fields(got, ref):
    exact, A = ref["exact"], ref["abs_sum"]
    e = abs(got - exact)
    return {"err_over_abs_sum": e / A if A else e, "rel_err": e / abs(exact) if exact else e,
            "err_vs_fp64_seq_over_abs": abs(got - ref["seq64"]) / A if A else 0.0}


# ---------------------------------------------------------------------------
# Headline: plain FP32 at bandwidth scale
# ---------------------------------------------------------------------------

def headline(args, torch, hdc, synth):
    dev = torch.device("cuda", 0)
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
    if args.with_copy:
        ycopy = torch.empty_like(x)
        ops.append(("copy_f32_identity", 2 * 4 * n, lambda: hdc.map(x, hdc.identity(), out=ycopy)))
    pairs = {name: [] for name, _, _ in ops}

    def step(record):
        for name, _, fn in ops:
            if record:
                s = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                s.record()
                fn()
                e.record()
                pairs[name].append((s, e))
            else:
                fn()

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    if args.with_copy:  # the calibration copy is not part of the step's bytes or time
        ms_per_step -= statistics.mean(s.elapsed_time(e) for s, e in pairs["copy_f32_identity"])

    per_op = {}
    for name, b, _ in ops:
        ms = statistics.mean(s.elapsed_time(e) for s, e in pairs[name])
        per_op[name] = {"ms": round(ms, 5), "GBps": round(gbps(b, ms), 1),
                        "frac_of_peak": round(gbps(b, ms) / HBM_PEAK_GBS, 4), "bytes": b}
    res = {"n": n, "step_bytes": step_bytes, "ms_per_step": ms_per_step, "per_op": per_op, "gen_s": gen_s}

    if not args.no_check:
        import oracle
        t1 = time.time()
        xc, xnc, znc, xic = x.cpu(), xn.cpu(), zn.cpu(), xi.cpu()
        ref_p = oracle.reduce(F_HOR, xc)
        ref_d = oracle.reduce(F_DOT, xnc, znc)
        ref_x = oracle.reduce(I_ID, xic)
        ref_y = oracle.reduce(I_AFF, xic)
        idx = torch.randint(0, n, (1 << 20,), generator=torch.Generator().manual_seed(5))
        map_ok = torch.equal(y.cpu()[idx].view(torch.int32), oracle.map(F_AFF, xc[idx]).view(torch.int32)) and \
            torch.equal(yi.cpu()[idx], oracle.map(I_AFF, xic[idx]))
        chk = {"sum_f32_horner": err_fields(r_p.item(), ref_p), "dot_f32": err_fields(r_d.item(), ref_d),
               "int_sums_bit_exact": r_x.item() == ref_x["isum"] and r_y.item() == ref_y["isum"],
               "maps_bit_exact_on_2^20_sampled_outputs": map_ok}
        chk["pass"] = (chk["sum_f32_horner"]["err_over_abs_sum"] <= 1e-6 and
                       chk["dot_f32"]["err_over_abs_sum"] <= 1e-6 and chk["int_sums_bit_exact"] and map_ok)
        chk["check_s"] = round(time.time() - t1, 1)
        res["accuracy"] = chk

    if not args.no_cpu_baseline:
        import oracle
        m = min(n, 1 << args.cpu_sample_log2)
        xc, xnc, znc, xic, yic = x[:m].cpu(), xn[:m].cpu(), zn[:m].cpu(), xi[:m].cpu(), yi[:m].cpu()
        t1 = time.perf_counter()
        oracle.map(F_AFF, xc)
        oracle.reduce(F_HOR, xc)
        oracle.reduce(F_DOT, xnc, znc)
        oracle.map(I_AFF, xic)
        oracle.reduce(I_ID, xic)
        oracle.reduce(I_ID, yic)
        cpu_s = time.perf_counter() - t1
        sample_bytes = step_bytes * m // n
        res["cpu_baseline"] = {
            "value": round(gbps(sample_bytes, cpu_s * 1e3), 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the six operations of one step on the first 2^{m.bit_length() - 1} elements of each "
                      f"array ({cpu_s:.1f} s on one thread; the oracle also forms the exact sum); host: "
                      f"{host_cores()} cores, {cpu_model()}"}
        # the same oracle on every core of the process: one contiguous range per thread, exact
        # accumulators joined in range order (best of 3)
        threads = host_cores()
        best = None
        for _ in range(3):
            t1 = time.perf_counter()
            oracle.map_mt(F_AFF, xc, threads)
            oracle.reduce_mt(F_HOR, xc, threads=threads)
            oracle.reduce_mt(F_DOT, xnc, znc, threads=threads)
            oracle.map_mt(I_AFF, xic, threads)
            oracle.reduce_mt(I_ID, xic, threads=threads)
            oracle.reduce_mt(I_ID, yic, threads=threads)
            dt = time.perf_counter() - t1
            best = dt if best is None else min(best, dt)
        res["cpu_baseline_multicore"] = {
            "value": round(gbps(sample_bytes, best * 1e3), 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle, one thread per core",
            "sample": f"the same sample on {threads} threads ({best:.2f} s, best of 3; exact and integer "
                      f"results identical to the one-thread oracle)"}
    del x, xn, zn, xi, y, yi
    torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------------------
# Precision form: 16-bit storage, compensated sums
# ---------------------------------------------------------------------------

def form_precision(args, torch, hdc, synth):
    dev = torch.device("cuda", 0)
    n = 1 << args.log2n
    seed = synth.seed_of(3)
    S = synth.STREAM
    out = {"n": n}
    xg64 = synth.normal_f64(seed, S["x"], n, dev)
    zg64 = synth.normal_f64(seed, S["z"], n, dev)
    for dt, name in ((torch.bfloat16, "bf16"), (torch.float16, "fp16")):
        x = synth.to_storage(xg64, dt)
        z = synth.to_storage(zg64, dt)
        v, info = synth.ill_conditioned(seed, n, dt, device=dev)
        # an ill-conditioned dot: products x2 * z2 are exactly the values v
        x2, z2, info2 = synth.ill_conditioned_dot(seed, n, dt, device=dev)
        xf, zf, vf = x.float(), z.float(), v.float()  # the plain-FP32 comparator reads widened copies
        x2f, z2f = x2.float(), z2.float()
        ident, prod = hdc.identity(), hdc.product()
        runs = {
            "sum_x": (lambda: hdc.transform_reduce(x, ident, "compensated"), 2 * n,
                      lambda: hdc.transform_reduce(xf, ident, "plain"), 4 * n),
            "dot_xz": (lambda: hdc.transform_reduce(x, prod, "compensated", z=z), 4 * n,
                       lambda: hdc.transform_reduce(xf, prod, "plain", z=zf), 8 * n),
            "sum_v_kappa": (lambda: hdc.transform_reduce(v, ident, "compensated"), 2 * n,
                            lambda: hdc.transform_reduce(vf, ident, "plain"), 4 * n),
            "dot_kappa": (lambda: hdc.transform_reduce(x2, prod, "compensated", z=z2), 4 * n,
                          lambda: hdc.transform_reduce(x2f, prod, "plain", z=z2f), 8 * n),
        }
        res = {"kappa": info["kappa"], "dot_kappa_kappa": info2["kappa"]}
        refs = {}
        for op, (fc, bc, fp, bp) in runs.items():
            tc = ev_time(torch, fc)
            tp = ev_time(torch, fp)
            rc, rp = fc().item(), fp().item()
            entry = {"comp_ms": round(tc, 5), "comp_GBps": round(gbps(bc, tc), 1),
                     "plain_f32_ms": round(tp, 5), "plain_f32_GBps": round(gbps(bp, tp), 1),
                     "speedup_vs_plain_f32": round(tp / tc, 3)}
            if not args.no_check:
                import oracle
                if op == "sum_v_kappa":
                    ref = oracle.reduce(ident, v)
                    entry["oracle_exact_equals_construction_target"] = ref["exact"] == info["target"]
                elif op == "dot_kappa":
                    ref = oracle.reduce(prod, x2, z2)
                    entry["oracle_exact_equals_construction_target"] = ref["exact"] == info2["target"]
                elif op == "sum_x":
                    ref = oracle.reduce(ident, x)
                else:
                    ref = oracle.reduce(prod, x, z)
                refs[op] = ref["exact"]
                entry["comp_err"] = err_fields(rc, ref)
                entry["plain_f32_err"] = err_fields(rp, ref)
            res[op] = entry
        # exact sums (and fp16 dots): the correctly rounded exact result, independent of order and tuning
        exact_runs = [("sum_x", lambda: hdc.transform_reduce(x, ident, "exact"), 2 * n),
                      ("sum_v_kappa", lambda: hdc.transform_reduce(v, ident, "exact"), 2 * n)]
        if dt == torch.float16:
            exact_runs += [("dot_xz", lambda: hdc.transform_reduce(x, prod, "exact", z=z), 4 * n),
                           ("dot_kappa", lambda: hdc.transform_reduce(x2, prod, "exact", z=z2), 4 * n)]
        for op, fe, be in exact_runs:
            te = ev_time(torch, fe)
            entry = {"exact_ms": round(te, 5), "exact_GBps": round(gbps(be, te), 1)}
            if not args.no_check:
                entry["exact_bits_equal_oracle"] = fe().item() == refs[op]
            res[op].update(entry)
        out[name] = res
        del x, z, v, xf, zf, vf, x2, z2, x2f, z2f
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Batching form: 100,000 lognormal segments in one persistent pass
# ---------------------------------------------------------------------------

def form_segmented(args, torch, hdc, synth):
    dev = torch.device("cuda", 0)
    seed = synth.seed_of(4)
    L = synth.segment_lengths(seed)
    off = synth.offsets_from_lengths(L)
    n = int(off[-1])
    S = L.numel()
    x = synth.uniform_pm1_f32(seed, synth.STREAM["x"], n, dev)
    og = off.to(dev)
    hor = hdc.horner(synth.horner_coefficients(8))
    nbytes = 4 * n + 8 * (S + 1)
    out = {"segments": S, "elements": n, "max_len": int(L.max()), "empty": int((L == 0).sum())}
    res = {}
    for acc in ("plain", "compensated"):
        ws = hdc.workspace(dev, hdc.OP_SEGMENTED_REDUCE, hdc.F32, hdc.ACC[acc], n, S)
        r = torch.empty(S, dtype=hdc.OUT_DTYPE[hdc.ACC[acc]], device=dev)
        t = ev_time(torch, lambda: hdc.segmented_reduce(x, og, hor, acc, out=r, ws=ws))
        res[acc] = {"ms": round(t, 5), "GBps": round(gbps(nbytes + r.element_size() * S, t), 1)}
        if not args.no_check:
            import oracle
            import numpy as np
            ref = oracle.segmented(hor, x.cpu(), off)
            got = r.cpu().double().numpy()
            e = np.abs(got - ref["exact"])
            A = ref["abs_sum"]
            res[acc]["max_err_over_abs_sum"] = float(np.max(np.where(A > 0, e / np.where(A > 0, A, 1), e)))
            res[acc]["segments_within_1e-6"] = int(np.sum(e <= 1e-6 * A))
    if args.no_per_call_comparator:
        out.update(res)
        del x
        torch.cuda.empty_cache()
        return out
    # Comparator: one plain transform_reduce call per segment (eager, from the host)
    r1 = torch.empty(S, dtype=torch.float32, device=dev)
    ws1 = hdc.workspace(dev, hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, 1 << 20)
    offl = off.tolist()
    f = hdc.make_functor(hor)
    import ctypes
    L_ = hdc.lib()
    stream = torch.cuda.current_stream().cuda_stream
    base, esz = x.data_ptr(), 4
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(S):
        L_.hdc_transform_reduce(ctypes.byref(f), hdc.F32, base + esz * offl[j], None, offl[j + 1] - offl[j], 0,
                                r1.data_ptr() + 4 * j, ws1.data_ptr(), ws1.numel(), stream)
    torch.cuda.synchronize()
    t_calls = (time.perf_counter() - t0) * 1e3
    res["per_segment_calls"] = {"ms": round(t_calls, 3), "GBps": round(gbps(nbytes, t_calls), 2),
                                "note": "100,000 plain hdc_transform_reduce calls issued from the host"}
    res["speedup_vs_per_segment_calls"] = round(t_calls / res["plain"]["ms"], 1)
    out.update(res)
    del x
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Graph form: 64 map + reduce calls in one captured graph
# ---------------------------------------------------------------------------

def form_graph(args, torch, hdc, synth):
    dev = torch.device("cuda", 0)
    seed = synth.seed_of(5)
    sizes = synth.call_sizes(seed)
    hor = hdc.horner(synth.horner_coefficients(8))
    faff, iaff, iid = hdc.affine(2.5, 0.5), hdc.affine(3, -7), hdc.identity()
    calls = []
    for i, n in enumerate(sizes):
        if i % 2 == 0:
            x = synth.to_storage(synth.uniform_pm1_f32(seed + i, synth.STREAM["x"], n, dev).double(), torch.float16)
            calls.append({"kind": "fp16", "n": n, "x": x, "y": torch.empty_like(x), "xf": x.float(),
                          "yf": torch.empty(n, dtype=torch.float32, device=dev),
                          "r": torch.empty((), dtype=torch.float64, device=dev),
                          "rf": torch.empty((), dtype=torch.float32, device=dev)})
        else:
            x = synth.uniform_int(seed + i, synth.STREAM["xi"], n, 20, dev)
            calls.append({"kind": "i32", "n": n, "x": x, "y": torch.empty_like(x),
                          "r": torch.empty((), dtype=torch.int64, device=dev)})
    bytes_sep = sum(6 * c["n"] if c["kind"] == "fp16" else 12 * c["n"] for c in calls)
    bytes_fused = sum(4 * c["n"] if c["kind"] == "fp16" else 8 * c["n"] for c in calls)
    bytes_f32 = sum(12 * c["n"] for c in calls)
    nmax = max(sizes)
    nbranch = 4
    streams = [torch.cuda.Stream(device=dev) for _ in range(nbranch)]
    wss = [hdc.workspace(dev, hdc.OP_TRANSFORM_REDUCE, hdc.F16, hdc.ACC_COMPENSATED, nmax) for _ in streams]
    wss = [torch.zeros_like(w) for w in wss]  # one workspace per branch
    order = sorted(range(len(calls)), key=lambda i: -calls[i]["n"])  # longest first, round-robin branches

    def issue(c, ws, fused):
        if c["kind"] == "fp16":
            if fused:
                hdc.map_reduce(c["x"], faff, hor, "compensated", out=c["y"], result=c["r"], ws=ws)
            else:
                hdc.map(c["x"], faff, out=c["y"])
                hdc.transform_reduce(c["x"], hor, "compensated", out=c["r"], ws=ws)
        else:
            if fused:
                hdc.map_reduce(c["x"], iaff, iid, "exact_int", out=c["y"], result=c["r"], ws=ws)
            else:
                hdc.map(c["x"], iaff, out=c["y"])
                hdc.transform_reduce(c["x"], iid, "exact_int", out=c["r"], ws=ws)

    def issue_f32(c, ws):
        if c["kind"] == "fp16":
            hdc.map(c["xf"], faff, out=c["yf"])
            hdc.transform_reduce(c["xf"], hor, "plain", out=c["rf"], ws=ws)
        else:
            hdc.map(c["x"], iaff, out=c["y"])
            hdc.transform_reduce(c["x"], iid, "exact_int", out=c["r"], ws=ws)

    def body(fused, branches):
        main = torch.cuda.current_stream()
        if branches == 1:
            for i in order:
                issue(calls[i], wss[0], fused)
            return
        for s in streams[:branches]:
            s.wait_stream(main)
        for k, i in enumerate(order):
            b = k % branches
            with torch.cuda.stream(streams[b]):
                issue(calls[i], wss[b], fused)
        for s in streams[:branches]:
            main.wait_stream(s)

    res = {"calls": len(calls), "elements": sum(sizes), "bytes_separate": bytes_sep, "bytes_fused": bytes_fused}
    graphs = {}
    for fused in (False, True):
        for branches in (1, nbranch):
            body(fused, branches)  # eager warm-up outside capture
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            cap = torch.cuda.Stream(device=dev)
            with torch.cuda.graph(g, stream=cap):
                body(fused, branches)
            torch.cuda.synchronize()
            graphs[(fused, branches)] = g
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.replays):
                g.replay()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.replays
            nb = bytes_fused if fused else bytes_sep
            key = ("fused" if fused else "separate") + f"_graph_{branches}branch"
            res[key] = {"ms_per_replay": round(ms, 4), "GBps": round(gbps(nb, ms), 1)}
    # grouped batch: the 32 fp16 calls in one grouped launch, the 32 int32 calls in another
    h_calls = [c for c in calls if c["kind"] == "fp16"]
    i_calls = [c for c in calls if c["kind"] == "i32"]
    wsb = [torch.zeros(hdc.workspace_size(hdc.OP_BATCH, dtc, accc, sum(c["n"] for c in cl), len(cl)),
                       dtype=torch.uint8, device=dev)
           for dtc, accc, cl in ((hdc.F16, hdc.ACC_COMPENSATED, h_calls), (hdc.I32, hdc.ACC_EXACT_INT, i_calls))]

    def grouped():
        hdc.batch_map_reduce([c["x"] for c in h_calls], faff, hor, "compensated", ys=[c["y"] for c in h_calls],
                             outs=[c["r"] for c in h_calls], ws=wsb[0])
        hdc.batch_map_reduce([c["x"] for c in i_calls], iaff, iid, "exact_int", ys=[c["y"] for c in i_calls],
                             outs=[c["r"] for c in i_calls], ws=wsb[1])
    grouped()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(5, args.replays // 4)
    for _ in range(reps):
        grouped()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    res["grouped_eager"] = {"ms_per_replay": round(ms, 4), "GBps": round(gbps(bytes_fused, ms), 1)}
    gg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gg, stream=torch.cuda.Stream(device=dev)):
        grouped()
    torch.cuda.synchronize()
    gg.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.replays):
        gg.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.replays
    res["grouped_graph"] = {"ms_per_replay": round(ms, 4), "GBps": round(gbps(bytes_fused, ms), 1)}

    # eager plain-FP32 comparator (f32 storage for the fp16 calls)
    def eager_f32():
        for i in order:
            issue_f32(calls[i], wss[0])
    eager_f32()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(5, args.replays // 20)
    for _ in range(reps):
        eager_f32()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    res["eager_plain_f32"] = {"ms": round(ms, 4), "GBps": round(gbps(bytes_f32, ms), 1)}
    best = min((v["ms_per_replay"], k) for k, v in res.items() if isinstance(v, dict) and "ms_per_replay" in v)
    res["best"] = best[1]
    res["speedup_vs_eager_plain_f32"] = round(ms / best[0], 2)
    # replay == eager, bit for bit (for the separate form)
    body(False, 1)
    torch.cuda.synchronize()
    eager = [(c["y"].clone(), c["r"].clone()) for c in calls]
    graphs[(False, nbranch)].replay()
    torch.cuda.synchronize()
    same = all(torch.equal(c["y"].view(torch.int16) if c["y"].element_size() == 2 else c["y"], e[0].view(
        torch.int16) if e[0].element_size() == 2 else e[0]) and torch.equal(c["r"], e[1])
        for c, e in zip(calls, eager))
    res["replay_equals_eager_bits"] = bool(same)
    if not args.no_check:
        # every call of the last replay against the oracle: its sum, and its map output on up to
        # 2^16 sampled positions (all of them for smaller calls)
        import oracle
        worst, ok_int, ok_map = 0.0, True, True
        gen = torch.Generator().manual_seed(17)
        for c in calls:
            xc = c["x"].cpu()
            n = c["n"]
            idx = torch.randint(0, n, (1 << 16,), generator=gen) if n > (1 << 16) else torch.arange(n)
            if c["kind"] == "fp16":
                ref = oracle.reduce(hor, xc)
                worst = max(worst, err_fields(c["r"].item(), ref)["err_over_abs_sum"])
                ok_map &= torch.equal(c["y"].cpu()[idx].view(torch.int16), oracle.map(faff, xc[idx]).view(torch.int16))
            else:
                ok_int &= c["r"].item() == oracle.reduce(iid, xc)["isum"]
                ok_map &= torch.equal(c["y"].cpu()[idx], oracle.map(iaff, xc[idx]))
        res["check"] = {"calls_checked": len(calls), "largest_call": max(sizes),
                        "fp16_max_err_over_abs_sum": worst, "int_bit_exact": bool(ok_int),
                        "maps_bit_exact_on_sampled_outputs": bool(ok_map)}
    del calls
    torch.cuda.empty_cache()
    return res


def form_small(args, torch, hdc, synth):
    """The small correctness workload, n = 2^20 f32 U[-1,1): map 2.5x + 0.5, then the plain sum of
    the degree-8 Horner p(x), and both fused in one pass.  4-8 MiB stay in the caches, so each
    call is bound by launch latency, not HBM: GB/s is reported, the HBM gate does not apply."""
    import oracle
    dev = torch.device("cuda", 0)
    n = 1 << 20
    x = synth.uniform_pm1_f32(synth.seed_of(1), synth.STREAM["x"], n)
    aff, hor = hdc.affine(2.5, 0.5), hdc.horner(synth.horner_coefficients(8))
    xg = x.to(dev)
    y = torch.empty_like(xg)
    r = torch.empty((), dtype=torch.float32, device=dev)
    ws = hdc.workspace(dev, hdc.OP_TRANSFORM_REDUCE, hdc.F32, hdc.ACC_PLAIN, n)
    t_map = ev_time(torch, lambda: hdc.map(xg, aff, out=y), reps=200)
    t_sum = ev_time(torch, lambda: hdc.transform_reduce(xg, hor, "plain", out=r, ws=ws), reps=200)
    t_both = ev_time(torch, lambda: (hdc.map(xg, aff, out=y), hdc.transform_reduce(xg, hor, "plain", out=r, ws=ws)),
                     reps=200)
    yf = torch.empty_like(xg)
    rf = torch.empty((), dtype=torch.float32, device=dev)
    t_fused = ev_time(torch, lambda: hdc.map_reduce(xg, aff, hor, "plain", out=yf, result=rf, ws=ws), reps=200)
    torch.cuda.synchronize()
    ref = oracle.reduce(hor, x)
    ym = oracle.map(aff, x).view(torch.int32)
    return {"n": n,
            "map_us": round(t_map * 1e3, 2), "map_GBps": round(gbps(8 * n, t_map), 1),
            "sum_us": round(t_sum * 1e3, 2), "sum_GBps": round(gbps(4 * n, t_sum), 1),
            "map_then_sum_us": round(t_both * 1e3, 2), "map_then_sum_GBps": round(gbps(12 * n, t_both), 1),
            "fused_map_sum_us": round(t_fused * 1e3, 2), "fused_map_sum_GBps": round(gbps(8 * n, t_fused), 1),
            "map_bit_exact": bool(torch.equal(y.cpu().view(torch.int32), ym)),
            "fused_map_bit_exact": bool(torch.equal(yf.cpu().view(torch.int32), ym)),
            "sum_err": err_fields(r.item(), ref), "fused_sum_err": err_fields(rf.item(), ref)}


def form_scan(args, torch, hdc, synth):
    """Prefix sums (inclusive) of p(x) over n f32 values and over the lognormal segments; GB/s of the
    algorithmic bytes (x read once, y written once)."""
    dev = torch.device("cuda", 0)
    n = 1 << args.log2n
    x = synth.uniform_pm1_f32(synth.seed_of(2), synth.STREAM["x"], n, dev)
    hor = hdc.horner(synth.horner_coefficients(8))
    y = torch.empty(n, dtype=torch.float32, device=dev)
    ws = hdc.workspace(dev, hdc.OP_SCAN, hdc.F32, hdc.ACC_PLAIN, n)
    t = ev_time(torch, lambda: hdc.scan(x, hor, "plain", out=y, ws=ws, check=False))
    ok = hdc.scan_status(ws) == 0  # the last timed call's output is valid
    xi = synth.uniform_int(synth.seed_of(2), synth.STREAM["xi"], n, 20, dev)
    yi = torch.empty(n, dtype=torch.int64, device=dev)
    wsi = hdc.workspace(dev, hdc.OP_SCAN, hdc.I32, hdc.ACC_EXACT_INT, n)
    ti = ev_time(torch, lambda: hdc.scan(xi, hdc.identity(), "exact_int", out=yi, ws=wsi, check=False))
    ok = ok and hdc.scan_status(wsi) == 0
    res = {"n": n, "f32_horner_ms": round(t, 5), "f32_horner_GBps": round(gbps(8 * n, t), 1),
           "i32_to_i64_ms": round(ti, 5), "i32_to_i64_GBps": round(gbps(12 * n, ti), 1),
           "bytes_per_element": "algorithmic: f32 4 read + 4 write; i32->i64 4 read + 8 write",
           "status_ok": bool(ok)}
    del x, y, xi, yi
    torch.cuda.empty_cache()
    # segmented scan over the segmented form's 100,000 lognormal segments
    seed = synth.seed_of(4)
    L = synth.segment_lengths(seed)
    off = synth.offsets_from_lengths(L)
    m = int(off[-1])
    xs = synth.uniform_pm1_f32(seed, synth.STREAM["x"], m, dev)
    ys = torch.empty(m, dtype=torch.float32, device=dev)
    offg = off.to(dev)
    wss = hdc.workspace(dev, hdc.OP_SCAN, hdc.F32, hdc.ACC_PLAIN, m)
    ts = ev_time(torch, lambda: hdc.segmented_scan(xs, offg, hor, "plain", out=ys, ws=wss, check=False))
    res["segmented_100k_lognormal"] = {"elements": m, "segments": int(L.numel()), "f32_horner_ms": round(ts, 5),
                                       "GBps": round(gbps(8 * m + 8 * (L.numel() + 1), ts), 1),
                                       "status_ok": hdc.scan_status(wss) == 0}
    del xs, ys
    torch.cuda.empty_cache()
    return res


def form_host(args, torch, hdc, synth):
    """The same callables on the host side (hdc_host_* on CPU tensors), on every core of the process:
    the step's map and Horner sum over a 2^26-element sample, against the GPU's per-op rate."""
    import oracle
    m = 1 << 26
    x = synth.uniform_pm1_f32(synth.seed_of(2), synth.STREAM["x"], m)
    hor = hdc.horner(synth.horner_coefficients(8))
    aff = hdc.affine(2.5, 0.5)
    threads = host_cores()
    y = torch.empty_like(x)
    hdc.host_map(x, aff, out=y, threads=threads)  # warm (pages touched)
    t0 = time.perf_counter()
    hdc.host_map(x, aff, out=y, threads=threads)
    t_map = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = hdc.host_transform_reduce(x, hor, "plain", threads=threads)
    t_sum = time.perf_counter() - t0
    ref = oracle.reduce(hor, x)
    res = {"n": m, "threads": threads,
           "map_f32_affine_GBps": round(8 * m / t_map / 1e9, 2),
           "sum_f32_horner_GBps": round(4 * m / t_sum / 1e9, 2),
           "sum_err_over_abs_sum": abs(float(r) - ref["exact"]) / ref["abs_sum"],
           "map_bit_exact": bool(torch.equal(y.view(torch.int32), oracle.map(aff, x).view(torch.int32)))}
    return res


def measured_traffic(op_name):
    """HBM bytes per launch of `op_name` from the committed counter summary, or None when the kernel
    sources changed since the counters were taken (or the op was not measured)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_headline.json")
    try:
        t = json.load(open(path))
        h = hashlib.sha256()
        for f in t["source_files"]:
            h.update(os.path.basename(f).encode())
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != t["source_sha256"]:
            return None
        return t["kernels"][op_name]["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; a multi-GPU run is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2309_03912_amd as hdc
    import synth

    torch.cuda.set_device(0)
    h = headline(args, torch, hdc, synth)
    value = gbps(h["step_bytes"], h["ms_per_step"])
    per_op = h["per_op"]
    dominant = max(per_op, key=lambda k: per_op[k]["ms"])
    d = per_op[dominant]
    out = {
        "metric": "HBM GB/s & % peak: plain FP32 vs BF16-compensated/batched at <=1e-6 rel err",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded counter-based generators)",
        "config": {"workload": "plain-fp32 bandwidth scale, n=2^%d per array: map 2.5x+0.5, sum Horner-8 p(x), "
                               "dot of N(0,1) arrays, int32 map 3x-7, int64 sums of x and y" % args.log2n,
                   "n": h["n"], "step_bytes": h["step_bytes"]},
        "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(d["GBps"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dominant),
                     "kernel": dominant,
                     "bytes_per_launch": d["bytes"], "launch_ms": d["ms"]},
        "per_op": per_op,
    }
    if "accuracy" in h:
        out["accuracy"] = h["accuracy"]
    if "cpu_baseline" in h:
        out["cpu_baseline"] = h["cpu_baseline"]
        out["cpu_baseline_multicore"] = h["cpu_baseline_multicore"]
    if not args.no_forms:
        forms = {}
        want = set(args.forms.split(","))
        if "c1" in want:
            forms["small_2^20"] = form_small(args, torch, hdc, synth)
        if "c3" in want:
            forms["precision_bf16_fp16_compensated"] = form_precision(args, torch, hdc, synth)
        if "c4" in want:
            forms["segmented_100k_lognormal"] = form_segmented(args, torch, hdc, synth)
        if "c5" in want:
            forms["graph_64_calls"] = form_graph(args, torch, hdc, synth)
        if "scan" in want:
            forms["scan"] = form_scan(args, torch, hdc, synth)
        if "host" in want:
            forms["host_side"] = form_host(args, torch, hdc, synth)
        out["forms"] = forms
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
