"""Seeded, counter-based synthetic inputs for every workload.

This module only *generates* inputs.  It holds none of the map/reduce
arithmetic: no functor is evaluated and no reduction of the method is
performed here.  Both the GPU path (through the tests and the bench) and the
CPU oracle read the tensors it returns, so neither side draws random numbers
of its own.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used counter-style.  Element ``i`` of stream
``s`` under seed ``seed`` is

    state0 = mix(mix(seed) ^ (s * GAMMA mod 2^64))
    u64(seed, s, i) = mix(state0 + (i + 1) * GAMMA mod 2^64)

which is exactly the (i+1)-th output of a SplitMix64 generator started at
``state0``; so every element is a pure function of (seed, stream, index) and
any slice can be produced on any device without producing the others.

All integer work is done in torch int64 (two's-complement wrap == arithmetic
mod 2^64); right shifts are made logical with a mask.  Integer-derived values
(uniforms, integers, segment lengths) are bit-identical on every device.
Transcendental steps (Box-Muller, exp) run in float64 and may differ by an ulp
between CPU and GPU libm; every consumer therefore hands the *same tensor*
(copied) to both the GPU path and the oracle.
"""
from __future__ import annotations

import math
from fractions import Fraction

import torch

GAMMA = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# Seed of workload k (k = 1..5).
SEED_BASE = 230903912

# Stream ids: one independent counter stream per quantity.
STREAM = {
    "x": 0,            # uniform / first operand
    "z": 1,            # second operand of a dot
    "sign": 2,         # random signs of the lognormal values
    "lengths": 3,      # segment-length normals
    "sizes": 4,        # per-call sizes of the batched workload
    "positions": 5,    # slot positions of the conditioning correction
    "v": 6,            # lognormal magnitudes (normal deviates)
    "target_sign": 7,  # sign of the ill-conditioned target sum
    "force": 8,        # index of the segment forced to the maximum length
    "xn": 9,           # normal first operand of the fp32 dot
    "xi": 10,          # integer operand
    "dot_scale": 11,   # signs and power-of-two splits of the ill-conditioned dot
}


def seed_of(k: int) -> int:
    """Seed of workload ``k`` (1-based)."""
    return SEED_BASE + k


def _s64(c: int) -> int:
    """Unsigned 64-bit constant -> the int64 with the same bits."""
    c &= MASK64
    return c - (1 << 64) if c >= (1 << 63) else c


def _mix_py(z: int) -> int:
    """SplitMix64 finaliser on Python ints (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MUL1) & MASK64
    z = ((z ^ (z >> 27)) * MUL2) & MASK64
    return z ^ (z >> 31)


def splitmix64_reference(state: int, count: int) -> list[int]:
    """Plain sequential SplitMix64 outputs (Python ints), for pinning."""
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        out.append(_mix_py(state))
    return out


def stream_state(seed: int, stream: int) -> int:
    """Starting state of stream ``stream`` under ``seed`` (Python int)."""
    return _mix_py(_mix_py(seed) ^ ((stream * GAMMA) & MASK64))


def _lsr(t: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (t >> k) & ((1 << (64 - k)) - 1)


def _mix_t(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _s64(MUL1)
    z = (z ^ _lsr(z, 27)) * _s64(MUL2)
    return z ^ _lsr(z, 31)


CHUNK = 1 << 24


def u64(seed: int, stream: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """Raw 64-bit words ``u64(seed, stream, i)`` for i in [start, start+count) (int64 bits)."""
    st = _s64(stream_state(seed, stream))
    out = torch.empty(count, dtype=torch.int64, device=device)
    for lo in range(0, count, CHUNK):
        hi = min(count, lo + CHUNK)
        i = torch.arange(start + lo + 1, start + hi + 1, dtype=torch.int64, device=device)
        out[lo:hi] = _mix_t(i * _s64(GAMMA) + st)
    return out


def _map_chunks(count, device, dtype, fn):
    out = torch.empty(count, dtype=dtype, device=device)
    for lo in range(0, count, CHUNK):
        hi = min(count, lo + CHUNK)
        out[lo:hi] = fn(lo, hi)
    return out


def uniform_pm1_f32(seed: int, stream: int, n: int, device="cpu") -> torch.Tensor:
    """x = (k - 2^23) * 2^-23 with k the top 24 bits: exact in fp32, x in [-1, 1)."""
    def f(lo, hi):
        k = _lsr(u64(seed, stream, lo, hi - lo, device), 40)
        return (k - (1 << 23)).to(torch.float32) * (2.0 ** -23)
    return _map_chunks(n, device, torch.float32, f)


def uniform_int(seed: int, stream: int, n: int, bits: int = 20, device="cpu") -> torch.Tensor:
    """Integers uniform on [0, 2^bits) from the top ``bits`` bits, as int32."""
    assert 1 <= bits <= 31
    def f(lo, hi):
        return _lsr(u64(seed, stream, lo, hi - lo, device), 64 - bits).to(torch.int32)
    return _map_chunks(n, device, torch.int32, f)


def uniform01_f64(seed: int, stream: int, start: int, count: int, device="cpu") -> torch.Tensor:
    """u = ((w >> 11) + 0.5) * 2^-53, in (0, 1), exact in float64."""
    w = _lsr(u64(seed, stream, start, count, device), 11)
    return (w.to(torch.float64) + 0.5) * (2.0 ** -53)


def normal_f64(seed: int, stream: int, n: int, device="cpu") -> torch.Tensor:
    """Box-Muller (cosine branch): element i uses the uniforms at counters 2i and 2i+1."""
    def f(lo, hi):
        u = uniform01_f64(seed, stream, 2 * lo, 2 * (hi - lo), device).view(-1, 2)
        return torch.sqrt(-2.0 * torch.log(u[:, 0])) * torch.cos((2.0 * math.pi) * u[:, 1])
    return _map_chunks(n, device, torch.float64, f)


def random_sign(seed: int, stream: int, n: int, device="cpu") -> torch.Tensor:
    """+1.0 / -1.0 (float64) from the top bit of each word."""
    def f(lo, hi):
        b = _lsr(u64(seed, stream, lo, hi - lo, device), 63)
        return 1.0 - 2.0 * b.to(torch.float64)
    return _map_chunks(n, device, torch.float64, f)


FP16_MAX = 65504.0


def to_storage(v: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    """Round float64 values to storage: v -> RN_f32 -> (clamp |.| <= 65504 for fp16) -> RN_T."""
    f = v.to(torch.float32)
    if dtype == torch.float32:
        return f
    if dtype == torch.float16:
        f = f.clamp(-FP16_MAX, FP16_MAX)
    return f.to(dtype)


# ---------------------------------------------------------------------------
# Exact sums of 16-bit storage values (for the conditioning construction).
# A value of either 16-bit format is m * 2^e with |m| < 2^11 an integer, so
# grouping by e and summing m in float64 is exact while n * 2^11 < 2^53.
# ---------------------------------------------------------------------------

def _sig_exp(t: torch.Tensor):
    """(signed integer significand as float64, exponent) of fp16/bf16 values."""
    bits = t.view(torch.int16).to(torch.int32) & 0xFFFF
    if t.dtype == torch.float16:
        e = (bits >> 10) & 0x1F
        f = bits & 0x3FF
        m = torch.where(e == 0, f, f | 0x400)
        ex = torch.where(e == 0, torch.full_like(e, -24), e - 25)
    elif t.dtype == torch.bfloat16:
        e = (bits >> 7) & 0xFF
        f = bits & 0x7F
        m = torch.where(e == 0, f, f | 0x80)
        ex = torch.where(e == 0, torch.full_like(e, -133), e - 134)
    else:
        raise TypeError(t.dtype)
    bad = (e == 0x1F) if t.dtype == torch.float16 else (e == 0xFF)
    if bool(bad.any()):
        raise ValueError("non-finite storage value")
    sign = 1.0 - 2.0 * ((bits >> 15) & 1).to(torch.float64)
    return sign * m.to(torch.float64), ex


def exact_sum_16(t: torch.Tensor, absolute: bool = False) -> Fraction:
    """Exact sum (or sum of magnitudes) of fp16/bf16 values as a Fraction."""
    assert t.numel() < (1 << 41)
    m, ex = _sig_exp(t.reshape(-1))
    if absolute:
        m = m.abs()
    off = int(ex.min().item()) if ex.numel() else 0
    w = torch.bincount((ex - off).to(torch.int64), weights=m)
    total = Fraction(0)
    for k, s in enumerate(w.cpu().tolist()):
        if s != 0.0:
            total += Fraction(int(s)) * Fraction(2) ** (k + off)
    return total


def _round_fraction_to(q: Fraction, dtype: torch.dtype) -> torch.Tensor:
    """RN_T of an exact rational (clamped to T's finite range); returns a 1-element tensor."""
    # float(Fraction) is correctly rounded to float64; a 16-bit rounding of that
    # double can double-round only if the double is exactly a tie, which the
    # check below resolves exactly.
    d = float(q)
    t = torch.tensor([d], dtype=torch.float64)
    cand = to_storage(t, dtype)
    # Exact correction for the double-rounding corner: compare with neighbours.
    best = cand
    best_err = abs(Fraction(float(cand.to(torch.float64).item())) - q)
    bits = cand.view(torch.int16).item()
    for delta in (-1, 1):
        nb = torch.tensor([(bits + delta + 32768) % 65536 - 32768], dtype=torch.int16).view(dtype)
        v = float(nb.to(torch.float64).item())
        if not math.isfinite(v):
            continue
        lim = FP16_MAX if dtype == torch.float16 else float(torch.finfo(dtype).max)
        if abs(v) > lim:
            continue
        err = abs(Fraction(v) - q)
        if err < best_err or (err == best_err and (nb.view(torch.int16).item() & 1) == 0):
            best, best_err = nb, err
    return best


def ill_conditioned(seed: int, n: int, dtype: torch.dtype, kappa: float = 1e8,
                    sigma: float = 4.0, device="cpu"):
    """Mixed-sign lognormal(0, sigma) values in 16-bit storage whose exact sum is a
    chosen target t with sum|v| / |t| ~= kappa.

    Steps: draw v = s * exp(sigma * g) and store it in ``dtype``; choose the target
    t = RN_T(+-A/kappa) with A the exact sum of magnitudes; pick seeded distinct
    slots, zero them, then greedily fill them with c = RN_T(t - S_cur) (clamped to
    the finite range) until the exact running sum equals t.

    Returns (tensor, info) where info holds the exact target and the achieved kappa.
    """
    g = normal_f64(seed, STREAM["v"], n, device)
    s = random_sign(seed, STREAM["sign"], n, device)
    v = to_storage(s * torch.exp(sigma * g), dtype)
    del g, s
    A = exact_sum_16(v, absolute=True)
    S = exact_sum_16(v)
    tsign = 1 if (stream_state(seed, STREAM["target_sign"]) >> 63) == 0 else -1
    t_val = _round_fraction_to(tsign * A / Fraction(kappa), dtype)
    t_exact = Fraction(float(t_val.to(torch.float64).item()))
    tmax = FP16_MAX if dtype == torch.float16 else float(torch.finfo(dtype).max)
    need = int(abs(t_exact - S) / Fraction(tmax)) + 1
    pool = int(need * 1.25) + 256
    if pool > n:
        raise ValueError("array too small for the conditioning construction")
    # Seeded distinct positions.
    pos, seen, j = [], set(), 0
    while len(pos) < pool:
        w = u64(seed, STREAM["positions"], j, 4 * pool, "cpu")
        for val in _lsr(w, 32).tolist():
            p = (val * n) >> 32
            if p not in seen:
                seen.add(p)
                pos.append(p)
                if len(pos) == pool:
                    break
        j += 4 * pool
    pos_t = torch.tensor(pos, dtype=torch.int64, device=device)
    removed = exact_sum_16(v[pos_t])
    cur = S - removed
    fill = []
    for _ in range(pool):
        r = t_exact - cur
        if r == 0:
            break
        c = _round_fraction_to(r, dtype)
        cv = Fraction(float(c.to(torch.float64).item()))
        if cv == 0:
            raise RuntimeError("conditioning construction stalled")
        fill.append(c)
        cur += cv
    if cur != t_exact:
        raise RuntimeError("conditioning construction ran out of slots")
    vals = torch.zeros(pool, dtype=dtype)
    if fill:
        vals[: len(fill)] = torch.cat(fill)
    v[pos_t] = vals.to(device)
    A_new = exact_sum_16(v, absolute=True)
    info = {
        "target": float(t_exact),
        "target_exact": t_exact,
        "abs_sum": float(A_new),
        "kappa": float(A_new / abs(t_exact)) if t_exact != 0 else math.inf,
        "slots_used": len(fill),
    }
    return v, info


def ill_conditioned_dot(seed: int, n: int, dtype: torch.dtype, kappa: float = 1e8, device="cpu"):
    """Operands x, z of a dot product whose products are exactly the ill-conditioned
    values v of ``ill_conditioned`` (so the exact dot is its target and its condition
    number is the same): z_i = s_i 2^k_i with a seeded sign s_i and k_i in [-2, 2],
    x_i = s_i v_i 2^-k_i; where that x_i is not representable, k_i = 0.

    Returns (x, z, info) with info as for ``ill_conditioned``.
    """
    v, info = ill_conditioned(seed, n, dtype, kappa, device=device)
    w = u64(seed, STREAM["dot_scale"], 0, n, device)
    k = ((_lsr(w, 32) * 5) >> 32).to(torch.float64) - 2.0     # uniform in {-2, ..., 2}
    s = 1.0 - 2.0 * (_lsr(w, 31) & 1).to(torch.float64)
    del w
    v64 = v.to(torch.float64)
    x64 = s * v64 * torch.exp2(-k)
    x = to_storage(x64, dtype)
    ok = x.to(torch.float64) == x64
    k = torch.where(ok, k, torch.zeros_like(k))
    x = torch.where(ok, x, to_storage(s * v64, dtype))
    z = (s * torch.exp2(k)).to(dtype)
    return x, z, info


# ---------------------------------------------------------------------------
# Segment lengths and batched call sizes.
# ---------------------------------------------------------------------------

def segment_lengths(seed: int, num_segments: int = 100_000, median: float = 256.0,
                    total_target: float = 2.0 ** 27, max_len: int = 1 << 20) -> torch.Tensor:
    """L_j = min(max_len, floor(exp(ln(median) + sigma * g_j))) with
    sigma = sqrt(2 ln(mean/median)) so that E[L] = total_target / num_segments;
    one seeded segment is forced to exactly ``max_len``.  int64, on the CPU."""
    mean = total_target / num_segments
    sigma = math.sqrt(2.0 * math.log(mean / median))
    g = normal_f64(seed, STREAM["lengths"], num_segments, "cpu")
    L = torch.floor(torch.exp(math.log(median) + sigma * g))
    L = torch.clamp(L, max=float(max_len)).to(torch.int64)
    j = (int(_lsr(u64(seed, STREAM["force"], 0, 1), 32).item()) * num_segments) >> 32
    L[j] = max_len
    return L


def offsets_from_lengths(L: torch.Tensor) -> torch.Tensor:
    """CSR offsets (int64, length S+1, off[0] = 0)."""
    off = torch.zeros(L.numel() + 1, dtype=torch.int64)
    off[1:] = torch.cumsum(L, 0)
    return off


def call_sizes(seed: int, calls: int = 64, lo_log2: int = 10, hi_log2: int = 26) -> list[int]:
    """n_i = floor(2^(lo + (hi-lo) u_i)); the first call is forced to 2^lo, the last to 2^hi."""
    u = uniform01_f64(seed, STREAM["sizes"], 0, calls, "cpu")
    n = torch.floor(torch.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).to(torch.int64).tolist()
    n[0] = 1 << lo_log2
    n[-1] = 1 << hi_log2
    return n


# ---------------------------------------------------------------------------
# Functor parameters of the workloads (plain data).
# ---------------------------------------------------------------------------

def horner_coefficients(degree: int = 8) -> list[float]:
    """c_k = RN_f32(1/(k+1)), k = 0..degree (computed on the host)."""
    return [float(torch.tensor(1.0 / (k + 1), dtype=torch.float64).to(torch.float32)) for k in range(degree + 1)]


AFFINE_F = (2.5, 0.5)
AFFINE_I = (3, -7)
