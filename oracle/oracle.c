/*
 * Oracle of the generic map / reduce path: TEST INFRASTRUCTURE ONLY.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  See oracle.h for the contract and the readings it follows.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (contraction is off so that every a*b+c below is either an explicit fma or
 * two roundings, exactly as written).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* 16-bit formats (IEEE 754 binary16, and bfloat16 = the top half of binary32) */
/* ------------------------------------------------------------------------ */

double or_decode_f16(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 0x1F, f = h & 0x3FF;
  double mag;
  if (e == 0)
    mag = ldexp((double)f, -24);             /* subnormal: f * 2^-24 */
  else if (e == 0x1F)
    mag = f ? NAN : INFINITY;
  else
    mag = ldexp((double)(1024 + f), e - 25); /* (1 + f/2^10) * 2^(e-15) */
  return s ? -mag : mag;
}

double or_decode_bf16(uint16_t h) {
  int s = h >> 15, e = (h >> 7) & 0xFF, f = h & 0x7F;
  double mag;
  if (e == 0)
    mag = ldexp((double)f, -133);            /* f * 2^-133 */
  else if (e == 0xFF)
    mag = f ? NAN : INFINITY;
  else
    mag = ldexp((double)(128 + f), e - 134); /* (1 + f/2^7) * 2^(e-127) */
  return s ? -mag : mag;
}

/* Round a non-negative double holding few significant bits to the nearest
 * integer, ties to the even neighbour (all steps exact). */
static double round_half_even(double k) {
  double r = floor(k), d = k - r;
  if (d > 0.5 || (d == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
  return r;
}

/* Nearest-even rounding to a binary format with `p` fraction bits, exponent
 * range [emin, emax] (emin = smallest normal exponent).  Returns the
 * magnitude bits (exponent field << p | fraction), or the infinity pattern. */
static uint32_t encode_mag(double d, int p, int emin, int emax, int bias) {
  uint32_t inf = (uint32_t)(emax + bias + 1) << p;
  if (d < ldexp(1.0, emin)) {
    /* subnormal range: quantum 2^(emin - p); r = 2^p is the smallest normal,
     * whose encoding is the same integer. */
    return (uint32_t)round_half_even(ldexp(d, p - emin));
  }
  int e;
  frexp(d, &e);            /* d in [2^(e-1), 2^e) */
  int E = e - 1;
  double r = round_half_even(ldexp(d, p - E)); /* in [2^p, 2^(p+1)] */
  if (r == ldexp(1.0, p + 1)) { r = ldexp(1.0, p); E += 1; }
  if (E > emax) return inf;
  return ((uint32_t)(E + bias) << p) | (uint32_t)(r - ldexp(1.0, p));
}

uint16_t or_encode_f16(float v) {
  uint16_t sign = signbit(v) ? 0x8000 : 0;
  if (isnan(v)) return sign | 0x7E00;
  if (isinf(v)) return sign | 0x7C00;
  return sign | (uint16_t)encode_mag(fabs((double)v), 10, -14, 15, 15);
}

uint16_t or_encode_bf16(float v) {
  uint16_t sign = signbit(v) ? 0x8000 : 0;
  if (isnan(v)) return sign | 0x7FC0;
  if (isinf(v)) return sign | 0x7F80;
  return sign | (uint16_t)encode_mag(fabs((double)v), 7, -126, 127, 127);
}

/* ------------------------------------------------------------------------ */
/* Element semantics                                                         */
/* ------------------------------------------------------------------------ */

float or_term_f32(const or_fn *f, float x) {
  switch (f->kind) {
  case OR_IDENTITY: return x;
  case OR_AFFINE:   return fmaf(f->a, x, f->b);
  case OR_HORNER: {
    float acc = f->coef[f->degree];
    for (int k = f->degree - 1; k >= 0; --k) acc = fmaf(acc, x, f->coef[k]);
    return acc;
  }
  default: return NAN;
  }
}

double or_term_f64(const or_fn *f, double x) {
  switch (f->kind) {
  case OR_IDENTITY: return x;
  case OR_AFFINE:   return fma((double)f->a, x, (double)f->b);
  case OR_HORNER: {
    double acc = f->coef[f->degree];
    for (int k = f->degree - 1; k >= 0; --k) acc = fma(acc, x, (double)f->coef[k]);
    return acc;
  }
  default: return NAN;
  }
}

static double widen(int dtype, const void *p, int64_t i) {
  switch (dtype) {
  case OR_F32:  return (double)((const float *)p)[i];
  case OR_F16:  return or_decode_f16(((const uint16_t *)p)[i]);
  case OR_BF16: return or_decode_bf16(((const uint16_t *)p)[i]);
  case OR_I32:  return (double)((const int32_t *)p)[i];
  default:      return NAN;
  }
}

static int valid(const or_fn *f, int dtype) {
  if (dtype < OR_F32 || dtype > OR_I32) return 0;
  if (f->kind == OR_HORNER && (f->degree < 0 || f->degree > OR_MAX_DEGREE)) return 0;
  if (dtype == OR_I32) return f->kind == OR_IDENTITY || f->kind == OR_AFFINE;
  return f->kind >= OR_IDENTITY && f->kind <= OR_PRODUCT;
}

int or_map(const or_fn *f, int dtype, const void *x, void *y, int64_t n) {
  if (!valid(f, dtype) || f->kind == OR_PRODUCT || n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) {
    switch (dtype) {
    case OR_F32:
      ((float *)y)[i] = or_term_f32(f, ((const float *)x)[i]);
      break;
    case OR_F16:
    case OR_BF16: {
      uint16_t h = ((const uint16_t *)x)[i];
      if (f->kind == OR_IDENTITY) { ((uint16_t *)y)[i] = h; break; }
      float t = or_term_f32(f, (float)widen(dtype, x, i)); /* widening is exact */
      ((uint16_t *)y)[i] = dtype == OR_F16 ? or_encode_f16(t) : or_encode_bf16(t);
      break;
    }
    case OR_I32: {
      int32_t v = ((const int32_t *)x)[i];
      if (f->kind == OR_IDENTITY) { ((int32_t *)y)[i] = v; break; }
      uint64_t w = (uint64_t)f->ia * (uint64_t)(int64_t)v + (uint64_t)f->ib;
      ((int32_t *)y)[i] = (int32_t)(uint32_t)w; /* two's-complement wrap */
      break;
    }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact summation: a fixed-point accumulator covering the whole fp64 range  */
/* ------------------------------------------------------------------------ */
/* Digit i holds bits [32 i, 32 i + 32) of the fixed-point value whose bit 0
 * weighs 2^-1074 (the smallest subnormal).  Digits are signed 64-bit so that
 * each accepts < 2^31 additions of a 32-bit chunk before a carry pass.  The
 * largest finite double reaches bit 1023 + 1074 = 2097, i.e. digit 65; the
 * digits above hold carries. */
#define SA_DIGITS 72
#define SA_RENORM (1 << 28)

typedef struct {
  int64_t d[SA_DIGITS];
  int64_t since_norm;
  int nan, pinf, ninf;
} sacc;

static void sa_init(sacc *s) { memset(s, 0, sizeof *s); }

static void sa_carry(sacc *s) {
  for (int i = 0; i < SA_DIGITS - 1; ++i) {
    int64_t c = s->d[i] >> 32;   /* floor division by 2^32 */
    s->d[i] -= c * ((int64_t)1 << 32);
    s->d[i + 1] += c;
  }
  s->since_norm = 0;
}

static void sa_add(sacc *s, double v) {
  if (isnan(v)) { s->nan = 1; return; }
  if (isinf(v)) { if (v > 0) s->pinf = 1; else s->ninf = 1; return; }
  if (v == 0.0) return;
  int e;
  double m = frexp(fabs(v), &e);        /* |v| = m 2^e, m in [0.5, 1) */
  uint64_t M = (uint64_t)ldexp(m, 53);  /* |v| = M 2^(e-53), exact */
  int p = e - 53 + 1074;                /* weight position of M's bit 0 */
  if (p < 0) { M >>= -p; p = 0; }       /* subnormal: the dropped bits are 0 */
  unsigned __int128 w = (unsigned __int128)M << (p % 32);
  int k = p / 32;
  int64_t sg = v < 0 ? -1 : 1;
  s->d[k]     += sg * (int64_t)(uint32_t)w;
  s->d[k + 1] += sg * (int64_t)(uint32_t)(w >> 32);
  s->d[k + 2] += sg * (int64_t)(uint32_t)(w >> 64);
  if (++s->since_norm >= SA_RENORM) sa_carry(s);
}

/* Bits [pos, pos + cnt) of the non-negative digit array (cnt <= 53,
 * pos >= 0), read as an integer. */
static uint64_t sa_bits(const int64_t *d, int pos, int cnt) {
  int w = pos / 32, sh = pos % 32;
  unsigned __int128 v = 0;
  for (int k = 2; k >= 0; --k) {
    v <<= 32;
    if (w + k < SA_DIGITS) v |= (uint32_t)d[w + k];
  }
  return (uint64_t)(v >> sh) & ((cnt == 64 ? 0 : ((uint64_t)1 << cnt)) - 1);
}

/* Whether any bit below position pos (exclusive) is set. */
static int sa_any_below(const int64_t *d, int pos) {
  if (pos <= 0) return 0;
  int w = pos / 32, sh = pos % 32;
  for (int k = 0; k < w; ++k)
    if (d[k]) return 1;
  return sh && ((uint32_t)d[w] & (((uint32_t)1 << sh) - 1)) != 0;
}

static double sa_round(sacc *s) {
  if (s->nan || (s->pinf && s->ninf)) return NAN;
  if (s->pinf) return INFINITY;
  if (s->ninf) return -INFINITY;
  sa_carry(s);
  int neg = s->d[SA_DIGITS - 1] < 0;
  int64_t d[SA_DIGITS];
  memcpy(d, s->d, sizeof d);
  if (neg) {
    for (int i = 0; i < SA_DIGITS; ++i) d[i] = -d[i];
    for (int i = 0; i < SA_DIGITS - 1; ++i) {
      int64_t c = d[i] >> 32;
      d[i] -= c * ((int64_t)1 << 32);
      d[i + 1] += c;
    }
  }
  /* Now every digit is in [0, 2^32): find the most significant set bit. */
  int h = SA_DIGITS - 1;
  while (h >= 0 && d[h] == 0) --h;
  if (h < 0) return 0.0;
  int top = 32 * h + (31 - __builtin_clz((uint32_t)d[h]));
  double r;
  if (top < 53) {
    r = ldexp((double)sa_bits(d, 0, top + 1), -1074);  /* exact */
  } else {
    int lo = top - 52;                                  /* keep bits [lo, top] */
    uint64_t M = sa_bits(d, lo, 53);
    int guard = (int)sa_bits(d, lo - 1, 1);
    int sticky = sa_any_below(d, lo - 1);
    if (guard && (sticky || (M & 1))) M += 1;           /* nearest, ties to even */
    r = ldexp((double)M, lo - 1074);                    /* M <= 2^53: exact or inf */
  }
  return neg ? -r : r;
}

double or_exact_sum(const double *v, int64_t n) {
  sacc s;
  sa_init(&s);
  for (int64_t i = 0; i < n; ++i) sa_add(&s, v[i]);
  return sa_round(&s);
}

/* ------------------------------------------------------------------------ */
/* Reductions                                                                */
/* ------------------------------------------------------------------------ */

/* The fold of the terms of [lo, hi) into caller-held accumulators (an exact
 * accumulator, the fp64 sum of f in fp64, the fp64 sum of |terms|, the
 * wrapping integer sum), so that the folds of consecutive ranges can be
 * joined without rounding. */
static void fold_range(const or_fn *f, int dtype, const void *x, const void *z,
                       int64_t lo, int64_t hi, sacc *s, double *seq,
                       double *abs_sum, uint64_t *isum) {
  if (dtype == OR_I32) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t v = ((const int32_t *)x)[i];
      uint64_t t = f->kind == OR_AFFINE
                       ? (uint64_t)f->ia * (uint64_t)v + (uint64_t)f->ib
                       : (uint64_t)v;
      *isum += t;                                    /* wraps mod 2^64 */
      *abs_sum += fabs((double)(int64_t)t);
    }
    return;
  }
  for (int64_t i = lo; i < hi; ++i) {
    double xi = widen(dtype, x, i), t, t64;
    if (f->kind == OR_PRODUCT) {
      t = xi * widen(dtype, z, i);  /* <= 48 significant bits: exact in fp64 */
      t64 = t;
    } else {
      t = (double)or_term_f32(f, (float)xi);
      t64 = or_term_f64(f, xi);
    }
    sa_add(s, t);
    *seq += t64;
    *abs_sum += fabs(t);
  }
}

static void reduce_range(const or_fn *f, int dtype, const void *x,
                         const void *z, int64_t lo, int64_t hi, or_result *r) {
  sacc s;
  sa_init(&s);
  double seq = 0.0, abs_sum = 0.0;
  uint64_t isum = 0;
  fold_range(f, dtype, x, z, lo, hi, &s, &seq, &abs_sum, &isum);
  if (dtype == OR_I32) {
    r->isum = (int64_t)isum;
    r->exact = r->seq64 = (double)(int64_t)isum;
  } else {
    r->exact = sa_round(&s);
    r->seq64 = seq;
    r->isum = 0;
  }
  r->abs_sum = abs_sum;
}

int or_reduce(const or_fn *f, int dtype, const void *x, const void *z,
              int64_t n, or_result *r) {
  if (!valid(f, dtype) || n < 0) return -1;
  if (f->kind == OR_PRODUCT && !z && n > 0) return -1;
  reduce_range(f, dtype, x, z, 0, n, r);
  return 0;
}

int or_segmented(const or_fn *f, int dtype, const void *x, const int64_t *off,
                 int64_t num_segments, or_result *r) {
  if (!valid(f, dtype) || f->kind == OR_PRODUCT || num_segments < 0) return -1;
  for (int64_t j = 0; j < num_segments; ++j) {
    if (off[j + 1] < off[j]) return -1;
    reduce_range(f, dtype, x, NULL, off[j], off[j + 1], &r[j]);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Prefix sums                                                               */
/* ------------------------------------------------------------------------ */

int or_scan(const or_fn *f, int dtype, const void *x, int64_t n, int exclusive,
            double *out_exact, double *out_abs, int64_t *out_int) {
  if (!valid(f, dtype) || f->kind == OR_PRODUCT || n < 0) return -1;
  if (dtype == OR_I32) {
    uint64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) {
      int64_t v = ((const int32_t *)x)[i];
      uint64_t t = f->kind == OR_AFFINE
                       ? (uint64_t)f->ia * (uint64_t)v + (uint64_t)f->ib
                       : (uint64_t)v;
      if (exclusive && out_int) out_int[i] = (int64_t)acc;
      acc += t;
      if (!exclusive && out_int) out_int[i] = (int64_t)acc;
    }
    return 0;
  }
  sacc s;
  sa_init(&s);
  double abs_sum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = (double)or_term_f32(f, (float)widen(dtype, x, i));
    if (exclusive) {
      if (out_exact) out_exact[i] = sa_round(&s);
      if (out_abs) out_abs[i] = abs_sum;
    }
    sa_add(&s, t);
    abs_sum += fabs(t);
    if (!exclusive) {
      if (out_exact) out_exact[i] = sa_round(&s);
      if (out_abs) out_abs[i] = abs_sum;
    }
  }
  return 0;
}
