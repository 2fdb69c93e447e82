/*
 * Oracle of the generic map / reduce path: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar C implementation of what the GPU library computes,
 * written from the definitions (element-wise application of one callable, and
 * the fold of its results), used only by the tests, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It shares no source, header, table
 * or helper with the GPU library and never calls it.
 *
 * The paper defines the *shape* of the computation: a generic callable taken
 * by value into a kernel and invoked once per thread (section 2.4, "ifdef
 * blocks with __CUDA_ARCH__", listing lst_solution_ifdef_cudaarch), and one
 * generic callable used from host and device code alike (section 2.6,
 * "Variant with lambdas: C++17").  It fixes no arithmetic.  The per-element
 * semantics below are this project's stated readings: single-rounding fma in
 * fp32 with round-to-nearest-even, 16-bit storage widened exactly and rounded
 * back to nearest-even, wrapping two's-complement integers.
 */
#ifndef HDC_ORACLE_H
#define HDC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types the oracle understands. */
enum { OR_F32 = 0, OR_F16 = 1, OR_BF16 = 2, OR_I32 = 3 };

/* Callables.  IDENTITY: t = x.  AFFINE: t = a*x + b (one rounding in fp32;
 * wrapping for integers).  HORNER: p(x) = sum_k coef[k] x^k evaluated as
 * acc = coef[d]; acc = fma(acc, x, coef[k]) for k = d-1 .. 0.  PRODUCT: the
 * two-operand term x*z of a dot product. */
enum { OR_IDENTITY = 0, OR_AFFINE = 1, OR_HORNER = 2, OR_PRODUCT = 3 };

#define OR_MAX_DEGREE 16

typedef struct {
  int kind;
  int degree;
  float a, b;
  float coef[OR_MAX_DEGREE + 1];
  int64_t ia, ib;
} or_fn;

/* Per-reduction reference values.
 *  exact   : the exact real sum of the per-element terms, rounded once to fp64
 *  seq64   : the plain left-to-right fp64 sum of the callable evaluated in fp64
 *  abs_sum : sum of |term| in fp64 (the tolerance denominator)
 *  isum    : integer sum, wrapping mod 2^64 (integer inputs only)
 */
typedef struct {
  double exact;
  double seq64;
  double abs_sum;
  int64_t isum;
} or_result;

/* 16-bit storage formats, decoded and encoded from their definitions. */
double   or_decode_f16(uint16_t h);
double   or_decode_bf16(uint16_t h);
uint16_t or_encode_f16(float v);   /* round to nearest, ties to even */
uint16_t or_encode_bf16(float v);  /* round to nearest, ties to even */

/* Scalar element semantics (exported for pinning). */
float  or_term_f32(const or_fn *f, float x);   /* fp32 value of f(x) */
double or_term_f64(const or_fn *f, double x);  /* f(x) evaluated in fp64 */

/* y[i] = f(x[i]) in the storage type.  Returns 0, or -1 on an unsupported
 * combination. */
int or_map(const or_fn *f, int dtype, const void *x, void *y, int64_t n);

/* Reference values of sum_i f(x[i]) (or sum_i x[i]*z[i] for PRODUCT). */
int or_reduce(const or_fn *f, int dtype, const void *x, const void *z,
              int64_t n, or_result *r);

/* Per segment j: the reduction over [off[j], off[j+1]). */
int or_segmented(const or_fn *f, int dtype, const void *x, const int64_t *off,
                 int64_t num_segments, or_result *r);

/* Prefix sums of the terms f(x[i]) (inclusive: terms 0..i; exclusive:
 * terms 0..i-1).  For floating-point storage out_exact[i] is the exact prefix
 * sum rounded once to fp64 and out_abs[i] the fp64 sum of |terms| over the
 * same range; for int32 storage out_int[i] is the prefix sum mod 2^64.
 * Unused output pointers may be NULL.  Returns 0, or -1. */
int or_scan(const or_fn *f, int dtype, const void *x, int64_t n, int exclusive,
            double *out_exact, double *out_abs, int64_t *out_int);

/* Exact sum of fp64 values rounded once to fp64 (IEEE results for
 * non-finite inputs). */
double or_exact_sum(const double *v, int64_t n);

#ifdef __cplusplus
}
#endif
#endif
