/*
 * The oracle run on several host threads: TEST INFRASTRUCTURE ONLY (the
 * multicore CPU baseline of the benchmark).
 *
 * It compiles the single-thread oracle (oracle.c) into itself and splits an
 * array into `nthreads` contiguous ranges.  Each thread folds its range with
 * the oracle's own per-element code into its own exact accumulator; the
 * accumulators are then added digit by digit in range order and rounded
 * once.  The exact result and the integer sum are therefore bit-identical to
 * the single-thread oracle's; seq64 becomes the in-order sum of the
 * per-range fp64 sums (not the single left-to-right sum).  Maps split the
 * same way and are element-wise, so they are identical too.
 */
#define _GNU_SOURCE
#include "oracle.c"

#include <pthread.h>

typedef struct {
  const or_fn *f;
  int dtype;
  const void *x;
  const void *z;
  void *y;
  int64_t lo, hi;
  sacc s;
  double seq, abs_sum;
  uint64_t isum;
  int rc;
} or_part;

static void *fold_part(void *arg) {
  or_part *p = (or_part *)arg;
  sa_init(&p->s);
  p->seq = p->abs_sum = 0.0;
  p->isum = 0;
  fold_range(p->f, p->dtype, p->x, p->z, p->lo, p->hi, &p->s, &p->seq, &p->abs_sum, &p->isum);
  return NULL;
}

static void *map_part(void *arg) {
  or_part *p = (or_part *)arg;
  const size_t es = p->dtype == OR_F16 || p->dtype == OR_BF16 ? 2 : 4;
  p->rc = or_map(p->f, p->dtype, (const char *)p->x + p->lo * es, (char *)p->y + p->lo * es, p->hi - p->lo);
  return NULL;
}

/* Run `body` over nthreads contiguous ranges of [0, n); parts[t] covers range t. */
static int run_parts(or_part *parts, int nthreads, int64_t n, void *(*body)(void *)) {
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  if (!th) return -1;
  int started = 0, rc = 0;
  for (int t = 0; t < nthreads; ++t) {
    parts[t].lo = n * t / nthreads;
    parts[t].hi = n * (t + 1) / nthreads;
    parts[t].rc = 0;
  }
  for (; started < nthreads; ++started)
    if (pthread_create(&th[started], NULL, body, &parts[started]) != 0) break;
  for (int t = started; t < nthreads; ++t) body(&parts[t]);  /* threads that did not start run here */
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  for (int t = 0; t < nthreads; ++t)
    if (parts[t].rc) rc = -1;
  free(th);
  return rc;
}

int or_reduce_mt(const or_fn *f, int dtype, const void *x, const void *z, int64_t n, int nthreads,
                 or_result *r) {
  if (!valid(f, dtype) || n < 0 || nthreads < 1) return -1;
  if (f->kind == OR_PRODUCT && !z && n > 0) return -1;
  or_part *parts = (or_part *)calloc((size_t)nthreads, sizeof(or_part));
  if (!parts) return -1;
  for (int t = 0; t < nthreads; ++t) {
    parts[t].f = f;
    parts[t].dtype = dtype;
    parts[t].x = x;
    parts[t].z = z;
  }
  int rc = run_parts(parts, nthreads, n, fold_part);
  sacc s;
  sa_init(&s);
  double seq = 0.0, abs_sum = 0.0;
  uint64_t isum = 0;
  for (int t = 0; t < nthreads; ++t) {  /* joined in range order */
    sa_carry(&parts[t].s);             /* digits in [0, 2^32) except the top one */
    for (int i = 0; i < SA_DIGITS; ++i) s.d[i] += parts[t].s.d[i];
    s.nan |= parts[t].s.nan;
    s.pinf |= parts[t].s.pinf;
    s.ninf |= parts[t].s.ninf;
    sa_carry(&s);
    seq += parts[t].seq;
    abs_sum += parts[t].abs_sum;
    isum += parts[t].isum;
  }
  if (dtype == OR_I32) {
    r->isum = (int64_t)isum;
    r->exact = r->seq64 = (double)(int64_t)isum;
  } else {
    r->exact = sa_round(&s);
    r->seq64 = seq;
    r->isum = 0;
  }
  r->abs_sum = abs_sum;
  free(parts);
  return rc;
}

int or_map_mt(const or_fn *f, int dtype, const void *x, void *y, int64_t n, int nthreads) {
  if (!valid(f, dtype) || f->kind == OR_PRODUCT || n < 0 || nthreads < 1) return -1;
  or_part *parts = (or_part *)calloc((size_t)nthreads, sizeof(or_part));
  if (!parts) return -1;
  for (int t = 0; t < nthreads; ++t) {
    parts[t].f = f;
    parts[t].dtype = dtype;
    parts[t].x = x;
    parts[t].y = y;
  }
  int rc = run_parts(parts, nthreads, n, map_part);
  free(parts);
  return rc;
}
