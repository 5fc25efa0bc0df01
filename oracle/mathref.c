/*
 * Reference values for the device's elementary functions.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle library; never linked into
 * the HIP library).  The running error bound of the oracle gives each device
 * elementary function an allowance f: its result may differ from the exact
 * value by f * u_c * |value|.  These routines measure, for device results
 * computed elsewhere, the largest such error against the C library:
 *   - FP32 results over a contiguous range of FP32 bit patterns (the inputs
 *     are regenerated here from the range, so nothing is read back from the
 *     device but its results), referenced to the FP64 libm value of the
 *     exactly widened input (its own error, about 2^-29 FP32 ulp, does not
 *     matter at the precision reported), taken as infinite where it lies
 *     beyond FP32's rounding threshold to infinity;
 *   - FP64 results for given FP64 inputs, referenced to the x87 extended
 *     precision (64-bit significand) libm value.
 *
 * Function codes: 0 exp, 1 log, 2 tanh, 3 sqrt, 4 pow(x, k).
 *
 * The error of a result r against the reference y is reported in two units:
 *   rel_u = |r - y| / (u_c |y|)   (the unit of the allowance f)
 *   ulp   = |r - y| / ulp(y)      (ulp of the result's binade)
 * A reference of 0 needs r == 0; an infinite or NaN reference needs r equal
 * to it.  Results whose reference is subnormal are measured in ulps only
 * (relative error is not meaningful there) and counted separately; they are
 * accepted within one subnormal ulp.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { MR_EXP = 0, MR_LOG = 1, MR_TANH = 2, MR_SQRT = 3, MR_POW = 4 };

typedef struct {
  double max_rel_u;       /* largest rel_u over normal references */
  double max_ulp;         /* largest ulp error over all finite references */
  int64_t argmax;         /* index of max_rel_u */
  int64_t first_bad;      /* first index beyond the allowance, or -1 */
  int64_t n_bad;          /* results beyond the allowance */
  int64_t n_subnormal;    /* references in the subnormal range */
  double max_sub_ulp;     /* largest ulp error among them */
} mr_stats;

static double ref64(int fn, double x, double k) {
  switch (fn) {
    case MR_EXP: return exp(x);
    case MR_LOG: return log(x);
    case MR_TANH: return tanh(x);
    case MR_SQRT: return sqrt(x);
    case MR_POW: return pow(x, k);
  }
  return NAN;
}

static long double ref80(int fn, long double x, long double k) {
  switch (fn) {
    case MR_EXP: return expl(x);
    case MR_LOG: return logl(x);
    case MR_TANH: return tanhl(x);
    case MR_SQRT: return sqrtl(x);
    case MR_POW: return powl(x, k);
  }
  return NAN;
}

/* One comparison; returns the rel_u error (INFINITY for a mismatch that no
 * allowance covers) and sets *ulp / *sub. */
static double judge(long double r, long double y, int mant_bits, int min_exp, double u_c,
                    double* ulp, int* sub) {
  *sub = 0;
  *ulp = 0.0;
  if (isnan(y)) return isnan(r) ? 0.0 : INFINITY;
  if (isinf(y)) return r == y ? 0.0 : INFINITY;
  if (y == 0) return r == 0 ? 0.0 : INFINITY;
  if (isnan(r) || isinf(r)) return INFINITY;
  const long double d = fabsl(r - y);
  int e;
  frexpl(y, &e); /* |y| in [2^(e-1), 2^e) */
  if (e - 1 < min_exp) { /* subnormal range: the spacing is fixed */
    *sub = 1;
    *ulp = (double)(d / ldexpl(1.0L, min_exp - mant_bits + 1));
    return 0.0;
  }
  *ulp = (double)(d / ldexpl(1.0L, e - mant_bits));
  return (double)(d / ((long double)u_c * fabsl(y)));
}

static void merge(mr_stats* a, const mr_stats* b) {
  if (b->max_rel_u > a->max_rel_u) { a->max_rel_u = b->max_rel_u; a->argmax = b->argmax; }
  if (b->max_ulp > a->max_ulp) a->max_ulp = b->max_ulp;
  if (b->first_bad >= 0 && (a->first_bad < 0 || b->first_bad < a->first_bad))
    a->first_bad = b->first_bad;
  a->n_bad += b->n_bad;
  a->n_subnormal += b->n_subnormal;
  if (b->max_sub_ulp > a->max_sub_ulp) a->max_sub_ulp = b->max_sub_ulp;
}

static void init(mr_stats* s) {
  memset(s, 0, sizeof *s);
  s->argmax = -1;
  s->first_bad = -1;
}

static void note(mr_stats* s, int64_t i, double rel, double ulp, int sub, double f_allow) {
  if (sub) {
    s->n_subnormal++;
    if (ulp > s->max_sub_ulp) s->max_sub_ulp = ulp;
    if (ulp > s->max_ulp) s->max_ulp = ulp;
    if (ulp > 1.0) {
      s->n_bad++;
      if (s->first_bad < 0 || i < s->first_bad) s->first_bad = i;
    }
    return;
  }
  if (rel > s->max_rel_u || s->argmax < 0) { s->max_rel_u = rel; s->argmax = i; }
  if (ulp > s->max_ulp) s->max_ulp = ulp;
  if (rel > f_allow) {
    s->n_bad++;
    if (s->first_bad < 0 || i < s->first_bad) s->first_bad = i;
  }
}

/* got[i] is the device's FP32 result for the input whose bit pattern is
 * bits0 + i (i < count; the range must not wrap).  k: the exponent of pow.
 * max_abs_x > 0 restricts the sweep to inputs with |x| <= max_abs_x (the
 * others, NaNs included, are skipped). */
int mr_sweep_f32(int fn, uint32_t bits0, int64_t count, double k, const float* got,
                 double f_allow, double max_abs_x, mr_stats* out) {
  if (fn < MR_EXP || fn > MR_POW || count < 0 || (uint64_t)bits0 + (uint64_t)count > 4294967296ull)
    return -1;
  init(out);
#pragma omp parallel
  {
    mr_stats loc;
    init(&loc);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
      const uint32_t b = bits0 + (uint32_t)i;
      float x;
      memcpy(&x, &b, 4);
      if (max_abs_x > 0 && !(fabs((double)x) <= max_abs_x)) continue;
      double y = ref64(fn, (double)x, k);
      /* a reference beyond FP32's rounding threshold to infinity is infinite
       * in FP32 (the FP64 libm value itself is finite there) */
      if (fabs(y) >= 0x1.ffffffp127) y = copysign(INFINITY, y);
      double ulp;
      int sub;
      const double rel = judge((long double)got[i], (long double)y, 24, -126, 0x1p-24, &ulp, &sub);
      note(&loc, i, rel, ulp, sub, f_allow);
    }
#pragma omp critical
    merge(out, &loc);
  }
  return 0;
}

/* got[i] is the device's FP64 result for x[i]. */
int mr_sweep_f64(int fn, const double* x, int64_t count, double k, const double* got,
                 double f_allow, mr_stats* out) {
  if (fn < MR_EXP || fn > MR_POW || count < 0) return -1;
  init(out);
#pragma omp parallel
  {
    mr_stats loc;
    init(&loc);
#pragma omp for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
      const long double y = ref80(fn, (long double)x[i], (long double)k);
      double ulp;
      int sub;
      /* a reference that rounds to infinity in FP64 is infinite */
      const long double yd = (long double)(double)y;
      const long double yr = isinf(yd) ? yd : y;
      const double rel = judge((long double)got[i], yr, 53, -1022, 0x1p-53, &ulp, &sub);
      note(&loc, i, rel, ulp, sub, f_allow);
    }
#pragma omp critical
    merge(out, &loc);
  }
  return 0;
}
