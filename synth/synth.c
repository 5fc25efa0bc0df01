/*
 * Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU
 * oracle.  This file holds none of the expression arithmetic: it only draws
 * numbers and rounds them to a storage format.
 *
 * Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used counter-style.  Draw k of tensor t
 * under configuration seed S is
 *     mix64(seed_t + (k + 1) * GAMMA),   seed_t = S ^ ((t + 1) * TGAMMA)
 * with GAMMA = 0x9E3779B97F4A7C15 (SplitMix64's golden gamma) and
 * TGAMMA = 0xD1B54A32D192ED03.  Element i of a tensor uses draw i (uniform,
 * integer) or draws 3i, 3i+1, 3i+2 (lognormal), so any element range can be
 * generated independently and in parallel.
 *
 * Storage rounding is IEEE round-to-nearest-even from the exact FP64 draw,
 * done directly (no double rounding through FP32).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL
#define TGAMMA 0xD1B54A32D192ED03ULL

enum { SY_F32 = 0, SY_F64 = 1, SY_BF16 = 2, SY_F16 = 3, SY_U32 = 4 };
enum { SY_UNIFORM = 0, SY_LOGNORMAL = 1, SY_UINT31 = 2, SY_ONES = 3, SY_UNIFORM12 = 4 };

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t synth_draw(uint64_t seed_cfg, uint64_t tensor, uint64_t k) {
  uint64_t st = seed_cfg ^ ((tensor + 1) * TGAMMA);
  return mix64(st + (k + 1) * GAMMA);
}

/* U[-1,1]: 2 * ((r >> 11) * 2^-53) - 1, exact in FP64. */
static inline double draw_uniform(uint64_t r) {
  return 2.0 * ((double)(r >> 11) * 0x1p-53) - 1.0;
}

/* Lognormal(mu=0, sigma): Box-Muller normal from two draws, random sign
 * from the top bit of a third. */
static inline double draw_lognormal(uint64_t r1, uint64_t r2, uint64_t r3,
                                    double sigma) {
  double u1 = ((double)(r1 >> 11) + 1.0) * 0x1p-53; /* (0,1] */
  double u2 = (double)(r2 >> 11) * 0x1p-53;         /* [0,1) */
  double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
  double mag = exp(sigma * g);
  return (r3 >> 63) ? -mag : mag;
}

/* Round x to a binary format with p significand bits (implicit bit
 * included) and minimum normal exponent emin, nearest-even, subnormals
 * kept.  Overflow is left to the caller. */
static double round_format(double x, int p, int emin) {
  if (x == 0.0 || isnan(x) || isinf(x)) return x;
  int e;
  frexp(x, &e); /* |x| = m * 2^e, m in [0.5, 1): unbiased exponent e-1 */
  int ex = e - 1;
  if (ex < emin) ex = emin;
  double ulp = ldexp(1.0, ex - (p - 1));
  return rint(x / ulp) * ulp; /* default rounding mode: nearest-even */
}

static uint16_t encode_bf16(double v) {
  /* v is exactly representable in bf16, hence in f32. */
  float f = (float)v;
  uint32_t b;
  memcpy(&b, &f, 4);
  return (uint16_t)(b >> 16);
}

static uint16_t encode_f16(double v) {
  uint16_t s = signbit(v) ? 0x8000u : 0u;
  double a = fabs(v);
  if (isnan(v)) return 0x7E00u;
  if (isinf(a)) return s | 0x7C00u;
  if (a == 0.0) return s;
  if (a < 0x1p-14) return s | (uint16_t)(a * 0x1p24); /* subnormal */
  int e;
  double m = frexp(a, &e); /* a = m 2^e, m in [0.5,1) */
  int E = e - 1 + 15;
  uint16_t man = (uint16_t)((m * 2.0 - 1.0) * 1024.0);
  return s | (uint16_t)(E << 10) | man;
}

/* Store an exact FP64 draw as dtype; returns 1 if it saturated (FP16 only). */
static int store(int dtype, void* out, int64_t i, double v) {
  switch (dtype) {
    case SY_F32: ((float*)out)[i] = (float)v; return 0;
    case SY_F64: ((double*)out)[i] = v; return 0;
    case SY_BF16: {
      double r = round_format(v, 8, -126);
      if (fabs(r) > 0x1.FEp127) r = copysign(INFINITY, v);
      ((uint16_t*)out)[i] = encode_bf16(r);
      return 0;
    }
    case SY_F16: {
      double r = round_format(v, 11, -14);
      int sat = 0;
      if (fabs(r) > 65504.0) { r = copysign(65504.0, v); sat = 1; }
      ((uint16_t*)out)[i] = encode_f16(r);
      return sat;
    }
    default: return 0;
  }
}

/* Fill out[0..n) with elements [start, start+n) of tensor `tensor`.
 * dist: SY_UNIFORM (U[-1,1]), SY_LOGNORMAL (sigma = param, random sign),
 * SY_UINT31 (u32 in [0,2^31)), SY_ONES (value = param), SY_UNIFORM12 (U[1,2)).  Returns the number
 * of FP16 saturations, or -1 for an unsupported combination. */
int64_t synth_fill(uint64_t seed_cfg, uint64_t tensor, int dist, double param,
                   int dtype, int64_t start, int64_t n, void* out) {
  int64_t sat = 0;
  if (dist == SY_UINT31) {
    if (dtype != SY_U32) return -1;
    uint32_t* o = (uint32_t*)out;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      o[i] = (uint32_t)(synth_draw(seed_cfg, tensor, (uint64_t)(start + i)) >> 33);
    return 0;
  }
  if (dtype == SY_U32) {
    if (dist != SY_ONES) return -1;
    uint32_t* o = (uint32_t*)out;
    for (int64_t i = 0; i < n; ++i) o[i] = (uint32_t)param;
    return 0;
  }
#pragma omp parallel for schedule(static) reduction(+ : sat)
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = (uint64_t)(start + i);
    double v;
    if (dist == SY_UNIFORM) {
      v = draw_uniform(synth_draw(seed_cfg, tensor, k));
    } else if (dist == SY_UNIFORM12) { /* U[1,2): 1 + (r >> 11) * 2^-53, exact in FP64 */
      v = 1.0 + (double)(synth_draw(seed_cfg, tensor, k) >> 11) * 0x1p-53;
    } else if (dist == SY_LOGNORMAL) {
      v = draw_lognormal(synth_draw(seed_cfg, tensor, 3 * k),
                         synth_draw(seed_cfg, tensor, 3 * k + 1),
                         synth_draw(seed_cfg, tensor, 3 * k + 2), param);
    } else {
      v = param;
    }
    sat += store(dtype, out, i, v);
  }
  return sat;
}

/* The unrounded FP64 draws (for error against the pre-storage values). */
int synth_fill_f64(uint64_t seed_cfg, uint64_t tensor, int dist, double param,
                   int64_t start, int64_t n, double* out) {
  if (dist == SY_UINT31) return -1;
  return (int)synth_fill(seed_cfg, tensor, dist, param, SY_F64, start, n, out);
}

/* Raw draws, for checking the generator against its published definition. */
void synth_raw(uint64_t seed_cfg, uint64_t tensor, int64_t start, int64_t n,
               uint64_t* out) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = synth_draw(seed_cfg, tensor, (uint64_t)(start + i));
}
