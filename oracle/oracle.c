/*
 * FP64 CPU oracle for fused element-wise expressions and their reductions.
 *
 * TEST INFRASTRUCTURE ONLY.  It is called by the test suite, by the smoke
 * check and by the benchmark's CPU-baseline leg, never by the HIP library,
 * and it shares no code with it.
 *
 * What it computes (the plain definition the fused kernels must reach):
 *   - An expression is a tree whose C++ type is its abstract syntax tree
 *     (Sec. 3, the X.t()+3 example); evaluating it fused gives, element by
 *     element, exactly what evaluating it one operator at a time gives
 *     (Sec. 3, "single pass", Sec. 5).  The oracle therefore evaluates the
 *     tree node by node, each node writing a full FP64 temporary.
 *   - Matrices are column-major: element (r, c) of an n_rows x n_cols matrix
 *     is linear index r + c*n_rows (Sec. 3, element-access rule of the
 *     plain matrix).
 *   - Scalar nodes combine a constant with the child's element (Sec. 3,
 *     scalar-add rule); here a constant is a node of its own.
 *   - accu() is the sum of all elements (Sec. 3 lists it among the
 *     user-facing functions); column sums sum(E,0), row sums sum(E,1) and the
 *     Frobenius norm follow Armadillo's definitions, which the API mirrors
 *     (Sec. 2).
 *
 * Inputs are the stored values widened exactly to FP64 (f32, bf16, f16 all
 * embed exactly).  Sums are Neumaier-compensated in FP64, accumulated in
 * element-index order (chunk partials combined in index order).
 *
 * Alongside each value it carries a first-order running error bound mu, in
 * units of the GPU compute unit roundoff u_c, for evaluating the same tree in
 * precision u_c in any order (Higham, Accuracy and Stability of Numerical
 * Algorithms, 2nd ed., Sec. 3.3, running error analysis):
 *     leaf, exact constant: 0      constant not exact in u_c: |c|
 *     a +- b: mu_a + mu_b + |v|    a*b: mu_a|b| + |a|mu_b + |v|
 *     a/b: (mu_a + |v| mu_b)/|b| + |v|      -a, |a|: mu_a
 *     exp(a): |v|(mu_a + f_exp)    sqrt(a): spread(a, mu_a) + |v|
 *     log(a): mu_a/|a| + f_log|v|   tanh(a): (1 - v^2) mu_a + f_tanh|v|
 *     pow(a, k) (k a constant): |k a^(k-1)| mu_a + f_pow|v|
 *     a > b: 0 (1 or 0; the comparison itself is exact)
 *     conversion to FP32 storage: mu_a + |v|
 *     sum of n terms t_i: sum mu_i + (ceil(log2 n) + 2) sum |t_i|
 * Each term is the first-order propagation of the operands' bounds through
 * the operator's derivative plus the operator's own error.  sqrt propagates
 * exactly instead (spread: the largest change of sqrt over the operand's
 * error interval, see sqrt_spread), because its derivative is unbounded at 0
 * and a cancellation just before it leaves an operand whose error is as
 * large as its value; away from 0 spread is mu_a/(2|v|) to first order.  Correctly
 * rounded operations (+ - * / sqrt, the conversion) contribute |v| (half an
 * ulp is at most u_c |v|); a device elementary function contributes f |v|,
 * where f (per function, in units of u_c relative to the result) is the
 * caller's allowance fop[] = {f_exp, f_log, f_tanh, f_pow}.  The allowances
 * are fixed by sweeping the device functions against libm (every FP32 input
 * of each function's domain; a sample of FP64 inputs): f must be at least
 * the largest relative error found there.
 *
 * Integer trees (u32) are evaluated in uint64 with every operation reduced
 * mod 2^32 (C unsigned semantics).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_F32 = 0, OR_F64 = 1, OR_BF16 = 2, OR_F16 = 3, OR_U32 = 4 };
enum {
  OR_LEAF = 0, OR_CONST = 1, OR_ADD = 2, OR_SUB = 3, OR_MUL = 4, OR_DIV = 5,
  OR_NEG = 6, OR_ABS = 7, OR_EXP = 8, OR_SQRT = 9, OR_XOR = 10,
  /* the paper's benchmark expressions (Sec. 4) add these */
  OR_LOG = 11, OR_TANH = 12, OR_POW = 13, OR_GT = 14, OR_TOF32 = 15
};
enum { OR_NONE = 0, OR_ACCU = 1, OR_COLSUM = 2, OR_ROWSUM = 3, OR_NORM = 4 };
enum { OR_OK = 0, OR_EBAD = -1, OR_ENOMEM = -2 };

#define CHUNK ((int64_t)1 << 18)
#define ACCU_BLOCKS 64 /* fixed partition of a chunk for the full sum */

/* Thread count for the timing of the oracle itself (not used by tests). */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---- exact widening of stored values ---------------------------------- */

static double widen_bf16(uint16_t h) {
  uint32_t b = (uint32_t)h << 16;
  float f;
  memcpy(&f, &b, 4);
  return (double)f;
}

static double widen_f16(uint16_t h) {
  int s = h >> 15, e = (h >> 10) & 0x1F, m = h & 0x3FF;
  double v;
  if (e == 0) v = ldexp((double)m, -24);
  else if (e == 31) v = m ? NAN : INFINITY;
  else v = ldexp((double)(m + 1024), e - 25);
  return s ? -v : v;
}

static double widen(int dtype, const void* p, int64_t i) {
  switch (dtype) {
    case OR_F32: return (double)((const float*)p)[i];
    case OR_F64: return ((const double*)p)[i];
    case OR_BF16: return widen_bf16(((const uint16_t*)p)[i]);
    case OR_F16: return widen_f16(((const uint16_t*)p)[i]);
    case OR_U32: return (double)((const uint32_t*)p)[i];
  }
  return NAN;
}

/* ---- Neumaier-compensated sum ----------------------------------------- */

typedef struct { double s, c, abs, mu; } acc_t;

/* s + c += t, Neumaier's variant of Kahan summation. */
static void neumaier(double* s, double* c, double t) {
  double u = *s + t;
  if (fabs(*s) >= fabs(t)) *c += (*s - u) + t;
  else *c += (t - u) + *s;
  *s = u;
}

static void acc_add(acc_t* a, double t, double mu_t) {
  neumaier(&a->s, &a->c, t);
  a->abs += fabs(t);
  a->mu += mu_t;
}

static void acc_merge(acc_t* a, const acc_t* b) {
  neumaier(&a->s, &a->c, b->s);
  neumaier(&a->s, &a->c, b->c);
  a->abs += b->abs;
  a->mu += b->mu;
}

static double ceil_log2(int64_t n) {
  double l = 0.0;
  int64_t p = 1;
  while (p < n) { p <<= 1; l += 1.0; }
  return l;
}

static void acc_final(const acc_t* a, int64_t nterms, double* out, double* mu) {
  *out = a->s + a->c;
  *mu = a->mu + (ceil_log2(nterms) + 2.0) * a->abs;
}

/* Largest change of sqrt(a) when a (>= 0) moves by at most D = u_c * mu_a,
 * in units of u_c.  sqrt is concave, so the worst move is downward unless it
 * would cross zero; upward is worse only once D > 3a:
 *   down = sqrt(a) - sqrt(a - D) = D / (sqrt(a) + sqrt(a - D))   (D <= a)
 *        = sqrt(a)                                              (D > a)
 *   up   = sqrt(a + D) - sqrt(a) = D / (sqrt(a + D) + sqrt(a)).
 * For D << a this is the first-order term mu_a / (2 sqrt(a)); unlike that
 * term it stays a bound when the operand's error is as large as the operand
 * (a cancellation just before the square root). */
static double sqrt_spread(double a, double mu_a, double u_c) {
  if (!(a >= 0.0)) return NAN;
  const double D = u_c * mu_a;
  if (D == 0.0) return 0.0;
  const double ra = sqrt(a);
  const double down = D <= a ? D / (ra + sqrt(a - D)) : ra;
  const double up = D / (sqrt(a + D) + ra);
  return (down > up ? down : up) / u_c;
}

/* ---- one tree node over a chunk ---------------------------------------- */

static int const_exact(double c, double u_c) {
  if (u_c >= 0x1p-24 * 0.99) return (double)(float)c == c;
  return 1;
}

/* Node arrays: op, a, b (child node indices, earlier than the node), leaf
 * (input index for OR_LEAF), cst (value for OR_CONST). */
/* A leaf's view of its input (NULL arrays: every leaf dense).  Element
 * (r, c) of the view is input[off + r * rs + c * cs]; a dense leaf of an
 * n_rows x n_cols expression is off = 0, rs = 1, cs = n_rows.  Transposes,
 * submatrices and diagonals are all of this form (Sec. 3: the transposed
 * access swaps row and column in the index). */
typedef struct {
  const int64_t* off;
  const int64_t* rs;
  const int64_t* cs;
  int64_t n_rows;
} views_t;

static void eval_node(int k, const int32_t* op, const int32_t* ca,
                      const int32_t* cb, const int32_t* leaf, const double* cst,
                      const void* const* inputs, const int* dtypes, int64_t e0,
                      int64_t len, double** V, double** M, double u_c,
                      const double* fop, const views_t* vw) {
  const double f_exp = fop[0], f_log = fop[1], f_tanh = fop[2], f_pow = fop[3];
  double* v = V[k];
  double* m = M[k];
  const double* va = ca[k] >= 0 ? V[ca[k]] : NULL;
  const double* ma = ca[k] >= 0 ? M[ca[k]] : NULL;
  const double* vb = cb[k] >= 0 ? V[cb[k]] : NULL;
  const double* mb = cb[k] >= 0 ? M[cb[k]] : NULL;
  int64_t i;
  switch (op[k]) {
    case OR_LEAF: {
      const void* p = inputs[leaf[k]];
      const int dt = dtypes[leaf[k]];
      if (vw->off) {
        const int64_t off = vw->off[k], rs = vw->rs[k], cs = vw->cs[k], R = vw->n_rows;
#pragma omp parallel for schedule(static)
        for (i = 0; i < len; ++i) {
          const int64_t r = (e0 + i) % R, c = (e0 + i) / R;
          v[i] = widen(dt, p, off + r * rs + c * cs);
          m[i] = 0.0;
        }
      } else {
#pragma omp parallel for schedule(static)
        for (i = 0; i < len; ++i) { v[i] = widen(dt, p, e0 + i); m[i] = 0.0; }
      }
      break;
    }
    case OR_CONST: {
      double c = cst[k], mc = const_exact(c, u_c) ? 0.0 : fabs(c);
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) { v[i] = c; m[i] = mc; }
      break;
    }
    case OR_ADD:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = va[i] + vb[i];
        m[i] = ma[i] + mb[i] + fabs(v[i]);
      }
      break;
    case OR_SUB:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = va[i] - vb[i];
        m[i] = ma[i] + mb[i] + fabs(v[i]);
      }
      break;
    case OR_MUL:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = va[i] * vb[i];
        m[i] = ma[i] * fabs(vb[i]) + fabs(va[i]) * mb[i] + fabs(v[i]);
      }
      break;
    case OR_DIV:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = va[i] / vb[i];
        m[i] = (ma[i] + fabs(v[i]) * mb[i]) / fabs(vb[i]) + fabs(v[i]);
      }
      break;
    case OR_NEG:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) { v[i] = -va[i]; m[i] = ma[i]; }
      break;
    case OR_ABS:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) { v[i] = fabs(va[i]); m[i] = ma[i]; }
      break;
    case OR_EXP:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = exp(va[i]);
        m[i] = fabs(v[i]) * (ma[i] + f_exp);
      }
      break;
    case OR_SQRT:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = sqrt(va[i]);
        m[i] = sqrt_spread(va[i], ma[i], u_c) + fabs(v[i]);
      }
      break;
    case OR_LOG:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = log(va[i]);
        m[i] = ma[i] / fabs(va[i]) + f_log * fabs(v[i]);
      }
      break;
    case OR_TANH:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = tanh(va[i]);
        m[i] = (1.0 - v[i] * v[i]) * ma[i] + f_tanh * fabs(v[i]);
      }
      break;
    case OR_POW:  /* b is a constant exponent */
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) {
        v[i] = pow(va[i], vb[i]);
        m[i] = fabs(vb[i] * pow(va[i], vb[i] - 1.0)) * ma[i] + f_pow * fabs(v[i]);
      }
      break;
    case OR_GT:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) { v[i] = va[i] > vb[i] ? 1.0 : 0.0; m[i] = 0.0; }
      break;
    case OR_TOF32:
#pragma omp parallel for schedule(static)
      for (i = 0; i < len; ++i) { v[i] = (double)(float)va[i]; m[i] = ma[i] + fabs(v[i]); }
      break;
  }
}

static int check_tree(int n_nodes, const int32_t* op, const int32_t* a,
                      const int32_t* b, const int32_t* leaf, int n_inputs) {
  if (n_nodes <= 0) return 0;
  for (int k = 0; k < n_nodes; ++k) {
    int o = op[k];
    if (o == OR_LEAF) {
      if (leaf[k] < 0 || leaf[k] >= n_inputs) return 0;
    } else if (o == OR_CONST) {
    } else if ((o >= OR_ADD && o <= OR_DIV) || o == OR_POW || o == OR_GT) {
      if (a[k] < 0 || a[k] >= k || b[k] < 0 || b[k] >= k) return 0;
    } else if ((o >= OR_NEG && o <= OR_SQRT) || o == OR_LOG || o == OR_TANH || o == OR_TOF32) {
      if (a[k] < 0 || a[k] >= k) return 0;
    } else {
      return 0;
    }
  }
  return 1;
}

/*
 * Evaluate a floating-point tree (root = last node) over an n_rows x n_cols
 * column-major operand set and optionally reduce it.  dtypes[q] is the
 * storage type of input q (u32 inputs widen to their integer value).
 *   reduce OR_NONE:   out[n], mu[n]            (n = n_rows * n_cols)
 *          OR_ACCU:   out[0] = sum of all elements
 *          OR_COLSUM: out[n_cols], column sums
 *          OR_ROWSUM: out[n_rows], row sums
 *          OR_NORM:   out[0] = sqrt(sum of squares)
 * u_c: unit roundoff of the compute type the bound mu refers to.
 * fop: allowances of the device elementary functions {exp, log, tanh, pow},
 *      in units of u_c relative to the result (2 = one ulp at most).
 */
int or_eval_views(int n_nodes, const int32_t* op, const int32_t* a, const int32_t* b,
                  const int32_t* leaf, const double* cst, int n_inputs,
                  const void* const* inputs, const int* dtypes, int64_t n_rows,
                  int64_t n_cols, int reduce, double u_c, const double* fop,
                  const int64_t* voff, const int64_t* vrs, const int64_t* vcs,
                  double* out, double* mu);

int or_eval(int n_nodes, const int32_t* op, const int32_t* a, const int32_t* b,
            const int32_t* leaf, const double* cst, int n_inputs,
            const void* const* inputs, const int* dtypes, int64_t n_rows,
            int64_t n_cols, int reduce, double u_c, const double* fop, double* out,
            double* mu) {
  return or_eval_views(n_nodes, op, a, b, leaf, cst, n_inputs, inputs, dtypes, n_rows, n_cols,
                       reduce, u_c, fop, NULL, NULL, NULL, out, mu);
}

/* or_eval with a view per node (voff/vrs/vcs indexed by node; only leaves
 * read them).  The caller keeps every view inside its input array. */
int or_eval_views(int n_nodes, const int32_t* op, const int32_t* a, const int32_t* b,
                  const int32_t* leaf, const double* cst, int n_inputs,
                  const void* const* inputs, const int* dtypes, int64_t n_rows,
                  int64_t n_cols, int reduce, double u_c, const double* fop,
                  const int64_t* voff, const int64_t* vrs, const int64_t* vcs,
                  double* out, double* mu) {
  const views_t vw = {voff, vrs, vcs, n_rows > 0 ? n_rows : 1};
  for (int q = 0; q < n_inputs; ++q)
    if (dtypes[q] < 0 || dtypes[q] > OR_U32) return OR_EBAD;
  if (n_rows < 0 || n_cols < 0 || reduce < OR_NONE || reduce > OR_NORM || !fop) return OR_EBAD;
  if (!check_tree(n_nodes, op, a, b, leaf, n_inputs)) return OR_EBAD;
  const int64_t n = n_rows * n_cols;

  double** V = (double**)calloc((size_t)n_nodes, sizeof(double*));
  double** M = (double**)calloc((size_t)n_nodes, sizeof(double*));
  acc_t* col = NULL;
  acc_t* part = NULL;
  int rc = OR_OK;
  const int64_t chunk = n < CHUNK ? (n > 0 ? n : 1) : CHUNK;
  for (int k = 0; k < n_nodes; ++k) {
    V[k] = (double*)malloc((size_t)chunk * sizeof(double));
    M[k] = (double*)malloc((size_t)chunk * sizeof(double));
    if (!V[k] || !M[k]) { rc = OR_ENOMEM; goto done; }
  }
  int64_t n_acc = reduce == OR_COLSUM ? n_cols : reduce == OR_ROWSUM ? n_rows : 1;
  col = (acc_t*)calloc((size_t)(n_acc > 0 ? n_acc : 1), sizeof(acc_t));
  part = (acc_t*)calloc(ACCU_BLOCKS, sizeof(acc_t));
  if (!col || !part) { rc = OR_ENOMEM; goto done; }

  const int root = n_nodes - 1;
  for (int64_t e0 = 0; e0 < n; e0 += chunk) {
    const int64_t len = (n - e0) < chunk ? (n - e0) : chunk;
    for (int k = 0; k < n_nodes; ++k)
      eval_node(k, op, a, b, leaf, cst, inputs, dtypes, e0, len, V, M, u_c, fop, &vw);
    const double* v = V[root];
    const double* m = M[root];
    if (reduce == OR_NONE) {
      memcpy(out + e0, v, (size_t)len * sizeof(double));
      memcpy(mu + e0, m, (size_t)len * sizeof(double));
    } else if (reduce == OR_ACCU || reduce == OR_NORM) {
      /* fixed partition of the chunk; partials merged in index order */
      const int64_t per = (len + ACCU_BLOCKS - 1) / ACCU_BLOCKS;
#pragma omp parallel for schedule(static)
      for (int p = 0; p < ACCU_BLOCKS; ++p) {
        acc_t t = {0, 0, 0, 0};
        int64_t lo = p * per, hi = lo + per < len ? lo + per : len;
        for (int64_t i = lo; i < hi; ++i) {
          if (reduce == OR_ACCU) acc_add(&t, v[i], m[i]);
          else acc_add(&t, v[i] * v[i], 2.0 * fabs(v[i]) * m[i] + v[i] * v[i]);
        }
        part[p] = t;
      }
      for (int p = 0; p < ACCU_BLOCKS; ++p) acc_merge(&col[0], &part[p]);
    } else if (reduce == OR_COLSUM) {
      const int64_t c0 = e0 / n_rows, c1 = (e0 + len - 1) / n_rows;
#pragma omp parallel for schedule(static)
      for (int64_t c = c0; c <= c1; ++c) {
        int64_t lo = c * n_rows - e0, hi = lo + n_rows;
        if (lo < 0) lo = 0;
        if (hi > len) hi = len;
        for (int64_t i = lo; i < hi; ++i) acc_add(&col[c], v[i], m[i]);
      }
    } else { /* OR_ROWSUM: each row visits its elements in column order */
#pragma omp parallel for schedule(static)
      for (int64_t r = 0; r < n_rows; ++r) {
        int64_t first = r - (e0 % n_rows);
        if (first < 0) first += n_rows;
        for (int64_t i = first; i < len; i += n_rows) acc_add(&col[r], v[i], m[i]);
      }
    }
  }

  if (reduce == OR_ACCU) {
    acc_final(&col[0], n, out, mu);
  } else if (reduce == OR_NORM) {
    double s, ms;
    acc_final(&col[0], n, &s, &ms);
    out[0] = sqrt(s);
    mu[0] = sqrt_spread(s, ms, u_c) + out[0];
  } else if (reduce == OR_COLSUM) {
    for (int64_t c = 0; c < n_cols; ++c) acc_final(&col[c], n_rows, &out[c], &mu[c]);
  } else if (reduce == OR_ROWSUM) {
    for (int64_t r = 0; r < n_rows; ++r) acc_final(&col[r], n_cols, &out[r], &mu[r]);
  }

done:
  for (int k = 0; k < n_nodes; ++k) { free(V[k]); free(M[k]); }
  free(V);
  free(M);
  free(col);
  free(part);
  return rc;
}

/*
 * Integer tree over u32 storage: ADD, SUB, MUL, XOR and CONST, each result
 * reduced mod 2^32.  out[n] receives the element values; if accu_out is not
 * NULL it receives the full (unwrapped) uint64 sum of the root.
 */
int or_eval_u32(int n_nodes, const int32_t* op, const int32_t* a,
                const int32_t* b, const int32_t* leaf, const double* cst,
                int n_inputs, const uint32_t* const* inputs, int64_t n,
                uint32_t* out, uint64_t* accu_out) {
  if (n < 0 || n_nodes <= 0) return OR_EBAD;
  for (int k = 0; k < n_nodes; ++k) {
    int o = op[k];
    if (o == OR_LEAF) { if (leaf[k] < 0 || leaf[k] >= n_inputs) return OR_EBAD; }
    else if (o == OR_CONST) {
      if (!(cst[k] >= 0 && cst[k] < 4294967296.0 && cst[k] == floor(cst[k]))) return OR_EBAD;
    } else if (o == OR_ADD || o == OR_SUB || o == OR_MUL || o == OR_XOR) {
      if (a[k] < 0 || a[k] >= k || b[k] < 0 || b[k] >= k) return OR_EBAD;
    } else return OR_EBAD;
  }
  const int64_t chunk = n < CHUNK ? (n > 0 ? n : 1) : CHUNK;
  uint64_t** T = (uint64_t**)calloc((size_t)n_nodes, sizeof(uint64_t*));
  int rc = OR_OK;
  uint64_t total = 0;
  for (int k = 0; k < n_nodes; ++k) {
    T[k] = (uint64_t*)malloc((size_t)chunk * sizeof(uint64_t));
    if (!T[k]) { rc = OR_ENOMEM; goto done; }
  }
  const uint64_t mask = 0xFFFFFFFFull;
  for (int64_t e0 = 0; e0 < n; e0 += chunk) {
    const int64_t len = (n - e0) < chunk ? (n - e0) : chunk;
    for (int k = 0; k < n_nodes; ++k) {
      uint64_t* t = T[k];
      const uint64_t* ta = a[k] >= 0 ? T[a[k]] : NULL;
      const uint64_t* tb = b[k] >= 0 ? T[b[k]] : NULL;
      switch (op[k]) {
        case OR_LEAF:
          for (int64_t i = 0; i < len; ++i) t[i] = inputs[leaf[k]][e0 + i];
          break;
        case OR_CONST:
          for (int64_t i = 0; i < len; ++i) t[i] = (uint64_t)cst[k];
          break;
        case OR_ADD: for (int64_t i = 0; i < len; ++i) t[i] = (ta[i] + tb[i]) & mask; break;
        case OR_SUB: for (int64_t i = 0; i < len; ++i) t[i] = (ta[i] - tb[i]) & mask; break;
        case OR_MUL: for (int64_t i = 0; i < len; ++i) t[i] = (ta[i] * tb[i]) & mask; break;
        case OR_XOR: for (int64_t i = 0; i < len; ++i) t[i] = (ta[i] ^ tb[i]) & mask; break;
      }
    }
    const uint64_t* r = T[n_nodes - 1];
    for (int64_t i = 0; i < len; ++i) {
      if (out) out[e0 + i] = (uint32_t)r[i];
      total += r[i];
    }
  }
  if (accu_out) *accu_out = total;
done:
  for (int k = 0; k < n_nodes; ++k) free(T[k]);
  free(T);
  return rc;
}
