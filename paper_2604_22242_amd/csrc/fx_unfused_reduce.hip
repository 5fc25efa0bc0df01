// Unfused baseline, reductions and whole expressions: reductions of
// materialised arrays, and each workload expression evaluated one operator
// at a time through caller-provided temporaries.
#include "fx.hpp"

using namespace fx;

static int elem_bytes(fx_dtype dt) {
  switch (dt) {
    case FX_F32: case FX_U32: return 4;
    case FX_F64: return 8;
    case FX_BF16: case FX_F16: return 2;
  }
  return 0;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Number of temporaries each workload expression needs when evaluated one
// operator at a time (buffers are reused once their value is consumed).
static int n_temporaries(int expr) {
  switch (expr) {
    case FX_EXPR_C1_Z: case FX_EXPR_C2_Z: case FX_EXPR_C2_COLSUM: case FX_EXPR_C2_ROWSUM:
    case FX_EXPR_AXY_EXPW:
      return 2;
    case FX_EXPR_ACCU_XY: case FX_EXPR_NORM_DIFF: case FX_EXPR_COLSUM_XY:
      return 1;
  }
  return -1;
}

extern "C" {

int fx_reduce(int kind, fx_dtype dt, const void* A, const void* B, fx_shape s, void* out,
              void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  if (dt == FX_U32) {
    auto a = leaf<uint32_t>(A, s.n_rows, s.n_cols);
    uint64_t* o = static_cast<uint64_t*>(out);
    if (kind == FX_R_ACCU) return accu(a, o, ws, ws_bytes, cfg, S(stream));
    if (kind == FX_R_DOT)
      return dot(a, leaf<uint32_t>(B, s.n_rows, s.n_cols), o, ws, ws_bytes, cfg, S(stream));
    return fail(FX_E_DTYPE, "reduction %d not defined for u32", kind);
  }
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto a = leaf<T>(A, s.n_rows, s.n_cols);
    double* o = static_cast<double*>(out);
    switch (kind) {
      case FX_R_ACCU: return accu(a, o, ws, ws_bytes, cfg, S(stream));
      case FX_R_NORM: return norm_fro(a, o, ws, ws_bytes, cfg, S(stream));
      case FX_R_DOT: return dot(a, leaf<T>(B, s.n_rows, s.n_cols), o, ws, ws_bytes, cfg, S(stream));
      case FX_R_COLSUM: case FX_R_ROWSUM:
        return sum(a, kind == FX_R_COLSUM ? 0 : 1, static_cast<acc_out_t<T>*>(out), ws, ws_bytes,
                   cfg, S(stream));
    }
    return fail(FX_E_ARG, "unknown reduction kind %d", kind);
  });
}

size_t fx_unfused_tmp_bytes(int expr, fx_dtype dt, fx_shape s) {
  const int nt = n_temporaries(expr), eb = elem_bytes(dt);
  if (nt < 0 || !eb || s.n_rows < 0 || s.n_cols < 0) return 0;
  return (size_t)nt * round256((size_t)(s.n_rows * s.n_cols) * eb);
}

int fx_unfused(int expr, fx_dtype dt, const void* const* in, double a, void* out, fx_shape s,
               void* tmp, size_t tmp_bytes, void* ws, size_t ws_bytes, const fx_launch* cfg,
               void* stream) {
  if (int rc = check_shape(s)) return rc;
  const int nt = n_temporaries(expr);
  if (nt < 0) return fail(FX_E_ARG, "unknown expression %d", expr);
  if (!in) return fail(FX_E_ARG, "NULL input list");
  if (dt == FX_U32 && expr != FX_EXPR_C1_Z && expr != FX_EXPR_ACCU_XY)
    return fail(FX_E_DTYPE, "expression %d has no u32 form", expr);
  const int64_t n = s.n_rows * s.n_cols;
  const size_t need = fx_unfused_tmp_bytes(expr, dt, s);
  if (n > 0 && (!tmp || tmp_bytes < need))
    return fail(FX_E_WORKSPACE, "temporaries of %zu bytes needed, %zu given", need, tmp_bytes);
  const void *X = in[0], *Y = in[1], *W = in[2];
  void* T0 = tmp;
  void* T1 = tmp ? static_cast<char*>(tmp) + round256((size_t)n * elem_bytes(dt)) : nullptr;
  const bool u = dt == FX_U32;
#define RUN(call) \
  do {            \
    int rc_ = (call); \
    if (rc_) return rc_; \
  } while (0)
  switch (expr) {
    case FX_EXPR_C1_Z:  // Z = X % Y + 2*W   (u32: (X ^ Y) + 3*W)
      RUN(fx_op_binary(u ? FX_OP_XOR : FX_OP_SCHUR, dt, X, Y, T0, n, cfg, stream));
      RUN(fx_op_scalar(FX_OP_SMUL, dt, W, u ? 3.0 : 2.0, T1, n, cfg, stream));
      return fx_op_binary(FX_OP_ADD, dt, T0, T1, out, n, cfg, stream);
    case FX_EXPR_ACCU_XY:
      RUN(fx_op_binary(FX_OP_SCHUR, dt, X, Y, T0, n, cfg, stream));
      return fx_reduce(FX_R_ACCU, dt, T0, nullptr, s, out, ws, ws_bytes, cfg, stream);
    case FX_EXPR_C2_Z: case FX_EXPR_C2_COLSUM: case FX_EXPR_C2_ROWSUM: {
      // ((X + Y) % exp(-abs(W))) / (1 + X % X)
      RUN(fx_op_binary(FX_OP_ADD, dt, X, Y, T0, n, cfg, stream));
      RUN(fx_op_unary(FX_OP_ABS, dt, W, T1, n, cfg, stream));
      RUN(fx_op_unary(FX_OP_NEG, dt, T1, T1, n, cfg, stream));
      RUN(fx_op_unary(FX_OP_EXP, dt, T1, T1, n, cfg, stream));
      RUN(fx_op_binary(FX_OP_SCHUR, dt, T0, T1, T0, n, cfg, stream));
      RUN(fx_op_binary(FX_OP_SCHUR, dt, X, X, T1, n, cfg, stream));
      RUN(fx_op_scalar(FX_OP_SADD, dt, T1, 1.0, T1, n, cfg, stream));
      if (expr == FX_EXPR_C2_Z) return fx_op_binary(FX_OP_DIV, dt, T0, T1, out, n, cfg, stream);
      RUN(fx_op_binary(FX_OP_DIV, dt, T0, T1, T0, n, cfg, stream));
      return fx_reduce(expr == FX_EXPR_C2_COLSUM ? FX_R_COLSUM : FX_R_ROWSUM, dt, T0, nullptr, s,
                       out, ws, ws_bytes, cfg, stream);
    }
    case FX_EXPR_NORM_DIFF:
      RUN(fx_op_binary(FX_OP_SUB, dt, X, Y, T0, n, cfg, stream));
      return fx_reduce(FX_R_NORM, dt, T0, nullptr, s, out, ws, ws_bytes, cfg, stream);
    case FX_EXPR_COLSUM_XY:
      RUN(fx_op_binary(FX_OP_SCHUR, dt, X, Y, T0, n, cfg, stream));
      return fx_reduce(FX_R_COLSUM, dt, T0, nullptr, s, out, ws, ws_bytes, cfg, stream);
    case FX_EXPR_AXY_EXPW:  // (a*X) % Y + exp(-W)
      RUN(fx_op_scalar(FX_OP_SMUL, dt, X, a, T0, n, cfg, stream));
      RUN(fx_op_binary(FX_OP_SCHUR, dt, T0, Y, T0, n, cfg, stream));
      RUN(fx_op_unary(FX_OP_NEG, dt, W, T1, n, cfg, stream));
      RUN(fx_op_unary(FX_OP_EXP, dt, T1, T1, n, cfg, stream));
      return fx_op_binary(FX_OP_ADD, dt, T0, T1, out, n, cfg, stream);
  }
#undef RUN
  return fail(FX_E_ARG, "unknown expression %d", expr);
}

}  // extern "C"
