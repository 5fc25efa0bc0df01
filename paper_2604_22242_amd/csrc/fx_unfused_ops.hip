// Unfused baseline, element-wise part: one kernel per operator, each reading
// its operands from memory and writing a full result array.  The kernels are
// the same skeleton with a one-node expression, so the only difference from
// the fused path is the temporaries (what toolkits without fusion pay,
// Sec. 4).
#include "fx_kernels.hpp"

using namespace fx;

extern "C" {

int fx_op_unary(int op, fx_dtype dt, const void* A, void* out, int64_t n, const fx_launch* cfg,
                void* stream) {
  if (int rc = check_n(n)) return rc;
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto a = leaf<T>(A, n, 1);
    T* z = static_cast<T*>(out);
    switch (op) {
      case FX_OP_NEG: return eval(z, -a, cfg, S(stream));
      case FX_OP_ABS: return eval(z, abs(a), cfg, S(stream));
      case FX_OP_EXP: return eval(z, exp(a), cfg, S(stream));
      case FX_OP_SQRT: return eval(z, sqrt(a), cfg, S(stream));
      case FX_OP_LOG: return eval(z, log(a), cfg, S(stream));
      case FX_OP_TANH: return eval(z, tanh(a), cfg, S(stream));
    }
    return fail(FX_E_ARG, "unknown unary operator %d", op);
  });
}

int fx_op_binary(int op, fx_dtype dt, const void* A, const void* B, void* out, int64_t n,
                 const fx_launch* cfg, void* stream) {
  if (int rc = check_n(n)) return rc;
  if (dt == FX_U32) {
    auto a = leaf<uint32_t>(A, n, 1), b = leaf<uint32_t>(B, n, 1);
    uint32_t* z = static_cast<uint32_t*>(out);
    switch (op) {
      case FX_OP_ADD: return eval(z, a + b, cfg, S(stream));
      case FX_OP_SUB: return eval(z, a - b, cfg, S(stream));
      case FX_OP_SCHUR: return eval(z, a % b, cfg, S(stream));
      case FX_OP_XOR: return eval(z, a ^ b, cfg, S(stream));
    }
    return fail(FX_E_ARG, "binary operator %d not defined for u32", op);
  }
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto a = leaf<T>(A, n, 1), b = leaf<T>(B, n, 1);
    T* z = static_cast<T*>(out);
    switch (op) {
      case FX_OP_ADD: return eval(z, a + b, cfg, S(stream));
      case FX_OP_SUB: return eval(z, a - b, cfg, S(stream));
      case FX_OP_SCHUR: return eval(z, a % b, cfg, S(stream));
      case FX_OP_DIV: return eval(z, a / b, cfg, S(stream));
    }
    return fail(FX_E_ARG, "binary operator %d not defined for floating point", op);
  });
}

int fx_op_scalar(int op, fx_dtype dt, const void* A, double k, void* out, int64_t n,
                 const fx_launch* cfg, void* stream) {
  if (int rc = check_n(n)) return rc;
  if (dt == FX_U32) {
    if (!(k >= 0 && k < 4294967296.0 && k == (double)(uint64_t)k))
      return fail(FX_E_ARG, "u32 scalar must be an integer in [0, 2^32)");
    const uint32_t ku = (uint32_t)k;
    auto a = leaf<uint32_t>(A, n, 1);
    uint32_t* z = static_cast<uint32_t*>(out);
    switch (op) {
      case FX_OP_SADD: return eval(z, ku + a, cfg, S(stream));
      case FX_OP_SMUL: return eval(z, ku * a, cfg, S(stream));
      case FX_OP_SSUB: return eval(z, a - ku, cfg, S(stream));
      case FX_OP_SRSUB: return eval(z, ku - a, cfg, S(stream));
    }
    return fail(FX_E_ARG, "scalar operator %d not defined for u32", op);
  }
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto a = leaf<T>(A, n, 1);
    T* z = static_cast<T*>(out);
    switch (op) {
      case FX_OP_SADD: return eval(z, k + a, cfg, S(stream));
      case FX_OP_SMUL: return eval(z, k * a, cfg, S(stream));
      case FX_OP_SDIV: return eval(z, a / k, cfg, S(stream));
      case FX_OP_SRDIV: return eval(z, k / a, cfg, S(stream));
      case FX_OP_SSUB: return eval(z, a - k, cfg, S(stream));
      case FX_OP_SRSUB: return eval(z, k - a, cfg, S(stream));
      case FX_OP_SPOW: return eval(z, pow(a, k), cfg, S(stream));
    }
    return fail(FX_E_ARG, "unknown scalar operator %d", op);
  });
}

}  // extern "C"
