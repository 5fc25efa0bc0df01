// The paper's element-wise benchmark expressions (Sec. 4), written with the
// expression-template front end and evaluated by the element-wise skeleton.
#include <math.h>

#include "fx_kernels.hpp"

using namespace fx;

namespace {

template <class F> int with_f32_bf16(fx_dtype dt, F&& f) {
  switch (dt) {
    case FX_F32: return f(tag<float>{});
    case FX_BF16: return f(tag<bf16_t>{});
    default: break;
  }
  return fail(FX_E_DTYPE, "the paper's expressions are compiled for FP32 and BF16 storage");
}

}  // namespace

extern "C" int fx_paper_expr(int which, fx_dtype dt, const void* const* in, const double* sc,
                             void* Z, fx_shape s, const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  if (!in) return fail(FX_E_ARG, "NULL input list");
  const int64_t R = s.n_rows, Cc = s.n_cols;
  return with_f32_bf16(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    T* z = static_cast<T*>(Z);
    auto X = leaf<T>(in[0], R, Cc);
    switch (which) {
      case FX_PAPER_ADD2: {
        auto Y = leaf<T>(in[1], R, Cc);
        return eval(z, X + Y, cfg, S(stream));
      }
      case FX_PAPER_ADD4: {
        auto B = leaf<T>(in[1], R, Cc), C = leaf<T>(in[2], R, Cc), D = leaf<T>(in[3], R, Cc);
        return eval(z, X + B + C + D, cfg, S(stream));
      }
      case FX_PAPER_RELU:
        return eval(z, X % (X > 0), cfg, S(stream));
      case FX_PAPER_SIGMOID:
        return eval(z, 1 / (1 + exp(-X)), cfg, S(stream));
      case FX_PAPER_SWISH: {
        if (!sc) return fail(FX_E_ARG, "swish needs beta");
        const double beta = sc[0];
        return eval(z, X / (1 + exp(-beta * X)), cfg, S(stream));
      }
      case FX_PAPER_GELU: {
        if (!sc) return fail(FX_E_ARG, "gelu needs alpha");
        const double alpha = sc[0];
        const double c = ::sqrt(2.0 / M_PI);
        return eval(z, (X / 2) % (1 + tanh(c * (X + alpha * pow(X, 3)))), cfg, S(stream));
      }
      case FX_PAPER_EXPR3: {
        auto Y = leaf<double>(in[1], R, Cc);
        auto W = leaf<T>(in[2], R, Cc);
        return eval(z, 1 / (X % conv_to<ct_t<T>>(Y) + log(log(X + 2) % W)), cfg, S(stream));
      }
    }
    return fail(FX_E_ARG, "unknown expression %d", which);
  });
}
