// The workload expressions through kernels generated as source text from
// their expression types at compile time and compiled by the driver at first
// use (Sec. 3; Sec. 4 counts that first compilation as the approach's only
// overhead).  The same types instantiate the ahead-of-time kernels of the
// fused entry points, so the two can be compared directly.
#include <algorithm>
#include <cstring>

#include "fx_source.hpp"
#include "fx_workloads.hpp"

using namespace fx;

namespace {

// The generated kernels' text must be a constant of the program: these
// assertions are evaluated by the compiler.
constexpr auto kC2Text = src_kernel<decltype(c2_expr(Leaf<float>{}, Leaf<float>{}, Leaf<float>{})),
                                    float, 0>::text;
static_assert(contains(kC2Text, "return (((x0 + x1) * expf((-__builtin_fabsf(x2)))) / (k0 + (x3 * x4)));"),
              "the matrix workload's element rule");
static_assert(contains(kC2Text, "#define FX_PARAMS const st_t* __restrict__ p0, const st_t* __restrict__ p1, "
                                "const st_t* __restrict__ p2, const st_t* __restrict__ p3, "
                                "const st_t* __restrict__ p4, ct_t k0, ct_t q0, int m0"),
              "one pointer per leaf occurrence, three arguments per scalar");
static_assert(contains(kC2Text, "fx_rtc_ew"), "the element-wise skeleton");

// An expression id's expression over storage T, handed to f with its result
// kind as a compile-time constant.
template <class T, class F>
int with_workload(int expr, const void* const* in, double a, fx_shape s, F&& f) {
  auto L = [&](int q) { return leaf<T>(in ? in[q] : nullptr, s.n_rows, s.n_cols); };
  using K0 = ic<0>;
  switch (expr) {
    case FX_EXPR_C1_Z: return f(c1_expr(L(0), L(1), L(2)), K0{});
    case FX_EXPR_AXY_EXPW:
      if constexpr (!std::is_same_v<T, uint32_t>) return f(axy_expw_expr(a, L(0), L(1), L(2)), K0{});
      break;
    case FX_EXPR_ACCU_XY:
      if constexpr (!std::is_same_v<T, uint32_t>) return f(xy_expr(L(0), L(1)), ic<FX_R_ACCU>{});
      break;
    case FX_EXPR_C2_Z:
      if constexpr (!std::is_same_v<T, uint32_t>) return f(c2_expr(L(0), L(1), L(2)), K0{});
      break;
    case FX_EXPR_C2_COLSUM:
      if constexpr (!std::is_same_v<T, uint32_t>)
        return f(c2_expr(L(0), L(1), L(2)), ic<FX_R_COLSUM>{});
      break;
    case FX_EXPR_C2_ROWSUM:
      if constexpr (!std::is_same_v<T, uint32_t>)
        return f(c2_expr(L(0), L(1), L(2)), ic<FX_R_ROWSUM>{});
      break;
    case FX_EXPR_NORM_DIFF:
      if constexpr (!std::is_same_v<T, uint32_t>) return f(diff_expr(L(0), L(1)), ic<FX_R_NORM>{});
      break;
    case FX_EXPR_COLSUM_XY:
      if constexpr (!std::is_same_v<T, uint32_t>) return f(xy_expr(L(0), L(1)), ic<FX_R_COLSUM>{});
      break;
    default:
      return fail(FX_E_ARG, "unknown expression %d", expr);
  }
  return fail(FX_E_DTYPE, "expression %d is floating point only", expr);
}

template <class F> int with_source_dtype(fx_dtype dt, F&& f) {
  if (dt == FX_U32) return f(tag<uint32_t>{});
  return with_fp(dt, f);
}

}  // namespace

extern "C" {

int fx_source_eval(int expr, fx_dtype dt, const void* const* inputs, double a, void* out,
                   fx_shape shape, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_shape(shape)) return rc;
  if (!inputs) return fail(FX_E_ARG, "NULL input list");
  return with_source_dtype(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    return with_workload<T>(expr, inputs, a, shape, [&](const auto& e, auto k) -> int {
      return eval_source<decltype(k)::value>(e, out, ws, ws_bytes, S(stream));
    });
  });
}

int fx_source_text(int expr, fx_dtype dt, char* buf, size_t cap, size_t* len) {
  return with_source_dtype(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    return with_workload<T>(expr, nullptr, 0.0, fx_shape{0, 0}, [&](const auto& e, auto k) -> int {
      using K = src_kernel<std::decay_t<decltype(e)>, T, decltype(k)::value>;
      if (len) *len = K::text.size;
      if (buf && cap) {
        const size_t m = std::min(cap - 1, K::text.size);
        std::memcpy(buf, K::text.data(), m);
        buf[m] = 0;
      }
      return FX_OK;
    });
  });
}

int fx_source_prepare(int expr, fx_dtype dt, double* compile_ms) {
  return with_source_dtype(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    return with_workload<T>(expr, nullptr, 0.0, fx_shape{0, 0}, [&](const auto& e, auto k) -> int {
      using K = src_kernel<std::decay_t<decltype(e)>, T, decltype(k)::value>;
      jit_program* p = nullptr;
      if (int rc = K::obtain(&p)) return rc;
      if (compile_ms) *compile_ms = K::compile_ms;
      return FX_OK;
    });
  });
}

}  // extern "C"
