// The paper's expressions over strided views (Sec. 4), written with the
// front end: submatrix sums, expressions with transposes, diagonal sums.
#include <math.h>

#include <algorithm>

#include "fx_views.hpp"

using namespace fx;

namespace {

int64_t diag_len(int64_t m, int64_t n, int64_t k) {
  return std::max<int64_t>(0, k >= 0 ? std::min(m, n - k) : std::min(m + k, n));
}

int view_shape(int which, fx_shape s, fx_shape* out) {
  const int64_t m = s.n_rows, n = s.n_cols;
  switch (which) {
    case FX_PAPER_ADDSUB2:
    case FX_PAPER_ADDSUB4:
      *out = fx_shape{m / 2, n / 2};
      return FX_OK;
    case FX_PAPER_EXPR1:
    case FX_PAPER_EXPR2:
      if (m != n) return fail(FX_E_SHAPE, "expression %d needs a square matrix (%lld x %lld)", which,
                              (long long)m, (long long)n);
      *out = s;
      return FX_OK;
    case FX_PAPER_DIAGSUM:
      *out = fx_shape{std::min(diag_len(m, n, -1), diag_len(m, n, 1)), 1};
      return FX_OK;
  }
  return fail(FX_E_ARG, "unknown view expression %d", which);
}

int view_inputs(int which) {
  return which == FX_PAPER_ADDSUB4 || which == FX_PAPER_EXPR2 ? 4 : 2;
}

// The output may not overlap an input that is read through a transposed,
// offset or diagonal view: a block would overwrite elements that another
// block still has to read.  The only aliasing allowed is the element-wise
// one of the global contract, for leaves read in place (A and D of expr2):
// Z exactly equal to that input.
int check_view_aliasing(int which, const void* const* in, const void* Z, fx_shape s, fx_shape o,
                        size_t esize) {
  const uintptr_t z0 = reinterpret_cast<uintptr_t>(Z);
  const uintptr_t z1 = z0 + (uintptr_t)(o.n_rows * o.n_cols) * esize;
  const uintptr_t bytes = (uintptr_t)(s.n_rows * s.n_cols) * esize;
  for (int q = 0; q < view_inputs(which); ++q) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(in[q]);
    if (!in[q]) return fail(FX_E_ARG, "NULL input %d", q);
    if (a0 >= z1 || a0 + bytes <= z0) continue;
    const bool in_place = which == FX_PAPER_EXPR2 && (q == 0 || q == 3) && a0 == z0;
    if (!in_place)
      return fail(FX_E_ARG, "the output overlaps input %d, which this expression reads through "
                  "a transposed, offset or diagonal view", q);
  }
  return FX_OK;
}

template <class F> int with_view_dtype(fx_dtype dt, F&& f) {
  switch (dt) {
    case FX_F32: return f(tag<float>{});
    case FX_F64: return f(tag<double>{});
    case FX_BF16: return f(tag<bf16_t>{});
    default: break;
  }
  return fail(FX_E_DTYPE, "the view expressions are compiled for FP32, FP64 and BF16 storage");
}

}  // namespace

extern "C" {

int fx_paper_view_shape(int which, fx_shape s, fx_shape* out) {
  if (!out) return fail(FX_E_ARG, "NULL output shape");
  if (int rc = check_shape(s)) return rc;
  return view_shape(which, s, out);
}

int fx_paper_view_expr(int which, fx_dtype dt, const void* const* in, const double* sc, void* Z,
                       fx_shape s, void* stream) {
  if (int rc = check_shape(s)) return rc;
  if (!in) return fail(FX_E_ARG, "NULL input list");
  fx_shape o;
  if (int rc = view_shape(which, s, &o)) return rc;
  if (o.n_rows * o.n_cols == 0) return FX_OK;
  const int64_t m = s.n_rows, n = s.n_cols;
  const int64_t r0 = (m - o.n_rows) / 2, c0 = (n - o.n_cols) / 2;
  return with_view_dtype(dt, [&](auto t_) {
    using T = typename decltype(t_)::type;
    if (!Z) return fail(FX_E_ARG, "NULL output pointer");
    if (int rc = check_view_aliasing(which, in, Z, s, o, sizeof(T))) return rc;
    T* z = static_cast<T*>(Z);
    auto L = [&](int q) { return leaf<T>(in[q], m, n); };
    switch (which) {
      case FX_PAPER_ADDSUB2:
        return eval_views(z, submat(L(0), r0, c0, o.n_rows, o.n_cols) +
                                 submat(L(1), r0, c0, o.n_rows, o.n_cols), S(stream));
      case FX_PAPER_ADDSUB4:
        return eval_views(z, submat(L(0), r0, c0, o.n_rows, o.n_cols) +
                                 submat(L(1), r0, c0, o.n_rows, o.n_cols) +
                                 submat(L(2), r0, c0, o.n_rows, o.n_cols) +
                                 submat(L(3), r0, c0, o.n_rows, o.n_cols), S(stream));
      case FX_PAPER_EXPR1: {
        auto X = L(0), Y = L(1);
        return eval_views(z, 2 * (t(X) + Y) + 2 * (X + t(Y)), S(stream));
      }
      case FX_PAPER_EXPR2: {
        if (!sc) return fail(FX_E_ARG, "expr2 needs the scalar a");
        auto A = L(0), B = L(1), C = L(2), D = L(3);
        return eval_views(z, sc[0] * A + t(B + C) + log(pow(D, 2)), S(stream));
      }
      case FX_PAPER_DIAGSUM: {
        auto X = L(0), Y = L(1);
        auto d = [&](const Leaf<T>& x, int64_t k) {
          Diag<T> v = diag(x, k);
          v.n_rows = o.n_rows;  // the common length
          return v;
        };
        // diagonal elements are one per column: every load is its own
        // scattered access, so vectors buy nothing and the few thousand
        // elements are spread thin (64-thread blocks, one element each)
        // to have as many loads in flight over as many CUs as possible
        const fx_launch thin{64, 1, (int32_t)sizeof(T),
                             (int32_t)std::max<int64_t>(1, std::min<int64_t>(ceil_div(o.n_rows, 64),
                                                                            1 << 20))};
        return eval(z, (d(X, -1) + d(X, 1)) % (d(Y, -1) + d(Y, 1)), &thin, S(stream));
      }
    }
    return fail(FX_E_ARG, "unknown view expression %d", which);
  });
}

}  // extern "C"
