// The library's fixed workload expressions, written once with the front end
// so that every mode that evaluates them (the compile-time kernels, the
// unfused baseline's reference shapes, the kernels generated from the same
// types as source text) sees the same expression type.
//   c1:       X % Y + 2*W          (u32: (X ^ Y) + 3*W)
//   xy:       X % Y                (accu, dot, sum(., 0))
//   c2:       (X + Y) % exp(-abs(W)) / (1 + X % X)
//   diff:     X - Y                (norm_fro)
//   axy_expw: a*X % Y + exp(-W)
#pragma once

#include "fx_expr.hpp"

namespace fx {

template <class X, class Y, class W> inline auto c1_expr(const X& x, const Y& y, const W& w) {
  if constexpr (std::is_same_v<typename X::ct, uint32_t>) return (x ^ y) + 3u * w;
  else return x % y + 2 * w;
}
template <class X, class Y> inline auto xy_expr(const X& x, const Y& y) { return x % y; }
template <class X, class Y, class W> inline auto c2_expr(const X& x, const Y& y, const W& w) {
  return (x + y) % exp(-abs(w)) / (1 + x % x);
}
template <class X, class Y> inline auto diff_expr(const X& x, const Y& y) { return x - y; }
template <class X, class Y, class W>
inline auto axy_expw_expr(double a, const X& x, const Y& y, const W& w) {
  return a * x % y + exp(-w);
}

}  // namespace fx
