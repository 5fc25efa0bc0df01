// The compile-time front end's user-facing reductions, under the names of the
// Armadillo-style functions the paper's library offers (Sec. 2 names accu;
// dot, norm_fro and sum(E, dim) are their siblings):
//   accu(E)      = sum of E's elements
//   dot(A, B)    = sum of A's and B's element-wise products
//   norm_fro(E)  = square root of the sum of E's squared elements
//   sum(E, 0|1)  = column sums | row sums
// Each fuses E into the reduction: one kernel, inputs read once, compensated
// per-thread sums and an FP64 combine (u64 for u32 expressions).  E may be an
// expression or a dmat view.  The scalar results go to device memory; the
// workspace is sized by fx_workspace_bytes and zeroed once by the caller.
// Z = E itself is eval(z, E, cfg, stream).
#pragma once

#include <type_traits>
#include <utility>

#include "fx_kernels.hpp"

namespace fx {

// expr_of<E>: the expression type of an operand (a dmat becomes its leaf).
template <class E> using total_of = typename wide<typename expr_of<E>::ct>::type;

template <class E>
int accu(const E& e, total_of<E>* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
         hipStream_t st) {
  return reduce_full<map_id>(as_expr(e), out, ws, ws_bytes, cfg, st);
}

template <class A, class B>
int dot(const A& a, const B& b, total_of<A>* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
        hipStream_t st) {
  return reduce_full<map_id>(as_expr(a) % as_expr(b), out, ws, ws_bytes, cfg, st);
}

template <class E>
int norm_fro(const E& e, double* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
             hipStream_t st) {
  static_assert(std::is_floating_point_v<typename expr_of<E>::ct>,
                "norm_fro takes floating-point expressions");
  return reduce_full<map_sq>(as_expr(e), out, ws, ws_bytes, cfg, st);
}

// dim 0: out[j] = sum over rows of column j; dim 1: out[i] = sum over
// columns of row i.  O is the accumulator type (the compute type).
template <class E, class O>
int sum(const E& e, int dim, O* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
        hipStream_t st) {
  if (dim != 0 && dim != 1) return fail(FX_E_ARG, "sum: dim must be 0 or 1, got %d", dim);
  return reduce_dim(dim == 0 ? FX_R_COLSUM : FX_R_ROWSUM, as_expr(e), out, ws, ws_bytes, cfg, st);
}

}  // namespace fx
