// Expression-template front end.
//
// The C++ type of an expression is its abstract syntax tree (Sec. 3: X.t()+3
// has a nested eOp/Op type).  Operator overloads on device views build that
// type at compile time; each node knows how to produce the element at a
// linear index from its children's elements (Sec. 3, the element-access
// macro built by recursing on the AST, one rule per node type):
//   leaf            p[r + c*n_rows]           (column-major, plain matrix rule)
//   scalar node     child(i) op k             (scalar-add rule, generalised)
//   unary node      f(child(i))
//   binary node     f(left(i), right(i))
// Here the rules are inline device functions rather than generated macro
// text, so hipcc instantiates one kernel per expression type ahead of time
// and no scaffolding survives compilation.  Each node also has a vector
// form at_vec<N>(i) that applies the same rule to N consecutive elements
// (one 16-byte load per leaf).
//
// Shapes are checked on the host before launch (the bounds-check macro of
// the generated set); on the device the only bound is the loop's i < n.
#pragma once

#include <math.h>

#include <type_traits>

#include "fx_core.hpp"

namespace fx {

struct expr_tag {};
template <class E> constexpr bool is_expr_v = std::is_base_of_v<expr_tag, E>;

// Host-side facts gathered from every leaf: common shape and alignment.
struct leaf_info {
  int64_t n_rows = -1, n_cols = -1;
  bool shape_ok = true;
  bool any_null = false;
  uintptr_t addr_or = 0;  // OR of all leaf addresses (alignment test)
  void add(const void* p, int64_t r, int64_t c) {
    if (!p && r * c > 0) any_null = true;
    if (n_rows < 0) { n_rows = r; n_cols = c; }
    else if (r != n_rows || c != n_cols) shape_ok = false;
    addr_or |= reinterpret_cast<uintptr_t>(p);
  }
  void add_shape(int64_t r, int64_t c) {  // an expression without array leaves
    if (n_rows < 0) { n_rows = r; n_cols = c; }
    else if (r != n_rows || c != n_cols) shape_ok = false;
  }
  bool aligned(int bytes) const { return (addr_or & (uintptr_t)(bytes - 1)) == 0; }
};

// ---- leaves ----------------------------------------------------------------

// A read-only, non-owning view of a dense column-major device matrix.
template <class T> struct Leaf : expr_tag {
  using storage = T;
  using ct = ct_t<T>;
  const T* p;
  int64_t n_rows, n_cols;

  __device__ __forceinline__ ct at(int64_t i) const { return static_cast<ct>(p[i]); }
  __device__ __forceinline__ ct at(int64_t r, int64_t c) const { return at(r + c * n_rows); }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    return load_lanes<N, NT>(p, i);
  }
  void collect(leaf_info& li) const { li.add(p, n_rows, n_cols); }
};

// Non-owning views handed to the front end (Armadillo-style dmat / dvec).
template <class T> struct dmat {
  T* p;
  int64_t n_rows, n_cols;
  Leaf<T> expr() const { return Leaf<T>{{}, p, n_rows, n_cols}; }
};
template <class T> inline dmat<T> dvec(T* p, int64_t n) { return dmat<T>{p, n, 1}; }
template <class T> inline Leaf<T> leaf(const void* p, int64_t rows, int64_t cols) {
  return Leaf<T>{{}, static_cast<const T*>(p), rows, cols};
}

template <class E> __host__ __device__ inline const E& as_expr(const E& e) { return e; }
template <class T> inline Leaf<T> as_expr(const dmat<T>& m) { return m.expr(); }

// ---- operators ---------------------------------------------------------------

struct op_add { template <class C> __device__ static C apply(C a, C b) { return a + b; } };
struct op_sub { template <class C> __device__ static C apply(C a, C b) { return a - b; } };
struct op_schur { template <class C> __device__ static C apply(C a, C b) { return a * b; } };
struct op_div { template <class C> __device__ static C apply(C a, C b) { return a / b; } };
struct op_xor {
  __device__ static uint32_t apply(uint32_t a, uint32_t b) { return a ^ b; }
};
struct op_neg { template <class C> __device__ static C apply(C a) { return -a; } };
struct op_abs {
  __device__ static float apply(float a) { return ::fabsf(a); }
  __device__ static double apply(double a) { return ::fabs(a); }
};
struct op_exp {
  __device__ static float apply(float a) { return ::expf(a); }
  __device__ static double apply(double a) { return ::exp(a); }
};
struct op_sqrt {
  __device__ static float apply(float a) { return ::sqrtf(a); }
  __device__ static double apply(double a) { return ::sqrt(a); }
};

// ---- inner nodes ---------------------------------------------------------------

template <class Op, class A> struct Unary : expr_tag {
  using ct = typename A::ct;
  using storage = typename A::storage;
  A a;
  __device__ __forceinline__ ct at(int64_t i) const { return Op::apply(a.at(i)); }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x = a.template at_vec<N, NT>(i);
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = Op::apply(x.v[j]);
    return x;
  }
  void collect(leaf_info& li) const { a.collect(li); }
};

template <class Op, class A, class B> struct Binary : expr_tag {
  static_assert(std::is_same_v<typename A::ct, typename B::ct>,
                "operands of an element-wise operator share one compute type");
  using ct = typename A::ct;
  using storage = typename A::storage;
  A a;
  B b;
  __device__ __forceinline__ ct at(int64_t i) const { return Op::apply(a.at(i), b.at(i)); }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x = a.template at_vec<N, NT>(i);
    lanes<ct, N> y = b.template at_vec<N, NT>(i);
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = Op::apply(x.v[j], y.v[j]);
    return x;
  }
  void collect(leaf_info& li) const { a.collect(li); b.collect(li); }
};

// k op child (LEFT = true) or child op k: the scalar node of Sec. 3, which
// adds `aux` to the child's element access.
template <class Op, class A, bool LEFT> struct Scalar : expr_tag {
  using ct = typename A::ct;
  using storage = typename A::storage;
  A a;
  ct k;
  __device__ __forceinline__ ct apply1(ct x) const {
    return LEFT ? Op::apply(k, x) : Op::apply(x, k);
  }
  __device__ __forceinline__ ct at(int64_t i) const { return apply1(a.at(i)); }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x = a.template at_vec<N, NT>(i);
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = apply1(x.v[j]);
    return x;
  }
  void collect(leaf_info& li) const { a.collect(li); }
};

// ---- operator overloads (host side: they build the type) -------------------------

template <class E> using expr_of = std::decay_t<decltype(as_expr(std::declval<E>()))>;
template <class E> constexpr bool is_operand_v =
    is_expr_v<std::decay_t<E>> || std::is_same_v<std::decay_t<E>, dmat<float>> ||
    std::is_same_v<std::decay_t<E>, dmat<double>> ||
    std::is_same_v<std::decay_t<E>, dmat<bf16_t>> ||
    std::is_same_v<std::decay_t<E>, dmat<f16_t>> ||
    std::is_same_v<std::decay_t<E>, dmat<uint32_t>>;
template <class E> constexpr bool is_scalar_v = std::is_arithmetic_v<std::decay_t<E>>;

#define FX_BINARY_OPERATOR(SYM, OP)                                                     \
  template <class A, class B, std::enable_if_t<is_operand_v<A> && is_operand_v<B>, int> = 0> \
  inline auto operator SYM(const A& a, const B& b) {                                   \
    return Binary<OP, expr_of<A>, expr_of<B>>{{}, as_expr(a), as_expr(b)};              \
  }                                                                                     \
  template <class A, class S, std::enable_if_t<is_operand_v<A> && is_scalar_v<S>, int> = 0> \
  inline auto operator SYM(const A& a, S k) {                                          \
    using E = expr_of<A>;                                                               \
    return Scalar<OP, E, false>{{}, as_expr(a), static_cast<typename E::ct>(k)};        \
  }                                                                                     \
  template <class S, class A, std::enable_if_t<is_scalar_v<S> && is_operand_v<A>, int> = 0> \
  inline auto operator SYM(S k, const A& a) {                                          \
    using E = expr_of<A>;                                                               \
    return Scalar<OP, E, true>{{}, as_expr(a), static_cast<typename E::ct>(k)};         \
  }

FX_BINARY_OPERATOR(+, op_add)
FX_BINARY_OPERATOR(-, op_sub)
FX_BINARY_OPERATOR(/, op_div)
#undef FX_BINARY_OPERATOR

// % is the Schur (element-wise) product between expressions (Sec. 4);
// * is only defined with a scalar (the matrix product is not element-wise).
template <class A, class B, std::enable_if_t<is_operand_v<A> && is_operand_v<B>, int> = 0>
inline auto operator%(const A& a, const B& b) {
  return Binary<op_schur, expr_of<A>, expr_of<B>>{{}, as_expr(a), as_expr(b)};
}
template <class A, class S, std::enable_if_t<is_operand_v<A> && is_scalar_v<S>, int> = 0>
inline auto operator*(const A& a, S k) {
  using E = expr_of<A>;
  return Scalar<op_schur, E, false>{{}, as_expr(a), static_cast<typename E::ct>(k)};
}
template <class S, class A, std::enable_if_t<is_scalar_v<S> && is_operand_v<A>, int> = 0>
inline auto operator*(S k, const A& a) {
  using E = expr_of<A>;
  return Scalar<op_schur, E, true>{{}, as_expr(a), static_cast<typename E::ct>(k)};
}
// ^ is bitwise XOR, defined for u32 expressions only.
template <class A, class B, std::enable_if_t<is_operand_v<A> && is_operand_v<B>, int> = 0>
inline auto operator^(const A& a, const B& b) {
  static_assert(std::is_same_v<typename expr_of<A>::ct, uint32_t>, "XOR needs u32 operands");
  return Binary<op_xor, expr_of<A>, expr_of<B>>{{}, as_expr(a), as_expr(b)};
}
template <class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto operator-(const A& a) {
  return Unary<op_neg, expr_of<A>>{{}, as_expr(a)};
}
template <class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto exp(const A& a) { return Unary<op_exp, expr_of<A>>{{}, as_expr(a)}; }
template <class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto abs(const A& a) { return Unary<op_abs, expr_of<A>>{{}, as_expr(a)}; }
template <class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto sqrt(const A& a) { return Unary<op_sqrt, expr_of<A>>{{}, as_expr(a)}; }

template <class E> inline leaf_info info_of(const E& e) {
  leaf_info li;
  e.collect(li);
  return li;
}

}  // namespace fx
