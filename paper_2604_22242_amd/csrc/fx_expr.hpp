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

#include <cmath>

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

// Identity of a leaf for de-duplication: the same address read as the same
// storage type.
struct leaf_id {
  const void* p;
  size_t size;
  int kind;
};
template <class T> constexpr int kind_of() {
  return std::is_same_v<T, float> ? 0 : std::is_same_v<T, double> ? 1
       : std::is_same_v<T, bf16_t> ? 2 : std::is_same_v<T, f16_t> ? 3 : 4;
}

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
  // two-phase evaluation (see Fused below): this leaf is register leaf OFF
  static constexpr int kLeaves = 1;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R* regs, const uint8_t* alias, int64_t i) const {
    if (!alias || alias[OFF] == OFF) regs[OFF] = load_lanes<N, NT>(p, i);
  }
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R* regs, int64_t) const {
    return regs[OFF];
  }
  void leaf_ids(leaf_id* out, int& k) const { out[k++] = leaf_id{p, sizeof(T), kind_of<T>()}; }
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
struct op_log {
  __device__ static float apply(float a) { return ::logf(a); }
  __device__ static double apply(double a) { return ::log(a); }
};
struct op_tanh {
  __device__ static float apply(float a) { return ::tanhf(a); }
  __device__ static double apply(double a) { return ::tanh(a); }
};
// a^k for a scalar exponent k
struct op_pow {
  __device__ static float apply(float a, float k) { return ::powf(a, k); }
  __device__ static double apply(double a, double k) { return ::pow(a, k); }
};
// a > b as 1 or 0 of the compute type (a relational operator yields a 0/1
// matrix that the Schur product can use)
struct op_gt {
  template <class C> __device__ static C apply(C a, C b) { return a > b ? C(1) : C(0); }
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
  static constexpr int kLeaves = A::kLeaves;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R* regs, const uint8_t* alias, int64_t i) const {
    a.template gather<OFF, N, NT>(regs, alias, i);
  }
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R* regs, int64_t i) const {
    lanes<ct, N> x = a.template at_regs<OFF, N, NT>(regs, i);
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = Op::apply(x.v[j]);
    return x;
  }
  void leaf_ids(leaf_id* out, int& k) const { a.leaf_ids(out, k); }
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
  static constexpr int kLeaves = A::kLeaves + B::kLeaves;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R* regs, const uint8_t* alias, int64_t i) const {
    a.template gather<OFF, N, NT>(regs, alias, i);
    b.template gather<OFF + A::kLeaves, N, NT>(regs, alias, i);
  }
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R* regs, int64_t i) const {
    lanes<ct, N> x = a.template at_regs<OFF, N, NT>(regs, i);
    lanes<ct, N> y = b.template at_regs<OFF + A::kLeaves, N, NT>(regs, i);
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = Op::apply(x.v[j], y.v[j]);
    return x;
  }
  void leaf_ids(leaf_id* out, int& k) const { a.leaf_ids(out, k); b.leaf_ids(out, k); }
};

// k op child (LEFT = true) or child op k: the scalar node of Sec. 3, which
// adds `aux` to the child's element access.
// Scalar-operand shortcuts chosen on the host when the node is built (the
// scalar is a run-time value): x / k with k a power of two whose reciprocal
// is exact becomes x * (1/k), bitwise the same; pow(x, k) for k = 1..4 is a
// product of x's (k = 2 is correctly rounded like pow; k = 3, 4 take two
// roundings, inside pow's error allowance).
enum : int32_t { SC_PLAIN = 0, SC_MUL_INV = 1, SC_POW1 = 2, SC_POW2, SC_POW3, SC_POW4 };

template <class Op, class A, bool LEFT> struct Scalar : expr_tag {
  using ct = typename A::ct;
  using storage = typename A::storage;
  A a;
  ct k;
  ct aux = ct(0);          // 1/k for SC_MUL_INV
  int32_t mode = SC_PLAIN;
  __device__ __forceinline__ ct apply1(ct x) const {
    if constexpr (std::is_same_v<Op, op_div> && !LEFT) {
      if (mode == SC_MUL_INV) return x * aux;
    }
    if constexpr (std::is_same_v<Op, op_pow>) {
      switch (mode) {
        case SC_POW1: return x;
        case SC_POW2: return x * x;
        case SC_POW3: return (x * x) * x;
        case SC_POW4: { const ct x2 = x * x; return x2 * x2; }
        default: break;
      }
    }
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
  static constexpr int kLeaves = A::kLeaves;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R* regs, const uint8_t* alias, int64_t i) const {
    a.template gather<OFF, N, NT>(regs, alias, i);
  }
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R* regs, int64_t i) const {
    lanes<ct, N> x = a.template at_regs<OFF, N, NT>(regs, i);
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = apply1(x.v[j]);
    return x;
  }
  void leaf_ids(leaf_id* out, int& k) const { a.leaf_ids(out, k); }
};

// conv_to<To>::from(child): the child's elements converted to compute type To
// (rounded to nearest-even when narrowing), so a leaf of another storage type
// can take part in the expression.
template <class To, class A> struct Convert : expr_tag {
  using ct = To;
  using storage = To;
  A a;
  __device__ __forceinline__ ct at(int64_t i) const { return static_cast<To>(a.at(i)); }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<typename A::ct, N> x = a.template at_vec<N, NT>(i);
    lanes<ct, N> r;
#pragma unroll
    for (int j = 0; j < N; ++j) r.v[j] = static_cast<To>(x.v[j]);
    return r;
  }
  void collect(leaf_info& li) const { a.collect(li); }
  // another compute type below: evaluated in place, its leaves not shared
  static constexpr int kLeaves = 0;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R*, const uint8_t*, int64_t) const {}
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R*, int64_t i) const {
    return at_vec<N, NT>(i);
  }
  void leaf_ids(leaf_id*, int&) const {}
};

// A1 + A2 + ... + AK over K leaves of one storage type, added left to right
// as the nested binary form would (the add-N expressions of Sec. 4).
template <class T, int K> struct SumN : expr_tag {
  using storage = T;
  using ct = ct_t<T>;
  const T* p[K];
  int64_t n_rows, n_cols;
  __device__ __forceinline__ ct at(int64_t i) const {
    ct s = static_cast<ct>(p[0][i]);
#pragma unroll
    for (int q = 1; q < K; ++q) s = s + static_cast<ct>(p[q][i]);
    return s;
  }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x[K];
#pragma unroll
    for (int q = 0; q < K; ++q) x[q] = load_lanes<N, NT>(p[q], i);
#pragma unroll
    for (int q = 1; q < K; ++q)
#pragma unroll
      for (int j = 0; j < N; ++j) x[0].v[j] = x[0].v[j] + x[q].v[j];
    return x[0];
  }
  void collect(leaf_info& li) const {
    for (int q = 0; q < K; ++q) li.add(p[q], n_rows, n_cols);
  }
  // its K loads are issued together already
  static constexpr int kLeaves = 0;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R*, const uint8_t*, int64_t) const {}
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R*, int64_t i) const {
    return at_vec<N, NT>(i);
  }
  void leaf_ids(leaf_id*, int&) const {}
};

// ---- reading a repeated leaf once -----------------------------------------
//
// An expression may name the same matrix several times ((X+Y)/(1+X%X)); each
// occurrence is its own leaf with its own pointer, so the compiler cannot
// merge their loads.  Fused<E> evaluates E in two phases: gather() loads
// every register leaf whose address and storage type were not already seen
// (in depth-first order; the host computes alias[k], the first leaf equal to
// leaf k), the repeats are copied register to register, and at_regs()
// evaluates the tree from those registers.  Leaf indices are fixed at
// compile time by the traversal, so no register is indexed at run time.
// The loads sit behind uniform branches, which makes the compiler wait for
// all of them before any arithmetic; the drivers therefore take Fused<E>
// only when some leaf does repeat.  Without repeats the same two phases run
// with no alias table (a null `alias`): every register leaf is loaded
// unconditionally, so the waits follow the loads one by one.
constexpr int kMaxFusedLeaves = 16;

template <class E, class = void> struct leaves_of { static constexpr int value = 0; };
template <class E> struct leaves_of<E, std::void_t<decltype(E::kLeaves)>> {
  static constexpr int value = E::kLeaves;
};

template <class E> struct Fused : expr_tag {
  using ct = typename E::ct;
  using storage = typename E::storage;
  static constexpr int L = E::kLeaves;
  static_assert(L >= 1 && L <= kMaxFusedLeaves, "register-leaf count out of range");
  E e;
  uint8_t alias[L];

  __device__ __forceinline__ ct at(int64_t i) const { return e.at(i); }
  // regs[k] for the first occurrence k of a leaf, copies for the repeats
  template <int N>
  __device__ __forceinline__ void resolve(lanes<ct, N>* regs) const {
#pragma unroll
    for (int k = 1; k < L; ++k)
#pragma unroll
      for (int j = 0; j < k; ++j)
        if (alias[k] == j) regs[k] = regs[j];
  }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> regs[L];
    e.template gather<0, N, NT>(regs, alias, i);
    resolve<N>(regs);
    return e.template at_regs<0, N, NT>(regs, i);
  }
  void collect(leaf_info& li) const { e.collect(li); }
  bool has_alias() const {
    for (int k = 0; k < L; ++k)
      if (alias[k] != k) return true;
    return false;
  }
};

// Host: wrap E when it has two or more register leaves.
template <class E> inline auto fuse_leaves(const E& e) {
  if constexpr (leaves_of<E>::value >= 2 && leaves_of<E>::value <= kMaxFusedLeaves) {
    Fused<E> f;
    f.e = e;
    leaf_id ids[kMaxFusedLeaves];
    int k = 0;
    e.leaf_ids(ids, k);
    for (int a = 0; a < Fused<E>::L; ++a) {
      f.alias[a] = (uint8_t)a;
      for (int b = 0; b < a; ++b)
        if (ids[b].p == ids[a].p && ids[b].size == ids[a].size && ids[b].kind == ids[a].kind) {
          f.alias[a] = (uint8_t)b;
          break;
        }
    }
    return f;
  } else {
    return e;
  }
}

// ---- operator overloads (host side: they build the type) -------------------------

template <class E> using expr_of = std::decay_t<decltype(as_expr(std::declval<E>()))>;
template <class E> constexpr bool is_operand_v =
    is_expr_v<std::decay_t<E>> || std::is_same_v<std::decay_t<E>, dmat<float>> ||
    std::is_same_v<std::decay_t<E>, dmat<double>> ||
    std::is_same_v<std::decay_t<E>, dmat<bf16_t>> ||
    std::is_same_v<std::decay_t<E>, dmat<f16_t>> ||
    std::is_same_v<std::decay_t<E>, dmat<uint32_t>>;
template <class E> constexpr bool is_scalar_v = std::is_arithmetic_v<std::decay_t<E>>;

// Host: pick the shortcut of a freshly built scalar node.
template <class Op, class E, bool LEFT> inline Scalar<Op, E, LEFT> tune_scalar(Scalar<Op, E, LEFT> s) {
  using C = typename E::ct;
  if constexpr (std::is_same_v<Op, op_div> && !LEFT && std::is_floating_point_v<C>) {
    int e = 0;
    const C m = std::frexp(s.k, &e);  // k = m * 2^e, |m| in [0.5, 1)
    const C inv = C(1) / s.k;
    if ((m == C(0.5) || m == C(-0.5)) && std::isnormal(s.k) && std::isnormal(inv)) {
      s.mode = SC_MUL_INV;
      s.aux = inv;
    }
  }
  if constexpr (std::is_same_v<Op, op_pow>) {
    if (s.k == C(1)) s.mode = SC_POW1;
    else if (s.k == C(2)) s.mode = SC_POW2;
    else if (s.k == C(3)) s.mode = SC_POW3;
    else if (s.k == C(4)) s.mode = SC_POW4;
  }
  return s;
}

#define FX_BINARY_OPERATOR(SYM, OP)                                                     \
  template <class A, class B, std::enable_if_t<is_operand_v<A> && is_operand_v<B>, int> = 0> \
  inline auto operator SYM(const A& a, const B& b) {                                   \
    return Binary<OP, expr_of<A>, expr_of<B>>{{}, as_expr(a), as_expr(b)};              \
  }                                                                                     \
  template <class A, class S, std::enable_if_t<is_operand_v<A> && is_scalar_v<S>, int> = 0> \
  inline auto operator SYM(const A& a, S k) {                                          \
    using E = expr_of<A>;                                                               \
    return tune_scalar(Scalar<OP, E, false>{{}, as_expr(a), static_cast<typename E::ct>(k)}); \
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
template <class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto log(const A& a) { return Unary<op_log, expr_of<A>>{{}, as_expr(a)}; }
template <class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto tanh(const A& a) { return Unary<op_tanh, expr_of<A>>{{}, as_expr(a)}; }
template <class A, class S, std::enable_if_t<is_operand_v<A> && is_scalar_v<S>, int> = 0>
inline auto pow(const A& a, S k) {
  using E = expr_of<A>;
  return tune_scalar(Scalar<op_pow, E, false>{{}, as_expr(a), static_cast<typename E::ct>(k)});
}
template <class A, class S, std::enable_if_t<is_operand_v<A> && is_scalar_v<S>, int> = 0>
inline auto operator>(const A& a, S k) {
  using E = expr_of<A>;
  return Scalar<op_gt, E, false>{{}, as_expr(a), static_cast<typename E::ct>(k)};
}
// conv_to<To>(A): Armadillo's conv_to<Mat<To>>::from(A)
template <class To, class A, std::enable_if_t<is_operand_v<A>, int> = 0>
inline auto conv_to(const A& a) { return Convert<To, expr_of<A>>{{}, as_expr(a)}; }

template <class E> inline leaf_info info_of(const E& e) {
  leaf_info li;
  e.collect(li);
  return li;
}

}  // namespace fx
