// Compile-time kernel source from an expression's type (Sec. 3, kernel
// generation): the front end's expression type is walked at compile time,
// node by node, by partial specialisation, and each node contributes the
// text of its element-access rule:
//   leaf k            x<k>                     (the k-th leaf occurrence)
//   unary node        f(<child>)
//   binary node       (<left> op <right>)
//   scalar node       (k<j> op <child>) or (<child> op k<j>)   (the j-th scalar)
// With the leaves' parameter list, their loads and the whole-kernel
// skeleton text, this gives the complete source of one fused kernel as a
// compile-time string constant embedded in the library (src_kernel<...>::
// text).  At first use the driver compiles it (hipRTC) and the code object is
// cached for the process; later calls only launch.
//
// As in the paper's generated kernels, every leaf occurrence is a kernel
// argument of its own (a matrix named three times is passed three times),
// and each scalar of the expression is a run-time argument (its value, the
// reciprocal or power shortcut the host chose, and that shortcut's mode).
// The element loop, the loads and the reductions are the skeleton text the
// run-time source mode uses too (fx_skel_src.hpp).
#pragma once

#include <math.h>

#include <atomic>
#include <type_traits>
#include <vector>

#include "fx_cstr.hpp"
#include "fx_jit.hpp"
#include "fx_kernels.hpp"
#include "fx_skel_src.hpp"

namespace fx {

// ---- names of the storage and compute types in the text ---------------------

template <class T> struct type_name;
template <> struct type_name<float> { static constexpr cstr name = "float"; };
template <> struct type_name<double> { static constexpr cstr name = "double"; };
template <> struct type_name<bf16_t> { static constexpr cstr name = "__bf16"; };
template <> struct type_name<f16_t> { static constexpr cstr name = "_Float16"; };
template <> struct type_name<uint32_t> { static constexpr cstr name = "unsigned int"; };

// ---- operator text ---------------------------------------------------------------

template <class Op, class C> struct unary_text;  // pre + child + post
template <class C> struct unary_text<op_neg, C> {
  static constexpr cstr pre = "(-"; static constexpr cstr post = ")";
};
template <> struct unary_text<op_abs, float> { static constexpr cstr pre = "__builtin_fabsf("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_abs, double> { static constexpr cstr pre = "__builtin_fabs("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_exp, float> { static constexpr cstr pre = "expf("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_exp, double> { static constexpr cstr pre = "exp("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_sqrt, float> { static constexpr cstr pre = "sqrtf("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_sqrt, double> { static constexpr cstr pre = "sqrt("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_log, float> { static constexpr cstr pre = "logf("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_log, double> { static constexpr cstr pre = "log("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_tanh, float> { static constexpr cstr pre = "tanhf("; static constexpr cstr post = ")"; };
template <> struct unary_text<op_tanh, double> { static constexpr cstr pre = "tanh("; static constexpr cstr post = ")"; };

template <class Op> struct infix_text;  // the operator between two operands
template <> struct infix_text<op_add> { static constexpr cstr op = " + "; };
template <> struct infix_text<op_sub> { static constexpr cstr op = " - "; };
template <> struct infix_text<op_schur> { static constexpr cstr op = " * "; };
template <> struct infix_text<op_div> { static constexpr cstr op = " / "; };
template <> struct infix_text<op_xor> { static constexpr cstr op = " ^ "; };

// ---- the element-access text of an expression type ------------------------------
//
// src<E, LOFF, SOFF>: E's element with its leaves numbered from LOFF and its
// scalars from SOFF (depth first, left to right: the order in which
// leaf_args / scalar_args below collect the run-time values).

template <class E, int LOFF, int SOFF> struct src {
  static_assert(sizeof(E) == 0, "this node type has no source rule");
};

template <class T, int LOFF, int SOFF> struct src<Leaf<T>, LOFF, SOFF> {
  static constexpr int leaves = 1, scalars = 0;
  static constexpr auto text = "x" + num<LOFF>();
};

template <class Op, class A, int LOFF, int SOFF> struct src<Unary<Op, A>, LOFF, SOFF> {
  using a = src<A, LOFF, SOFF>;
  static constexpr int leaves = a::leaves, scalars = a::scalars;
  using U = unary_text<Op, typename A::ct>;
  static constexpr auto text = U::pre + a::text + U::post;
};

template <class Op, class A, class B, int LOFF, int SOFF> struct src<Binary<Op, A, B>, LOFF, SOFF> {
  using a = src<A, LOFF, SOFF>;
  using b = src<B, LOFF + a::leaves, SOFF + a::scalars>;
  static constexpr int leaves = a::leaves + b::leaves, scalars = a::scalars + b::scalars;
  static constexpr auto text = "(" + a::text + infix_text<Op>::op + b::text + ")";
};
template <class A, class B, int LOFF, int SOFF> struct src<Binary<op_gt, A, B>, LOFF, SOFF> {
  using a = src<A, LOFF, SOFF>;
  using b = src<B, LOFF + a::leaves, SOFF + a::scalars>;
  static constexpr int leaves = a::leaves + b::leaves, scalars = a::scalars + b::scalars;
  static constexpr auto text = "(" + a::text + " > " + b::text + " ? (ct_t)1 : (ct_t)0)";
};

// A scalar node is scalar SOFF; its child's scalars follow it.  Its value is
// kernel argument k<j>, the reciprocal shortcut q<j>, the shortcut mode m<j>.
template <class Op, class A, bool LEFT, int LOFF, int SOFF>
struct src<Scalar<Op, A, LEFT>, LOFF, SOFF> {
  using a = src<A, LOFF, SOFF + 1>;
  static constexpr int leaves = a::leaves, scalars = 1 + a::scalars;
  static constexpr auto j = num<SOFF>();
  static constexpr auto text_of() {
    if constexpr (std::is_same_v<Op, op_pow>) {
      return "fx_spow(" + a::text + ", k" + j + ", m" + j + ")";
    } else if constexpr (std::is_same_v<Op, op_div> && !LEFT) {
      return "fx_sdiv(" + a::text + ", k" + j + ", q" + j + ", m" + j + ")";
    } else if constexpr (std::is_same_v<Op, op_gt>) {
      return "(" + a::text + " > k" + j + " ? (ct_t)1 : (ct_t)0)";
    } else if constexpr (LEFT) {
      return "(k" + j + infix_text<Op>::op + a::text + ")";
    } else {
      return "(" + a::text + infix_text<Op>::op + "k" + j + ")";
    }
  }
  static constexpr auto text = text_of();
};

// ---- run-time values of the kernel arguments -------------------------------------

struct scalar_arg {
  double k, aux;  // the value and its reciprocal shortcut, in the compute type
  int32_t mode;
};

template <class T> void leaf_args(const Leaf<T>& e, std::vector<const void*>& p) { p.push_back(e.p); }
template <class Op, class A> void leaf_args(const Unary<Op, A>& e, std::vector<const void*>& p) {
  leaf_args(e.a, p);
}
template <class Op, class A, class B>
void leaf_args(const Binary<Op, A, B>& e, std::vector<const void*>& p) {
  leaf_args(e.a, p);
  leaf_args(e.b, p);
}
template <class Op, class A, bool L> void leaf_args(const Scalar<Op, A, L>& e, std::vector<const void*>& p) {
  leaf_args(e.a, p);
}

template <class T> void scalar_args(const Leaf<T>&, std::vector<scalar_arg>&) {}
template <class Op, class A> void scalar_args(const Unary<Op, A>& e, std::vector<scalar_arg>& s) {
  scalar_args(e.a, s);
}
template <class Op, class A, class B>
void scalar_args(const Binary<Op, A, B>& e, std::vector<scalar_arg>& s) {
  scalar_args(e.a, s);
  scalar_args(e.b, s);
}
template <class Op, class A, bool L> void scalar_args(const Scalar<Op, A, L>& e, std::vector<scalar_arg>& s) {
  s.push_back(scalar_arg{(double)e.k, (double)e.aux, e.mode});
  scalar_args(e.a, s);
}

// ---- the generated part of the program text ------------------------------------

// "<pre>0<post><sep><pre>1<post>...": K numbered items (empty for K = 0)
template <int I, int K, size_t P, size_t Q, size_t S>
constexpr auto numbered(const char (&pre)[P], const char (&post)[Q], const char (&sep)[S]) {
  if constexpr (I >= K) return cstr<0>();
  else if constexpr (I + 1 == K) return pre + num<I>() + post;
  else return pre + num<I>() + post + sep + numbered<I + 1, K>(pre, post, sep);
}

// ", ct_t k0, ct_t q0, int m0, ..." and ", k0, q0, m0, ..." for J scalars
template <int I, int J> constexpr auto scalar_params() {
  if constexpr (I >= J) return cstr<0>();
  else return ", ct_t k" + num<I>() + ", ct_t q" + num<I>() + ", int m" + num<I>() +
              scalar_params<I + 1, J>();
}
template <int I, int J> constexpr auto scalar_names() {
  if constexpr (I >= J) return cstr<0>();
  else return ", k" + num<I>() + ", q" + num<I>() + ", m" + num<I>() + scalar_names<I + 1, J>();
}

// one load per leaf occurrence, and the leaves' values for fx_expr
template <int I, int L> constexpr auto load_lines() {
  if constexpr (I >= L) return cstr<0>();
  else return "  fx_ld<N>::run(p" + num<I>() + " + i, r.v[" + num<I>() + "]);\n" +
              load_lines<I + 1, L>();
}
template <int I, int L> constexpr auto lane_values() {
  if constexpr (I + 1 >= L) return "(ct_t)r.v[" + num<I>() + "][j]";
  else return "(ct_t)r.v[" + num<I>() + "][j], " + lane_values<I + 1, L>();
}
template <int I, int L> constexpr auto element_values() {
  if constexpr (I + 1 >= L) return "(ct_t)p" + num<I>() + "[i]";
  else return "(ct_t)p" + num<I>() + "[i], " + element_values<I + 1, L>();
}

template <class C> constexpr auto pow_name() {
  if constexpr (std::is_same_v<C, float>) return cstr("powf");
  else return cstr("pow");
}

// Scalar-node shortcuts the host may choose (the modes of the front end's
// scalar node): x / k as x * (1/k) when that is exact, pow(x, 1..4) as
// products.
template <class C> constexpr auto scalar_helpers() {
  auto div = "__device__ __forceinline__ ct_t fx_sdiv(ct_t x, ct_t k, ct_t q, int m) {\n"
             "  return m == " + num<SC_MUL_INV>() + " ? x * q : x / k;\n}\n";
  if constexpr (std::is_floating_point_v<C>) {
    return div + "__device__ __forceinline__ ct_t fx_spow(ct_t x, ct_t k, int m) {\n"
                 "  if (m == " + num<SC_POW1>() + ") return x;\n"
                 "  if (m == " + num<SC_POW2>() + ") return x * x;\n"
                 "  if (m == " + num<SC_POW3>() + ") return (x * x) * x;\n"
                 "  if (m == " + num<SC_POW4>() + ") { const ct_t x2 = x * x; return x2 * x2; }\n"
                 "  return " + pow_name<C>() + "(x, k);\n}\n";
  } else {
    return div;
  }
}

template <int KIND> constexpr auto map_text() {
  if constexpr (KIND == FX_R_NORM)
    return cstr("#define FX_MAP(x) ((x) * (x))\n#define FX_FINISH(s) __builtin_sqrt(s)\n");
  else
    return cstr("#define FX_MAP(x) (x)\n#define FX_FINISH(s) (s)\n");
}

template <int KIND> constexpr auto skeleton_text() {
  if constexpr (KIND == 0) return cstr(kElementwise);
  else if constexpr (KIND == FX_R_COLSUM) return kSums + cstr(kColsum);
  else if constexpr (KIND == FX_R_ROWSUM) return kSums + cstr(kRowsum);
  else return kSums + cstr(kFull);
}

// The complete program text of expression type E over storage T for result
// kind KIND (0 element-wise, FX_R_ACCU, FX_R_NORM, FX_R_COLSUM, FX_R_ROWSUM).
template <class E, class T, int KIND> constexpr auto program_text() {
  using S = src<E, 0, 0>;
  using C = typename E::ct;
  static_assert(KIND == 0 || std::is_floating_point_v<C>,
                "generated reductions are compensated floating-point sums");
  constexpr int L = S::leaves, J = S::scalars;
  constexpr int elem = (int)sizeof(T);
  constexpr int rk = KIND == FX_R_NORM ? FX_R_ACCU : KIND;
  using O = std::conditional_t<std::is_same_v<C, double>, double, float>;
  return "// generated at compile time from an expression type\n"
         "typedef " + type_name<T>::name + " st_t;\n"
         "typedef " + type_name<C>::name + " ct_t;\n"
         "typedef " + type_name<O>::name + " acc_out_t;\n"
         "#define FX_N " + num<16 / elem>() + "\n"
         "#define FX_NIN " + num<L>() + "\n"
         "#define FX_BLOCK " + num<default_block(rk, elem)>() + "\n"
         "#define FX_EPT " + num<default_ept(rk, elem)>() + "\n" + map_text<KIND>() +
         "#define FX_PARAMS " + numbered<0, L>("const st_t* __restrict__ p", "", ", ") +
         scalar_params<0, J>() + "\n#define FX_ARGS " + numbered<0, L>("p", "", ", ") +
         scalar_names<0, J>() + "\n" + kLoads + scalar_helpers<C>() +
         "__device__ __forceinline__ ct_t fx_expr(" + numbered<0, L>("ct_t x", "", ", ") +
         scalar_params<0, J>() + ") {\n  return " + S::text + ";\n}\n"
         "template <int N> __device__ __forceinline__ void fx_load(FX_PARAMS, long i, "
         "fx_raw<N>& r) {\n" + load_lines<0, L>() + "}\n"
         "template <int N> __device__ __forceinline__ void fx_eval(FX_PARAMS, const fx_raw<N>& r, "
         "ct_t* o) {\n#pragma unroll\n  for (int j = 0; j < N; ++j) o[j] = fx_expr(" +
         lane_values<0, L>() + scalar_names<0, J>() + ");\n}\n"
         "__device__ __forceinline__ ct_t fx_at(FX_PARAMS, long i) {\n  return fx_expr(" +
         element_values<0, L>() + scalar_names<0, J>() + ");\n}\n" + skeleton_text<KIND>();
}

// One generated kernel: its text, a constant of the program, and the compiled
// program, obtained through the driver at first use and kept.
template <class E, class T, int KIND> struct src_kernel {
  static constexpr auto text = program_text<E, T, KIND>();
  static inline std::atomic<jit_program*> prog{nullptr};
  static inline double compile_ms = 0;  // the first use's compilation time
  static int obtain(jit_program** p) {
    jit_program* q = prog.load(std::memory_order_acquire);
    if (!q) {
      double ms = 0;
      if (int rc = jit_obtain(text.data(), text.size, &q, &ms)) return rc;
      jit_program* expected = nullptr;
      if (prog.compare_exchange_strong(expected, q)) compile_ms = ms;
    }
    *p = q;
    return FX_OK;
  }
};

// Evaluate expression e through its generated kernel: out is Z (element-wise,
// storage type), a double (accu / norm) or the accumulator-type dimension
// sums.  Needs 16-byte aligned arrays (the text's loads are 16-byte vectors).
template <int KIND, class E>
int eval_source(const E& e, void* out, void* ws, size_t ws_bytes, hipStream_t st) {
  using T = typename E::storage;
  using C = typename E::ct;
  using O = std::conditional_t<std::is_same_v<C, double>, double, float>;
  using K = src_kernel<E, T, KIND>;
  constexpr int elem = (int)sizeof(T);
  constexpr bool full = KIND == FX_R_ACCU || KIND == FX_R_NORM;
  constexpr int rk = KIND == FX_R_NORM ? FX_R_ACCU : KIND;
  int64_t rows, cols;
  if (int rc = check_expr(e, &rows, &cols)) return rc;
  const int64_t n = rows * cols;
  const int64_t nout = KIND == 0 ? n : KIND == FX_R_COLSUM ? cols : KIND == FX_R_ROWSUM ? rows : 1;
  if (nout == 0) return FX_OK;
  if (!out) return fail(FX_E_ARG, "NULL output pointer");
  std::vector<const void*> ptrs;
  leaf_args(e, ptrs);
  uintptr_t addr_or = KIND == 0 ? reinterpret_cast<uintptr_t>(out) : 0;
  for (const void* p : ptrs) addr_or |= reinterpret_cast<uintptr_t>(p);
  if (addr_or & 15) return fail(FX_E_ARG, "the generated kernels need 16-byte aligned arrays");
  if (n == 0 && !full) {  // sums over an empty dimension
    const int grid = (int)std::min<int64_t>(ceil_div(nout, 256), 1024);
    hipLaunchKernelGGL((k_fill_zero<O>), dim3(grid), dim3(256), 0, st, static_cast<O*>(out), nout);
    return hip_check(hipGetLastError(), "k_fill_zero launch");
  }
  const launch L = resolve(rk, elem, rows, cols, nullptr, true);
  constexpr int N = 16 / elem;
  const int vec = KIND == 0 || full || rows % N == 0 ? N : 1;
  const ws_layout W = workspace_for(rk, rows, cols, L, vec);
  if (W.total() > 0 && (!ws || ws_bytes < W.total()))
    return fail(FX_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", W.total(), ws_bytes);
  jit_program* prog = nullptr;
  if (int rc = K::obtain(&prog)) return rc;
  const char* names[2] = {nullptr, nullptr};
  skeleton_kernels(KIND, names);
  const char* name = (KIND == FX_R_COLSUM || KIND == FX_R_ROWSUM) && vec == 1 ? names[1] : names[0];
  hipFunction_t fn;
  if (int rc = jit_function(prog, name, &fn)) return rc;
  // kernel arguments: the leaves, the scalars, then the skeleton's own
  std::vector<scalar_arg> sc;
  scalar_args(e, sc);
  std::vector<C> kv(sc.size()), qv(sc.size());
  std::vector<int> mv(sc.size());
  std::vector<void*> args;
  for (auto& p : ptrs) args.push_back(&p);
  for (size_t j = 0; j < sc.size(); ++j) {
    kv[j] = (C)sc[j].k;
    qv[j] = (C)sc[j].aux;
    mv[j] = sc[j].mode;
    args.push_back(&kv[j]);
    args.push_back(&qv[j]);
    args.push_back(&mv[j]);
  }
  long n_l = (long)n, rows_l = (long)rows, cols_l = (long)cols;
  void* o = out;
  void* parts = W.total() > 0 ? static_cast<char*>(ws) + W.counter_bytes : nullptr;
  void* ctr = W.total() > 0 ? ws : nullptr;
  int split = std::max(1, L.split);  // thin columns run as one chunk per column
  long rpc = 0, cpc = 0;
  if constexpr (KIND == 0) {
    args.insert(args.end(), {&o, &n_l});
    return jit_launch(fn, L.split, 1, L.block, args.data(), st);
  } else if constexpr (full) {
    args.insert(args.end(), {&n_l, &parts, &ctr, &o});
    return jit_launch(fn, L.split, 1, L.block, args.data(), st);
  } else if constexpr (KIND == FX_R_COLSUM) {
    rpc = (long)(ceil_div(ceil_div(rows, split), vec) * vec);
    args.insert(args.end(), {&rows_l, &split, &rpc, &parts, &ctr, &o});
    return jit_launch(fn, cols, split, L.block, args.data(), st);
  } else {
    cpc = (long)ceil_div(cols, split);
    args.insert(args.end(), {&rows_l, &cols_l, &split, &cpc, &parts, &ctr, &o});
    return jit_launch(fn, ceil_div(rows, (int64_t)L.block * vec), split, L.block, args.data(), st);
  }
}

}  // namespace fx
