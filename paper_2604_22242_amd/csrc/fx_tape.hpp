// Run-time expression tapes.
//
// Expressions whose tree is only known at run time cannot be C++ types, so
// the host compiles the tree into a short register program (three-address
// code over at most kTapeMaxSlots slots, constants as immediates) and the
// device interprets it per element.  The program travels inside the kernel
// argument, so every instruction fetch is a wave-uniform scalar load.  Each
// lane's slot file is one 16-wide vector value indexed with those uniform
// slot numbers, which gfx950 serves from VGPRs in indexed mode
// (s_set_gpr_idx_on) rather than from private memory; lanes are interpreted
// in passes of 4 (FP32 compute) or 2 (FP64) so the files stay in registers.  TapeExpr<T> has the same
// interface as a compile-time expression, so the element-wise, full
// reduction, column-sum and row-sum skeletons (and their single-pass
// finish) serve tapes unchanged; its eval_tile overload loads every input
// of all EPT vectors before interpreting them one vector at a time.
#pragma once

#include "fx_kernels.hpp"

namespace fx {

constexpr int kTapeMaxIn = 4;
constexpr int kTapeMaxIns = 128;
constexpr int kTapeMaxSlots = 16;
constexpr uint8_t kImm = 0xFF;

enum : uint8_t { T_ADD = 0, T_SUB, T_MUL, T_DIV, T_NEG, T_ABS, T_EXP, T_SQRT, T_MOV };

struct tape_ins {
  uint8_t op, dst, a, b;  // a/b: slot index or kImm
  float kf;               // immediate for FP32 compute
  double kd;              // immediate for FP64 compute
};

struct tape_prog {
  int32_t n_ins, n_in, root, n_slots;
  tape_ins ins[kTapeMaxIns];
};

template <class C> __device__ __forceinline__ C tape_imm(const tape_ins& I);
template <> __device__ __forceinline__ float tape_imm<float>(const tape_ins& I) { return I.kf; }
template <> __device__ __forceinline__ double tape_imm<double>(const tape_ins& I) { return I.kd; }

template <class C> struct slot_file;
template <> struct slot_file<float> { typedef float type __attribute__((ext_vector_type(16))); };
template <> struct slot_file<double> { typedef double type __attribute__((ext_vector_type(16))); };
template <class C> using slots_t = typename slot_file<C>::type;
template <class C> constexpr int kPassLanes = sizeof(C) == 4 ? 4 : 2;

// Interpret `prog` on L lanes whose inputs already sit in slots [0, n_in).
template <class C, int L>
__device__ __forceinline__ void tape_run(const tape_prog& prog, slots_t<C> (&s)[L]) {
  for (int pc = 0; pc < prog.n_ins; ++pc) {
    const tape_ins I = prog.ins[pc];
    const C k = tape_imm<C>(I);
    C x[L], y[L];
    if (I.a == kImm) {
#pragma unroll
      for (int j = 0; j < L; ++j) x[j] = k;
    } else {
#pragma unroll
      for (int j = 0; j < L; ++j) x[j] = s[j][I.a];
    }
    if (I.op <= T_DIV) {
      if (I.b == kImm) {
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = k;
      } else {
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = s[j][I.b];
      }
    }
    switch (I.op) {
      case T_ADD:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_add::apply(x[j], y[j]);
        break;
      case T_SUB:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_sub::apply(x[j], y[j]);
        break;
      case T_MUL:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_schur::apply(x[j], y[j]);
        break;
      case T_DIV:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_div::apply(x[j], y[j]);
        break;
      case T_NEG:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_neg::apply(x[j]);
        break;
      case T_ABS:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_abs::apply(x[j]);
        break;
      case T_EXP:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_exp::apply(x[j]);
        break;
      case T_SQRT:
#pragma unroll
        for (int j = 0; j < L; ++j) x[j] = op_sqrt::apply(x[j]);
        break;
      default:  // T_MOV
        break;
    }
#pragma unroll
    for (int j = 0; j < L; ++j) s[j][I.dst] = x[j];
  }
}

// BYREF = false: the program is held by value (it travels in the kernel
// argument); BYREF = true: it is read through a pointer into device memory
// (the batch kernel, where each tile may run a different program).
template <class T, bool BYREF = false> struct TapeExpr : expr_tag {
  using storage = T;
  using ct = ct_t<T>;
  const T* p[kTapeMaxIn];
  int64_t n_rows, n_cols;
  std::conditional_t<BYREF, const tape_prog*, tape_prog> prog;

  __host__ __device__ __forceinline__ const tape_prog& P() const {
    if constexpr (BYREF) return *prog;
    else return prog;
  }

  // Values of N lanes whose inputs are in[q].v[0..N): passes of G lanes.
  template <int N>
  __device__ __forceinline__ lanes<ct, N> interpret(const lanes<ct, N> (&in)[kTapeMaxIn]) const {
    constexpr int G = N < kPassLanes<ct> ? N : kPassLanes<ct>;
    const tape_prog& pr = P();
    lanes<ct, N> r;
#pragma unroll
    for (int g = 0; g < N; g += G) {
      slots_t<ct> s[G];
#pragma unroll
      for (int j = 0; j < G; ++j) {
        s[j] = slots_t<ct>{};
#pragma unroll
        for (int q = 0; q < kTapeMaxIn; ++q)
          if (q < pr.n_in) s[j][q] = in[q].v[g + j];
      }
      tape_run<ct, G>(pr, s);
#pragma unroll
      for (int j = 0; j < G; ++j) r.v[g + j] = s[j][pr.root];
    }
    return r;
  }
  __device__ __forceinline__ ct at(int64_t i) const {
    lanes<ct, 1> in[kTapeMaxIn];
    const int n_in = P().n_in;
#pragma unroll
    for (int q = 0; q < kTapeMaxIn; ++q) in[q].v[0] = q < n_in ? static_cast<ct>(p[q][i]) : ct(0);
    return interpret<1>(in).v[0];
  }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> in[kTapeMaxIn];
    const int n_in = P().n_in;
#pragma unroll
    for (int q = 0; q < kTapeMaxIn; ++q)
      if (q < n_in) in[q] = load_lanes<N, NT>(p[q], i);
    return interpret<N>(in);
  }
  void collect(leaf_info& li) const {
    for (int q = 0; q < P().n_in; ++q) li.add(p[q], n_rows, n_cols);
    if (P().n_in == 0) li.add_shape(n_rows, n_cols);
  }
};

template <int N, int EPT, class T, bool BYREF>
__device__ __forceinline__ void eval_tile(const TapeExpr<T, BYREF>& e, int64_t base, int64_t stride,
                                          lanes<ct_t<T>, N> (&r)[EPT]) {
  using C = ct_t<T>;
  lanes<C, N> in[EPT][kTapeMaxIn];
  const int n_in = e.P().n_in;
#pragma unroll
  for (int q = 0; q < kTapeMaxIn; ++q)
    if (q < n_in)
#pragma unroll
      for (int k = 0; k < EPT; ++k) in[k][q] = load_lanes<N, kNT>(e.p[q], base + k * stride);
#pragma unroll
  for (int k = 0; k < EPT; ++k) r[k] = e.template interpret<N>(in[k]);
}

template <class T, bool B> struct max_ept<TapeExpr<T, B>> { static constexpr int value = 2; };

// Evaluate a tape of storage type T (defined once per dtype, in its own
// translation unit, to keep compile times short).
template <class T>
int tape_eval_typed(const tape_prog& prog, const void* const* inputs, fx_shape s, int kind,
                    void* out, void* ws, size_t ws_bytes, const fx_launch* cfg, hipStream_t st);

#define FX_TAPE_EVAL_DEFINE(T)                                                                    \
  template <>                                                                                     \
  int tape_eval_typed<T>(const tape_prog& prog, const void* const* inputs, fx_shape s, int kind, \
                         void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,              \
                         hipStream_t st) {                                                        \
    TapeExpr<T> e;                                                                                \
    for (int q = 0; q < kTapeMaxIn; ++q)                                                          \
      e.p[q] = q < prog.n_in ? static_cast<const T*>(inputs[q]) : nullptr;                       \
    e.n_rows = s.n_rows;                                                                          \
    e.n_cols = s.n_cols;                                                                          \
    e.prog = prog;                                                                                \
    switch (kind) {                                                                               \
      case 0: return eval(static_cast<T*>(out), e, cfg, st);                                      \
      case FX_R_ACCU: return reduce_full<map_id>(e, out, ws, ws_bytes, cfg, st);                 \
      case FX_R_NORM: return reduce_full<map_sq>(e, out, ws, ws_bytes, cfg, st);                 \
      case FX_R_COLSUM: case FX_R_ROWSUM:                                                         \
        return reduce_dim(kind, e, static_cast<acc_out_t<T>*>(out), ws, ws_bytes, cfg, st);      \
    }                                                                                             \
    return fail(FX_E_ARG, "unknown kind %d for a tape", kind);                                    \
  }

// Host: compile a node list (children first, root last) into a program.
// Returns FX_OK or an fx_status with fx_last_error set.
int tape_compile(const fx_node* nodes, int32_t n_nodes, tape_prog* prog, fx_tape_info* info);

}  // namespace fx

// The opaque handle of the C ABI.
struct fx_tape {
  fx::tape_prog prog;
  fx_tape_info info;
};
