// Run-time expression tapes.
//
// Expressions whose tree is only known at run time cannot be C++ types, so
// the host compiles the tree into a short accumulator program and the device
// interprets it per element.  The running value lives in ordinary registers
// (the accumulator); values needed later (inputs, spilled partial results,
// nodes used more than once) live in a slot file of at most kTapeMaxSlots
// entries, and constants travel as immediates.  An instruction combines the
// accumulator with at most one slot or immediate, so a chain of operators
// such as exp(0 - abs(a)) costs only its arithmetic.  The program travels
// inside the kernel argument (or, for batches, in device memory), so every
// instruction fetch is a wave-uniform scalar load and the dispatch is a
// uniform branch.  Each lane's slot file is one 16-wide vector value indexed
// with those uniform slot numbers, which gfx950 serves from VGPRs in indexed
// mode (s_set_gpr_idx_on) rather than from private memory; lanes are
// interpreted in passes of 4 (FP32 compute) or 2 (FP64) so the files stay in
// registers.  TapeExpr<T> has the same interface as a compile-time
// expression, so the element-wise, full reduction, column-sum and row-sum
// skeletons (and their single-pass finish) serve tapes unchanged; its
// eval_tile overload loads every input of all EPT vectors before
// interpreting them one vector at a time.
#pragma once

#include <mutex>
#include "fx_kernels.hpp"

namespace fx {

constexpr int kTapeMaxIn = 4;
constexpr int kTapeMaxIns = 128;
constexpr int kTapeMaxSlots = 16;

// acc is the accumulator, y the operand: slot s[a] (suffix S) or the
// immediate (suffix I).  R-forms put the operand on the left.  The codes are
// the fx_tape_opcode values of the C interface.
enum : uint8_t {
  A_LD = 0,  // acc = s[a]
  A_LDI,     // acc = k
  A_ST,      // s[a] = acc
  A_ADD_S, A_ADD_I,    // acc = acc + y
  A_SUB_S, A_SUB_I,    // acc = acc - y
  A_RSUB_S, A_RSUB_I,  // acc = y - acc
  A_MUL_S, A_MUL_I,    // acc = acc % y
  A_DIV_S, A_DIV_I,    // acc = acc / y
  A_RDIV_S, A_RDIV_I,  // acc = y / acc
  A_NEG, A_ABS, A_EXP, A_SQRT,  // acc = f(acc)
  A_STLD,                        // s[a] = acc, then acc = s[a2]
  A_N_OPS
};
static_assert(A_LD == FX_TI_LD && A_ST == FX_TI_ST && A_ADD_S == FX_TI_ADD_S &&
                  A_RDIV_I == FX_TI_RDIV_I && A_SQRT == FX_TI_SQRT && A_STLD == FX_TI_STLD,
              "interpreter opcodes follow fx_tape_opcode");
// Input modifiers of an instruction that reads the accumulator, applied in
// this order before the operation: acc = s[a2] (a load folded into its
// consumer), acc = |acc|, acc = -acc (abs and neg nodes folded likewise;
// both are exact).
constexpr uint16_t kAbsIn = FX_TI_ABS_IN, kNegIn = FX_TI_NEG_IN, kLdIn = FX_TI_LD_IN;

// op and a fill the first 32-bit word together so that a fetch through a
// device pointer (batches) stays one scalar load: a narrower field would let
// the compiler shrink it to a 16-bit vector load, whose wait also waits for
// every input load in flight.
struct tape_ins {
  uint16_t op, a;  // a: slot index (LD, ST and S-forms) | second slot a2 << 8
  float kf;        // immediate for FP32 compute
  double kd;       // immediate for FP64 compute
};

// ins[n_ins] is always readable (the array has one spare zero entry): the
// interpreter fetches instruction pc + 1 while it executes instruction pc.
struct tape_prog {
  int32_t n_ins, n_in, n_slots, pad;
  tape_ins ins[kTapeMaxIns + 1];
};

template <class C> __device__ __forceinline__ C tape_imm(const tape_ins& I);
template <> __device__ __forceinline__ float tape_imm<float>(const tape_ins& I) { return I.kf; }
template <> __device__ __forceinline__ double tape_imm<double>(const tape_ins& I) { return I.kd; }

// Slot files.  Each is one 16-wide vector value, the width for which the
// compiler indexes registers in place (narrower vectors get select chains).
// A program needing at most 8 slots keeps two lanes per file, interleaved
// (element 2 * slot + lane): half the registers, higher occupancy; every
// generated tree so far fits.  Otherwise each lane has a file of 16 slots.
template <class C> struct slot_vec;
template <> struct slot_vec<float> { typedef float type __attribute__((ext_vector_type(16))); };
template <> struct slot_vec<double> { typedef double type __attribute__((ext_vector_type(16))); };
template <class C> using slots_t = typename slot_vec<C>::type;
constexpr int kTapeSmallSlots = 8;
// lanes per file, files for L lanes
template <int S> constexpr int kLanesPerFile = 16 / S;
template <int S, int L> constexpr int kFiles = (L + kLanesPerFile<S> - 1) / kLanesPerFile<S>;
#define FX_SLOT(f, j, a) f[(j) / P][(a) * P + (j) % P]
// Lanes interpreted per pass: every interpreted instruction is one fetch and
// one dispatch for all of them.
#ifndef FX_TAPE_PASS_LANES
#define FX_TAPE_PASS_LANES 8
#endif
template <class C> constexpr int kPassLanes = sizeof(C) == 4 ? FX_TAPE_PASS_LANES
                                                              : (FX_TAPE_PASS_LANES + 1) / 2;

// acc[j] = OP(acc[j], y) for slot and immediate operands (and the reversed
// forms): each case computes straight into the accumulator so no operand
// copies survive the branch merge.
#define FX_TAPE_BIN(NAME, OPK)                                                     \
  case A_##NAME##_S:                                                              \
    _Pragma("unroll") for (int j = 0; j < L; ++j) acc[j] = OPK::apply(acc[j], FX_SLOT(s, j, a)); \
    break;                                                                        \
  case A_##NAME##_I:                                                              \
    _Pragma("unroll") for (int j = 0; j < L; ++j) acc[j] = OPK::apply(acc[j], k); \
    break;                                                                        \
  case A_R##NAME##_S:                                                             \
    _Pragma("unroll") for (int j = 0; j < L; ++j) acc[j] = OPK::apply(FX_SLOT(s, j, a), acc[j]); \
    break;                                                                        \
  case A_R##NAME##_I:                                                             \
    _Pragma("unroll") for (int j = 0; j < L; ++j) acc[j] = OPK::apply(k, acc[j]); \
    break;

#define FX_TAPE_UN(NAME, OPK)                                                     \
  case A_##NAME:                                                                  \
    _Pragma("unroll") for (int j = 0; j < L; ++j) acc[j] = OPK::apply(acc[j]);    \
    break;

// Interpret `prog` on L lanes whose inputs already sit in slots [0, n_in);
// the result is left in acc.
template <class C, int L, int S>
__device__ __forceinline__ void tape_run(const tape_prog& prog, slots_t<C> (&s)[kFiles<S, L>],
                                         C (&acc)[L]) {
  constexpr int P = kLanesPerFile<S>;
  const int n = prog.n_ins;
  tape_ins I = prog.ins[0];
  for (int pc = 0; pc < n; ++pc) {
    const tape_ins next = prog.ins[pc + 1];
    const C k = tape_imm<C>(I);
    const unsigned op = I.op;
    const unsigned a = I.a & 0xFFu, a2 = I.a >> 8;
    if (op & (kAbsIn | kNegIn | kLdIn)) {
      if (op & kLdIn)
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = FX_SLOT(s, j, a2);
      if (op & kAbsIn)
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = op_abs::apply(acc[j]);
      if (op & kNegIn)
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = op_neg::apply(acc[j]);
    }
    switch (op & 0xFFu) {
      case A_LD:
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = FX_SLOT(s, j, a);
        break;
      case A_LDI:
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = k;
        break;
      case A_ST:
#pragma unroll
        for (int j = 0; j < L; ++j) FX_SLOT(s, j, a) = acc[j];
        break;
      case A_ADD_S:
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = op_add::apply(acc[j], FX_SLOT(s, j, a));
        break;
      case A_ADD_I:
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = op_add::apply(acc[j], k);
        break;
      FX_TAPE_BIN(SUB, op_sub)
      case A_MUL_S:
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = op_schur::apply(acc[j], FX_SLOT(s, j, a));
        break;
      case A_MUL_I:
#pragma unroll
        for (int j = 0; j < L; ++j) acc[j] = op_schur::apply(acc[j], k);
        break;
      FX_TAPE_BIN(DIV, op_div)
      FX_TAPE_UN(NEG, op_neg)
      FX_TAPE_UN(ABS, op_abs)
      FX_TAPE_UN(EXP, op_exp)
      FX_TAPE_UN(SQRT, op_sqrt)
      case A_STLD:
#pragma unroll
        for (int j = 0; j < L; ++j) {
          FX_SLOT(s, j, a) = acc[j];
          acc[j] = FX_SLOT(s, j, a2);
        }
        break;
      default:
        break;
    }
    I = next;
  }
}

#undef FX_TAPE_BIN
#undef FX_TAPE_UN

// BYREF = false: the program is held by value (it travels in the kernel
// argument); BYREF = true: it is read through a pointer into device memory
// (the batch kernel, where each tile may run a different program).
template <class T, bool BYREF = false, int SLOTS = kTapeSmallSlots> struct TapeExpr : expr_tag {
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
      constexpr int P = kLanesPerFile<SLOTS>;
      slots_t<ct> s[kFiles<SLOTS, G>];
#pragma unroll
      for (int f = 0; f < kFiles<SLOTS, G>; ++f) s[f] = slots_t<ct>{};
#pragma unroll
      for (int j = 0; j < G; ++j)
#pragma unroll
        for (int q = 0; q < kTapeMaxIn; ++q)
          if (q < pr.n_in) FX_SLOT(s, j, q) = in[q].v[g + j];
      ct acc[G];
#pragma unroll
      for (int j = 0; j < G; ++j) acc[j] = ct(0);
      tape_run<ct, G, SLOTS>(pr, s, acc);
#pragma unroll
      for (int j = 0; j < G; ++j) r.v[g + j] = acc[j];
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

template <int N, int EPT, class T, bool BYREF, int SLOTS>
__device__ __forceinline__ void eval_tile(const TapeExpr<T, BYREF, SLOTS>& e, int64_t base, int64_t stride,
                                          lanes<ct_t<T>, N> (&r)[EPT]) {
  using C = ct_t<T>;
  lanes<C, N> in[EPT][kTapeMaxIn];
  const int n_in = e.P().n_in;
#pragma unroll
  for (int q = 0; q < kTapeMaxIn; ++q)
    if (q < n_in)
#pragma unroll
      for (int k = 0; k < EPT; ++k) in[k][q] = load_lanes<N, kNT>(e.p[q], base + k * stride);
  // the EPT vectors are interpreted together, in passes of kPassLanes lanes
  lanes<C, N * EPT> flat[kTapeMaxIn];
#pragma unroll
  for (int q = 0; q < kTapeMaxIn; ++q)
#pragma unroll
    for (int k = 0; k < EPT; ++k)
#pragma unroll
      for (int j = 0; j < N; ++j) flat[q].v[k * N + j] = in[k][q].v[j];
  const lanes<C, N * EPT> out = e.template interpret<N * EPT>(flat);
#pragma unroll
  for (int k = 0; k < EPT; ++k)
#pragma unroll
    for (int j = 0; j < N; ++j) r[k].v[j] = out.v[k * N + j];
}

template <class T, bool B, int S> struct max_ept<TapeExpr<T, B, S>> { static constexpr int value = 2; };

// The launch configuration of an interpreted tape: the fields of cfg (NULL:
// all) left at 0 take the interpreter's defaults for the kind and storage
// width; split may stay 0 (the library's heuristic).  Defined with the other
// launch heuristics in fx_host.hip.
fx_launch tape_launch(int kind, int elem, int64_t n_rows, int64_t n_cols, const fx_launch* cfg);

// Evaluate a tape of storage type T (defined once per dtype, in its own
// translation unit, to keep compile times short).
template <class T>
int tape_eval_typed(const tape_prog& prog, const void* const* inputs, fx_shape s, int kind,
                    void* out, void* ws, size_t ws_bytes, const fx_launch* cfg, hipStream_t st);

template <class T, int SLOTS>
int tape_eval_impl(const tape_prog& prog, const void* const* inputs, fx_shape s, int kind,
                   void* out, void* ws, size_t ws_bytes, const fx_launch* cfg, hipStream_t st) {
  TapeExpr<T, false, SLOTS> e;
  for (int q = 0; q < kTapeMaxIn; ++q)
    e.p[q] = q < prog.n_in ? static_cast<const T*>(inputs[q]) : nullptr;
  e.n_rows = s.n_rows;
  e.n_cols = s.n_cols;
  e.prog = prog;
  // fields left at 0 take the interpreter's own defaults, not the library's
  const fx_launch c = tape_launch(kind, (int)sizeof(T), s.n_rows, s.n_cols, cfg);
  switch (kind) {
    case 0: return eval(static_cast<T*>(out), e, &c, st);
    case FX_R_ACCU: return reduce_full<map_id>(e, out, ws, ws_bytes, &c, st);
    case FX_R_NORM: return reduce_full<map_sq>(e, out, ws, ws_bytes, &c, st);
    case FX_R_COLSUM: case FX_R_ROWSUM:
      return reduce_dim(kind, e, static_cast<acc_out_t<T>*>(out), ws, ws_bytes, &c, st);
  }
  return fail(FX_E_ARG, "unknown kind %d for a tape", kind);
}

#define FX_TAPE_EVAL_DEFINE(T)                                                                    \
  template <>                                                                                     \
  int tape_eval_typed<T>(const tape_prog& prog, const void* const* inputs, fx_shape s, int kind, \
                         void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,              \
                         hipStream_t st) {                                                        \
    if (prog.n_slots <= kTapeSmallSlots)                                                          \
      return tape_eval_impl<T, kTapeSmallSlots>(prog, inputs, s, kind, out, ws, ws_bytes, cfg, st); \
    return tape_eval_impl<T, kTapeMaxSlots>(prog, inputs, s, kind, out, ws, ws_bytes, cfg, st);  \
  }

// Host: compile a node list (children first, root last) into a program.
// Returns FX_OK or an fx_status with fx_last_error set.
int tape_compile(const fx_node* nodes, int32_t n_nodes, tape_prog* prog, fx_tape_info* info);

}  // namespace fx

// The opaque handle of the C ABI.  With a model attached, evaluations that
// leave the launch configuration to the library take the model's choice;
// the last choice is cached (one key: dtype, shape, kind) under `mu`.
struct fx_tape {
  fx::tape_prog prog;
  fx_tape_info info;
  const fx_model* model = nullptr;
  mutable std::mutex mu;
  mutable bool have_choice = false;
  mutable fx_dtype choice_dt = FX_F32;
  mutable fx_shape choice_shape{0, 0};
  mutable int choice_kind = 0;
  mutable long choice_version = 0;  // the model's version the choice was made with
  mutable fx_launch choice{0, 0, 0, 0};
};

namespace fx {
// Counts the changes of a model's parameters and standardisation.
long model_version(const fx_model* m);
// fx_tape_eval without the model: `cfg` as given (fx_tune_time times the
// all-default configuration as the library's defaults).
int tape_eval_exact(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                    fx_shape s, int kind, void* out, void* ws, size_t ws_bytes,
                    const fx_launch* cfg, hipStream_t st);
}  // namespace fx
