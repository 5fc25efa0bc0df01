// Run-time expression tapes.
//
// Expressions whose tree is only known at run time cannot be C++ types, so
// the host compiles the tree into a short accumulator program and the device
// interprets it per element.  Two forms of the program exist.
//
// The architectural form (tape_code, listed by fx_tape_program): the running
// value lives in an accumulator; values needed later (inputs, spilled
// partial results, nodes used more than once) live in at most kTapeMaxSlots
// slots; an instruction combines the accumulator with at most one slot or
// immediate, so a chain of operators such as exp(0 - abs(a)) costs only its
// arithmetic.
//
// The device form (tape_prog): the host lowers every architectural
// instruction into micro-operations whose slot operand is part of the
// operation code (U_ADD + 3 adds slot 3).  Each case of the device's
// dispatch names its slot registers statically, so slot values stay in
// fixed VGPRs and an operand costs nothing beyond the arithmetic that uses
// it: no register-indexing mode, no moves.  Guard patterns of the form
// exp(-|a|), sqrt(|a|) and |a| + k are single micro-operations whose
// absolute value and negation become free source modifiers.  Divisions
// share one body per slot-file size (the operand is copied in first; the
// divide itself costs more than ten times the copy).  The program travels
// inside the kernel argument (or, for batches, in device memory), so every
// fetch is a wave-uniform scalar load and the dispatch is a uniform branch
// tree.  Lanes are interpreted in passes sized so that the slot file holds
// 64 VGPRs.  TapeExpr<T> has the same interface as a compile-time expression,
// so the element-wise, full reduction, column-sum and row-sum skeletons (and
// their single-pass finish) serve tapes unchanged; its eval_tile overload
// loads every input of all EPT vectors before interpreting them.
#pragma once

#include <mutex>
#include "fx_kernels.hpp"

namespace fx {

constexpr int kTapeMaxIn = 4;
constexpr int kTapeMaxIns = 128;     // architectural instructions
constexpr int kTapeMaxSlots = 16;
constexpr int kTapeMaxUops = 320;    // micro-operations of the lowered form
constexpr int kTapeMaxConsts = 128;  // FP64 immediates of the lowered form

// ---- architectural form (host) ---------------------------------------------
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
              "architectural opcodes follow fx_tape_opcode");
// Input modifiers of an instruction that reads the accumulator, applied in
// this order before the operation: acc = s[a2] (a load folded into its
// consumer), acc = |acc|, acc = -acc (abs and neg nodes folded likewise;
// both are exact).
constexpr uint16_t kAbsIn = FX_TI_ABS_IN, kNegIn = FX_TI_NEG_IN, kLdIn = FX_TI_LD_IN;

struct tape_ins {
  uint16_t op, a;  // a: slot index (LD, ST and S-forms) | second slot a2 << 8
  float kf;        // immediate rounded to FP32
  double kd;       // immediate
};

struct tape_code {
  int32_t n_ins, n_in, n_slots, pad;
  tape_ins ins[kTapeMaxIns + 1];
};

// ---- device form -----------------------------------------------------------
// Slot families (code = family + slot) and slot-free operations.
enum : uint8_t {
  U_LD = 0x00,    // acc = s[k]
  U_ST = 0x10,    // s[k] = acc
  U_ADD = 0x20,   // acc = acc + s[k]
  U_SUB = 0x30,   // acc = acc - s[k]
  U_RSUB = 0x40,  // acc = s[k] - acc
  U_MUL = 0x50,   // acc = acc % s[k]
  U_DIV = 0x60,   // acc = acc / s[k]
  U_RDIV = 0x70,  // acc = s[k] / acc
  U_LDI = 0x80,   // acc = imm
  U_ADDI,         // acc = acc + imm   (also acc - imm, as acc + (-imm): the same IEEE result)
  U_ADDI_ABS,     // acc = |acc| + imm
  U_RSUBI,        // acc = imm - acc
  U_MULI,         // acc = acc % imm
  U_DIVI,         // acc = acc / imm
  U_RDIVI,        // acc = imm / acc
  U_NEG, U_ABS, U_EXP, U_SQRT,
  U_EXP_NABS,     // acc = exp(-|acc|)
  U_SQRT_ABS,     // acc = sqrt(|acc|)
  U_END
};

struct tape_uop {
  uint8_t op;    // U_*
  uint8_t ki;    // index of the immediate in tape_prog::kd
  uint16_t pad;
  float kf;      // the immediate rounded to FP32 (FP32 compute)
};

// ins[n_ins] is always readable (the array has one spare zero entry): the
// interpreter fetches micro-operation pc + 1 while it executes pc.
struct tape_prog {
  int32_t n_ins, n_in, n_slots, n_consts;
  double kd[kTapeMaxConsts];  // immediates for FP64 compute
  tape_uop ins[kTapeMaxUops + 1];
};

template <class C> __device__ __forceinline__ C tape_imm(const tape_prog& p, const tape_uop& I);
template <> __device__ __forceinline__ float tape_imm<float>(const tape_prog&, const tape_uop& I) {
  return I.kf;
}
template <> __device__ __forceinline__ double tape_imm<double>(const tape_prog& p, const tape_uop& I) {
  return p.kd[I.ki];
}

// Slot-file sizes the device is compiled for, and the lanes of one pass:
// the file holds 64 VGPRs (16 slots: half the lanes).
constexpr int kTapeSmallSlots = 8;
template <class C, int S> constexpr int kPassLanes = (64 * 4) / (S * (int)sizeof(C));

// One case per slot of a family; BODY(K) is the statement for slot K.
#define FX_SLOT_CASES8(FAM, BODY)                                                    \
  case (FAM) + 0: BODY(0) case (FAM) + 1: BODY(1) case (FAM) + 2: BODY(2)             \
  case (FAM) + 3: BODY(3) case (FAM) + 4: BODY(4) case (FAM) + 5: BODY(5)             \
  case (FAM) + 6: BODY(6) case (FAM) + 7: BODY(7)
#define FX_SLOT_CASES16(FAM, BODY)                                                   \
  FX_SLOT_CASES8(FAM, BODY)                                                          \
  case (FAM) + 8: BODY(8) case (FAM) + 9: BODY(9) case (FAM) + 10: BODY(10)           \
  case (FAM) + 11: BODY(11) case (FAM) + 12: BODY(12) case (FAM) + 13: BODY(13)       \
  case (FAM) + 14: BODY(14) case (FAM) + 15: BODY(15)

#define FX_LANES(STMT) _Pragma("unroll") for (int j = 0; j < L; ++j) { STMT; }
#define FX_U_LD(K) FX_LANES(acc[j] = s[K][j]) break;
#define FX_U_ST(K) FX_LANES(s[K][j] = acc[j]) break;
#define FX_U_ADD(K) FX_LANES(acc[j] = acc[j] + s[K][j]) break;
#define FX_U_SUB(K) FX_LANES(acc[j] = acc[j] - s[K][j]) break;
#define FX_U_RSUB(K) FX_LANES(acc[j] = s[K][j] - acc[j]) break;
#define FX_U_MUL(K) FX_LANES(acc[j] = acc[j] * s[K][j]) break;
#define FX_U_DIV(K) FX_LANES(acc[j] = acc[j] / s[K][j]) break;
#define FX_U_RDIV(K) FX_LANES(acc[j] = s[K][j] / acc[j]) break;

// The whole dispatch for one slot-file size (SC: FX_SLOT_CASES8 or 16).
#define FX_TAPE_SWITCH(SC)                                                            \
  switch (I.op) {                                                                     \
    SC(U_LD, FX_U_LD)                                                                 \
    SC(U_ST, FX_U_ST)                                                                 \
    SC(U_ADD, FX_U_ADD)                                                               \
    SC(U_SUB, FX_U_SUB)                                                               \
    SC(U_RSUB, FX_U_RSUB)                                                             \
    SC(U_MUL, FX_U_MUL)                                                               \
    SC(U_DIV, FX_U_DIV)                                                               \
    SC(U_RDIV, FX_U_RDIV)                                                             \
    case U_LDI: FX_LANES(acc[j] = k) break;                                           \
    case U_ADDI: FX_LANES(acc[j] = acc[j] + k) break;                                 \
    case U_ADDI_ABS: FX_LANES(acc[j] = op_abs::apply(acc[j]) + k) break;              \
    case U_RSUBI: FX_LANES(acc[j] = k - acc[j]) break;                                \
    case U_MULI: FX_LANES(acc[j] = acc[j] * k) break;                                 \
    case U_DIVI: FX_LANES(acc[j] = acc[j] / k) break;                                 \
    case U_RDIVI: FX_LANES(acc[j] = k / acc[j]) break;                                \
    case U_NEG: FX_LANES(acc[j] = -acc[j]) break;                                     \
    case U_ABS: FX_LANES(acc[j] = op_abs::apply(acc[j])) break;                       \
    case U_EXP: FX_LANES(acc[j] = op_exp::apply(acc[j])) break;                       \
    case U_SQRT: FX_LANES(acc[j] = op_sqrt::apply(acc[j])) break;                     \
    case U_EXP_NABS: FX_LANES(acc[j] = op_exp::apply(-op_abs::apply(acc[j]))) break;  \
    case U_SQRT_ABS: FX_LANES(acc[j] = op_sqrt::apply(op_abs::apply(acc[j]))) break;  \
    default: break;                                                                   \
  }

// Interpret `prog` on L lanes whose inputs already sit in slots [0, n_in);
// the result is left in acc.  Each micro-operation is one IEEE operation (or
// library function) per lane, exactly as in the architectural form, so the
// lowering changes no result bit.  One function per slot-file size (each
// has its own divide labels).
#define FX_TAPE_RUN(NAME, S, SC)                                                      \
  template <class C, int L>                                                           \
  __device__ __forceinline__ void NAME(const tape_prog& prog, C (&s)[S][L], C (&acc)[L]) { \
    const int n = prog.n_ins;                                                         \
    tape_uop I = prog.ins[0];                                                         \
    for (int pc = 0; pc < n; ++pc) {                                                  \
      const tape_uop next = prog.ins[pc + 1];                                         \
      const C k = tape_imm<C>(prog, I);                                               \
      FX_TAPE_SWITCH(SC)                                                              \
      I = next;                                                                       \
    }                                                                                 \
  }
FX_TAPE_RUN(tape_run8, 8, FX_SLOT_CASES8)
FX_TAPE_RUN(tape_run16, 16, FX_SLOT_CASES16)
#undef FX_TAPE_RUN

template <class C, int L, int S>
__device__ __forceinline__ void tape_run(const tape_prog& prog, C (&s)[S][L], C (&acc)[L]) {
  static_assert(S == 8 || S == 16, "slot files of 8 or 16");
  if constexpr (S == 8) tape_run8<C, L>(prog, s, acc);
  else tape_run16<C, L>(prog, s, acc);
}

#undef FX_TAPE_SWITCH
#undef FX_U_LD
#undef FX_U_ST
#undef FX_U_ADD
#undef FX_U_SUB
#undef FX_U_RSUB
#undef FX_U_MUL
#undef FX_U_DIV
#undef FX_U_RDIV
#undef FX_LANES
#undef FX_SLOT_CASES8
#undef FX_SLOT_CASES16

// Lanes of an input the program does not read: unspecified values, no code.
template <class C, int N> __device__ __forceinline__ lanes<C, N> unset_lanes() {
  lanes<C, N> r;
#pragma unroll
  for (int j = 0; j < N; ++j) r.v[j] = __builtin_nondeterministic_value(r.v[j]);
  return r;
}

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
  // Slots past the inputs start with unspecified values (every program
  // stores a slot before it reads it), which costs no instruction.
  template <int N>
  __device__ __forceinline__ lanes<ct, N> interpret(const lanes<ct, N> (&in)[kTapeMaxIn]) const {
    constexpr int G = N < kPassLanes<ct, SLOTS> ? N : kPassLanes<ct, SLOTS>;
    const tape_prog& pr = P();
    lanes<ct, N> r;
#pragma unroll
    for (int g = 0; g < N; g += G) {
      ct s[SLOTS][G];
#pragma unroll
      for (int j = 0; j < G; ++j) {
#pragma unroll
        for (int a = 0; a < kTapeMaxIn; ++a) s[a][j] = in[a].v[g + j];
#pragma unroll
        for (int a = kTapeMaxIn; a < SLOTS; ++a) s[a][j] = __builtin_nondeterministic_value(s[a][j]);
      }
      ct acc[G];
#pragma unroll
      for (int j = 0; j < G; ++j) acc[j] = __builtin_nondeterministic_value(acc[j]);
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
      in[q] = q < n_in ? load_lanes<N, NT>(p[q], i) : unset_lanes<ct, N>();
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
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      in[k][q] = q < n_in ? load_lanes<N, kNT>(e.p[q], base + k * stride) : unset_lanes<C, N>();
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

template <class T, bool B, int S> struct max_ept<TapeExpr<T, B, S>> { static constexpr int value = 4; };
template <class T, bool B, int S> struct vec8_compiled<TapeExpr<T, B, S>> {
  static constexpr bool value = true;
};

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

// Host: compile a node list (children first, root last) into the
// architectural program, and lower that into the device program.  Return
// FX_OK or an fx_status with fx_last_error set.
int tape_compile(const fx_node* nodes, int32_t n_nodes, tape_code* code, fx_tape_info* info);
int tape_lower(const tape_code& code, tape_prog* prog);

}  // namespace fx

// The opaque handle of the C ABI.  With a model attached, evaluations that
// leave the launch configuration to the library take the model's choice;
// the last choice is cached (one key: dtype, shape, kind) under `mu`.
struct fx_tape {
  fx::tape_code code;  // architectural form (fx_tape_program)
  fx::tape_prog prog;  // device form
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
