// Run-time tapes: host compiler (tree -> register program) and the C entry
// points; evaluation reuses the skeleton kernels through TapeExpr<T>.
#include <algorithm>
#include <new>
#include <vector>

#include "fx_tape.hpp"

namespace fx {

namespace {

bool is_unary(int op) {
  return op == FX_OP_NEG || op == FX_OP_ABS || op == FX_OP_EXP || op == FX_OP_SQRT;
}
bool is_binary(int op) {
  return op == FX_OP_ADD || op == FX_OP_SUB || op == FX_OP_SCHUR || op == FX_OP_DIV;
}
int op_index(int op) {  // position in fx_tape_info::op_count
  switch (op) {
    case FX_OP_ADD: return 0;
    case FX_OP_SUB: return 1;
    case FX_OP_SCHUR: return 2;
    case FX_OP_DIV: return 3;
    case FX_OP_NEG: return 4;
    case FX_OP_ABS: return 5;
    case FX_OP_EXP: return 6;
    default: return 7;
  }
}

// Where a node's value is: in the accumulator (and, for a node used more
// than once, also in `slot`), in a slot (inputs, stored values), or an
// immediate constant.
enum where { IN_ACC, IN_SLOT, IMMED };

struct operand {
  where w = IN_SLOT;
  int slot = -1;
  double value = 0;
};

// Accumulator code generation.  A node's code leaves its value in the
// accumulator.  A binary node whose operands both need code evaluates the
// one needing more slots first (Sethi-Ullman order for an accumulator
// machine), stores it, evaluates the other and combines them with the
// operand order kept through the reversed forms (y - acc, y / acc).
struct compiler {
  const fx_node* nodes;
  int n;
  int n_in = 0;
  std::vector<int> uses, need, depth;
  std::vector<char> done;
  std::vector<operand> result;
  std::vector<int> free_slots;
  int next_slot = 0, max_slot = 0;
  tape_code* prog;
  int status = FX_OK;

  int alloc() {
    if (!free_slots.empty()) {
      std::sort(free_slots.begin(), free_slots.end(), std::greater<int>());
      int s = free_slots.back();
      free_slots.pop_back();
      return s;
    }
    int s = next_slot++;
    max_slot = std::max(max_slot, next_slot);
    return s;
  }
  // One use of node k is consumed; its slot is free after the last.
  void release(int k) {
    if (--uses[k] == 0 && result[k].slot >= n_in && result[k].w != IMMED)
      free_slots.push_back(result[k].slot);
  }
  // abs / neg of the accumulator not yet applied: they become input
  // modifiers of the next instruction that reads it
  uint16_t pending = 0;
  void modify(uint16_t m) {
    if (m == kAbsIn) pending = kAbsIn;  // |x|, |-x|, |-|x|| all equal |x|
    else pending ^= kNegIn;
  }
  void flush() {  // apply pending modifiers as instructions of their own
    const uint16_t m = pending;
    pending = 0;
    if (m & kAbsIn) emit_ins(A_ABS);
    if (m & kNegIn) emit_ins(A_NEG);
  }
  void emit_ins(uint8_t op, int slot = 0, double k = 0.0) {
    if (op == A_LD || op == A_LDI) {
      if (pending) flush();  // never happens for a tree: acc is consumed first
    }
    if (prog->n_ins >= kTapeMaxIns) {
      if (status == FX_OK) status = fail(FX_E_UNSUPPORTED, "tape longer than %d instructions", kTapeMaxIns);
      return;
    }
    tape_ins& I = prog->ins[prog->n_ins++];
    I = tape_ins{};
    I.op = (uint16_t)(op | ((op == A_LD || op == A_LDI) ? 0 : pending));
    if (op != A_LD && op != A_LDI) pending = 0;
    I.a = (uint16_t)slot;
    I.kf = (float)k;
    I.kd = k;
  }
  // Does evaluating node k emit code (and so overwrite the accumulator)?
  bool needs_code(int k) const {
    return !done[k] && nodes[k].op != FX_OP_LEAF && nodes[k].op != FX_OP_CONST;
  }
  void load(const operand& o) {
    if (o.w == IMMED) emit_ins(A_LDI, 0, o.value);
    else if (o.w == IN_SLOT) emit_ins(A_LD, o.slot);
  }
  // acc = x OP y where one of x, y is in the accumulator (acc_left says
  // which); the other is a slot or an immediate.
  void combine(int op, bool acc_left, const operand& other) {
    const bool imm = other.w == IMMED;
    uint8_t code;
    switch (op) {
      case FX_OP_ADD: code = imm ? A_ADD_I : A_ADD_S; break;            // commutes exactly
      case FX_OP_SCHUR: code = imm ? A_MUL_I : A_MUL_S; break;          // commutes exactly
      case FX_OP_SUB:
        code = acc_left ? (imm ? A_SUB_I : A_SUB_S) : (imm ? A_RSUB_I : A_RSUB_S);
        break;
      default:  // FX_OP_DIV
        code = acc_left ? (imm ? A_DIV_I : A_DIV_S) : (imm ? A_RDIV_I : A_RDIV_S);
        break;
    }
    emit_ins(code, imm ? 0 : other.slot, imm ? other.value : 0.0);
  }
  operand emit(int k) {
    if (done[k]) return result[k];
    const fx_node& nd = nodes[k];
    operand r;
    if (nd.op == FX_OP_LEAF) {
      r.slot = nd.input;
    } else if (nd.op == FX_OP_CONST) {
      r.w = IMMED;
      r.value = nd.value;
    } else if (is_unary(nd.op)) {
      operand a = emit(nd.a);
      if (a.w != IN_ACC) load(a);
      release(nd.a);
      if (nd.op == FX_OP_ABS) modify(kAbsIn);
      else if (nd.op == FX_OP_NEG) modify(kNegIn);
      else emit_ins(nd.op == FX_OP_EXP ? A_EXP : A_SQRT);
      r.w = IN_ACC;
    } else {
      const bool a_first = need[nd.a] >= need[nd.b];
      const int f = a_first ? nd.a : nd.b, g = a_first ? nd.b : nd.a;
      operand x = emit(f);
      int spill = -1;
      if (x.w == IN_ACC && needs_code(g)) {  // keep x while g is computed
        if (x.slot < 0) {
          x.slot = spill = alloc();
          emit_ins(A_ST, x.slot);
        }
        x.w = IN_SLOT;
      }
      operand y = emit(g);
      // x: first-evaluated operand, y: second; map back to (left, right)
      const operand& L = a_first ? x : y;
      const operand& R = a_first ? y : x;
      if (L.w == IN_ACC) {
        combine(nd.op, true, R);
      } else if (R.w == IN_ACC) {
        combine(nd.op, false, L);
      } else if (L.w == IN_SLOT || R.w == IMMED) {
        load(L);
        combine(nd.op, true, R);
      } else {  // L immediate, R in a slot
        load(R);
        combine(nd.op, false, L);
      }
      release(nd.a);
      release(nd.b);
      if (spill >= 0) free_slots.push_back(spill);
      r.w = IN_ACC;
    }
    if (r.w == IN_ACC && uses[k] > 1) {  // a shared node: keep a copy
      r.slot = alloc();
      emit_ins(A_ST, r.slot);
    }
    done[k] = 1;
    result[k] = r;
    if (r.w == IN_ACC && r.slot >= 0) {  // later uses read the slot
      result[k].w = IN_SLOT;
    }
    return r;
  }
};

// Peephole over the emitted program: "ST a; LD b" becomes one STLD a, b, and
// a plain "LD b" followed by an instruction that reads the accumulator is
// folded into it as the load-in modifier (slot b in the high byte of a).
// Each removed instruction saves one fetch and one dispatch per lane group.
void fuse_loads(tape_code* p) {
  int o = 0;
  for (int i = 0; i < p->n_ins; ++i) {
    tape_ins I = p->ins[i];
    const bool has_next = i + 1 < p->n_ins;
    const tape_ins N = has_next ? p->ins[i + 1] : tape_ins{};
    const int op = I.op & 0xFF, nop = N.op & 0xFF;
    if (has_next && op == A_ST && nop == A_LD && (N.op & ~0xFF) == 0) {
      I.op = (uint16_t)((I.op & ~0xFF) | A_STLD);  // the ST's abs/neg modifiers stay
      I.a = (uint16_t)((I.a & 0xFF) | ((N.a & 0xFF) << 8));
      p->ins[o++] = I;
      ++i;
      continue;
    }
    if (has_next && op == A_LD && (I.op & ~0xFF) == 0 && nop != A_LD && nop != A_LDI &&
        nop != A_STLD && !(N.op & kLdIn)) {
      tape_ins F = N;
      F.op = (uint16_t)(N.op | kLdIn);
      F.a = (uint16_t)((N.a & 0xFF) | ((I.a & 0xFF) << 8));
      p->ins[o++] = F;
      ++i;
      continue;
    }
    p->ins[o++] = I;
  }
  for (int i = o; i <= p->n_ins && i <= kTapeMaxIns; ++i) p->ins[i] = tape_ins{};
  p->n_ins = o;
}

}  // namespace

int tape_compile(const fx_node* nodes, int32_t n, tape_code* prog, fx_tape_info* info) {
  if (!nodes || n <= 0) return fail(FX_E_ARG, "empty tree");
  if (n > 4 * kTapeMaxIns) return fail(FX_E_UNSUPPORTED, "tree of %d nodes is too large", n);
  compiler c;
  c.nodes = nodes;
  c.n = n;
  c.uses.assign(n, 0);
  c.need.assign(n, 0);
  c.depth.assign(n, 0);
  c.done.assign(n, 0);
  c.result.assign(n, operand{});
  *info = fx_tape_info{};
  info->n_nodes = n;
  for (int k = 0; k < n; ++k) {
    const fx_node& nd = nodes[k];
    if (nd.op == FX_OP_LEAF) {
      if (nd.input < 0 || nd.input >= kTapeMaxIn)
        return fail(FX_E_UNSUPPORTED, "node %d: input %d outside [0, %d)", k, nd.input, kTapeMaxIn);
      c.n_in = std::max(c.n_in, nd.input + 1);
    } else if (nd.op == FX_OP_CONST) {
    } else if (is_unary(nd.op)) {
      if (nd.a < 0 || nd.a >= k) return fail(FX_E_ARG, "node %d: operand %d not earlier", k, nd.a);
      c.uses[nd.a]++;
      c.need[k] = c.need[nd.a];
      c.depth[k] = c.depth[nd.a] + 1;
    } else if (is_binary(nd.op)) {
      if (nd.a < 0 || nd.a >= k || nd.b < 0 || nd.b >= k)
        return fail(FX_E_ARG, "node %d: operands %d, %d not earlier", k, nd.a, nd.b);
      c.uses[nd.a]++;
      c.uses[nd.b]++;
      // slots needed beyond the accumulator: a computed operand is held in
      // a slot while the other is computed, if that one needs code too
      const bool ca = is_unary(nodes[nd.a].op) || is_binary(nodes[nd.a].op);
      const bool cb = is_unary(nodes[nd.b].op) || is_binary(nodes[nd.b].op);
      const int na = c.need[nd.a], nb = c.need[nd.b];
      c.need[k] = (ca && cb) ? (na == nb ? na + 1 : std::max(na, nb)) : std::max(na, nb);
      c.depth[k] = std::max(c.depth[nd.a], c.depth[nd.b]) + 1;
    } else {
      return fail(FX_E_ARG, "node %d: unknown operator %d", k, nd.op);
    }
  }
  c.uses[n - 1]++;  // the root's value is the output
  *prog = tape_code{};
  prog->n_in = c.n_in;
  c.next_slot = c.max_slot = c.n_in;
  c.prog = prog;
  operand root = c.emit(n - 1);
  if (root.w != IN_ACC) c.load(root);  // a leaf, a constant or a stored node
  c.flush();                           // a root abs / neg
  if (c.status != FX_OK) return c.status;
  fuse_loads(prog);
  if (c.max_slot > kTapeMaxSlots)
    return fail(FX_E_UNSUPPORTED, "tape needs %d live slots (at most %d)", c.max_slot, kTapeMaxSlots);
  prog->n_slots = c.max_slot;
  info->n_inputs = c.n_in;
  info->depth = c.depth[n - 1];
  info->n_instructions = prog->n_ins;
  info->n_slots = c.max_slot;
  for (int k = 0; k < n; ++k) {
    if (!c.done[k]) continue;  // count only what the root reaches
    if (nodes[k].op == FX_OP_CONST) info->n_consts++;
    else if (nodes[k].op != FX_OP_LEAF) info->op_count[op_index(nodes[k].op)]++;
  }
  return FX_OK;
}

// Lower the architectural program into device micro-operations.  Every
// micro-operation performs exactly the IEEE operations of the instruction it
// comes from, so the two forms give the same bits:
//   a folded load (LD_IN) becomes LD of that slot; STLD becomes ST then LD;
//   abs / neg input modifiers become ABS / NEG, except where the consumer
//   takes them as an operand modifier: exp(-|a|), sqrt(|a|), |a| + k;
//   "0 - |a|" directly followed by exp becomes exp(-|a|) (0 - |a| and -|a|
//   differ only in the sign of a zero result, which exp maps to 1 either way);
//   acc - k becomes acc + (-k) (IEEE defines x - y as x + (-y)).
int tape_lower(const tape_code& code, tape_prog* prog) {
  *prog = tape_prog{};
  prog->n_in = code.n_in;
  prog->n_slots = code.n_slots <= kTapeSmallSlots ? kTapeSmallSlots : kTapeMaxSlots;
  int n = 0;
  auto emit = [&](uint8_t op, double k = 0.0) -> bool {
    if (n >= kTapeMaxUops) return false;
    tape_uop& u = prog->ins[n++];
    u = tape_uop{};
    u.op = op;
    if (op >= U_LDI && op != U_NEG && op != U_ABS && op != U_EXP && op != U_SQRT &&
        op != U_EXP_NABS && op != U_SQRT_ABS) {
      int ki = -1;  // FP64 immediates, deduplicated by bit pattern
      for (int c = 0; c < prog->n_consts; ++c)
        if (__builtin_memcmp(&prog->kd[c], &k, sizeof k) == 0) ki = c;
      if (ki < 0) {
        if (prog->n_consts >= kTapeMaxConsts) return false;
        ki = prog->n_consts++;
        prog->kd[ki] = k;
      }
      u.ki = (uint8_t)ki;
      u.kf = (float)k;
    }
    return true;
  };
  bool ok = true;
  for (int i = 0; i < code.n_ins && ok; ++i) {
    const tape_ins& I = code.ins[i];
    const int op = I.op & 0xFF;
    const int a = I.a & 0xFF, a2 = I.a >> 8;
    const bool ld_in = (I.op & kLdIn) != 0, abs_in = (I.op & kAbsIn) != 0,
               neg_in = (I.op & kNegIn) != 0;
    const double k = I.kd;
    if (ld_in) ok = ok && emit(U_LD + a2);
    // consumers that take the modifiers as operand modifiers
    if (op == A_EXP && abs_in && neg_in) { ok = ok && emit(U_EXP_NABS); continue; }
    if (op == A_SQRT && abs_in && !neg_in) { ok = ok && emit(U_SQRT_ABS); continue; }
    if (op == A_ADD_I && abs_in && !neg_in) { ok = ok && emit(U_ADDI_ABS, k); continue; }
    if (op == A_RSUB_I && k == 0.0 && abs_in && !neg_in && i + 1 < code.n_ins &&
        code.ins[i + 1].op == A_EXP) {
      ok = ok && emit(U_EXP_NABS);
      ++i;
      continue;
    }
    if (abs_in) ok = ok && emit(U_ABS);
    if (neg_in) ok = ok && emit(U_NEG);
    switch (op) {
      case A_LD: ok = ok && emit(U_LD + a); break;
      case A_LDI: ok = ok && emit(U_LDI, k); break;
      case A_ST: ok = ok && emit(U_ST + a); break;
      case A_STLD: ok = ok && emit(U_ST + a) && emit(U_LD + a2); break;
      case A_ADD_S: ok = ok && emit(U_ADD + a); break;
      case A_SUB_S: ok = ok && emit(U_SUB + a); break;
      case A_RSUB_S: ok = ok && emit(U_RSUB + a); break;
      case A_MUL_S: ok = ok && emit(U_MUL + a); break;
      case A_DIV_S: ok = ok && emit(U_DIV + a); break;
      case A_RDIV_S: ok = ok && emit(U_RDIV + a); break;
      case A_ADD_I: ok = ok && emit(U_ADDI, k); break;
      case A_SUB_I: ok = ok && emit(U_ADDI, -k); break;
      case A_RSUB_I: ok = ok && emit(U_RSUBI, k); break;
      case A_MUL_I: ok = ok && emit(U_MULI, k); break;
      case A_DIV_I: ok = ok && emit(U_DIVI, k); break;
      case A_RDIV_I: ok = ok && emit(U_RDIVI, k); break;
      case A_NEG: ok = ok && emit(U_NEG); break;
      case A_ABS: ok = ok && emit(U_ABS); break;
      case A_EXP: ok = ok && emit(U_EXP); break;
      case A_SQRT: ok = ok && emit(U_SQRT); break;
      default: return fail(FX_E_ARG, "instruction %d: unknown opcode %d", i, op);
    }
  }
  if (!ok)
    return fail(FX_E_UNSUPPORTED, "tape lowers to more than %d device operations or %d constants",
                kTapeMaxUops, kTapeMaxConsts);
  prog->n_ins = n;  // ins[n] stays zero: the prefetch past the end reads it
  return FX_OK;
}

}  // namespace fx

using namespace fx;

namespace fx {

int tape_eval_exact(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                    fx_shape s, int kind, void* out, void* ws, size_t ws_bytes,
                    const fx_launch* cfg, hipStream_t st) {
  if (!t) return fail(FX_E_ARG, "NULL tape");
  if (int rc = check_shape(s)) return rc;
  if (n_inputs < t->prog.n_in || (t->prog.n_in > 0 && !inputs))
    return fail(FX_E_ARG, "tape reads %d inputs, %d given", t->prog.n_in, n_inputs);
  switch (dt) {
    case FX_F32: return tape_eval_typed<float>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, st);
    case FX_F64: return tape_eval_typed<double>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, st);
    case FX_BF16: return tape_eval_typed<bf16_t>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, st);
    case FX_F16: return tape_eval_typed<f16_t>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, st);
    default: break;
  }
  return fail(FX_E_DTYPE, "tapes evaluate floating-point dtypes only");
}

}  // namespace fx

extern "C" {

int fx_tape_create(const fx_node* nodes, int32_t n_nodes, fx_tape** out) {
  if (!out) return fail(FX_E_ARG, "NULL output handle");
  *out = nullptr;
  fx_tape* t = new (std::nothrow) fx_tape;
  if (!t) return fail(FX_E_ARG, "out of host memory");
  int rc = tape_compile(nodes, n_nodes, &t->code, &t->info);
  if (rc == FX_OK) rc = tape_lower(t->code, &t->prog);
  if (rc != FX_OK) {
    delete t;
    return rc;
  }
  *out = t;
  return FX_OK;
}

void fx_tape_destroy(fx_tape* t) { delete t; }

int32_t fx_tape_program(const fx_tape* t, uint16_t* op, uint8_t* slot, uint8_t* slot2, double* imm,
                        int32_t cap) {
  if (!t) return -fail(FX_E_ARG, "NULL tape");
  const int32_t n = t->code.n_ins;
  if (cap > 0 && (!op || !slot || !slot2 || !imm)) return -fail(FX_E_ARG, "NULL output array");
  for (int32_t i = 0; i < n && i < cap; ++i) {
    op[i] = t->code.ins[i].op;
    slot[i] = (uint8_t)(t->code.ins[i].a & 0xFF);
    slot2[i] = (uint8_t)(t->code.ins[i].a >> 8);
    imm[i] = t->code.ins[i].kd;
  }
  return n;
}

int fx_tape_describe(const fx_tape* t, fx_tape_info* out) {
  if (!t || !out) return fail(FX_E_ARG, "NULL argument");
  *out = t->info;
  return FX_OK;
}

int fx_tape_set_model(fx_tape* t, const fx_model* m) {
  if (!t) return fail(FX_E_ARG, "NULL tape");
  std::lock_guard<std::mutex> g(t->mu);
  t->model = m;
  t->have_choice = false;
  return FX_OK;
}

int fx_tape_eval(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                 fx_shape s, int kind, void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
                 void* stream) {
  if (!t) return fail(FX_E_ARG, "NULL tape");
  const bool library_choice =
      !cfg || (!cfg->block && !cfg->ept && !cfg->vec_bytes && !cfg->split);
  if (!library_choice || !t->model)
    return tape_eval_exact(t, dt, inputs, n_inputs, s, kind, out, ws, ws_bytes, cfg, S(stream));
  if (int rc = check_shape(s)) return rc;
  fx_launch pick;
  {
    std::lock_guard<std::mutex> g(t->mu);
    const long version = model_version(t->model);
    if (!(t->have_choice && t->choice_dt == dt && t->choice_kind == kind &&
          t->choice_shape.n_rows == s.n_rows && t->choice_shape.n_cols == s.n_cols &&
          t->choice_version == version)) {
      float f[32];
      const int32_t nf = fx_tape_features(t, dt, s, kind, f, 32);
      if (nf < 0) return -nf;
      if (int rc = fx_model_predict(t->model, f, kind, dt, &t->choice)) return rc;
      t->have_choice = true;
      t->choice_dt = dt;
      t->choice_kind = kind;
      t->choice_shape = s;
      t->choice_version = version;
    }
    pick = t->choice;
  }
  // a choice whose workspace the caller did not provide falls back to the
  // defaults (whose workspace fx_workspace_bytes covers)
  if (kind != 0 && fx_workspace_bytes(kind, dt, s, &pick) > ws_bytes) pick = fx_launch{0, 0, 0, 0};
  return tape_eval_exact(t, dt, inputs, n_inputs, s, kind, out, ws, ws_bytes, &pick, S(stream));
}

}  // extern "C"
