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
uint8_t tape_op(int op) {
  switch (op) {
    case FX_OP_ADD: return T_ADD;
    case FX_OP_SUB: return T_SUB;
    case FX_OP_SCHUR: return T_MUL;
    case FX_OP_DIV: return T_DIV;
    case FX_OP_NEG: return T_NEG;
    case FX_OP_ABS: return T_ABS;
    case FX_OP_EXP: return T_EXP;
    default: return T_SQRT;
  }
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

// An operand of an instruction: a slot or an immediate.
struct operand {
  bool imm = false;
  int slot = -1;
  double value = 0;
};

struct compiler {
  const fx_node* nodes;
  int n;
  int n_in = 0;
  std::vector<int> uses, need, depth;
  std::vector<char> done;
  std::vector<operand> result;
  std::vector<int> free_slots;
  int next_slot = 0, max_slot = 0;
  tape_prog* prog;
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
  void release(int k) {
    if (--uses[k] == 0 && !result[k].imm && result[k].slot >= n_in)
      free_slots.push_back(result[k].slot);
  }
  void emit_ins(uint8_t op, int dst, const operand& a, const operand* b) {
    if (prog->n_ins >= kTapeMaxIns) {
      if (status == FX_OK) status = fail(FX_E_UNSUPPORTED, "tape longer than %d instructions", kTapeMaxIns);
      return;
    }
    tape_ins& I = prog->ins[prog->n_ins++];
    I.op = op;
    I.dst = (uint8_t)dst;
    I.a = a.imm ? kImm : (uint8_t)a.slot;
    I.b = (b && !b->imm) ? (uint8_t)b->slot : kImm;
    const double k = a.imm ? a.value : (b && b->imm ? b->value : 0.0);
    I.kf = (float)k;
    I.kd = k;
  }
  operand emit(int k) {
    if (done[k]) return result[k];
    const fx_node& nd = nodes[k];
    operand r;
    if (nd.op == FX_OP_LEAF) {
      r.slot = nd.input;
    } else if (nd.op == FX_OP_CONST) {
      r.imm = true;
      r.value = nd.value;
    } else if (is_unary(nd.op)) {
      operand a = emit(nd.a);
      release(nd.a);
      int dst = alloc();
      emit_ins(tape_op(nd.op), dst, a, nullptr);
      r.slot = dst;
    } else {
      // the operand needing more slots first (Sethi-Ullman order)
      const bool a_first = need[nd.a] >= need[nd.b];
      operand a, b;
      if (a_first) { a = emit(nd.a); b = emit(nd.b); }
      else { b = emit(nd.b); a = emit(nd.a); }
      int mov = -1;
      if (a.imm && b.imm) {  // two immediates: materialise one
        mov = alloc();
        emit_ins(T_MOV, mov, a, nullptr);
        a.imm = false;
        a.slot = mov;
      }
      release(nd.a);
      release(nd.b);
      if (mov >= 0) free_slots.push_back(mov);
      int dst = alloc();
      emit_ins(tape_op(nd.op), dst, a, &b);
      r.slot = dst;
    }
    done[k] = 1;
    result[k] = r;
    return r;
  }
};

}  // namespace

int tape_compile(const fx_node* nodes, int32_t n, tape_prog* prog, fx_tape_info* info) {
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
      c.need[k] = std::max(1, c.need[nd.a]);
      c.depth[k] = c.depth[nd.a] + 1;
    } else if (is_binary(nd.op)) {
      if (nd.a < 0 || nd.a >= k || nd.b < 0 || nd.b >= k)
        return fail(FX_E_ARG, "node %d: operands %d, %d not earlier", k, nd.a, nd.b);
      c.uses[nd.a]++;
      c.uses[nd.b]++;
      const int na = c.need[nd.a], nb = c.need[nd.b];
      c.need[k] = std::max(1, na == nb ? na + 1 : std::max(na, nb));
      c.depth[k] = std::max(c.depth[nd.a], c.depth[nd.b]) + 1;
    } else {
      return fail(FX_E_ARG, "node %d: unknown operator %d", k, nd.op);
    }
  }
  c.uses[n - 1]++;  // the root's value is the output
  *prog = tape_prog{};
  prog->n_in = c.n_in;
  c.next_slot = c.max_slot = c.n_in;
  c.prog = prog;
  operand root = c.emit(n - 1);
  if (c.status != FX_OK) return c.status;
  if (root.imm) {  // a constant expression
    int dst = c.alloc();
    c.emit_ins(T_MOV, dst, root, nullptr);
    root.imm = false;
    root.slot = dst;
  }
  if (c.status != FX_OK) return c.status;
  if (c.max_slot > kTapeMaxSlots)
    return fail(FX_E_UNSUPPORTED, "tape needs %d live slots (at most %d)", c.max_slot, kTapeMaxSlots);
  prog->root = root.slot;
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

}  // namespace fx

using namespace fx;

extern "C" {

int fx_tape_create(const fx_node* nodes, int32_t n_nodes, fx_tape** out) {
  if (!out) return fail(FX_E_ARG, "NULL output handle");
  *out = nullptr;
  fx_tape* t = new (std::nothrow) fx_tape;
  if (!t) return fail(FX_E_ARG, "out of host memory");
  int rc = tape_compile(nodes, n_nodes, &t->prog, &t->info);
  if (rc != FX_OK) {
    delete t;
    return rc;
  }
  *out = t;
  return FX_OK;
}

void fx_tape_destroy(fx_tape* t) { delete t; }

int fx_tape_describe(const fx_tape* t, fx_tape_info* out) {
  if (!t || !out) return fail(FX_E_ARG, "NULL argument");
  *out = t->info;
  return FX_OK;
}

int fx_tape_eval(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                 fx_shape s, int kind, void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
                 void* stream) {
  if (!t) return fail(FX_E_ARG, "NULL tape");
  if (int rc = check_shape(s)) return rc;
  if (n_inputs < t->prog.n_in || (t->prog.n_in > 0 && !inputs))
    return fail(FX_E_ARG, "tape reads %d inputs, %d given", t->prog.n_in, n_inputs);
  switch (dt) {
    case FX_F32: return tape_eval_typed<float>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, S(stream));
    case FX_F64: return tape_eval_typed<double>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, S(stream));
    case FX_BF16: return tape_eval_typed<bf16_t>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, S(stream));
    case FX_F16: return tape_eval_typed<f16_t>(t->prog, inputs, s, kind, out, ws, ws_bytes, cfg, S(stream));
    default: break;
  }
  return fail(FX_E_DTYPE, "tapes evaluate floating-point dtypes only");
}

}  // extern "C"
