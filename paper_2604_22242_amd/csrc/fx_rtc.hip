// Run-time source mode.  A tree known only at run time is turned into the
// source text of one fused kernel (one SSA value per node, constants as
// exact hexadecimal literals) for one result kind (element-wise, accu,
// norm, column sums or row sums), compiled with hipRTC for the device at
// first use and cached per process by its text.  This follows the paper's
// own mechanism (Sec. 3: kernel source generated from the expression and
// compiled through the driver at first use, then reused), next to the
// ahead-of-time template instantiation and the tape interpreter.  The
// generated kernel does the reads and writes of a compile-time one with no
// interpreter cost; its skeletons take the same per-thread element
// assignment, compensated per-thread sums in the compute type, wave64 + LDS
// block sums in FP64 and single-pass ticket finish as the compile-time
// skeletons, with the library's default block size and EPT of the kind and
// storage type written into the text.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "fx_kernels.hpp"
#include "fx_jit.hpp"
#include "fx_skel_src.hpp"

namespace fx {

namespace {

constexpr int kRtcMaxIn = 4;

bool is_unary(int op) {
  return op == FX_OP_NEG || op == FX_OP_ABS || op == FX_OP_EXP || op == FX_OP_SQRT;
}
bool is_binary(int op) {
  return op == FX_OP_ADD || op == FX_OP_SUB || op == FX_OP_SCHUR || op == FX_OP_DIV;
}

// Storage, compute and dimension-sum output types of a storage dtype.
struct rtc_types {
  const char* st;
  const char* ct;
  const char* acc_out;
  int elem;
};
bool types_of(fx_dtype dt, rtc_types* t) {
  switch (dt) {
    case FX_F32: *t = {"float", "float", "float", 4}; return true;
    case FX_F64: *t = {"double", "double", "double", 8}; return true;
    case FX_BF16: *t = {"__bf16", "float", "float", 2}; return true;
    case FX_F16: *t = {"_Float16", "float", "float", 2}; return true;
    default: return false;
  }
}

std::string literal(double v, bool f32) {
  if (std::isnan(v)) return f32 ? "__builtin_nanf(\"\")" : "__builtin_nan(\"\")";
  if (std::isinf(v)) return std::string(v < 0 ? "-" : "") + (f32 ? "__builtin_inff()" : "__builtin_inf()");
  char b[64];
  if (f32) std::snprintf(b, sizeof b, "%af", (double)(float)v);
  else std::snprintf(b, sizeof b, "%a", v);
  return b;
}

// The expression as straight-line code over t0..t{n-1}; `x{q}` are the
// input values of the element, in the compute type.
int emit_body(const fx_node* nd, int n, bool f32, std::string& body, int* n_in) {
  const char* T = f32 ? "float" : "double";
  *n_in = 0;
  char line[256];
  for (int k = 0; k < n; ++k) {
    const fx_node& e = nd[k];
    std::string rhs;
    if (e.op == FX_OP_LEAF) {
      if (e.input < 0 || e.input >= kRtcMaxIn)
        return fail(FX_E_UNSUPPORTED, "node %d: input %d outside [0, %d)", k, e.input, kRtcMaxIn);
      *n_in = std::max(*n_in, e.input + 1);
      rhs = "x" + std::to_string(e.input);
    } else if (e.op == FX_OP_CONST) {
      rhs = literal(e.value, f32);
    } else if (is_unary(e.op)) {
      if (e.a < 0 || e.a >= k) return fail(FX_E_ARG, "node %d: operand %d not earlier", k, e.a);
      const std::string a = "t" + std::to_string(e.a);
      switch (e.op) {
        case FX_OP_NEG: rhs = "-" + a; break;
        case FX_OP_ABS: rhs = std::string(f32 ? "fabsf(" : "fabs(") + a + ")"; break;
        case FX_OP_EXP: rhs = std::string(f32 ? "expf(" : "exp(") + a + ")"; break;
        default: rhs = std::string(f32 ? "sqrtf(" : "sqrt(") + a + ")"; break;
      }
    } else if (is_binary(e.op)) {
      if (e.a < 0 || e.a >= k || e.b < 0 || e.b >= k)
        return fail(FX_E_ARG, "node %d: operands %d, %d not earlier", k, e.a, e.b);
      const char* o = e.op == FX_OP_ADD ? " + " : e.op == FX_OP_SUB ? " - "
                    : e.op == FX_OP_SCHUR ? " * " : " / ";
      rhs = "t" + std::to_string(e.a) + o + "t" + std::to_string(e.b);
    } else {
      return fail(FX_E_ARG, "node %d: unknown operator %d", k, e.op);
    }
    std::snprintf(line, sizeof line, "  const %s t%d = %s;\n", T, k, rhs.c_str());
    body += line;
  }
  return FX_OK;
}

const char* kind_name(int kind) {
  switch (kind) {
    case 0: return "element-wise";
    case FX_R_ACCU: return "accu";
    case FX_R_NORM: return "norm_fro";
    case FX_R_COLSUM: return "column sums";
    case FX_R_ROWSUM: return "row sums";
  }
  return "?";
}

// The whole program text for one tree, dtype and kind.
std::string kernel_source(const std::string& body, int n_in, const rtc_types& ty, int kind,
                          int block, int ept, int root) {
  const int N = 16 / ty.elem;
  const int nin = std::max(1, n_in);
  std::string s;
  s += std::string("// generated: ") + kind_name(kind) + " of one fused expression, " + ty.st +
       " storage\n";
  s += std::string("typedef ") + ty.st + " st_t;\n";
  s += std::string("typedef ") + ty.ct + " ct_t;\n";
  s += std::string("typedef ") + ty.acc_out + " acc_out_t;\n";
  s += "#define FX_N " + std::to_string(N) + "\n";
  s += "#define FX_NIN " + std::to_string(nin) + "\n";
  s += "#define FX_BLOCK " + std::to_string(block) + "\n";
  s += "#define FX_EPT " + std::to_string(ept) + "\n";
  if (kind == FX_R_NORM) {
    s += "#define FX_MAP(x) ((x) * (x))\n";
    s += "#define FX_FINISH(s) __builtin_sqrt(s)\n";
  } else {
    s += "#define FX_MAP(x) (x)\n";
    s += "#define FX_FINISH(s) (s)\n";
  }
  s += "#define FX_PARAMS const st_t* __restrict__ p0, const st_t* __restrict__ p1, "
       "const st_t* __restrict__ p2, const st_t* __restrict__ p3\n";
  s += "#define FX_ARGS p0, p1, p2, p3\n";
  s += kLoads;
  s += "\n__device__ __forceinline__ ct_t fx_expr(ct_t x0, ct_t x1, ct_t x2, ct_t x3) {\n";
  s += body;
  s += "  return t" + std::to_string(root) + ";\n}\n";
  // the used inputs' loads, then the expression per lane
  s += "template <int N> __device__ __forceinline__ void fx_load(FX_PARAMS, long i, fx_raw<N>& r) {\n";
  for (int q = 0; q < n_in; ++q)
    s += "  fx_ld<N>::run(p" + std::to_string(q) + " + i, r.v[" + std::to_string(q) + "]);\n";
  s += "}\n";
  auto arg = [&](int q, const std::string& x) {
    return q < n_in ? "(ct_t)" + x : std::string("(ct_t)0");
  };
  s += "template <int N> __device__ __forceinline__ void fx_eval(FX_PARAMS, const fx_raw<N>& r, "
       "ct_t* o) {\n";
  s += "#pragma unroll\n";
  s += "  for (int j = 0; j < N; ++j) o[j] = fx_expr(";
  for (int q = 0; q < kRtcMaxIn; ++q)
    s += arg(q, "r.v[" + std::to_string(q) + "][j]") + (q + 1 < kRtcMaxIn ? ", " : ");\n");
  s += "}\n";
  s += "__device__ __forceinline__ ct_t fx_at(FX_PARAMS, long i) {\n  return fx_expr(";
  for (int q = 0; q < kRtcMaxIn; ++q)
    s += arg(q, "p" + std::to_string(q) + "[i]") + (q + 1 < kRtcMaxIn ? ", " : ");\n");
  s += "}\n";
  if (kind == 0) {
    s += kElementwise;
  } else {
    s += kSums;
    s += kind == FX_R_COLSUM ? kColsum : kind == FX_R_ROWSUM ? kRowsum : kFull;
  }
  return s;
}

}  // namespace

}  // namespace fx

using namespace fx;

struct fx_rtc {
  fx_dtype dt;
  int kind;
  int n_in;
  int elem;
  int block, ept;  // the launch configuration written into the source
  std::string source;
  jit_program* prog;
  double compile_ms;  // 0 when the source was found in the cache
};

namespace {

template <class O> int fill_zero(void* out, int64_t n, hipStream_t st) {
  const int grid = (int)std::min<int64_t>(ceil_div(n, 256), 1024);
  hipLaunchKernelGGL((k_fill_zero<O>), dim3(grid), dim3(256), 0, st, static_cast<O*>(out), n);
  return hip_check(hipGetLastError(), "k_fill_zero launch");
}

}  // namespace

extern "C" {

int fx_rtc_create(const fx_node* nodes, int32_t n_nodes, fx_dtype dt, int kind, fx_rtc** out) {
  if (!out) return fail(FX_E_ARG, "NULL output handle");
  *out = nullptr;
  if (!nodes || n_nodes <= 0) return fail(FX_E_ARG, "empty tree");
  rtc_types ty;
  if (!types_of(dt, &ty))
    return fail(FX_E_DTYPE, "the run-time source mode takes FP32, FP64, BF16 or FP16 storage");
  if (kind != 0 && kind != FX_R_ACCU && kind != FX_R_NORM && kind != FX_R_COLSUM &&
      kind != FX_R_ROWSUM)
    return fail(FX_E_ARG, "unknown result kind %d", kind);
  std::string body;
  int n_in = 0;
  if (int rc = emit_body(nodes, n_nodes, dt != FX_F64, body, &n_in)) return rc;
  // the library's default block size and EPT of this kind and storage type
  // (they do not depend on the shape; the split does, and is chosen per call)
  const launch L = resolve(kind == FX_R_NORM ? FX_R_ACCU : kind, ty.elem, 1, 1, nullptr, true);
  std::string src = kernel_source(body, n_in, ty, kind, L.block, L.ept, n_nodes - 1);
  fx_rtc* h = new (std::nothrow) fx_rtc;
  if (!h) return fail(FX_E_ARG, "out of host memory");
  h->dt = dt;
  h->kind = kind;
  h->n_in = n_in;
  h->elem = ty.elem;
  h->block = L.block;
  h->ept = L.ept;
  h->source = src;
  if (int rc = jit_obtain(src.data(), src.size(), &h->prog, &h->compile_ms)) {
    delete h;
    return rc;
  }
  *out = h;
  return FX_OK;
}

void fx_rtc_destroy(fx_rtc* r) { delete r; }  // the compiled code stays cached

int fx_rtc_source(const fx_rtc* r, char* buf, size_t cap, size_t* len) {
  if (!r) return fail(FX_E_ARG, "NULL handle");
  if (len) *len = r->source.size();
  if (buf && cap) {
    const size_t m = std::min(cap - 1, r->source.size());
    std::memcpy(buf, r->source.data(), m);
    buf[m] = 0;
  }
  return FX_OK;
}

double fx_rtc_compile_ms(const fx_rtc* r) { return r ? r->compile_ms : -1.0; }

int fx_rtc_eval(fx_rtc* r, const void* const* inputs, int32_t n_inputs, fx_shape shape, void* out,
                void* ws, size_t ws_bytes, void* stream) {
  if (!r) return fail(FX_E_ARG, "NULL handle");
  const int64_t rows = shape.n_rows, cols = shape.n_cols;
  if (rows < 0 || cols < 0) return fail(FX_E_ARG, "negative shape");
  if (rows > 0 && cols > INT64_MAX / rows) return fail(FX_E_ARG, "shape overflows");
  const int64_t n = rows * cols;
  const int kind = r->kind;
  const bool full = kind == FX_R_ACCU || kind == FX_R_NORM;
  const int64_t nout = kind == 0 ? n : kind == FX_R_COLSUM ? cols : kind == FX_R_ROWSUM ? rows : 1;
  if (nout == 0) return FX_OK;
  if (n_inputs < r->n_in || (r->n_in > 0 && !inputs))
    return fail(FX_E_ARG, "the kernel reads %d inputs, %d given", r->n_in, n_inputs);
  if (!out) return fail(FX_E_ARG, "NULL output pointer");
  uintptr_t addr_or = kind == 0 ? reinterpret_cast<uintptr_t>(out) : 0;
  void* p[kRtcMaxIn] = {nullptr, nullptr, nullptr, nullptr};
  for (int q = 0; q < r->n_in; ++q) {
    if (!inputs[q]) return fail(FX_E_ARG, "NULL input %d", q);
    p[q] = const_cast<void*>(inputs[q]);
    addr_or |= reinterpret_cast<uintptr_t>(inputs[q]);
  }
  if (addr_or & 15) return fail(FX_E_ARG, "the run-time kernels need 16-byte aligned arrays");
  hipStream_t st = S(stream);
  if (n == 0 && !full)  // sums over an empty dimension
    return r->dt == FX_F64 ? fill_zero<double>(out, nout, st) : fill_zero<float>(out, nout, st);
  const int rkind = kind == FX_R_NORM ? FX_R_ACCU : kind;
  const launch L = resolve(rkind, r->elem, rows, cols, nullptr, true);
  if (L.block != r->block || L.ept != r->ept)
    return fail(FX_E_CONFIG, "launch configuration differs from the generated kernel's");
  const int N = 16 / r->elem;
  const int vec = kind == 0 || full || rows % N == 0 ? N : 1;
  const ws_layout W = workspace_for(rkind, rows, cols, L, vec);
  if (W.total() > 0 && (!ws || ws_bytes < W.total()))
    return fail(FX_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", W.total(), ws_bytes);
  const char* names[2] = {nullptr, nullptr};
  const int nf = skeleton_kernels(kind, names);
  hipFunction_t fn[2] = {nullptr, nullptr};
  for (int f = 0; f < nf; ++f)
    if (int rc = jit_function(r->prog, names[f], &fn[f])) return rc;
  long n_l = (long)n, rows_l = (long)rows, cols_l = (long)cols;
  void* o = out;
  void* parts = W.total() > 0 ? static_cast<char*>(ws) + W.counter_bytes : nullptr;
  void* ctr = W.total() > 0 ? ws : nullptr;
  if (kind == 0) {
    void* args[] = {&p[0], &p[1], &p[2], &p[3], &o, &n_l};
    return jit_launch(fn[0], L.split, 1, r->block, args, st);
  }
  if (full) {
    void* args[] = {&p[0], &p[1], &p[2], &p[3], &n_l, &parts, &ctr, &o};
    return jit_launch(fn[0], L.split, 1, r->block, args, st);
  }
  hipFunction_t f = vec > 1 ? fn[0] : fn[1];
  int split = std::max(1, L.split);  // thin columns run as one chunk per column
  if (kind == FX_R_COLSUM) {
    long rpc = (long)(ceil_div(ceil_div(rows, split), vec) * vec);
    void* args[] = {&p[0], &p[1], &p[2], &p[3], &rows_l, &split, &rpc, &parts, &ctr, &o};
    return jit_launch(f, cols, split, r->block, args, st);
  }
  long cpc = (long)ceil_div(cols, split);
  const int64_t rblocks = ceil_div(rows, (int64_t)r->block * vec);
  void* args[] = {&p[0], &p[1], &p[2], &p[3], &rows_l, &cols_l, &split, &cpc, &parts, &ctr, &o};
  return jit_launch(f, rblocks, split, r->block, args, st);
}

}  // extern "C"
