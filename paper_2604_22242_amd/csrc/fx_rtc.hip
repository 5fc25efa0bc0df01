// Run-time source mode.  A tree known only at run time is turned into the
// source text of one fused element-wise kernel (one SSA value per node,
// constants as exact hexadecimal literals), compiled with hipRTC for the
// device at first use and cached per process by its text.  This follows the
// paper's own mechanism (Sec. 3: kernel source generated from the expression
// and compiled through the driver at first use, then reused), next to the
// ahead-of-time template instantiation and the tape interpreter; the
// compiled kernel does the same reads and writes as a compile-time one and
// has no interpreter overhead, at the price of a compilation per new tree.
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fx_kernels.hpp"

namespace fx {

namespace {

constexpr int kRtcBlock = 256;
constexpr int kRtcMaxIn = 4;

// One compiled source: its code object and, per device, the loaded module.
struct rtc_entry {
  std::vector<char> code;
  std::map<int, std::pair<hipModule_t, hipFunction_t>> loaded;
};

std::mutex& cache_mutex() {
  static std::mutex m;
  return m;
}
std::map<std::string, rtc_entry*>& cache() {
  static std::map<std::string, rtc_entry*> c;  // entries live until the process ends
  return c;
}

bool is_unary(int op) {
  return op == FX_OP_NEG || op == FX_OP_ABS || op == FX_OP_EXP || op == FX_OP_SQRT;
}
bool is_binary(int op) {
  return op == FX_OP_ADD || op == FX_OP_SUB || op == FX_OP_SCHUR || op == FX_OP_DIV;
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
// input values of the element.
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
    std::snprintf(line, sizeof line, "    const %s t%d = %s;\n", T, k, rhs.c_str());
    body += line;
  }
  return FX_OK;
}

// Element-wise kernel: each thread one 16-byte vector of every input (N
// elements), a scalar tail for the last n % N elements.
std::string kernel_source(const std::string& body, int n_in, bool f32, int root) {
  const char* T = f32 ? "float" : "double";
  const int N = f32 ? 4 : 2;
  const char* V = "vec_t";
  std::string s;
  s += "// generated: one fused element-wise kernel\n";
  s += std::string("typedef ") + T + " vec_t __attribute__((ext_vector_type(" + std::to_string(N) +
       ")));\n";
  s += "extern \"C\" __global__ __launch_bounds__(" + std::to_string(kRtcBlock) +
       ") void fx_rtc_ew(";
  for (int q = 0; q < kRtcMaxIn; ++q)
    s += std::string("const ") + T + "* __restrict__ p" + std::to_string(q) + ", ";
  s += std::string(T) + "* __restrict__ z, long n) {\n";
  s += "  const long i0 = ((long)blockIdx.x * " + std::to_string(kRtcBlock) +
       " + threadIdx.x) * " + std::to_string(N) + ";\n";
  s += "  if (i0 + " + std::to_string(N) + " <= n) {\n";
  for (int q = 0; q < n_in; ++q)
    s += std::string("    const ") + V + " v" + std::to_string(q) +
         " = __builtin_nontemporal_load((const " + V + "*)(p" + std::to_string(q) + " + i0));\n";
  s += std::string("    ") + T + " r[" + std::to_string(N) + "];\n";
  s += "    #pragma unroll\n";
  s += "    for (int j = 0; j < " + std::to_string(N) + "; ++j) {\n";
  for (int q = 0; q < n_in; ++q)
    s += std::string("      const ") + T + " x" + std::to_string(q) + " = v" + std::to_string(q) +
         "[j];\n";
  std::string ind;
  for (size_t a = 0, b; a < body.size(); a = b + 1) {
    b = body.find('\n', a);
    ind += "  " + body.substr(a, b - a + 1);
  }
  s += ind;
  s += "      r[j] = t" + std::to_string(root) + ";\n";
  s += "    }\n";
  s += std::string("    *(") + V + "*)(z + i0) = (" + V + "){" +
       (f32 ? "r[0], r[1], r[2], r[3]" : "r[0], r[1]") + "};\n";
  s += "  } else {\n";
  s += "    for (long i = i0; i < n; ++i) {\n";
  for (int q = 0; q < n_in; ++q)
    s += std::string("      const ") + T + " x" + std::to_string(q) + " = p" + std::to_string(q) +
         "[i];\n";
  s += ind;
  s += "      z[i] = t" + std::to_string(root) + ";\n";
  s += "    }\n";
  s += "  }\n";
  s += "}\n";
  return s;
}

int compile(const std::string& src, std::vector<char>& code, std::string& log) {
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, src.c_str(), "fx_rtc.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(FX_E_HIP, "hiprtcCreateProgram failed");
  // the library's own flags: gfx950, -O3, IEEE divide/sqrt and denormals,
  // no packed FP32 instructions
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(p, 6, opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(p, &ls);
  if (ls > 1) {
    log.resize(ls);
    hiprtcGetProgramLog(p, &log[0]);
  }
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&p);
    return fail(FX_E_HIP, "hipRTC compilation failed (%s): %.400s", hiprtcGetErrorString(r),
                log.c_str());
  }
  size_t cs = 0;
  hiprtcGetCodeSize(p, &cs);
  code.resize(cs);
  hiprtcGetCode(p, code.data());
  hiprtcDestroyProgram(&p);
  return FX_OK;
}

}  // namespace

}  // namespace fx

using namespace fx;

struct fx_rtc {
  fx_dtype dt;
  int n_in;
  std::string source;
  rtc_entry* entry;
  double compile_ms;  // 0 when the source was found in the cache
};

extern "C" {

int fx_rtc_create(const fx_node* nodes, int32_t n_nodes, fx_dtype dt, fx_rtc** out) {
  if (!out) return fail(FX_E_ARG, "NULL output handle");
  *out = nullptr;
  if (!nodes || n_nodes <= 0) return fail(FX_E_ARG, "empty tree");
  if (dt != FX_F32 && dt != FX_F64)
    return fail(FX_E_DTYPE, "the run-time source mode is built for FP32 and FP64 storage");
  const bool f32 = dt == FX_F32;
  std::string body;
  int n_in = 0;
  if (int rc = emit_body(nodes, n_nodes, f32, body, &n_in)) return rc;
  std::string src = kernel_source(body, n_in, f32, n_nodes - 1);
  fx_rtc* h = new (std::nothrow) fx_rtc;
  if (!h) return fail(FX_E_ARG, "out of host memory");
  h->dt = dt;
  h->n_in = n_in;
  h->source = src;
  h->compile_ms = 0;
  std::lock_guard<std::mutex> g(cache_mutex());
  auto it = cache().find(src);
  if (it == cache().end()) {
    rtc_entry* e = new (std::nothrow) rtc_entry;
    if (!e) {
      delete h;
      return fail(FX_E_ARG, "out of host memory");
    }
    std::string log;
    const auto t0 = std::chrono::steady_clock::now();
    if (int rc = compile(src, e->code, log)) {
      delete e;
      delete h;
      return rc;
    }
    h->compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    it = cache().emplace(src, e).first;
  }
  h->entry = it->second;
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

int fx_rtc_eval(fx_rtc* r, const void* const* inputs, int32_t n_inputs, int64_t n, void* out,
                void* stream) {
  if (!r) return fail(FX_E_ARG, "NULL handle");
  if (n < 0) return fail(FX_E_ARG, "negative size");
  if (n == 0) return FX_OK;
  if (n_inputs < r->n_in || (r->n_in > 0 && !inputs))
    return fail(FX_E_ARG, "the kernel reads %d inputs, %d given", r->n_in, n_inputs);
  if (!out) return fail(FX_E_ARG, "NULL output pointer");
  const size_t elem = r->dt == FX_F32 ? 4 : 8;
  uintptr_t addr_or = reinterpret_cast<uintptr_t>(out);
  const void* p[kRtcMaxIn] = {nullptr, nullptr, nullptr, nullptr};
  for (int q = 0; q < r->n_in; ++q) {
    if (!inputs[q]) return fail(FX_E_ARG, "NULL input %d", q);
    p[q] = inputs[q];
    addr_or |= reinterpret_cast<uintptr_t>(inputs[q]);
  }
  if (addr_or & 15) return fail(FX_E_ARG, "the run-time kernels need 16-byte aligned arrays");
  int dev = 0;
  if (int rc = hip_check(hipGetDevice(&dev), "hipGetDevice")) return rc;
  hipFunction_t fn;
  {
    std::lock_guard<std::mutex> g(cache_mutex());
    auto it = r->entry->loaded.find(dev);
    if (it == r->entry->loaded.end()) {
      hipModule_t m;
      if (int rc = hip_check(hipModuleLoadData(&m, r->entry->code.data()), "hipModuleLoadData"))
        return rc;
      hipFunction_t f;
      if (int rc = hip_check(hipModuleGetFunction(&f, m, "fx_rtc_ew"), "hipModuleGetFunction"))
        return rc;
      it = r->entry->loaded.emplace(dev, std::make_pair(m, f)).first;
    }
    fn = it->second.second;
  }
  const int64_t N = 16 / (int64_t)elem;
  const int64_t blocks = ceil_div(ceil_div(n, N), kRtcBlock);
  if (blocks > 0x7fffffff) return fail(FX_E_UNSUPPORTED, "%lld elements exceed the grid", (long long)n);
  long nl = (long)n;
  void* z = out;
  void* args[] = {&p[0], &p[1], &p[2], &p[3], &z, &nl};
  return hip_check(hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, kRtcBlock, 1, 1, 0,
                                         S(stream), args, nullptr),
                   "fx_rtc_ew launch");
}

}  // extern "C"
