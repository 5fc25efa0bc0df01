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
// assignment, Neumaier per-thread sums in the compute type, wave64 + LDS
// block sums in FP64 and single-pass ticket finish as the compile-time
// skeletons, with the library's default block size and EPT of the kind and
// storage type written into the text.
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
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

constexpr int kRtcMaxIn = 4;
constexpr int kRtcMaxFns = 2;  // a vector and a one-element variant

// One compiled source: its code object and, per device, the loaded module
// and its kernels.
struct rtc_module {
  hipModule_t mod;
  hipFunction_t fn[kRtcMaxFns];
};
struct rtc_entry {
  std::vector<char> code;
  std::map<int, rtc_module> loaded;
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

// ---- fixed parts of the generated text ------------------------------------

// Loads: N consecutive elements at p, one 16-byte streaming load (N = FX_N)
// or one element (N = 1).
const char kLoads[] = R"(typedef unsigned int fx_u32x4 __attribute__((ext_vector_type(4)));
#define FX_PARAMS const st_t* __restrict__ p0, const st_t* __restrict__ p1, \
                  const st_t* __restrict__ p2, const st_t* __restrict__ p3
#define FX_ARGS p0, p1, p2, p3
template <int N> struct fx_ld {
  __device__ static __forceinline__ void run(const st_t* p, st_t* o) {
    const fx_u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const fx_u32x4*>(p));
    __builtin_memcpy(o, &v, 16);
  }
};
template <> struct fx_ld<1> {
  __device__ static __forceinline__ void run(const st_t* p, st_t* o) { o[0] = *p; }
};
template <int N> struct fx_raw { st_t v[FX_NIN][N]; };
)";

// Element-wise: tiles of FX_BLOCK * FX_EPT vectors, the EPT loads of every
// input issued before any arithmetic; the last block also does the
// n % FX_N scalar tail.
const char kElementwise[] = R"(
__device__ __forceinline__ void fx_store(st_t* z, const ct_t* r) {
  st_t s[FX_N];
#pragma unroll
  for (int j = 0; j < FX_N; ++j) s[j] = (st_t)r[j];
  fx_u32x4 v;
  __builtin_memcpy(&v, s, 16);
  *reinterpret_cast<fx_u32x4*>(z) = v;
}

extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_ew(FX_PARAMS, st_t* __restrict__ z,
                                                                 long n) {
  const long nv = n / FX_N;
  const long tile = (long)FX_BLOCK * FX_EPT;
  for (long t = blockIdx.x; t * tile < nv; t += gridDim.x) {
    const long v0 = t * tile + threadIdx.x;
    if ((t + 1) * tile <= nv) {
      fx_raw<FX_N> raw[FX_EPT];
      ct_t r[FX_EPT][FX_N];
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_load<FX_N>(FX_ARGS, (v0 + (long)k * FX_BLOCK) * FX_N, raw[k]);
      __builtin_amdgcn_sched_barrier(0);  // every load ahead of the arithmetic
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_eval<FX_N>(raw[k], r[k]);
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_store(z + (v0 + (long)k * FX_BLOCK) * FX_N, r[k]);
    } else {
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) {
        const long v = v0 + (long)k * FX_BLOCK;
        if (v < nv) {
          fx_raw<FX_N> raw;
          ct_t r[FX_N];
          fx_load<FX_N>(FX_ARGS, v * FX_N, raw);
          fx_eval<FX_N>(raw, r);
          fx_store(z + v * FX_N, r);
        }
      }
    }
  }
  if (blockIdx.x == gridDim.x - 1)
    for (long i = nv * FX_N + threadIdx.x; i < n; i += FX_BLOCK) z[i] = (st_t)fx_at(FX_ARGS, i);
}
)";

// Sums: Neumaier's compensated per-thread sum in the compute type, of the
// pairwise pre-added values of each tile, handed upward in FP64; the block sum is a wave64 butterfly and then the waves'
// results in order; partials are published with agent-scope stores and the
// block that draws the last ticket of an agent-scope counter adds them in
// index order after one acquire, then clears the counter.
const char kSums[] = R"(
__device__ __forceinline__ float fx_abs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double fx_abs(double x) { return __builtin_fabs(x); }
struct fx_acc {
  ct_t s, c;
};
__device__ __forceinline__ void fx_add(fx_acc& a, ct_t t) {
#pragma clang fp contract(off)
  const ct_t u = a.s + t;
  const ct_t e = fx_abs(a.s) >= fx_abs(t) ? (a.s - u) + t : (t - u) + a.s;
  a.c += e;
  a.s = u;
}
__device__ __forceinline__ double fx_value(const fx_acc& a) { return (double)a.s + (double)a.c; }
// a thread's K values of one tile, pre-added as a balanced pairwise tree and
// handed to the compensated sum as one term
template <int K> __device__ __forceinline__ ct_t fx_tree(ct_t (&v)[K]) {
#pragma unroll
  for (int w = 1; w < K; w *= 2)
#pragma unroll
    for (int i = 0; i + w < K; i += 2 * w) v[i] += v[i + w];
  return v[0];
}

__device__ __forceinline__ double fx_block_sum(double v, double* lds) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < FX_BLOCK / 64; ++w) t += lds[w];
  return t;
}

__device__ __forceinline__ void fx_publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool fx_last_ticket(unsigned* counter, unsigned expected) {
  __shared__ bool last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
           expected - 1;
  __syncthreads();
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}
__device__ __forceinline__ void fx_reset(unsigned* counter) {
  __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
)";

// Full reduction: out = FX_FINISH(sum FX_MAP(E_i)), one FP64 value; blocks
// walk tiles of FX_BLOCK * FX_EPT vectors grid-stride.
const char kFull[] = R"(
extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_full(FX_PARAMS, long n, double* partials,
                                                                   unsigned* counter, double* out) {
  __shared__ double lds[FX_BLOCK / 64];
  fx_acc acc = {0, 0};
  const long nv = n / FX_N;
  const long tile = (long)FX_BLOCK * FX_EPT;
  for (long t = blockIdx.x; t * tile < nv; t += gridDim.x) {
    const long v0 = t * tile + threadIdx.x;
    if ((t + 1) * tile <= nv) {
      fx_raw<FX_N> raw[FX_EPT];
      ct_t r[FX_EPT][FX_N];
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_load<FX_N>(FX_ARGS, (v0 + (long)k * FX_BLOCK) * FX_N, raw[k]);
      __builtin_amdgcn_sched_barrier(0);  // every load ahead of the arithmetic
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_eval<FX_N>(raw[k], r[k]);
      ct_t v[FX_EPT * FX_N];
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k)
#pragma unroll
        for (int j = 0; j < FX_N; ++j) v[k * FX_N + j] = FX_MAP(r[k][j]);
      fx_add(acc, fx_tree<FX_EPT * FX_N>(v));
    } else {
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) {
        const long v = v0 + (long)k * FX_BLOCK;
        if (v < nv) {
          fx_raw<FX_N> raw;
          ct_t r[FX_N];
          fx_load<FX_N>(FX_ARGS, v * FX_N, raw);
          fx_eval<FX_N>(raw, r);
#pragma unroll
          for (int j = 0; j < FX_N; ++j) r[j] = FX_MAP(r[j]);
          fx_add(acc, fx_tree<FX_N>(r));
        }
      }
    }
  }
  if (blockIdx.x == gridDim.x - 1)
    for (long i = nv * FX_N + threadIdx.x; i < n; i += FX_BLOCK) fx_add(acc, FX_MAP(fx_at(FX_ARGS, i)));
  const double s = fx_block_sum(fx_value(acc), lds);
  if (gridDim.x == 1) {
    if (threadIdx.x == 0) *out = FX_FINISH(s);
    return;
  }
  if (threadIdx.x == 0) fx_publish(partials + blockIdx.x, s);
  if (fx_last_ticket(counter, gridDim.x)) {
    double t = 0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += FX_BLOCK) t += partials[b];
    t = fx_block_sum(t, lds);
    if (threadIdx.x == 0) {
      *out = FX_FINISH(t);
      fx_reset(counter);
    }
  }
}
)";

// Column sums: block (column c, chunk s) sums rows [s*rpc, (s+1)*rpc) of
// column c, a contiguous run; with split > 1 the chunk partials go to
// partials[c*split + s] and the last block of column c adds them in chunk
// order.  The vector variant needs FX_N | n_rows (rpc is then a multiple of
// FX_N).
const char kColsum[] = R"(
template <int N>
__device__ __forceinline__ void fx_colsum(FX_PARAMS, long n_rows, int split, long rpc, double* partials,
                                          unsigned* counters, acc_out_t* out) {
  __shared__ double lds[FX_BLOCK / 64];
  const long col = blockIdx.x;
  const int s = blockIdx.y;
  const long r0 = (long)s * rpc;
  const long r1 = n_rows < r0 + rpc ? n_rows : r0 + rpc;
  const long base = col * n_rows + r0;
  const long nv = r1 > r0 ? (r1 - r0) / N : 0;
  fx_acc acc = {0, 0};
  const long tile = (long)FX_BLOCK * FX_EPT;
  for (long t0 = 0; t0 < nv; t0 += tile) {
    const long v0 = t0 + threadIdx.x;
    if (t0 + tile <= nv) {
      fx_raw<N> raw[FX_EPT];
      ct_t r[FX_EPT][N];
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_load<N>(FX_ARGS, base + (v0 + (long)k * FX_BLOCK) * N, raw[k]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_eval<N>(raw[k], r[k]);
      ct_t v[FX_EPT * N];
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k)
#pragma unroll
        for (int j = 0; j < N; ++j) v[k * N + j] = r[k][j];
      fx_add(acc, fx_tree<FX_EPT * N>(v));
    } else {
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) {
        const long v = v0 + (long)k * FX_BLOCK;
        if (v < nv) {
          fx_raw<N> raw;
          ct_t r[N];
          fx_load<N>(FX_ARGS, base + v * N, raw);
          fx_eval<N>(raw, r);
          fx_add(acc, fx_tree<N>(r));
        }
      }
    }
  }
  const double sum = fx_block_sum(fx_value(acc), lds);
  if (split == 1) {
    if (threadIdx.x == 0) out[col] = (acc_out_t)sum;
    return;
  }
  if (threadIdx.x == 0) fx_publish(partials + col * split + s, sum);
  if (fx_last_ticket(counters + col, split)) {
    if (threadIdx.x == 0) {
      double t = 0;
      for (int q = 0; q < split; ++q) t += partials[col * split + q];
      out[col] = (acc_out_t)t;
      fx_reset(counters + col);
    }
  }
}
extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_colsum_v(FX_PARAMS, long n_rows, int split,
    long rpc, double* partials, unsigned* counters, acc_out_t* out) {
  fx_colsum<FX_N>(FX_ARGS, n_rows, split, rpc, partials, counters, out);
}
extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_colsum_s(FX_PARAMS, long n_rows, int split,
    long rpc, double* partials, unsigned* counters, acc_out_t* out) {
  fx_colsum<1>(FX_ARGS, n_rows, split, rpc, partials, counters, out);
}
)";

// Row sums: a thread owns rows [r0, r0 + N) (one vector per column, so a
// wave reads consecutive vectors of one column) and walks the columns of its
// chunk FX_EPT at a time; with split > 1 the chunk partials go to
// partials[s*n_rows + r] and the last block of a row block adds them in
// chunk order.  The vector variant needs FX_N | n_rows.
const char kRowsum[] = R"(
template <int N>
__device__ __forceinline__ void fx_rowsum(FX_PARAMS, long n_rows, long n_cols, int split, long cpc,
                                          double* partials, unsigned* counters, acc_out_t* out) {
  const int s = blockIdx.y;
  const long r0 = ((long)blockIdx.x * FX_BLOCK + threadIdx.x) * N;
  const bool active = r0 < n_rows;
  const long c0 = (long)s * cpc;
  const long c1 = n_cols < c0 + cpc ? n_cols : c0 + cpc;
  fx_acc acc[N];
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = fx_acc{0, 0};
  if (active) {
    long c = c0;
    for (; c + FX_EPT <= c1; c += FX_EPT) {
      fx_raw<N> raw[FX_EPT];
      ct_t r[FX_EPT][N];
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_load<N>(FX_ARGS, r0 + (c + k) * n_rows, raw[k]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) fx_eval<N>(raw[k], r[k]);
#pragma unroll
      for (int j = 0; j < N; ++j) {  // row j's FX_EPT columns, pre-added
        ct_t v[FX_EPT];
#pragma unroll
        for (int k = 0; k < FX_EPT; ++k) v[k] = r[k][j];
        fx_add(acc[j], fx_tree<FX_EPT>(v));
      }
    }
    for (; c < c1; ++c) {
      fx_raw<N> raw;
      ct_t r[N];
      fx_load<N>(FX_ARGS, r0 + c * n_rows, raw);
      fx_eval<N>(raw, r);
#pragma unroll
      for (int j = 0; j < N; ++j) fx_add(acc[j], r[j]);
    }
  }
  if (split == 1) {
    if (active)
#pragma unroll
      for (int j = 0; j < N; ++j) out[r0 + j] = (acc_out_t)fx_value(acc[j]);
    return;
  }
  if (active)
#pragma unroll
    for (int j = 0; j < N; ++j) fx_publish(partials + (long)s * n_rows + r0 + j, fx_value(acc[j]));
  if (fx_last_ticket(counters + blockIdx.x, split)) {
    if (active) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        double t = 0;
        for (int q = 0; q < split; ++q) t += partials[(long)q * n_rows + r0 + j];
        out[r0 + j] = (acc_out_t)t;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) fx_reset(counters + blockIdx.x);
  }
}
extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_rowsum_v(FX_PARAMS, long n_rows, long n_cols,
    int split, long cpc, double* partials, unsigned* counters, acc_out_t* out) {
  fx_rowsum<FX_N>(FX_ARGS, n_rows, n_cols, split, cpc, partials, counters, out);
}
extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_rowsum_s(FX_PARAMS, long n_rows, long n_cols,
    int split, long cpc, double* partials, unsigned* counters, acc_out_t* out) {
  fx_rowsum<1>(FX_ARGS, n_rows, n_cols, split, cpc, partials, counters, out);
}
)";

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
  s += "template <int N> __device__ __forceinline__ void fx_eval(const fx_raw<N>& r, ct_t* o) {\n";
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

// Kernel names of a kind: [vector variant, one-element variant].
int kernel_names(int kind, const char** names) {
  switch (kind) {
    case 0: names[0] = "fx_rtc_ew"; return 1;
    case FX_R_ACCU: case FX_R_NORM: names[0] = "fx_rtc_full"; return 1;
    case FX_R_COLSUM: names[0] = "fx_rtc_colsum_v"; names[1] = "fx_rtc_colsum_s"; return 2;
    default: names[0] = "fx_rtc_rowsum_v"; names[1] = "fx_rtc_rowsum_s"; return 2;
  }
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
  int kind;
  int n_in;
  int elem;
  int block, ept;  // the launch configuration written into the source
  std::string source;
  rtc_entry* entry;
  double compile_ms;  // 0 when the source was found in the cache
};

namespace {

// The kernels of r on the current device, loading the module at first use.
int functions(fx_rtc* r, hipFunction_t* fn) {
  int dev = 0;
  if (int rc = hip_check(hipGetDevice(&dev), "hipGetDevice")) return rc;
  std::lock_guard<std::mutex> g(cache_mutex());
  auto it = r->entry->loaded.find(dev);
  if (it == r->entry->loaded.end()) {
    rtc_module m{};
    if (int rc = hip_check(hipModuleLoadData(&m.mod, r->entry->code.data()), "hipModuleLoadData"))
      return rc;
    const char* names[kRtcMaxFns] = {nullptr, nullptr};
    const int nf = kernel_names(r->kind, names);
    for (int f = 0; f < nf; ++f) {
      if (int rc = hip_check(hipModuleGetFunction(&m.fn[f], m.mod, names[f]), names[f])) {
        (void)hipModuleUnload(m.mod);
        return rc;
      }
    }
    it = r->entry->loaded.emplace(dev, m).first;
  }
  for (int f = 0; f < kRtcMaxFns; ++f) fn[f] = it->second.fn[f];
  return FX_OK;
}

int launch_fn(hipFunction_t f, int64_t gx, int64_t gy, int block, void** args, hipStream_t st) {
  if (gx > 0x7fffffff || gy > 65535)
    return fail(FX_E_UNSUPPORTED, "grid %lld x %lld too large", (long long)gx, (long long)gy);
  return hip_check(hipModuleLaunchKernel(f, (unsigned)gx, (unsigned)gy, 1, (unsigned)block, 1, 1, 0,
                                         st, args, nullptr),
                   "run-time kernel launch");
}

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
  hipFunction_t fn[kRtcMaxFns] = {nullptr, nullptr};
  if (int rc = functions(r, fn)) return rc;
  long n_l = (long)n, rows_l = (long)rows, cols_l = (long)cols;
  void* o = out;
  void* parts = W.total() > 0 ? static_cast<char*>(ws) + W.counter_bytes : nullptr;
  void* ctr = W.total() > 0 ? ws : nullptr;
  if (kind == 0) {
    void* args[] = {&p[0], &p[1], &p[2], &p[3], &o, &n_l};
    return launch_fn(fn[0], L.split, 1, r->block, args, st);
  }
  if (full) {
    void* args[] = {&p[0], &p[1], &p[2], &p[3], &n_l, &parts, &ctr, &o};
    return launch_fn(fn[0], L.split, 1, r->block, args, st);
  }
  hipFunction_t f = vec > 1 ? fn[0] : fn[1];
  int split = std::max(1, L.split);  // thin columns run as one chunk per column
  if (kind == FX_R_COLSUM) {
    long rpc = (long)(ceil_div(ceil_div(rows, split), vec) * vec);
    void* args[] = {&p[0], &p[1], &p[2], &p[3], &rows_l, &split, &rpc, &parts, &ctr, &o};
    return launch_fn(f, cols, split, r->block, args, st);
  }
  long cpc = (long)ceil_div(cols, split);
  const int64_t rblocks = ceil_div(rows, (int64_t)r->block * vec);
  void* args[] = {&p[0], &p[1], &p[2], &p[3], &rows_l, &cols_l, &split, &cpc, &parts, &ctr, &o};
  return launch_fn(f, rblocks, split, r->block, args, st);
}

}  // extern "C"
