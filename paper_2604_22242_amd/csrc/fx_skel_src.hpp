// The fixed parts of generated kernel source: skeleton kernels written as
// text, shared by both source modes (the run-time one, from a tape's node
// list, and the compile-time one, from an expression's type).  Each piece
// relies on the generated part to define:
//   st_t, ct_t, acc_out_t   storage, compute and dimension-sum output types
//   FX_N, FX_BLOCK, FX_EPT  vector width (elements), block size, EPT
//   FX_NIN                  number of loaded input streams
//   FX_PARAMS / FX_ARGS     the kernel's expression parameters and their names
//   FX_MAP, FX_FINISH       the map before summation and the finish after it
//   fx_load<N>(FX_ARGS, i, raw)   the inputs' N elements at i into raw
//   fx_eval<N>(FX_ARGS, raw, r)   the expression on those N elements
//   fx_at(FX_ARGS, i)             the expression at element i
// The skeletons are those of the compile-time kernels: EPT vectors per input
// loaded before any arithmetic, compensated per-thread sums in the compute type,
// FP64 wave64 + LDS block sums and the single-pass agent-scope ticket finish.
#pragma once

#include "fx.h"

namespace fx {

// Kernel names of a result kind: [vector variant, one-element variant].
inline int skeleton_kernels(int kind, const char** names) {
  switch (kind) {
    case 0: names[0] = "fx_rtc_ew"; return 1;
    case FX_R_ACCU: case FX_R_NORM: names[0] = "fx_rtc_full"; return 1;
    case FX_R_COLSUM: names[0] = "fx_rtc_colsum_v"; names[1] = "fx_rtc_colsum_s"; return 2;
    default: names[0] = "fx_rtc_rowsum_v"; names[1] = "fx_rtc_rowsum_s"; return 2;
  }
}


// Loads: N consecutive elements at p, one 16-byte streaming load (N = FX_N)
// or one element (N = 1).
inline constexpr char kLoads[] = R"(typedef unsigned int fx_u32x4 __attribute__((ext_vector_type(4)));
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
inline constexpr char kElementwise[] = R"(
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
      for (int k = 0; k < FX_EPT; ++k) fx_eval<FX_N>(FX_ARGS, raw[k], r[k]);
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
          fx_eval<FX_N>(FX_ARGS, raw, r);
          fx_store(z + v * FX_N, r);
        }
      }
    }
  }
  if (blockIdx.x == gridDim.x - 1)
    for (long i = nv * FX_N + threadIdx.x; i < n; i += FX_BLOCK) z[i] = (st_t)fx_at(FX_ARGS, i);
}
)";

// Sums: compensated per-thread sums in the compute type (Neumaier's
// refinement of Kahan's method: c collects the exact rounding error of every
// addition into s, taken with Knuth's TwoSum), one compensated add per
// element, handed upward in FP64; the block sum is a
// wave64 butterfly and then the waves' results in order; partials are
// published with agent-scope stores and the block that draws the last ticket
// of an agent-scope counter adds them in index order after one acquire, then
// clears the counter.
inline constexpr char kSums[] = R"(
struct fx_acc {
  ct_t s, c;
};
__device__ __forceinline__ void fx_add(fx_acc& a, ct_t t) {
#pragma clang fp contract(off)
  const ct_t u = a.s + t;
  const ct_t tv = u - a.s, sv = u - tv;  // TwoSum: the exact error of a.s + t
  a.c += (a.s - sv) + (t - tv);
  a.s = u;
}
__device__ __forceinline__ double fx_value(const fx_acc& a) {
  return __builtin_isfinite(a.s) ? (double)a.s + (double)a.c : (double)a.s;
}
// one chain per vector lane, added in FP64 in lane order
template <int N> __device__ __forceinline__ double fx_lanes_value(const fx_acc (&a)[N]) {
  double t = fx_value(a[0]);
#pragma unroll
  for (int j = 1; j < N; ++j) t += fx_value(a[j]);
  return t;
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
inline constexpr char kFull[] = R"(
extern "C" __global__ __launch_bounds__(FX_BLOCK) void fx_rtc_full(FX_PARAMS, long n, double* partials,
                                                                   unsigned* counter, double* out) {
  __shared__ double lds[FX_BLOCK / 64];
  fx_acc acc[FX_N];
#pragma unroll
  for (int j = 0; j < FX_N; ++j) acc[j] = fx_acc{0, 0};
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
      for (int k = 0; k < FX_EPT; ++k) fx_eval<FX_N>(FX_ARGS, raw[k], r[k]);
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k)
#pragma unroll
        for (int j = 0; j < FX_N; ++j) fx_add(acc[j], FX_MAP(r[k][j]));
    } else {
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) {
        const long v = v0 + (long)k * FX_BLOCK;
        if (v < nv) {
          fx_raw<FX_N> raw;
          ct_t r[FX_N];
          fx_load<FX_N>(FX_ARGS, v * FX_N, raw);
          fx_eval<FX_N>(FX_ARGS, raw, r);
#pragma unroll
          for (int j = 0; j < FX_N; ++j) fx_add(acc[j], FX_MAP(r[j]));
        }
      }
    }
  }
  if (blockIdx.x == gridDim.x - 1)
    for (long i = nv * FX_N + threadIdx.x; i < n; i += FX_BLOCK) fx_add(acc[0], FX_MAP(fx_at(FX_ARGS, i)));
  const double s = fx_block_sum(fx_lanes_value(acc), lds);
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
inline constexpr char kColsum[] = R"(
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
  fx_acc acc[N];
#pragma unroll
  for (int j = 0; j < N; ++j) acc[j] = fx_acc{0, 0};
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
      for (int k = 0; k < FX_EPT; ++k) fx_eval<N>(FX_ARGS, raw[k], r[k]);
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k)
#pragma unroll
        for (int j = 0; j < N; ++j) fx_add(acc[j], r[k][j]);
    } else {
#pragma unroll
      for (int k = 0; k < FX_EPT; ++k) {
        const long v = v0 + (long)k * FX_BLOCK;
        if (v < nv) {
          fx_raw<N> raw;
          ct_t r[N];
          fx_load<N>(FX_ARGS, base + v * N, raw);
          fx_eval<N>(FX_ARGS, raw, r);
#pragma unroll
          for (int j = 0; j < N; ++j) fx_add(acc[j], r[j]);
        }
      }
    }
  }
  const double sum = fx_block_sum(fx_lanes_value(acc), lds);
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
inline constexpr char kRowsum[] = R"(
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
      for (int k = 0; k < FX_EPT; ++k) fx_eval<N>(FX_ARGS, raw[k], r[k]);
#pragma unroll
      for (int j = 0; j < N; ++j)  // row j's FX_EPT columns, in column order
#pragma unroll
        for (int k = 0; k < FX_EPT; ++k) fx_add(acc[j], r[k][j]);
    }
    for (; c < c1; ++c) {
      fx_raw<N> raw;
      ct_t r[N];
      fx_load<N>(FX_ARGS, r0 + c * n_rows, raw);
      fx_eval<N>(FX_ARGS, raw, r);
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

}  // namespace fx
