// Core device/host helpers of the fused-expression library for gfx950:
// storage/compute type traits, 16-byte vector loads and stores, compensated
// per-thread accumulation, wave64 + LDS block reduction, launch
// configuration and error reporting.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "fx.h"

namespace fx {

// ---------------------------------------------------------------------------
// Storage types and their compute types.  Half formats are stored as clang's
// __bf16 / _Float16 and computed in FP32 (low-precision storage, FP32
// arithmetic); FP64 computes in FP64; u32 in u32 (mod 2^32).

using bf16_t = __bf16;
using f16_t = _Float16;

template <class T> struct traits;
template <> struct traits<float> {
  using ct = float; using acc = float;
  static constexpr fx_dtype id = FX_F32;
};
template <> struct traits<double> {
  using ct = double; using acc = double;
  static constexpr fx_dtype id = FX_F64;
};
template <> struct traits<bf16_t> {
  using ct = float; using acc = float;
  static constexpr fx_dtype id = FX_BF16;
};
template <> struct traits<f16_t> {
  using ct = float; using acc = float;
  static constexpr fx_dtype id = FX_F16;
};
template <> struct traits<uint32_t> {
  using ct = uint32_t; using acc = uint64_t;
  static constexpr fx_dtype id = FX_U32;
};
template <class T> using ct_t = typename traits<T>::ct;

// A short array of N compute-type lanes (one vector load's worth).
template <class C, int N> struct lanes {
  C v[N];
};

// Raw bit containers for one load of B bytes.
template <int B> struct raw;
template <> struct raw<2> { using type = unsigned short; };
template <> struct raw<4> { using type = unsigned int; };
template <> struct raw<8> { using type = unsigned int __attribute__((ext_vector_type(2))); };
template <> struct raw<16> { using type = unsigned int __attribute__((ext_vector_type(4))); };

// Load N consecutive elements at p + i (p + i aligned to N*sizeof(T)) and
// widen them to the compute type.  NT selects the nontemporal (streaming)
// cache policy.
// Vectors wider than 16 bytes (a wide leaf inside an expression of a
// narrower storage type) are read as several 16-byte loads.
template <int N, bool NT, class T>
__device__ __forceinline__ lanes<ct_t<T>, N> load_lanes(const T* __restrict__ p, int64_t i) {
  constexpr int BYTES = N * (int)sizeof(T);
  constexpr int CHUNK = BYTES > 16 ? 16 : BYTES;
  constexpr int PER = CHUNK / (int)sizeof(T);  // elements per load
  using R = typename raw<CHUNK>::type;
  T s[N];
#pragma unroll
  for (int c = 0; c < N / PER; ++c) {
    const R* q = reinterpret_cast<const R*>(p + i + c * PER);
    R r = NT ? __builtin_nontemporal_load(q) : *q;
    __builtin_memcpy(s + c * PER, &r, sizeof(R));
  }
  lanes<ct_t<T>, N> out;
#pragma unroll
  for (int j = 0; j < N; ++j) out.v[j] = static_cast<ct_t<T>>(s[j]);
  return out;
}

// Round N compute-type lanes to the storage type (IEEE nearest-even) and
// store them at p + i.
template <int N, bool NT, class T>
__device__ __forceinline__ void store_lanes(T* __restrict__ p, int64_t i, const lanes<ct_t<T>, N>& x) {
  using R = typename raw<N * (int)sizeof(T)>::type;
  T s[N];
#pragma unroll
  for (int j = 0; j < N; ++j) s[j] = static_cast<T>(x.v[j]);
  R r;
  __builtin_memcpy(&r, s, sizeof(R));
  R* q = reinterpret_cast<R*>(p + i);
  if (NT) __builtin_nontemporal_store(r, q);
  else *q = r;
}

// ---------------------------------------------------------------------------
// Per-thread accumulation.  Floating point: compensated summation in the
// compute type with Neumaier's refinement of Kahan's method, one compensated
// add per element: the running sum s, and c, the sum of the exact rounding
// errors of the additions into s; the thread's sum is s + c, handed upward in
// FP64.  Each error is taken with Knuth's branch-free TwoSum (six additions,
// exact whichever operand is larger), which on gfx950 avoids the compare and
// selects of the magnitude test, and the hazard waits between them.  The
// error of the sum is about u |sum| plus a term of order n u^2 times the sum
// of the magnitudes of the thread's terms, so cancellation costs no accuracy.
// Integers: plain u64, exact.

__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }

template <class C> struct accum {
  C s = 0, c = 0;
  __device__ __forceinline__ void add(C t) {
#pragma clang fp contract(off)
    const C u = s + t;
    const C tv = u - s;          // the part of t that reached u
    const C sv = u - tv;         // the part of s that reached u
    c += (s - sv) + (t - tv);    // what u lost of each, exactly
    s = u;
  }
  // an infinite or NaN running sum is the sum (its compensation is NaN)
  __device__ __forceinline__ double value() const {
    return __builtin_isfinite(s) ? (double)s + (double)c : (double)s;
  }
};
template <> struct accum<uint32_t> {
  uint64_t s = 0;
  __device__ __forceinline__ void add(uint64_t t) { s += t; }
  __device__ __forceinline__ uint64_t value() const { return s; }
};

// A thread's compensated sums, one per vector lane: the elements at lane j
// of the vectors a thread visits form chain j, added in the order the thread
// visits its vectors.  Separate chains keep the dependent additions apart so
// that they overlap (one long chain per thread is latency-bound when few
// waves share a SIMD); the thread's sum is the chains' values added in FP64
// in lane order.  Scalar tails join chain 0.
template <class C, int N> struct lane_accum {
  accum<C> a[N];
  __device__ __forceinline__ auto value() const {
    auto t = a[0].value();
#pragma unroll
    for (int j = 1; j < N; ++j) t += a[j].value();
    return t;
  }
};

// Combination type above the thread: FP64 for floating point, u64 for u32.
template <class C> struct wide { using type = double; };
template <> struct wide<uint32_t> { using type = uint64_t; };

// Sum one value per thread over the block in a fixed order (wave64 butterfly,
// then the per-wave results through LDS).  Every thread gets the total.
// `lds` must hold blockDim.x / 64 values.
template <class D>
__device__ __forceinline__ D block_sum(D v, D* lds) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  D t = 0;
  for (int w = 0; w < nw; ++w) t += lds[w];
  return t;
}

// ---------------------------------------------------------------------------
// Cross-block finish.  Each block publishes its partials with agent-scope
// atomic stores (written through to the point of coherence of all eight
// XCDs: `global_store ... sc1`), waits for its own stores to complete, then
// takes a ticket on an agent-scope counter.  Only the block that draws the
// last ticket then performs an agent-scope acquire (one L2 invalidate,
// `buffer_inv sc1`) and reads the partials with ordinary loads, which it can
// batch, adding them in index order.  Publishing never needs an L2
// write-back (an agent-scope release fence), which would cost one per block.

template <class D> __device__ __forceinline__ void publish(D* p, D v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool take_last_ticket(unsigned* counter, unsigned expected) {
  __shared__ bool last;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's published partials have landed
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == expected - 1);
  }
  __syncthreads();
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

__device__ __forceinline__ void reset_counter(unsigned* counter) {
  __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum p[0], p[stride], ..., p[(m-1)*stride] left to right; loads are issued
// eight at a time ahead of the additions (the order of the additions is the
// plain serial one).
template <class D>
__device__ __forceinline__ D sum_strided(const D* p, int64_t stride, int m) {
  D t = 0;
  int q = 0;
  for (; q + 8 <= m; q += 8) {
    D v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[(int64_t)(q + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) t += v[k];
  }
  for (; q < m; ++q) t += p[(int64_t)q * stride];
  return t;
}

// ---------------------------------------------------------------------------
// Host side.

std::string& last_error();
int fail(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);

// Number of compute units of the current device (cached).
int device_cus();

// A resolved launch configuration.
struct launch {
  int block;      // threads per block (64..512, multiple of 64)
  int ept;        // independent vector loads per leaf per thread (1,2,4,8)
  int vec_bytes;  // bytes per vector load (storage bytes, 2..16)
  int split;      // grid size / blocks per column / column chunks
};

inline bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// The library's default block size and EPT of a result kind (0 element-wise,
// FX_R_*) for storage elements of `elem` bytes.  They do not depend on the
// shape (the grid does), so generated kernel source can fix them in its text.
constexpr int default_block(int kind, int elem) {
  return kind == 0 ? 512
       : kind == FX_R_COLSUM ? (elem >= 4 ? 512 : 256)
       : kind == FX_R_ROWSUM ? (elem >= 4 ? 256 : 64)
       : elem >= 4 ? 256 : 512;  // full reductions
}
constexpr int default_ept(int kind, int elem) {
  return kind == 0 ? 1 : kind == FX_R_COLSUM ? (elem >= 4 ? 2 : 1) : 2;
}

// Validate the user-facing fields (zeros mean "choose").
int check_launch(const fx_launch* cfg);

}  // namespace fx
