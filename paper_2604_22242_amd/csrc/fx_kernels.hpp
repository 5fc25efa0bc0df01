// Skeleton kernels for gfx950 and their host launchers.
//
// Each skeleton is a fixed recipe with the expression as a template
// parameter (Sec. 3: one skeleton kernel serves virtually every expression of
// the form Y = <rhs>).  The skeletons here:
//   k_ew        Z[i] = E(i)                      ("copy" skeleton)
//   k_full      sum_i map(E(i)) -> one value     (accu, dot, norm_fro)
//   k_colsum    sum over rows, per column        (sum(E, 0))
//   k_colsum_thin  same for very short columns (one thread per column)
//   k_rowsum    sum over columns, per row        (sum(E, 1))
//
// Memory access: wave64, each lane moves one vector of N elements (16 bytes
// by default) per load; a block covers a contiguous tile of
// blockDim * EPT vectors, the EPT loads of every leaf are independent and
// issued before any result is stored.  Full reductions combine the block
// partials in FP64 in one pass: the last block to finish (agent-scope
// ticket) adds them in index order, so a fixed launch configuration gives
// bitwise-reproducible results.
#pragma once

#include <algorithm>
#include <type_traits>
#include <utility>

#include "fx_expr.hpp"

// Cache policy of streamed loads and stores (measured on MI355X: streaming
// loads raise the read ceiling from 6.4 to 7.1 TB/s).  FX_NT_STORES forces
// streaming stores everywhere; by default the element-wise kernel chooses
// per launch from the size of its output (kStreamStoresAbove).
#ifndef FX_NT_LOADS
#define FX_NT_LOADS 1
#endif
#ifndef FX_NT_STORES
#define FX_NT_STORES 0
#endif


namespace fx {

constexpr int kMaxBlock = 512;
constexpr bool kNT = FX_NT_LOADS != 0;    // streaming policy for loads
constexpr bool kNTS = FX_NT_STORES != 0;  // streaming policy for stores

// Outputs larger than MI355X's 256 MiB last-level cache (the Infinity Cache)
// are written with streaming stores.  Measured for X%Y + 2W in FP32: up to a
// 256 MiB output, ordinary stores run at 6.6-6.7 TB/s (the output stays in
// that cache) against 6.1-6.2 streaming; from 320 MiB on, ordinary stores
// fall to 6.0-6.1 TB/s and streaming stores keep 6.2-6.3.
constexpr uint64_t kStreamStoresAbove = uint64_t(256) << 20;

// Maps applied to each element before summation.
struct map_id {
  template <class C> __device__ static C f(C x) { return x; }
  __host__ __device__ static double finish(double s) { return s; }
  __host__ __device__ static uint64_t finish(uint64_t s) { return s; }
};
struct map_sq {
  template <class C> __device__ static C f(C x) { return x * x; }
  __device__ static double finish(double s) { return ::sqrt(s); }
};

// Add the map M of a thread's EPT x N values of one tile to its compensated
// lane sums, one element at a time (lane j's chain takes vector 0's, then
// vector 1's ... element j).
template <class M, int N, int EPT, class C>
__device__ __forceinline__ void add_tile(lane_accum<C, N>& acc, const lanes<C, N> (&r)[EPT]) {
#pragma unroll
  for (int k = 0; k < EPT; ++k)
#pragma unroll
    for (int j = 0; j < N; ++j) acc.a[j].add(M::f(r[k].v[j]));
}
template <class M, int N, class C>
__device__ __forceinline__ void add_lanes(lane_accum<C, N>& acc, const lanes<C, N>& r) {
#pragma unroll
  for (int j = 0; j < N; ++j) acc.a[j].add(M::f(r.v[j]));
}

// EPT vectors of N elements at base, base + stride, ...: every leaf's loads
// are issued before any arithmetic (two phases: the register leaves of all
// EPT vectors, then the tree from registers, with a scheduling barrier
// between them; left to itself the scheduler may hold a vector's loads back
// until the previous one has arrived when little arithmetic follows).
// Expression types with their own evaluation strategy (the run-time tape)
// overload this.
template <int N, int EPT, class E>
__device__ __forceinline__ void eval_tile(const E& e, int64_t base, int64_t stride,
                                          lanes<typename E::ct, N> (&r)[EPT]) {
  constexpr int L = leaves_of<E>::value;
  if constexpr (L >= 1 && L <= kMaxFusedLeaves) {
    lanes<typename E::ct, N> regs[EPT][L];
    const uint8_t* no_alias = nullptr;
#pragma unroll
    for (int k = 0; k < EPT; ++k) e.template gather<0, N, kNT>(regs[k], no_alias, base + k * stride);
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the arithmetic
#pragma unroll
    for (int k = 0; k < EPT; ++k) r[k] = e.template at_regs<0, N, kNT>(regs[k], base + k * stride);
  } else {
#pragma unroll
    for (int k = 0; k < EPT; ++k) r[k] = e.template at_vec<N, kNT>(base + k * stride);
  }
}

// Fused<E>: the loads of all EPT vectors first, then the arithmetic.
template <int N, int EPT, class E>
__device__ __forceinline__ void eval_tile(const Fused<E>& f, int64_t base, int64_t stride,
                                          lanes<typename E::ct, N> (&r)[EPT]) {
  lanes<typename E::ct, N> regs[EPT][Fused<E>::L];
#pragma unroll
  for (int k = 0; k < EPT; ++k) f.e.template gather<0, N, kNT>(regs[k], f.alias, base + k * stride);
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    f.template resolve<N>(regs[k]);
    r[k] = f.e.template at_regs<0, N, kNT>(regs[k], base + k * stride);
  }
}

// ============================================================================
// Element-wise: Z[i] = E(i), i < n.

// NTS: streaming stores.  The policy is a template parameter: a run-time
// choice between two otherwise identical stores is merged by the compiler
// into one store, which drops the streaming hint.
template <class E, class T, int N, int EPT, bool NTS>
__global__ __launch_bounds__(kMaxBlock) void k_ew(E e, T* __restrict__ z, int64_t n) {
  using C = typename E::ct;
  const int64_t nv = n / N;  // whole vectors
  const int64_t tile = (int64_t)blockDim.x * EPT;
  // tile t exists while t * tile < nv (no 64-bit division: gfx950 has no
  // scalar divide, and its emulation would delay every wave's first load)
  for (int64_t t = blockIdx.x; t * tile < nv; t += gridDim.x) {
    const int64_t v0 = t * tile + threadIdx.x;
    if ((t + 1) * tile <= nv) {
      lanes<C, N> r[EPT];
      eval_tile<N, EPT>(e, v0 * N, (int64_t)blockDim.x * N, r);
#pragma unroll
      for (int k = 0; k < EPT; ++k) store_lanes<N, NTS>(z, (v0 + k * blockDim.x) * N, r[k]);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int64_t v = v0 + k * blockDim.x;
        if (v < nv) store_lanes<N, NTS>(z, v * N, e.template at_vec<N, kNT>(v * N));
      }
    }
  }
  if (N > 1 && blockIdx.x == gridDim.x - 1) {
    for (int64_t i = nv * N + threadIdx.x; i < n; i += blockDim.x) z[i] = static_cast<T>(e.at(i));
  }
}

// ============================================================================
// Full reduction: out = finish(sum_i map(E(i))).  partials: gridDim.x wide
// values; counter: one unsigned, zero on entry, zero again on exit.

template <class E, class M, class O, int N, int EPT>
__global__ __launch_bounds__(kMaxBlock) void k_full(E e, int64_t n, typename wide<typename E::ct>::type* partials,
                                                  unsigned* counter, O* out) {
  using C = typename E::ct;
  using D = typename wide<C>::type;
  __shared__ D lds[kMaxBlock / 64];
  lane_accum<C, N> acc;
  const int64_t nv = n / N;
  const int64_t tile = (int64_t)blockDim.x * EPT;
  // tile t exists while t * tile < nv (no 64-bit division: gfx950 has no
  // scalar divide, and its emulation would delay every wave's first load)
  for (int64_t t = blockIdx.x; t * tile < nv; t += gridDim.x) {
    const int64_t v0 = t * tile + threadIdx.x;
    if ((t + 1) * tile <= nv) {
      lanes<C, N> r[EPT];
      eval_tile<N, EPT>(e, v0 * N, (int64_t)blockDim.x * N, r);
      add_tile<M>(acc, r);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int64_t v = v0 + k * blockDim.x;
        if (v < nv) add_lanes<M>(acc, e.template at_vec<N, kNT>(v * N));
      }
    }
  }
  if (N > 1 && blockIdx.x == gridDim.x - 1) {
    for (int64_t i = nv * N + threadIdx.x; i < n; i += blockDim.x) acc.a[0].add(M::f(e.at(i)));
  }
  D s = block_sum<D>(acc.value(), lds);
  if (gridDim.x == 1) {
    if (threadIdx.x == 0) *out = static_cast<O>(M::finish(s));
    return;
  }
  if (threadIdx.x == 0) publish(partials + blockIdx.x, s);
  if (take_last_ticket(counter, gridDim.x)) {
    D t = 0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) t += partials[b];
    t = block_sum<D>(t, lds);
    if (threadIdx.x == 0) {
      *out = static_cast<O>(M::finish(t));
      reset_counter(counter);
    }
  }
}

// ============================================================================
// Column sums.  Block (column c, chunk s) sums rows [s*rpc, (s+1)*rpc) of
// column c: a contiguous run read blockDim * N elements at a time, EPT loads
// per input in flight.  With split > 1 the chunk partials go to
// partials[c*split + s] and the block that draws the last ticket on
// counters[c] adds them in chunk order.  N > 1 requires N | n_rows and
// aligned leaves; rpc is a multiple of N.

template <class E, class O, int N, int EPT>
__global__ __launch_bounds__(kMaxBlock) void k_colsum(E e, int64_t n_rows, int split, int64_t rpc,
                                                    typename wide<typename E::ct>::type* partials,
                                                    unsigned* counters, O* out) {
  using C = typename E::ct;
  using D = typename wide<C>::type;
  __shared__ D lds[kMaxBlock / 64];
  const int64_t col = blockIdx.x;
  const int s = blockIdx.y;
  const int64_t r0 = (int64_t)s * rpc;
  const int64_t r1 = min(n_rows, r0 + rpc);
  const int64_t base = col * n_rows + r0;
  const int64_t nv = r1 > r0 ? (r1 - r0) / N : 0;
  lane_accum<C, N> acc;
  const int64_t tile = (int64_t)blockDim.x * EPT;
  for (int64_t t0 = 0; t0 < nv; t0 += tile) {
    const int64_t v0 = t0 + threadIdx.x;
    if (t0 + tile <= nv) {
      lanes<C, N> r[EPT];
      eval_tile<N, EPT>(e, base + v0 * N, (int64_t)blockDim.x * N, r);
      add_tile<map_id>(acc, r);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int64_t v = v0 + k * blockDim.x;
        if (v < nv) add_lanes<map_id>(acc, e.template at_vec<N, kNT>(base + v * N));
      }
    }
  }
  const D sum = block_sum<D>(acc.value(), lds);
  if (split == 1) {
    if (threadIdx.x == 0) out[col] = static_cast<O>(sum);
    return;
  }
  if (threadIdx.x == 0) publish(partials + col * split + s, sum);
  if (take_last_ticket(counters + col, split)) {
    if (threadIdx.x == 0) {
      out[col] = static_cast<O>(sum_strided<D>(partials + col * split, 1, split));
      reset_counter(counters + col);
    }
  }
}

// Short columns: thread c sums column c serially (no cross-thread combine).
template <class E, class O>
__global__ __launch_bounds__(kMaxBlock) void k_colsum_thin(E e, int64_t n_rows, int64_t n_cols, O* out) {
  using C = typename E::ct;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cols;
       c += (int64_t)gridDim.x * blockDim.x) {
    accum<C> acc;
    for (int64_t r = 0; r < n_rows; ++r) acc.add(e.at(r + c * n_rows));
    out[c] = static_cast<O>(acc.value());
  }
}

// ============================================================================
// Row sums.  Thread owns rows [r0, r0+N) (one vector per column, so a wave
// reads 64 consecutive vectors of a column) and walks the columns
// [s*cpc, (s+1)*cpc) of its chunk EPT at a time (EPT loads per input in
// flight), keeping N compensated row sums.  With split > 1 the chunk
// partials go to partials[s*n_rows + r]; the block that draws the last
// ticket of its row block (counters[blockIdx.x]) adds them in chunk order.
// N > 1 requires N | n_rows and aligned leaves.

template <class E, class O, int N, int EPT>
__global__ __launch_bounds__(kMaxBlock) void k_rowsum(E e, int64_t n_rows, int64_t n_cols, int split,
                                                    int64_t cpc,
                                                    typename wide<typename E::ct>::type* partials,
                                                    unsigned* counters, O* out) {
  using C = typename E::ct;
  using D = typename wide<C>::type;
  const int s = blockIdx.y;
  const int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * N;
  const bool active = r0 < n_rows;
  const int64_t c0 = (int64_t)s * cpc;
  const int64_t c1 = min(n_cols, c0 + cpc);
  accum<C> acc[N];
  if (active) {
    int64_t c = c0;
    for (; c + EPT <= c1; c += EPT) {
      lanes<C, N> r[EPT];
      eval_tile<N, EPT>(e, r0 + c * n_rows, n_rows, r);
#pragma unroll
      for (int j = 0; j < N; ++j)  // row j's EPT columns, in column order
#pragma unroll
        for (int k = 0; k < EPT; ++k) acc[j].add(r[k].v[j]);
    }
    for (; c < c1; ++c) {
      lanes<C, N> r = e.template at_vec<N, kNT>(r0 + c * n_rows);
#pragma unroll
      for (int j = 0; j < N; ++j) acc[j].add(r.v[j]);
    }
  }
  if (split == 1) {
    if (active)
#pragma unroll
      for (int j = 0; j < N; ++j) out[r0 + j] = static_cast<O>(acc[j].value());
    return;
  }
  if (active)
#pragma unroll
    for (int j = 0; j < N; ++j) publish(partials + (int64_t)s * n_rows + r0 + j, acc[j].value());
  if (take_last_ticket(counters + blockIdx.x, split)) {
    if (active) {
#pragma unroll
      for (int j = 0; j < N; ++j)
        out[r0 + j] = static_cast<O>(sum_strided<D>(partials + r0 + j, n_rows, split));
    }
    __syncthreads();
    if (threadIdx.x == 0) reset_counter(counters + blockIdx.x);
  }
}

// Zero-fill (used for sums over empty dimensions; a kernel rather than a
// memset node, so the call can sit inside a captured graph).
template <class O>
__global__ __launch_bounds__(256) void k_fill_zero(O* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = O(0);
}

// ============================================================================
// Host side: configuration resolution and dispatch.

template <int V> using ic = std::integral_constant<int, V>;

// Largest EPT compiled for an expression type (the run-time tape keeps one
// slot file per lane in registers and caps it lower).
template <class E> struct max_ept { static constexpr int value = 8; };
template <class E> struct max_ept<Fused<E>> { static constexpr int value = max_ept<E>::value; };

template <int MAX = 8, class F> inline int with_ept(int ept, F&& f) {
  switch (ept) {
    case 1: return f(ic<1>{});
    case 2: if constexpr (MAX >= 2) return f(ic<2>{}); break;
    case 4: if constexpr (MAX >= 4) return f(ic<4>{}); break;
    case 8: if constexpr (MAX >= 8) return f(ic<8>{}); break;
  }
  return fail(FX_E_UNSUPPORTED, "ept %d not compiled for this expression (max %d)", ept, MAX);
}

// Expression types compiled for 8-byte vectors as well (the run-time tape,
// whose launch the autotuner searches); the others take one element (any
// alignment) or 16 bytes.
template <class E> struct vec8_compiled { static constexpr bool value = false; };
template <class E> struct vec8_compiled<Fused<E>> { static constexpr bool value = vec8_compiled<E>::value; };
template <class E> constexpr bool vec8_compiled_v = vec8_compiled<E>::value;

// Vector width in elements: one element, 8 bytes (where compiled) or 16 bytes.
template <class T, class E = void, class F> inline int with_vec(int vec_elems, F&& f) {
  constexpr int W = 16 / (int)sizeof(T);
  constexpr bool V8 = W >= 4 && vec8_compiled_v<E>;
  if (vec_elems == 1) return f(ic<1>{});
  if (vec_elems == W) return f(ic<W>{});
  if constexpr (V8) {
    if (vec_elems == W / 2) return f(ic<W / 2>{});
  }
  return fail(FX_E_UNSUPPORTED, "vector of %d elements not compiled (1 or %d%s)", vec_elems, W,
              V8 ? " or half of it" : "");
}

// Resolve a configuration for `n_elems` elements of storage size `elem` with
// `n_leaves` distinct inputs.  kind: 0 element-wise, FX_R_* reductions.
launch resolve(int kind, int elem, int64_t n_rows, int64_t n_cols, const fx_launch* cfg,
               bool aligned16);

// Workspace layout: [counters, 256-byte aligned][FP64/u64 partials].
struct ws_layout {
  size_t counter_bytes = 0, partial_bytes = 0;
  size_t total() const { return counter_bytes + partial_bytes; }
};
ws_layout workspace_for(int kind, int64_t n_rows, int64_t n_cols, const launch& L, int vec_elems);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <class E> int check_expr(const E& e, int64_t* n_rows, int64_t* n_cols) {
  leaf_info li = info_of(e);
  if (!li.shape_ok) return fail(FX_E_SHAPE, "operands of the expression differ in shape");
  if (li.any_null) return fail(FX_E_ARG, "NULL input pointer");
  if (li.n_rows < 0 || li.n_cols < 0) return fail(FX_E_ARG, "negative dimension");
  *n_rows = li.n_rows;
  *n_cols = li.n_cols;
  return FX_OK;
}

// A defaulted EPT never exceeds what is compiled for the expression type.
template <class E> inline void clamp_ept(launch& L, const fx_launch* cfg) {
  if (!(cfg && cfg->ept)) L.ept = std::min(L.ept, max_ept<E>::value);
}

// Z = E element-wise (Sec. 3: assignment through the copy skeleton).
template <class E, class T>
int eval_direct(T* z, const E& e, const fx_launch* cfg, hipStream_t st);
template <class E, class T>
int eval(T* z, const E& e, const fx_launch* cfg, hipStream_t st) {
  if constexpr (leaves_of<E>::value >= 2 && leaves_of<E>::value <= kMaxFusedLeaves) {
    const auto f = fuse_leaves(e);
    if (f.has_alias()) return eval_direct(z, f, cfg, st);
  }
  return eval_direct(z, e, cfg, st);
}
template <class E, class T>
int eval_direct(T* z, const E& e, const fx_launch* cfg, hipStream_t st) {
  int64_t rows, cols;
  if (int rc = check_expr(e, &rows, &cols)) return rc;
  const int64_t n = rows * cols;
  if (n == 0) return FX_OK;
  if (!z) return fail(FX_E_ARG, "NULL output pointer");
  if (int rc = check_launch(cfg)) return rc;
  leaf_info li = info_of(e);
  li.addr_or |= reinterpret_cast<uintptr_t>(z);
  launch L = resolve(0, sizeof(T), rows, cols, cfg, li.aligned(16));
  clamp_ept<E>(L, cfg);
  const int vec = L.vec_bytes / (int)sizeof(T);
  return with_vec<T, E>(vec, [&](auto Nc) {
    return with_ept<max_ept<E>::value>(L.ept, [&](auto Ec) {
      constexpr int N = decltype(Nc)::value, EPT = decltype(Ec)::value;
      // (streaming stores are compiled for 16-byte vectors, the default for
      // outputs of that size)
      if constexpr (N * sizeof(T) == 16) {
        if (kNTS || (uint64_t)n * sizeof(T) > kStreamStoresAbove) {
          hipLaunchKernelGGL((k_ew<E, T, N, EPT, true>), dim3(L.split), dim3(L.block), 0, st, e, z, n);
          return hip_check(hipGetLastError(), "k_ew launch");
        }
      }
      hipLaunchKernelGGL((k_ew<E, T, N, EPT, kNTS>), dim3(L.split), dim3(L.block), 0, st, e, z, n);
      return hip_check(hipGetLastError(), "k_ew launch");
    });
  });
}

inline unsigned* ws_counters(void* ws) { return static_cast<unsigned*>(ws); }
template <class D> inline D* ws_partials(void* ws, const ws_layout& W) {
  return reinterpret_cast<D*>(static_cast<char*>(ws) + W.counter_bytes);
}

// out = finish(sum map(E)) as FP64 (u64 for u32 expressions).
template <class M, class E>
int reduce_full_direct(const E& e, void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
                       hipStream_t st);
template <class M, class E>
int reduce_full(const E& e, void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
                hipStream_t st) {
  if constexpr (leaves_of<E>::value >= 2 && leaves_of<E>::value <= kMaxFusedLeaves) {
    const auto f = fuse_leaves(e);
    if (f.has_alias()) return reduce_full_direct<M>(f, out, ws, ws_bytes, cfg, st);
  }
  return reduce_full_direct<M>(e, out, ws, ws_bytes, cfg, st);
}
template <class M, class E>
int reduce_full_direct(const E& e, void* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
                       hipStream_t st) {
  using T = typename E::storage;
  using D = typename wide<typename E::ct>::type;
  int64_t rows, cols;
  if (int rc = check_expr(e, &rows, &cols)) return rc;
  if (!out) return fail(FX_E_ARG, "NULL output pointer");
  if (int rc = check_launch(cfg)) return rc;
  const int64_t n = rows * cols;
  leaf_info li = info_of(e);
  launch L = resolve(FX_R_ACCU, sizeof(T), rows, cols, cfg, li.aligned(16));
  clamp_ept<E>(L, cfg);
  const int vec = L.vec_bytes / (int)sizeof(T);
  ws_layout W = workspace_for(FX_R_ACCU, rows, cols, L, vec);
  if (L.split > 1 && (!ws || ws_bytes < W.total()))
    return fail(FX_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", W.total(), ws_bytes);
  return with_vec<T, E>(vec, [&](auto Nc) {
    return with_ept<max_ept<E>::value>(L.ept, [&](auto Ec) {
      constexpr int N = decltype(Nc)::value, EPT = decltype(Ec)::value;
      hipLaunchKernelGGL((k_full<E, M, D, N, EPT>), dim3(L.split), dim3(L.block), 0, st, e, n,
                         ws ? ws_partials<D>(ws, W) : nullptr, ws ? ws_counters(ws) : nullptr,
                         static_cast<D*>(out));
      return hip_check(hipGetLastError(), "k_full launch");
    });
  });
}

// sum(E, 0) or sum(E, 1) into out (accumulator dtype O).
template <class O, class E>
int reduce_dim_direct(int kind, const E& e, O* out, void* ws, size_t ws_bytes,
                      const fx_launch* cfg, hipStream_t st);
template <class O, class E>
int reduce_dim(int kind, const E& e, O* out, void* ws, size_t ws_bytes, const fx_launch* cfg,
               hipStream_t st) {
  if constexpr (leaves_of<E>::value >= 2 && leaves_of<E>::value <= kMaxFusedLeaves) {
    const auto f = fuse_leaves(e);
    if (f.has_alias()) return reduce_dim_direct(kind, f, out, ws, ws_bytes, cfg, st);
  }
  return reduce_dim_direct(kind, e, out, ws, ws_bytes, cfg, st);
}
template <class O, class E>
int reduce_dim_direct(int kind, const E& e, O* out, void* ws, size_t ws_bytes,
                      const fx_launch* cfg, hipStream_t st) {
  using T = typename E::storage;
  using D = typename wide<typename E::ct>::type;
  int64_t rows, cols;
  if (int rc = check_expr(e, &rows, &cols)) return rc;
  if (int rc = check_launch(cfg)) return rc;
  const int64_t nout = kind == FX_R_COLSUM ? cols : rows;
  if (nout == 0) return FX_OK;
  if (!out) return fail(FX_E_ARG, "NULL output pointer");
  if (rows * cols == 0) {
    const int grid = (int)std::min<int64_t>(ceil_div(nout, 256), 1024);
    hipLaunchKernelGGL((k_fill_zero<O>), dim3(grid), dim3(256), 0, st, out, nout);
    return hip_check(hipGetLastError(), "k_fill_zero launch");
  }
  leaf_info li = info_of(e);
  const int W16 = 16 / (int)sizeof(T);
  launch L = resolve(kind, sizeof(T), rows, cols, cfg, li.aligned(16) && rows % W16 == 0);
  clamp_ept<E>(L, cfg);
  const int vec = L.vec_bytes / (int)sizeof(T);
  ws_layout W = workspace_for(kind, rows, cols, L, vec);
  if (W.total() > 0 && (!ws || ws_bytes < W.total()))
    return fail(FX_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", W.total(), ws_bytes);
  D* parts = ws ? ws_partials<D>(ws, W) : nullptr;
  unsigned* ctr = ws ? ws_counters(ws) : nullptr;
  if (kind == FX_R_COLSUM) {
    if (L.split == 0) {  // thin columns: one thread per column
      const int grid = (int)std::min<int64_t>(ceil_div(cols, L.block), 1 << 20);
      hipLaunchKernelGGL((k_colsum_thin<E, O>), dim3(grid), dim3(L.block), 0, st, e, rows, cols, out);
      return hip_check(hipGetLastError(), "k_colsum_thin launch");
    }
    const int64_t rpc = ceil_div(ceil_div(rows, L.split), vec) * vec;
    return with_vec<T, E>(vec, [&](auto Nc) {
      return with_ept<max_ept<E>::value>(L.ept, [&](auto Ec) {
        constexpr int N = decltype(Nc)::value, EPT = decltype(Ec)::value;
        hipLaunchKernelGGL((k_colsum<E, O, N, EPT>), dim3((unsigned)cols, L.split), dim3(L.block), 0,
                           st, e, rows, L.split, rpc, parts, ctr, out);
        return hip_check(hipGetLastError(), "k_colsum launch");
      });
    });
  }
  const int64_t cpc = ceil_div(cols, L.split);
  const int64_t rblocks = ceil_div(rows, (int64_t)L.block * vec);
  return with_vec<T, E>(vec, [&](auto Nc) {
    return with_ept<max_ept<E>::value>(L.ept, [&](auto Ec) {
      constexpr int N = decltype(Nc)::value, EPT = decltype(Ec)::value;
      hipLaunchKernelGGL((k_rowsum<E, O, N, EPT>), dim3((unsigned)rblocks, L.split), dim3(L.block), 0,
                         st, e, rows, cols, L.split, cpc, parts, ctr, out);
      return hip_check(hipGetLastError(), "k_rowsum launch");
    });
  });
}

// ---- dtype dispatch shared by the C entry points -------------------------

template <class T> struct tag { using type = T; };

// Floating-point storage dtypes.
template <class F> int with_fp(fx_dtype dt, F&& f) {
  switch (dt) {
    case FX_F32: return f(tag<float>{});
    case FX_F64: return f(tag<double>{});
    case FX_BF16: return f(tag<bf16_t>{});
    case FX_F16: return f(tag<f16_t>{});
    default: break;
  }
  return fail(FX_E_DTYPE, "dtype %d not supported here (floating point only)", (int)dt);
}

template <class T> using acc_out_t = std::conditional_t<std::is_same_v<T, double>, double, float>;

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

inline int check_n(int64_t n) { return n < 0 ? fail(FX_E_ARG, "negative size %lld", (long long)n) : FX_OK; }
inline int check_shape(fx_shape s) {
  return (s.n_rows < 0 || s.n_cols < 0) ? fail(FX_E_ARG, "negative dimension") : FX_OK;
}

}  // namespace fx
