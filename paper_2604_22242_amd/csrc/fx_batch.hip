// Batches: one persistent launch over thousands of uneven expressions.
//
// Host: each item's compiled program is copied into a device array, the
// items are cut into fixed-size tiles (consecutive per item) and a tile
// table maps tile -> item; the table lists tiles by decreasing estimated
// cost (device operations x elements), so that the work queue hands out the
// long tiles first and the short ones fill the end.  Device: a grid of
// persistent blocks takes tiles from that queue (one atomic ticket per tile);
// the program of a tile is read through a pointer (wave-uniform loads) and
// interpreted with the same TapeExpr code as fx_tape_eval, element-wise
// tiles write their slice of the output and reducing items publish one FP64
// partial per tile; the tile that draws the item's last ticket adds the
// item's partials in tile order and resets the counter.  The last block to
// leave resets the queue, so the launch can be replayed as it is.
#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "fx_tape.hpp"

namespace fx {

struct batch_desc {
  const void* in[kTapeMaxIn];
  void* out;
  int64_t n;
  int32_t kind;
  int32_t n_tiles;
  int64_t first_tile;
};

// One tile of the queue: its item and its index within the item.
struct batch_tile {
  uint32_t item, index;
};

// The batch reads its item pointers from device memory, so the compiler
// cannot tell that they point to global memory and would use flat
// instructions, whose completion the scalar instruction fetches of the
// interpreter then also wait for.  These helpers access them through the
// global address space.
#define FX_GLOBAL __attribute__((address_space(1)))
template <int N, class T>
__device__ __forceinline__ lanes<ct_t<T>, N> gload_lanes(const T* p, int64_t i) {
  constexpr int BYTES = N * (int)sizeof(T);
  static_assert(BYTES <= 16, "one load per vector");
  using R = typename raw<BYTES>::type;
  const FX_GLOBAL R* q = (const FX_GLOBAL R*)(p + i);
  const R r = kNT ? __builtin_nontemporal_load(q) : *q;
  T s[N];
  __builtin_memcpy(s, &r, sizeof(R));
  lanes<ct_t<T>, N> out;
#pragma unroll
  for (int j = 0; j < N; ++j) out.v[j] = static_cast<ct_t<T>>(s[j]);
  return out;
}
template <class T> __device__ __forceinline__ ct_t<T> gload(const T* p, int64_t i) {
  return static_cast<ct_t<T>>(*(const FX_GLOBAL T*)(p + i));
}
template <int N, bool NTS, class T>
__device__ __forceinline__ void gstore_lanes(T* p, int64_t i, const lanes<ct_t<T>, N>& x) {
  using R = typename raw<N * (int)sizeof(T)>::type;
  T s[N];
#pragma unroll
  for (int j = 0; j < N; ++j) s[j] = static_cast<T>(x.v[j]);
  R r;
  __builtin_memcpy(&r, s, sizeof(R));
  FX_GLOBAL R* q = (FX_GLOBAL R*)(p + i);
  if (NTS) __builtin_nontemporal_store(r, q);
  else *q = r;
}
template <class T> __device__ __forceinline__ void gstore(T* p, int64_t i, ct_t<T> v) {
  *(FX_GLOBAL T*)(p + i) = static_cast<T>(v);
}

// Inputs of EPT vectors at base + k * stride, of which only the elements
// below `end` exist (the last pass of an item): whole vectors load as
// vectors, the vector that straddles `end` element by element.
template <int N, int EPT, class X>
__device__ __forceinline__ void batch_load_tail(const X& x, int n_in, int64_t base, int64_t stride,
                                                int64_t end,
                                                lanes<typename X::ct, N> (&in)[EPT][kTapeMaxIn]) {
  using C = typename X::ct;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int64_t e = base + k * stride;
#pragma unroll
    for (int q = 0; q < kTapeMaxIn; ++q) {
      if (q < n_in && e + N <= end) {
        in[k][q] = gload_lanes<N>(x.p[q], e);
      } else {
        in[k][q] = unset_lanes<C, N>();
        if (q < n_in)
#pragma unroll
          for (int j = 0; j < N; ++j)
            if (e + j < end) in[k][q].v[j] = gload(x.p[q], e + j);
      }
    }
  }
}

// NTS: streaming stores for the element-wise outputs (chosen by the host when
// they add up to more than the last-level cache, as for single launches).
template <class T, int N, int EPT, int SLOTS, bool NTS>
__global__ __launch_bounds__(kMaxBlock) void k_batch(const batch_desc* __restrict__ descs,
                                                   const tape_prog* __restrict__ progs,
                                                   const batch_tile* __restrict__ tiles,
                                                   int64_t n_tiles, int64_t tile_elems,
                                                   double* __restrict__ partials,
                                                   unsigned* __restrict__ counters,
                                                   unsigned* __restrict__ queue) {
  using C = ct_t<T>;
  __shared__ double lds[kMaxBlock / 64];
  __shared__ unsigned next;
  const int64_t stride = (int64_t)blockDim.x * N;  // between a thread's vectors
  const int64_t pass = stride * EPT;               // elements per block pass
  for (;;) {
    if (threadIdx.x == 0)
      next = __hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned t = next;
    __syncthreads();  // every thread has read `next` before it changes
    if (t >= n_tiles) break;
    const batch_tile tl = tiles[t];
    const batch_desc d = descs[tl.item];
    TapeExpr<T, true, SLOTS> x;
#pragma unroll
    for (int q = 0; q < kTapeMaxIn; ++q) x.p[q] = static_cast<const T*>(d.in[q]);
    x.n_rows = d.n;
    x.n_cols = 1;
    x.prog = progs + tl.item;
    const int n_in = x.P().n_in;
    const bool ew = d.kind == 0;
    T* z = static_cast<T*>(d.out);
    const int64_t i0 = (int64_t)tl.index * tile_elems;
    const int64_t i1 = min(d.n, i0 + tile_elems);
    // one compensated chain per thread (the interpreter between two passes
    // leaves the chain's dependent additions ample time; a chain per vector
    // lane would cost registers, and with them occupancy)
    accum<C> acc;
    for (int64_t e0 = i0; e0 < i1; e0 += pass) {
      const int64_t base = e0 + (int64_t)threadIdx.x * N;
      const bool whole = e0 + pass <= i1;  // uniform
      lanes<C, N> in[EPT][kTapeMaxIn];
      if (whole) {
#pragma unroll
        for (int q = 0; q < kTapeMaxIn; ++q)
#pragma unroll
          for (int k = 0; k < EPT; ++k)
            in[k][q] = q < n_in ? gload_lanes<N>(x.p[q], base + k * stride) : unset_lanes<C, N>();
      } else {
        batch_load_tail<N, EPT>(x, n_in, base, stride, i1, in);
      }
      // one interpreter for whole and partial passes
      lanes<C, N * EPT> flat[kTapeMaxIn];
#pragma unroll
      for (int q = 0; q < kTapeMaxIn; ++q)
#pragma unroll
        for (int k = 0; k < EPT; ++k)
#pragma unroll
          for (int j = 0; j < N; ++j) flat[q].v[k * N + j] = in[k][q].v[j];
      const lanes<C, N * EPT> r = x.template interpret<N * EPT>(flat);
      if (whole) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          lanes<C, N> v;
#pragma unroll
          for (int j = 0; j < N; ++j) v.v[j] = r.v[k * N + j];
          if (ew) {
            gstore_lanes<N, NTS>(z, base + k * stride, v);
          } else {
#pragma unroll
            for (int j = 0; j < N; ++j) acc.add(v.v[j]);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const int64_t e = base + k * stride;
#pragma unroll
          for (int j = 0; j < N; ++j) {
            if (e + j < i1) {
              if (ew) gstore(z, e + j, r.v[k * N + j]);
              else acc.add(r.v[k * N + j]);
            }
          }
        }
      }
    }
    if (!ew) {
      const double s = block_sum<double>(acc.value(), lds);
      if (d.n_tiles == 1) {
        if (threadIdx.x == 0) *(FX_GLOBAL double*)d.out = s;
      } else {
        const int64_t pt = d.first_tile + tl.index;  // partials in tile order per item
        if (threadIdx.x == 0) publish(partials + pt, s);
        if (take_last_ticket(counters + tl.item, d.n_tiles)) {
          if (threadIdx.x == 0) {
            *(FX_GLOBAL double*)d.out = sum_strided<double>(partials + d.first_tile, 1, d.n_tiles);
            reset_counter(counters + tl.item);
          }
        }
      }
      __syncthreads();  // the next tile reuses lds
    }
  }
  // the last block out resets the queue for the next launch (every block's
  // final ticket, which found the queue empty, precedes its exit ticket)
  if (threadIdx.x == 0) {
    const unsigned done = __hip_atomic_fetch_add(queue + 1, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(queue + 1, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace fx

using namespace fx;

struct fx_batch {
  fx_dtype dt;
  fx_batch_info info;
  std::vector<fx_batch_item> items;  // for separate launches
  std::vector<tape_prog> progs;
  std::vector<size_t> ws_off;        // workspace offset per reducing item
  void* d_ws = nullptr;
  batch_desc* d_descs = nullptr;
  tape_prog* d_progs = nullptr;
  batch_tile* d_tiles = nullptr;
  double* d_partials = nullptr;
  unsigned* d_counters = nullptr;
  unsigned* d_queue = nullptr;  // tile tickets, exit tickets (zero between launches)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last_stream = nullptr;
  int vec;
  bool small_slots;  // every program fits the 8-slot file
  bool nts;          // streaming stores (element-wise outputs beyond the last-level cache)
};

// Release paths cannot report errors: a failure here only means the context
// is already gone.
static void batch_free(fx_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  (void)hipFree(b->d_descs);
  (void)hipFree(b->d_progs);
  (void)hipFree(b->d_tiles);
  (void)hipFree(b->d_partials);
  (void)hipFree(b->d_counters);
  (void)hipFree(b->d_queue);
  (void)hipFree(b->d_ws);
}

static int elem_of(fx_dtype dt) {
  switch (dt) {
    case FX_F32: return 4;
    case FX_F64: return 8;
    case FX_BF16: case FX_F16: return 2;
    default: return 0;
  }
}

template <class F> static int batch_dispatch(fx_dtype dt, int vec, int ept, F&& f) {
  return with_fp(dt, [&](auto tg) {
    using T = typename decltype(tg)::type;
    return with_vec<T>(vec, [&](auto Nc) {
      return with_ept<2>(ept, [&](auto Ec) {
        return f(tag<T>{}, Nc, Ec);
      });
    });
  });
}

// Blocks of the batch kernel that one CU holds at once (the persistent grid
// is that many per CU: more would only wait for the queue to drain).
static int batch_resident_blocks(fx_dtype dt, int vec, int ept, bool small_slots, int block,
                                 int* out) {
  return batch_dispatch(dt, vec, ept, [&](auto tg, auto Nc, auto Ec) {
    using T = typename decltype(tg)::type;
    constexpr int N = decltype(Nc)::value, EPT = decltype(Ec)::value;
    int nb = 0;
    const hipError_t e =
        small_slots ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                          &nb, k_batch<T, N, EPT, kTapeSmallSlots, false>, block, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                          &nb, k_batch<T, N, EPT, kTapeMaxSlots, false>, block, 0);
    if (int rc = hip_check(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor")) return rc;
    *out = nb > 0 ? nb : 1;
    return (int)FX_OK;
  });
}

static int batch_run(fx_batch* b, hipStream_t st) {
  const fx_batch_info& I = b->info;
  if (I.n_tiles == 0) return FX_OK;
  return batch_dispatch(b->dt, b->vec, I.ept, [&](auto tg, auto Nc, auto Ec) {
    using T = typename decltype(tg)::type;
    constexpr int N = decltype(Nc)::value, EPT = decltype(Ec)::value;
    auto go = [&](auto kernel) {
      hipLaunchKernelGGL(kernel, dim3(I.grid), dim3(I.block), 0, st, b->d_descs, b->d_progs,
                         b->d_tiles, I.n_tiles, I.tile_elems, b->d_partials, b->d_counters,
                         b->d_queue);
      return hip_check(hipGetLastError(), "k_batch launch");
    };
    // streaming stores are compiled for 16-byte vectors only
    if constexpr (N * sizeof(T) == 16) {
      if (b->nts)
        return b->small_slots ? go(k_batch<T, N, EPT, kTapeSmallSlots, true>)
                              : go(k_batch<T, N, EPT, kTapeMaxSlots, true>);
    }
    return b->small_slots ? go(k_batch<T, N, EPT, kTapeSmallSlots, kNTS>)
                          : go(k_batch<T, N, EPT, kTapeMaxSlots, kNTS>);
  });
}

extern "C" {

int fx_batch_create(const fx_batch_item* items, int32_t count, fx_dtype dt, const fx_launch* cfg,
                    int64_t tile_elems, fx_batch** out) {
  if (!out) return fail(FX_E_ARG, "NULL output handle");
  *out = nullptr;
  const int elem = elem_of(dt);
  if (!elem) return fail(FX_E_DTYPE, "batches evaluate floating-point dtypes only");
  if (count < 0 || (count > 0 && !items)) return fail(FX_E_ARG, "bad item list");
  if (int rc = check_launch(cfg)) return rc;
  if (tile_elems < 0) return fail(FX_E_ARG, "negative tile size");
  fx_launch c = cfg ? *cfg : fx_launch{0, 0, 0, 0};
  uintptr_t addr_or = 0;
  for (int i = 0; i < count; ++i) {
    const fx_batch_item& it = items[i];
    if (!it.tape) return fail(FX_E_ARG, "item %d: NULL tape", i);
    if (it.n < 0) return fail(FX_E_ARG, "item %d: negative size", i);
    if (it.kind != 0 && it.kind != FX_R_ACCU) return fail(FX_E_ARG, "item %d: kind %d", i, it.kind);
    if (it.n > 0 && !it.out) return fail(FX_E_ARG, "item %d: NULL output", i);
    if (it.kind == FX_R_ACCU && !it.out) return fail(FX_E_ARG, "item %d: NULL output", i);
    for (int q = 0; q < it.tape->prog.n_in; ++q) {
      if (it.n > 0 && !it.inputs[q]) return fail(FX_E_ARG, "item %d: NULL input %d", i, q);
      addr_or |= reinterpret_cast<uintptr_t>(it.inputs[q]);
    }
    if (it.kind == 0) addr_or |= reinterpret_cast<uintptr_t>(it.out);
  }
  fx_batch* b = new (std::nothrow) fx_batch;
  if (!b) return fail(FX_E_ARG, "out of host memory");
  b->dt = dt;
  b->small_slots = true;
  for (int i = 0; i < count; ++i)
    if (items[i].tape->prog.n_slots > kTapeSmallSlots) b->small_slots = false;
  fx_batch_info& I = b->info;
  I = fx_batch_info{};
  I.count = count;
  // 512 threads for 4- and 8-byte storage, 256 for half storage (4096-tree
  // batch, graph replays: FP32 0.355 against 0.367 ms with 256; half storage
  // 0.322 with 256 against 0.355 with 512)
  I.block = c.block ? c.block : (elem >= 4 ? 512 : 256);
  I.vec_bytes = (c.vec_bytes ? std::max(c.vec_bytes, elem) : 16);
  if (addr_or & 15) I.vec_bytes = elem;  // every pointer must be 16-byte aligned for vectors
  b->vec = I.vec_bytes / elem;
  // default: as many vectors per thread as fill one interpreter pass (8
  // FP32-compute lanes, 4 FP64), at most 2
  {
    const int pass_lanes = elem == 8 ? kPassLanes<double, kTapeSmallSlots>
                                     : kPassLanes<float, kTapeSmallSlots>;
    I.ept = c.ept ? c.ept : std::max(1, std::min(2, pass_lanes / b->vec));
  }
  const int64_t pass = (int64_t)I.block * I.ept * b->vec;
  // default tile: 16 block passes (65536 FP32 elements, 32768 FP64 or half)
  const int64_t want = tile_elems ? tile_elems : 16 * pass;
  I.tile_elems = ceil_div(want, pass) * pass;
  // tile table
  std::vector<batch_desc> descs(count);
  std::vector<tape_prog> progs(count);
  std::vector<batch_tile> tiles;
  std::vector<double> cost;
  int64_t first = 0;
  for (int i = 0; i < count; ++i) {
    const fx_batch_item& it = items[i];
    batch_desc& d = descs[i];
    for (int q = 0; q < kTapeMaxIn; ++q) d.in[q] = q < it.tape->prog.n_in ? it.inputs[q] : nullptr;
    d.out = it.out;
    d.n = it.n;
    d.kind = it.kind;
    const int64_t nt = std::max<int64_t>(1, ceil_div(it.n, I.tile_elems));  // accu of n=0 writes 0
    if (it.kind == 0 && it.n == 0) {
      d.n_tiles = 0;
      d.first_tile = first;
      progs[i] = it.tape->prog;
      continue;
    }
    d.n_tiles = (int32_t)nt;
    d.first_tile = first;
    for (int64_t k = 0; k < nt; ++k) {
      tiles.push_back(batch_tile{(uint32_t)i, (uint32_t)k});
      // device operations and memory streams per element, times the elements
      const int64_t elems = std::min(it.n - k * I.tile_elems, I.tile_elems);
      cost.push_back((double)elems *
                     (it.tape->prog.n_ins + 2.0 * (it.tape->prog.n_in + (it.kind == 0 ? 1 : 0))));
    }
    first += nt;
    progs[i] = it.tape->prog;
    I.bytes += (int64_t)elem * it.n * (it.tape->prog.n_in + (it.kind == 0 ? 1 : 0));
  }
  I.n_tiles = first;
  {
    uint64_t ew_bytes = 0;
    for (int i = 0; i < count; ++i)
      if (items[i].kind == 0) ew_bytes += (uint64_t)elem * (uint64_t)items[i].n;
    b->nts = kNTS || ew_bytes > kStreamStoresAbove;
  }
  {  // the queue hands out the costliest tiles first (ties: table order)
    std::vector<int64_t> order(tiles.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
    std::vector<batch_tile> sorted(tiles.size());
    for (size_t q = 0; q < order.size(); ++q) sorted[q] = tiles[order[q]];
    tiles.swap(sorted);
  }
  int resident = 1;
  if (!c.split) {
    if (int rc = batch_resident_blocks(dt, b->vec, I.ept, b->small_slots, I.block, &resident)) {
      delete b;
      return rc;
    }
  }
  const int64_t grid_default = (int64_t)device_cus() * resident;
  I.grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(c.split ? c.split : grid_default,
                                                          std::max<int64_t>(1, I.n_tiles)));
  // workspaces for launching the items one by one (default configuration)
  b->items.assign(items, items + count);
  b->progs = progs;
  b->ws_off.assign(count, 0);
  size_t ws_total = 0;
  for (int i = 0; i < count; ++i) {
    if (items[i].kind != FX_R_ACCU) continue;
    b->ws_off[i] = ws_total;
    ws_total += (fx_workspace_bytes(FX_R_ACCU, dt, fx_shape{items[i].n, 1}, nullptr) + 255) & ~(size_t)255;
  }
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMalloc(p, bytes);
  };
  alloc((void**)&b->d_descs, sizeof(batch_desc) * std::max(1, count));
  alloc((void**)&b->d_progs, sizeof(tape_prog) * std::max(1, count));
  alloc((void**)&b->d_tiles, sizeof(batch_tile) * std::max<int64_t>(1, I.n_tiles));
  alloc((void**)&b->d_partials, sizeof(double) * std::max<int64_t>(1, I.n_tiles));
  alloc((void**)&b->d_counters, sizeof(unsigned) * std::max(1, count));
  alloc((void**)&b->d_queue, 2 * sizeof(unsigned));
  if (e == hipSuccess && count)
    e = hipMemcpy(b->d_descs, descs.data(), sizeof(batch_desc) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess && count)
    e = hipMemcpy(b->d_progs, progs.data(), sizeof(tape_prog) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess && I.n_tiles)
    e = hipMemcpy(b->d_tiles, tiles.data(), sizeof(batch_tile) * I.n_tiles, hipMemcpyHostToDevice);
  alloc(&b->d_ws, std::max<size_t>(256, ws_total));
  if (e == hipSuccess) e = hipMemset(b->d_counters, 0, sizeof(unsigned) * std::max(1, count));
  if (e == hipSuccess) e = hipMemset(b->d_queue, 0, 2 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(b->d_ws, 0, std::max<size_t>(256, ws_total));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    int rc = hip_check(e, "fx_batch_create");
    batch_free(b);
    delete b;
    return rc;
  }
  // reject configurations that are not compiled before anything is enqueued
  int rc = batch_dispatch(dt, b->vec, I.ept, [](auto, auto, auto) { return FX_OK; });
  if (rc != FX_OK) {
    batch_free(b);
    delete b;
    return rc;
  }
  *out = b;
  return FX_OK;
}

int fx_batch_launch(fx_batch* b, void* stream) {
  if (!b) return fail(FX_E_ARG, "NULL batch");
  b->last_stream = S(stream);
  return batch_run(b, S(stream));
}

int fx_batch_graph(fx_batch* b, void* stream) {
  if (!b) return fail(FX_E_ARG, "NULL batch");
  hipStream_t st = S(stream);
  if (!st) return fail(FX_E_ARG, "graph capture needs a non-default stream");
  b->last_stream = st;
  if (!b->exec) {
    if (int rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal),
                           "hipStreamBeginCapture"))
      return rc;
    int rc = batch_run(b, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != FX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (int rc2 = hip_check(e, "hipStreamEndCapture")) return rc2;
    hipGraphExec_t x = nullptr;
    if (int rc3 = hip_check(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "hipGraphInstantiate")) {
      (void)hipGraphDestroy(g);
      return rc3;
    }
    b->graph = g;
    b->exec = x;
  }
  return hip_check(hipGraphLaunch(b->exec, st), "hipGraphLaunch");
}

int fx_batch_launch_each(fx_batch* b, void* stream) {
  if (!b) return fail(FX_E_ARG, "NULL batch");
  b->last_stream = S(stream);
  for (size_t i = 0; i < b->items.size(); ++i) {
    const fx_batch_item& it = b->items[i];
    const fx_shape sh{it.n, 1};
    void* ws = it.kind == FX_R_ACCU ? static_cast<char*>(b->d_ws) + b->ws_off[i] : nullptr;
    const size_t wsb = it.kind == FX_R_ACCU ? fx_workspace_bytes(FX_R_ACCU, b->dt, sh, nullptr) : 0;
    int rc = FX_OK;
    switch (b->dt) {
      case FX_F32: rc = tape_eval_typed<float>(b->progs[i], it.inputs, sh, it.kind, it.out, ws, wsb, nullptr, S(stream)); break;
      case FX_F64: rc = tape_eval_typed<double>(b->progs[i], it.inputs, sh, it.kind, it.out, ws, wsb, nullptr, S(stream)); break;
      case FX_BF16: rc = tape_eval_typed<bf16_t>(b->progs[i], it.inputs, sh, it.kind, it.out, ws, wsb, nullptr, S(stream)); break;
      case FX_F16: rc = tape_eval_typed<f16_t>(b->progs[i], it.inputs, sh, it.kind, it.out, ws, wsb, nullptr, S(stream)); break;
      default: rc = fail(FX_E_DTYPE, "bad dtype");
    }
    if (rc != FX_OK) return rc;
  }
  return FX_OK;
}

int fx_batch_describe(const fx_batch* b, fx_batch_info* out) {
  if (!b || !out) return fail(FX_E_ARG, "NULL argument");
  *out = b->info;
  return FX_OK;
}

void fx_batch_destroy(fx_batch* b) {
  if (!b) return;
  // queued work may still use the buffers; a destroy cannot report errors
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  else (void)hipDeviceSynchronize();
  batch_free(b);
  delete b;
}

}  // extern "C"
