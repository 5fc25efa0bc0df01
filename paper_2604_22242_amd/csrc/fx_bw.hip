// Bandwidth ceilings of this device, the analogue of the copy benchmark the
// paper uses for its achievable-bandwidth figure (Sec. 4): copy (through the
// same element-wise skeleton as every fused expression), read, write, and a
// three-read one-write triad (the read/write mix of the matrix workload).
#include "fx_kernels.hpp"

using namespace fx;

namespace {

using u32x4 = raw<16>::type;

// Each block streams a contiguous tile of blockDim * EPT 16-byte vectors per
// step and folds them with XOR; one value per block goes to sink (so the
// loads cannot be removed).
template <int EPT>
__global__ __launch_bounds__(kMaxBlock) void k_bw_read(const u32x4* __restrict__ src, int64_t nv,
                                                     double* sink) {
  __shared__ unsigned lds[kMaxBlock / 64];
  unsigned acc = 0;
  const int64_t tile = (int64_t)blockDim.x * EPT;
  for (int64_t t = (int64_t)blockIdx.x * tile; t < nv; t += (int64_t)gridDim.x * tile) {
    u32x4 r[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int64_t v = t + threadIdx.x + k * blockDim.x;
      r[k] = v < nv ? (kNT ? __builtin_nontemporal_load(src + v) : src[v]) : u32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) acc ^= r[k].x ^ r[k].y ^ r[k].z ^ r[k].w;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc ^= __shfl_xor(acc, m, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t ^= lds[w];
    sink[blockIdx.x] = (double)t;
  }
}

template <int EPT>
__global__ __launch_bounds__(kMaxBlock) void k_bw_write(u32x4* __restrict__ dst, int64_t nv,
                                                      unsigned value) {
  const u32x4 v4 = {value, value, value, value};
  const int64_t tile = (int64_t)blockDim.x * EPT;
  for (int64_t t = (int64_t)blockIdx.x * tile; t < nv; t += (int64_t)gridDim.x * tile) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int64_t v = t + threadIdx.x + k * blockDim.x;
      if (v < nv) {
        if (kNTS) __builtin_nontemporal_store(v4, dst + v);
        else dst[v] = v4;
      }
    }
  }
}

// dst = a + b + c (u32 lanes, wrapping): three streams read for every one
// written, the mix of the matrix workload's Z, with no arithmetic to speak
// of.  Grid-stride over tiles of blockDim * EPT vectors per array; all 3*EPT
// loads of a tile are issued before its stores.  NTS: streaming stores.
template <int EPT, bool NTS>
__global__ __launch_bounds__(kMaxBlock) void k_bw_triad(const u32x4* __restrict__ a,
                                                      const u32x4* __restrict__ b,
                                                      const u32x4* __restrict__ c,
                                                      u32x4* __restrict__ dst, int64_t nv) {
  const int64_t tile = (int64_t)blockDim.x * EPT;
  for (int64_t t = (int64_t)blockIdx.x * tile; t < nv; t += (int64_t)gridDim.x * tile) {
    u32x4 ra[EPT], rb[EPT], rc[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int64_t v = t + threadIdx.x + k * blockDim.x;
      if (v < nv) {
        ra[k] = kNT ? __builtin_nontemporal_load(a + v) : a[v];
        rb[k] = kNT ? __builtin_nontemporal_load(b + v) : b[v];
        rc[k] = kNT ? __builtin_nontemporal_load(c + v) : c[v];
      }
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int64_t v = t + threadIdx.x + k * blockDim.x;
      if (v < nv) {
        const u32x4 s = ra[k] + rb[k] + rc[k];
        if (NTS) __builtin_nontemporal_store(s, dst + v);
        else dst[v] = s;
      }
    }
  }
}

int check_bytes(const void* p, size_t bytes) {
  if (bytes % 16) return fail(FX_E_ARG, "byte count %zu is not a multiple of 16", bytes);
  if (reinterpret_cast<uintptr_t>(p) % 16) return fail(FX_E_ARG, "pointer not 16-byte aligned");
  if (bytes && !p) return fail(FX_E_ARG, "NULL pointer");
  return FX_OK;
}

}  // namespace

extern "C" {

int fx_bw_copy(const void* src, void* dst, size_t bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_bytes(src, bytes)) return rc;
  if (int rc = check_bytes(dst, bytes)) return rc;
  const int64_t n = (int64_t)(bytes / 4);
  return eval(static_cast<uint32_t*>(dst), leaf<uint32_t>(src, n, 1), cfg, S(stream));
}

int fx_bw_read(const void* src, size_t bytes, double* sink, const fx_launch* cfg, void* stream) {
  if (int rc = check_bytes(src, bytes)) return rc;
  if (int rc = check_launch(cfg)) return rc;
  if (!sink) return fail(FX_E_ARG, "NULL sink");
  launch L = resolve(0, 4, (int64_t)(bytes / 4), 1, cfg, true);
  const int64_t nv = (int64_t)(bytes / 16);
  return with_ept(L.ept, [&](auto Ec) {
    constexpr int EPT = decltype(Ec)::value;
    hipLaunchKernelGGL((k_bw_read<EPT>), dim3(L.split), dim3(L.block), 0, S(stream),
                       static_cast<const u32x4*>(src), nv, sink);
    return hip_check(hipGetLastError(), "k_bw_read launch");
  });
}

int fx_bw_write(void* dst, size_t bytes, uint32_t value, const fx_launch* cfg, void* stream) {
  if (int rc = check_bytes(dst, bytes)) return rc;
  if (int rc = check_launch(cfg)) return rc;
  launch L = resolve(0, 4, (int64_t)(bytes / 4), 1, cfg, true);
  const int64_t nv = (int64_t)(bytes / 16);
  return with_ept(L.ept, [&](auto Ec) {
    constexpr int EPT = decltype(Ec)::value;
    hipLaunchKernelGGL((k_bw_write<EPT>), dim3(L.split), dim3(L.block), 0, S(stream),
                       static_cast<u32x4*>(dst), nv, value);
    return hip_check(hipGetLastError(), "k_bw_write launch");
  });
}

int fx_bw_triad(const void* a, const void* b, const void* c, void* dst, size_t bytes, int flags,
                const fx_launch* cfg, void* stream) {
  for (const void* p : {a, b, c, (const void*)dst})
    if (int rc = check_bytes(p, bytes)) return rc;
  if (int rc = check_launch(cfg)) return rc;
  if (flags & ~1) return fail(FX_E_ARG, "unknown flags 0x%x", flags);
  launch L = resolve(0, 4, (int64_t)(bytes / 4), 1, cfg, true);
  const int64_t nv = (int64_t)(bytes / 16);
  if (nv == 0) return FX_OK;
  return with_ept(L.ept, [&](auto Ec) {
    constexpr int EPT = decltype(Ec)::value;
    auto A = static_cast<const u32x4*>(a), B = static_cast<const u32x4*>(b),
         C = static_cast<const u32x4*>(c);
    auto D = static_cast<u32x4*>(dst);
    if (flags & 1)
      hipLaunchKernelGGL((k_bw_triad<EPT, true>), dim3(L.split), dim3(L.block), 0, S(stream), A, B,
                         C, D, nv);
    else
      hipLaunchKernelGGL((k_bw_triad<EPT, false>), dim3(L.split), dim3(L.block), 0, S(stream), A,
                         B, C, D, nv);
    return hip_check(hipGetLastError(), "k_bw_triad launch");
  });
}

}  // extern "C"
