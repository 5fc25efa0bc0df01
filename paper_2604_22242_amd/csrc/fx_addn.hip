// Z = A1 + ... + An for n = 1..16: one SumN<T, n> instantiation per n.
#include "fx_kernels.hpp"

using namespace fx;

namespace {

template <class T, int K>
int addn_k(const void* const* in, int32_t n, T* z, fx_shape s, const fx_launch* cfg, hipStream_t st) {
  if constexpr (K > 16) {
    return fail(FX_E_ARG, "add-N takes 1 to 16 inputs, %d given", n);
  } else {
    if (n != K) return addn_k<T, K + 1>(in, n, z, s, cfg, st);
    SumN<T, K> e;
    for (int q = 0; q < K; ++q) e.p[q] = static_cast<const T*>(in[q]);
    e.n_rows = s.n_rows;
    e.n_cols = s.n_cols;
    return eval(z, e, cfg, st);
  }
}

}  // namespace

extern "C" int fx_addn(fx_dtype dt, const void* const* in, int32_t n, void* Z, fx_shape s,
                       const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  if (!in) return fail(FX_E_ARG, "NULL input list");
  if (n < 1 || n > 16) return fail(FX_E_ARG, "add-N takes 1 to 16 inputs, %d given", n);
  switch (dt) {
    case FX_F32: return addn_k<float, 1>(in, n, static_cast<float*>(Z), s, cfg, S(stream));
    case FX_BF16: return addn_k<bf16_t, 1>(in, n, static_cast<bf16_t*>(Z), s, cfg, S(stream));
    default: break;
  }
  return fail(FX_E_DTYPE, "add-N is compiled for FP32 and BF16 storage");
}
