// Fused column and row sums of the matrix workload's expression.
#include "fx_kernels.hpp"
#include "fx_workloads.hpp"

using namespace fx;

static int c2_dimsum(int kind, fx_dtype dt, const void* X, const void* Y, const void* W, void* out,
                     fx_shape s, void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, s.n_rows, s.n_cols), y = leaf<T>(Y, s.n_rows, s.n_cols),
         w = leaf<T>(W, s.n_rows, s.n_cols);
    return reduce_dim(kind, c2_expr(x, y, w),
                      static_cast<acc_out_t<T>*>(out), ws, ws_bytes, cfg, S(stream));
  });
}

extern "C" {

int fx_c2_colsum(fx_dtype dt, const void* X, const void* Y, const void* W, void* out, fx_shape s,
                 void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream) {
  return c2_dimsum(FX_R_COLSUM, dt, X, Y, W, out, s, ws, ws_bytes, cfg, stream);
}

int fx_c2_rowsum(fx_dtype dt, const void* X, const void* Y, const void* W, void* out, fx_shape s,
                 void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream) {
  return c2_dimsum(FX_R_ROWSUM, dt, X, Y, W, out, s, ws, ws_bytes, cfg, stream);
}

}  // extern "C"
