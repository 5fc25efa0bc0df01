// Fused reductions of two-input expressions: norm_fro(X - Y), sum(X % Y, 0).
#include "fx_kernels.hpp"
#include "fx_workloads.hpp"

using namespace fx;

extern "C" {

int fx_norm_fro_diff(fx_dtype dt, const void* X, const void* Y, fx_shape s, double* d_out,
                     void* ws, size_t ws_bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, s.n_rows, s.n_cols), y = leaf<T>(Y, s.n_rows, s.n_cols);
    return reduce_full<map_sq>(diff_expr(x, y), d_out, ws, ws_bytes, cfg, S(stream));
  });
}

int fx_colsum_xy(fx_dtype dt, const void* X, const void* Y, void* out, fx_shape s, void* ws,
                 size_t ws_bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, s.n_rows, s.n_cols), y = leaf<T>(Y, s.n_rows, s.n_cols);
    return reduce_dim(FX_R_COLSUM, xy_expr(x, y), static_cast<acc_out_t<T>*>(out), ws, ws_bytes, cfg,
                      S(stream));
  });
}

}  // extern "C"
