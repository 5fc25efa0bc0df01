// Fused C-ABI entry point of the matrix workload's element-wise result.
#include "fx_kernels.hpp"
#include "fx_workloads.hpp"

using namespace fx;

extern "C" {

int fx_c2_z(fx_dtype dt, const void* X, const void* Y, const void* W, void* Z, fx_shape s,
            const fx_launch* cfg, void* stream) {
  if (int rc = check_shape(s)) return rc;
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, s.n_rows, s.n_cols), y = leaf<T>(Y, s.n_rows, s.n_cols),
         w = leaf<T>(W, s.n_rows, s.n_cols);
    return eval(static_cast<T*>(Z), c2_expr(x, y, w), cfg, S(stream));
  });
}

}  // extern "C"
