// Fused C-ABI entry points: each is one expression written with the
// expression-template front end and evaluated by one skeleton kernel.
#include "fx.hpp"
#include "fx_workloads.hpp"

using namespace fx;

extern "C" {

int fx_c1_z(fx_dtype dt, const void* X, const void* Y, const void* W, void* Z, int64_t n,
            const fx_launch* cfg, void* stream) {
  if (int rc = check_n(n)) return rc;
  if (dt == FX_U32) {
    auto x = leaf<uint32_t>(X, n, 1), y = leaf<uint32_t>(Y, n, 1), w = leaf<uint32_t>(W, n, 1);
    return eval(static_cast<uint32_t*>(Z), c1_expr(x, y, w), cfg, S(stream));
  }
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, n, 1), y = leaf<T>(Y, n, 1), w = leaf<T>(W, n, 1);
    return eval(static_cast<T*>(Z), c1_expr(x, y, w), cfg, S(stream));
  });
}

int fx_axy_expw(fx_dtype dt, double a, const void* X, const void* Y, const void* W, void* Z,
                int64_t n, const fx_launch* cfg, void* stream) {
  if (int rc = check_n(n)) return rc;
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, n, 1), y = leaf<T>(Y, n, 1), w = leaf<T>(W, n, 1);
    return eval(static_cast<T*>(Z), axy_expw_expr(a, x, y, w), cfg, S(stream));
  });
}

int fx_accu_xy(fx_dtype dt, const void* X, const void* Y, int64_t n, void* d_out, void* ws,
               size_t ws_bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_n(n)) return rc;
  if (dt == FX_U32) {
    auto x = leaf<uint32_t>(X, n, 1), y = leaf<uint32_t>(Y, n, 1);
    return accu(xy_expr(x, y), static_cast<uint64_t*>(d_out), ws, ws_bytes, cfg, S(stream));
  }
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    auto x = leaf<T>(X, n, 1), y = leaf<T>(Y, n, 1);
    return accu(xy_expr(x, y), static_cast<double*>(d_out), ws, ws_bytes, cfg, S(stream));
  });
}

int fx_dot(fx_dtype dt, const void* X, const void* Y, int64_t n, void* d_out, void* ws,
           size_t ws_bytes, const fx_launch* cfg, void* stream) {
  if (int rc = check_n(n)) return rc;
  if (dt == FX_U32) {
    const dmat<uint32_t> x{static_cast<uint32_t*>(const_cast<void*>(X)), n, 1},
        y{static_cast<uint32_t*>(const_cast<void*>(Y)), n, 1};
    return dot(x, y, static_cast<uint64_t*>(d_out), ws, ws_bytes, cfg, S(stream));
  }
  return with_fp(dt, [&](auto t) {
    using T = typename decltype(t)::type;
    const dmat<T> x{static_cast<T*>(const_cast<void*>(X)), n, 1},
        y{static_cast<T*>(const_cast<void*>(Y)), n, 1};
    return dot(x, y, static_cast<double*>(d_out), ws, ws_bytes, cfg, S(stream));
  });
}

}  // extern "C"
