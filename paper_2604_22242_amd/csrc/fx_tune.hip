// Timing core of the autotuner: one tape under many launch configurations,
// timed with HIP events on the caller's stream.
#include <math.h>

#include <vector>

#include "fx_tape.hpp"

using namespace fx;

extern "C" int fx_tape_eval(const fx_tape* t, fx_dtype dt, const void* const* inputs,
                            int32_t n_inputs, fx_shape s, int kind, void* out, void* ws,
                            size_t ws_bytes, const fx_launch* cfg, void* stream);

extern "C" int fx_tune_time(const fx_tape* t, fx_dtype dt, const void* const* inputs,
                            int32_t n_inputs, fx_shape shape, int kind, void* out, void* ws,
                            size_t ws_bytes, const fx_launch* cfgs, int32_t n_cfgs, int32_t warmup,
                            int32_t reps, float* ms, void* stream) {
  if (!t || !cfgs || !ms || n_cfgs < 0 || warmup < 0 || reps <= 0)
    return fail(FX_E_ARG, "bad arguments");
  hipStream_t st = S(stream);
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  for (auto& e : ev)
    if (int rc = hip_check(hipEventCreate(&e), "hipEventCreate")) {
      for (auto& x : ev) if (x) (void)hipEventDestroy(x);
      return rc;
    }
  int status = FX_OK;
  for (int c = 0; c < n_cfgs && status == FX_OK; ++c) {
    float* row = ms + (size_t)c * reps;
    auto run = [&]() {
      return fx_tape_eval(t, dt, inputs, n_inputs, shape, kind, out, ws, ws_bytes, &cfgs[c], stream);
    };
    int rc = run();  // the first launch also validates the configuration
    if (rc == FX_E_UNSUPPORTED || rc == FX_E_CONFIG || rc == FX_E_WORKSPACE) {
      for (int r = 0; r < reps; ++r) row[r] = NAN;
      continue;
    }
    if (rc != FX_OK) { status = rc; break; }
    for (int w = 1; w < warmup && status == FX_OK; ++w) status = run();
    for (int r = 0; r < reps && status == FX_OK; ++r) {
      status = hip_check(hipEventRecord(ev[2 * r], st), "hipEventRecord");
      if (status == FX_OK) status = run();
      if (status == FX_OK) status = hip_check(hipEventRecord(ev[2 * r + 1], st), "hipEventRecord");
    }
    if (status != FX_OK) break;
    if ((status = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize")) != FX_OK) break;
    for (int r = 0; r < reps; ++r) {
      float m = NAN;
      if (hipEventElapsedTime(&m, ev[2 * r], ev[2 * r + 1]) != hipSuccess) m = NAN;
      row[r] = m;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return status;
}
