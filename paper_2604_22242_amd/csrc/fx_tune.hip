// The autotuner's native part: one tape timed under many launch
// configurations with HIP events on the caller's stream, the configuration
// grid, and the exhaustive search over it.
#include <math.h>

#include <algorithm>
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

// ---- exhaustive search -------------------------------------------------------
//
// The grid: block {64, 128, 256, 512} x EPT {1, 2} x vector {one element, 16
// bytes} x four split values of the kind, in that nesting order, then the
// library default (all fields 0).  The split values are: element-wise 0 (one
// tile per block), 2, 8 and 32 blocks per CU; accu / norm 1, 2, 4 and 8
// blocks per CU; column sums 0 (the heuristic), 1, 4 and 16 chunks per
// column; row sums 0 (the heuristic), 16, 64 and 256 column chunks.

namespace {

constexpr int kGridBlocks[4] = {64, 128, 256, 512};
constexpr int kGridEpts[2] = {1, 2};
constexpr int kGridSize = 4 * 2 * 2 * 4 + 1;

void grid_splits(int kind, int cus, int* s) {
  switch (kind) {
    case FX_R_ACCU: case FX_R_NORM: s[0] = cus; s[1] = 2 * cus; s[2] = 4 * cus; s[3] = 8 * cus; break;
    case FX_R_COLSUM: s[0] = 0; s[1] = 1; s[2] = 4; s[3] = 16; break;
    case FX_R_ROWSUM: s[0] = 0; s[1] = 16; s[2] = 64; s[3] = 256; break;
    default: s[0] = 0; s[1] = 2 * cus; s[2] = 8 * cus; s[3] = 32 * cus; break;
  }
}

int elem_of(fx_dtype dt) {
  switch (dt) {
    case FX_F32: return 4;
    case FX_F64: return 8;
    case FX_BF16: case FX_F16: return 2;
    default: return 0;
  }
}

float median_of(float* v, int n) {
  std::sort(v, v + n);
  return n % 2 ? v[n / 2] : 0.5f * (v[n / 2 - 1] + v[n / 2]);
}

}  // namespace

extern "C" int32_t fx_tune_grid(int kind, fx_dtype dt, fx_launch* out, int32_t cap) {
  const int elem = elem_of(dt);
  if (!elem) return fail(FX_E_DTYPE, "tapes take floating-point dtypes");
  if (kind < 0 || kind > FX_R_NORM) return fail(FX_E_ARG, "unknown kind %d", kind);
  if (!out || cap < kGridSize) return kGridSize;
  int sp[4];
  grid_splits(kind, device_cus(), sp);
  int k = 0;
  for (int b : kGridBlocks)
    for (int e : kGridEpts)
      for (int vb : {elem, 16})
        for (int s : sp) out[k++] = fx_launch{b, e, vb, s};
  out[k++] = fx_launch{0, 0, 0, 0};
  return k;
}

extern "C" int fx_autotune(const fx_tape* t, fx_dtype dt, const void* const* inputs,
                           int32_t n_inputs, fx_shape shape, int kind, void* out, void* ws,
                           size_t ws_bytes, int32_t warmup, int32_t reps, fx_launch* best,
                           float* best_ms, void* stream) {
  if (!t || !best || !best_ms || warmup < 0 || reps <= 0) return fail(FX_E_ARG, "bad arguments");
  fx_launch grid[kGridSize];
  const int32_t n = fx_tune_grid(kind, dt, grid, kGridSize);
  if (n < 0) return n;
  std::vector<float> ms((size_t)n * reps);
  if (int rc = fx_tune_time(t, dt, inputs, n_inputs, shape, kind, out, ws, ws_bytes, grid, n,
                            warmup, reps, ms.data(), stream))
    return rc;
  int arg = -1;
  float lo = INFINITY;
  for (int c = 0; c + 1 < n; ++c) {  // the default (last) is timed, never chosen
    float* row = ms.data() + (size_t)c * reps;
    bool ok = true;
    for (int r = 0; r < reps; ++r) ok = ok && !isnan(row[r]);
    if (!ok) continue;
    const float m = median_of(row, reps);
    if (m < lo) { lo = m; arg = c; }
  }
  if (arg < 0) return fail(FX_E_UNSUPPORTED, "no configuration of the grid runs this tape");
  *best = grid[arg];
  *best_ms = lo;
  return FX_OK;
}
