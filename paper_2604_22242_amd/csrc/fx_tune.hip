// The autotuner's native part: one tape timed under many launch
// configurations with HIP events on the caller's stream, the configuration
// grid, and the exhaustive search over it.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "fx_tape.hpp"

using namespace fx;

extern "C" int fx_model_create(int32_t n_features, int32_t hidden, const int32_t* head_sizes,
                               int32_t n_heads, fx_model** out);
extern "C" int fx_model_set(fx_model* m, const float* params, const float* mean, const float* stdv);
extern "C" int fx_model_choose(const fx_model* m, const float* features, int32_t* choice);
extern "C" void fx_model_destroy(fx_model* m);

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
      return tape_eval_exact(t, dt, inputs, n_inputs, shape, kind, out, ws, ws_bytes, &cfgs[c], st);
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
// The grid: block {64, 128, 256, 512} x EPT {1, 2, 4} x vector {one element,
// 8 bytes, 16 bytes} x four split values of the kind, in that nesting order,
// then the library default (all fields 0).  Blocks stop at 512 threads: every
// kernel is compiled for at most 512 (a 1024-thread bound would cap the
// interpreter at 128 registers per lane, and it keeps up to 90 live in its
// loop).  EPT 8 is not compiled for tapes (four interpreter passes of code per
// loop, for no gain in the sweeps).  The split values are: element-wise 0 (one
// tile per block), 2, 8 and 32 blocks per CU; accu / norm 1, 2, 4 and 8
// blocks per CU; column sums 0 (the heuristic), 1, 4 and 16 chunks per
// column; row sums 0 (the heuristic), 16, 64 and 256 column chunks.

namespace {

constexpr int kGridBlocks[4] = {64, 128, 256, 512};
constexpr int kGridEpts[3] = {1, 2, 4};
constexpr int kGridVecs[3] = {0, 8, 16};  // 0: one element
constexpr int kGridSize = 4 * 3 * 3 * 4 + 1;

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
  if (!elem) return -fail(FX_E_DTYPE, "tapes take floating-point dtypes");
  if (kind < 0 || kind > FX_R_NORM) return -fail(FX_E_ARG, "unknown kind %d", kind);
  if (!out || cap < kGridSize) return kGridSize;
  int sp[4];
  grid_splits(kind, device_cus(), sp);
  int k = 0;
  for (int b : kGridBlocks)
    for (int e : kGridEpts)
      for (int v : kGridVecs)
        for (int s : sp) out[k++] = fx_launch{b, e, v ? std::max(v, elem) : elem, s};
  out[k++] = fx_launch{0, 0, 0, 0};
  return k;
}

namespace {

// A 64-bit FNV-1a hash of a tape's program (opcodes, slots, immediates),
// storage dtype, shape and kind: the database key of a tuned item.
uint64_t tape_key(const fx_tape* t, fx_dtype dt, fx_shape shape, int kind) {
  const int32_t n = fx_tape_program(t, nullptr, nullptr, nullptr, nullptr, 0);
  std::vector<uint16_t> op(n);
  std::vector<uint8_t> s1(n), s2(n);
  std::vector<double> imm(n);
  fx_tape_program(t, op.data(), s1.data(), s2.data(), imm.data(), n);
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t bytes) {
    for (size_t i = 0; i < bytes; ++i) h = (h ^ ((const uint8_t*)p)[i]) * 1099511628211ull;
  };
  mix(op.data(), op.size() * sizeof(uint16_t));
  mix(s1.data(), s1.size());
  mix(s2.data(), s2.size());
  mix(imm.data(), imm.size() * sizeof(double));
  const int64_t tail[4] = {(int64_t)dt, shape.n_rows, shape.n_cols, kind};
  mix(tail, sizeof(tail));
  return h;
}

const char* dtype_name(fx_dtype dt) {
  switch (dt) {
    case FX_F32: return "f32";
    case FX_F64: return "f64";
    case FX_BF16: return "bf16";
    default: return "f16";
  }
}

const char* kind_name(int kind) {
  switch (kind) {
    case FX_R_ACCU: return "accu";
    case FX_R_COLSUM: return "colsum";
    case FX_R_ROWSUM: return "rowsum";
    case FX_R_NORM: return "norm";
    default: return nullptr;  // element-wise
  }
}

// Append one JSON line: the tuned item's features, every configuration's
// median time (null where it did not run), the argmin and the default's time.
int append_record(const char* path, const fx_tape* t, fx_dtype dt, fx_shape shape, int kind,
                  const float* med, int n, int arg, double seconds) {
  float feat[32];
  const int nf = fx_tape_features(t, dt, shape, kind, feat, 32);
  if (nf < 0) return -nf;
  FILE* f = fopen(path, "a");
  if (!f) return fail(FX_E_ARG, "cannot open %s for appending", path);
  const char* kn = kind_name(kind);
  fprintf(f, "{\"key\": \"%016llx:%lldx%lld:%s:%s\", \"dtype\": \"%s\", \"reduce\": ",
          (unsigned long long)tape_key(t, dt, shape, kind), (long long)shape.n_rows,
          (long long)shape.n_cols, dtype_name(dt), kn ? kn : "None", dtype_name(dt));
  if (kn) fprintf(f, "\"%s\"", kn);
  else fprintf(f, "null");
  fprintf(f, ", \"shape\": [%lld, %lld], \"cus\": %d, \"features\": [",
          (long long)shape.n_rows, (long long)shape.n_cols, device_cus());
  for (int i = 0; i < nf; ++i) fprintf(f, "%s%.4g", i ? ", " : "", feat[i]);
  fprintf(f, "], \"ms\": [");
  for (int c = 0; c < n; ++c) {
    if (isnan(med[c])) fprintf(f, "%snull", c ? ", " : "");
    else fprintf(f, "%s%.4g", c ? ", " : "", med[c]);
  }
  fprintf(f, "], \"best\": %d, \"best_ms\": %.9g, \"default_ms\": %.9g, "
          "\"mode\": \"native\", \"tune_seconds\": %.4f}\n",
          arg, med[arg], med[n - 1], seconds);
  const bool bad = ferror(f) != 0;
  if (fclose(f) != 0 || bad) return fail(FX_E_ARG, "writing %s failed", path);
  return FX_OK;
}

}  // namespace

extern "C" int fx_autotune(const fx_tape* t, fx_dtype dt, const void* const* inputs,
                           int32_t n_inputs, fx_shape shape, int kind, void* out, void* ws,
                           size_t ws_bytes, int32_t warmup, int32_t reps, fx_launch* best,
                           float* best_ms, const char* db_path, void* stream) {
  if (!t || !best || !best_ms || warmup < 0 || reps <= 0) return fail(FX_E_ARG, "bad arguments");
  const auto t0 = std::chrono::steady_clock::now();
  fx_launch grid[kGridSize];
  const int32_t n = fx_tune_grid(kind, dt, grid, kGridSize);
  if (n < 0) return -n;
  std::vector<float> ms((size_t)n * reps), med(n);
  if (int rc = fx_tune_time(t, dt, inputs, n_inputs, shape, kind, out, ws, ws_bytes, grid, n,
                            warmup, reps, ms.data(), stream))
    return rc;
  for (int c = 0; c < n; ++c) {
    float* row = ms.data() + (size_t)c * reps;
    bool ok = true;
    for (int r = 0; r < reps; ++r) ok = ok && !isnan(row[r]);
    med[c] = ok ? median_of(row, reps) : NAN;
  }
  int arg = -1;
  for (int c = 0; c + 1 < n; ++c)  // the default (last) is timed, never chosen
    if (!isnan(med[c]) && (arg < 0 || med[c] < med[arg])) arg = c;
  if (arg < 0) return fail(FX_E_UNSUPPORTED, "no configuration of the grid runs this tape");
  *best = grid[arg];
  *best_ms = med[arg];
  if (db_path) {
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return append_record(db_path, t, dt, shape, kind, med.data(), n, arg, sec);
  }
  return FX_OK;
}

// ---- the learned model, natively -------------------------------------------
//
// Features of a tape (the model's 25 inputs, in the order the model was
// trained on): the 8 operator counts (add, sub, schur, div, neg, abs, exp,
// sqrt); constants, depth, instructions, slots, inputs; 1 for 2-byte
// storage; log2 of the size, rows and columns (n x 1 for element-wise
// results and full reductions); the result kind one-hot
// (element-wise, accu, column sums, row sums, norm); bytes per element
// (inputs plus the output of an element-wise result); the transcendental
// count (div + exp + sqrt); log2 of the bytes moved.

constexpr int kModelFeatures = 25;

extern "C" int32_t fx_tape_features(const fx_tape* t, fx_dtype dt, fx_shape shape, int kind,
                                    float* out, int32_t cap) {
  if (!t) return -fail(FX_E_ARG, "NULL tape");
  const int elem = elem_of(dt);
  if (!elem) return -fail(FX_E_DTYPE, "tapes take floating-point dtypes");
  if (kind < 0 || kind > FX_R_NORM || kind == FX_R_DOT)
    return -fail(FX_E_ARG, "unknown kind %d", kind);
  if (shape.n_rows < 0 || shape.n_cols < 0) return -fail(FX_E_ARG, "negative shape");
  if (!out || cap < kModelFeatures) return kModelFeatures;
  const fx_tape_info& I = t->info;
  // Element-wise results and full reductions see the data as one flat
  // vector, so their rows / columns features are those of an n x 1 shape.
  const bool flat = kind == 0 || kind == FX_R_ACCU || kind == FX_R_NORM;
  const double rows = flat ? (double)shape.n_rows * (double)shape.n_cols : (double)shape.n_rows;
  const double cols = flat ? 1.0 : (double)shape.n_cols;
  const double n = std::max(1.0, rows * cols);
  const double bpe = (double)elem * (I.n_inputs + (kind == 0 ? 1 : 0));
  int k = 0;
  for (int q = 0; q < 8; ++q) out[k++] = (float)I.op_count[q];
  out[k++] = (float)I.n_consts;
  out[k++] = (float)I.depth;
  out[k++] = (float)I.n_instructions;
  out[k++] = (float)I.n_slots;
  out[k++] = (float)I.n_inputs;
  out[k++] = elem == 2 ? 1.0f : 0.0f;
  out[k++] = (float)log2(n);
  out[k++] = (float)log2(std::max(1.0, rows));
  out[k++] = (float)log2(std::max(1.0, cols));
  const int onehot[5] = {0, FX_R_ACCU, FX_R_COLSUM, FX_R_ROWSUM, FX_R_NORM};
  for (int r : onehot) out[k++] = kind == r ? 1.0f : 0.0f;
  out[k++] = (float)bpe;
  out[k++] = (float)(I.op_count[3] + I.op_count[6] + I.op_count[7]);
  out[k++] = (float)log2(std::max(1.0, bpe * n));
  return k;
}

// The model file: "FXM1", int32 n_features, hidden, n_heads, head sizes,
// float mean[n_features], std[n_features], int32 n_params, float params.
extern "C" int fx_model_load(const char* path, fx_model** out) {
  if (!path || !out) return fail(FX_E_ARG, "NULL argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(FX_E_ARG, "cannot open %s", path);
  auto rd = [&](void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; };
  char magic[4];
  int32_t F = 0, H = 0, nh = 0, heads[8], np = 0;
  bool ok = rd(magic, 4) && memcmp(magic, "FXM1", 4) == 0 && rd(&F, 4) && rd(&H, 4) && rd(&nh, 4) &&
            F > 0 && F <= 64 && H > 0 && H <= 256 && nh > 0 && nh <= 8 && rd(heads, 4 * (size_t)nh);
  int32_t C = 0;
  for (int h = 0; ok && h < nh; ++h) {
    ok = heads[h] >= 2;
    C += heads[h];
  }
  std::vector<float> mean(ok ? F : 0), stdv(ok ? F : 0), params;
  ok = ok && rd(mean.data(), 4 * (size_t)F) && rd(stdv.data(), 4 * (size_t)F) && rd(&np, 4) &&
       np == H * F + H + C * H + C;
  if (ok) {
    params.resize(np);
    ok = rd(params.data(), 4 * (size_t)np);
  }
  fclose(f);
  if (!ok) return fail(FX_E_ARG, "%s is not a model file (FXM1) of valid dimensions", path);
  fx_model* m = nullptr;
  if (int rc = fx_model_create(F, H, heads, nh, &m)) return rc;
  if (int rc = fx_model_set(m, params.data(), mean.data(), stdv.data())) {
    fx_model_destroy(m);
    return rc;
  }
  *out = m;
  return FX_OK;
}

// The model's classes onto the grid: heads block / EPT / vector / split.
extern "C" int fx_model_predict(const fx_model* m, const float* features, int kind, fx_dtype dt,
                                fx_launch* out) {
  if (!m || !features || !out) return fail(FX_E_ARG, "NULL argument");
  const int elem = elem_of(dt);
  if (!elem) return fail(FX_E_DTYPE, "tapes take floating-point dtypes");
  if (kind < 0 || kind > FX_R_NORM || kind == FX_R_DOT) return fail(FX_E_ARG, "unknown kind %d", kind);
  int32_t choice[8] = {0};
  if (int rc = fx_model_choose(m, features, choice)) return rc;
  if (choice[0] < 0 || choice[0] > 3 || choice[1] < 0 || choice[1] > 2 || choice[2] < 0 ||
      choice[2] > 2 || choice[3] < 0 || choice[3] > 3)
    return fail(FX_E_ARG, "the model's heads are not block (4) / EPT (3) / vector (3) / split (4)");
  int sp[4];
  grid_splits(kind, device_cus(), sp);
  const int v = kGridVecs[choice[2]];
  *out = fx_launch{kGridBlocks[choice[0]], kGridEpts[choice[1]], v ? std::max(v, elem) : elem,
                   sp[choice[3]]};
  return FX_OK;
}
