// Host-side pieces shared by every entry point: error reporting, launch
// configuration resolution and workspace layout.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>

#include "fx_kernels.hpp"

namespace fx {

std::string& last_error() {
  thread_local std::string s;
  return s;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return FX_OK;
  return fail(FX_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

int check_launch(const fx_launch* c) {
  if (!c) return FX_OK;
  if (c->block != 0 && (c->block < 64 || c->block > kMaxBlock || c->block % 64))
    return fail(FX_E_CONFIG, "block %d: need a multiple of 64 in [64, %d]", c->block, kMaxBlock);
  if (c->ept != 0 && c->ept != 1 && c->ept != 2 && c->ept != 4 && c->ept != 8)
    return fail(FX_E_CONFIG, "ept %d: need 1, 2, 4 or 8", c->ept);
  if (c->vec_bytes != 0 && c->vec_bytes != 2 && c->vec_bytes != 4 && c->vec_bytes != 8 &&
      c->vec_bytes != 16)
    return fail(FX_E_CONFIG, "vec_bytes %d: need 2, 4, 8 or 16", c->vec_bytes);
  if (c->split < 0 || c->split > 65535 * 64)
    return fail(FX_E_CONFIG, "split %d out of range", c->split);
  return FX_OK;
}

// Defaults, from launch-configuration sweeps on MI355X (C2 expression
// 8192 x 8192 in FP32, FP64 and BF16; accu at 2^28 in BF16):
//   element-wise: one tile per block, no grid-stride loop, 512 threads x one
//     16-byte vector per input (6.6 TB/s FP32 on the C2 expression);
//   full reductions: two blocks per CU, EPT 2 (each block takes one ticket:
//     tens of thousands of tickets on one counter serialise); 256 threads
//     for 4- and 8-byte types, 512 for half types, whose compensated sums
//     cost twice the arithmetic per byte and need the extra waves to hide
//     the loads (BF16 accu at 2^28: 0.156 against 0.213 ms);
//   column sums: one block per column (512 threads, EPT 2 for 4- and
//     8-byte types; 256 threads, EPT 1 for half types), a column split into
//     chunks when there are fewer columns than blocks to fill the chip;
//   row sums: each thread owns one row vector and keeps EPT columns in
//     flight (256 threads for 4- and 8-byte types, 64 for half types; EPT 2:
//     0.130 against 0.146 ms for EPT 4 on the FP32 matrix workload once each
//     tile's loads are issued together), with enough column chunks for 8
//     waves per CU.
static constexpr int kReduceBlocksPerCU = 2;
static constexpr int kReduceMinBlocks = 32;
static constexpr int kReduceMinTilesPerBlock = 4;
static constexpr int kColsumBlocksPerCU = 8;
static constexpr int kRowsumWavesPerCU = 8;
constexpr int kRowsumMinCols = 32;

launch resolve(int kind, int elem, int64_t n_rows, int64_t n_cols, const fx_launch* cfg,
               bool aligned16) {
  fx_launch c = cfg ? *cfg : fx_launch{0, 0, 0, 0};
  launch L;
  const bool ew = kind == 0;
  const bool full = kind == FX_R_ACCU || kind == FX_R_NORM || kind == FX_R_DOT;
  const int vec16 = 16 / elem;  // sizing always assumes 16-byte vectors
  const int64_t n = n_rows * n_cols;
  const int64_t cus = device_cus();
  int vb = c.vec_bytes ? c.vec_bytes : 16;
  if (vb < elem) vb = elem;
  if (!aligned16) vb = elem;
  L.vec_bytes = vb;
  if (ew || full) {
    L.block = c.block ? c.block : default_block(kind, elem);
    L.ept = c.ept ? c.ept : default_ept(kind, elem);
    const int64_t tiles = std::max<int64_t>(1, ceil_div(n, (int64_t)L.block * L.ept * vec16));
    // full reductions: one ticket per block; below 2^24 elements the tickets
    // of two blocks per CU cost more than the extra bandwidth buys (measured:
    // 8.0 vs 10.3 us at 2^20), above it two per CU keep HBM busier.  Small
    // ones also give every block at least four tiles (but keep 32 blocks):
    // the single-pass finish is a few serial round trips plus one ticket per
    // block, which the work of a one- or two-tile block does not cover
    // (2^20 elements: 128 blocks 6.3 us, 256 blocks 7.3 us).
    const int64_t per_cu = n < ((int64_t)1 << 24) ? 1 : kReduceBlocksPerCU;
    const int64_t want =
        ew ? tiles
           : std::min<int64_t>(std::min<int64_t>(tiles, cus * per_cu),
                               std::max<int64_t>(kReduceMinBlocks, tiles / kReduceMinTilesPerBlock));
    L.split = c.split ? c.split : (int)std::min<int64_t>(want, 1 << 30);
  } else if (kind == FX_R_COLSUM) {
    L.block = c.block ? c.block : default_block(kind, elem);
    L.ept = c.ept ? c.ept : default_ept(kind, elem);
    if (!c.split && n_rows <= 32) {
      L.split = 0;  // thin columns: one thread per column
    } else {
      const int64_t target = cus * kColsumBlocksPerCU;
      int64_t s = c.split ? c.split : ceil_div(target, std::max<int64_t>(1, n_cols));
      // every chunk holds at least one full pass of the block
      s = std::min<int64_t>(s, std::max<int64_t>(1, ceil_div(n_rows, (int64_t)L.block * vec16)));
      L.split = (int)std::max<int64_t>(1, std::min<int64_t>(s, 65535));
    }
  } else {  // FX_R_ROWSUM
    L.block = c.block ? c.block : default_block(kind, elem);
    L.ept = c.ept ? c.ept : default_ept(kind, elem);
    const int64_t rblocks = std::max<int64_t>(1, ceil_div(n_rows, (int64_t)L.block * vec16));
    const int64_t target = cus * kRowsumWavesPerCU * 64 / L.block;
    int64_t s = c.split ? c.split : ceil_div(target, rblocks);
    // a defaulted split keeps at least kRowsumMinCols columns per chunk: the
    // finish adds `split` partials per row one after another, so thousands of
    // one-column chunks (a short, wide matrix) cost more than they spread
    if (!c.split) s = std::min<int64_t>(s, std::max<int64_t>(1, n_cols / kRowsumMinCols));
    s = std::min<int64_t>(s, std::max<int64_t>(1, n_cols));
    L.split = (int)std::max<int64_t>(1, std::min<int64_t>(s, 65535));
  }
  return L;
}

// Interpreted tapes want other configurations than compiled expressions:
// the interpreter's per-instruction cost shifts the balance towards more,
// smaller blocks.  Each default below is the single configuration with the
// best geometric-mean time (over each item's best) on the autotuner's
// 20,000 random training trees, per kind and storage width; on the 2,000
// held-out trees these give 1.10x the best against 1.47x for the library
// defaults.  Element-wise FP32 / FP64 tapes of 2^20 elements or more take
// two vectors per thread.  Column sums keep the split heuristic when there are fewer
// columns than CUs (one block per column would leave the chip idle); row
// sums use one row per thread in 64 column chunks.  The split default
// applies only when the whole configuration is left at 0: a caller that
// sets any field and leaves split at 0 gets the library's split heuristic.
fx_launch tape_launch(int kind, int elem, int64_t n_rows, int64_t n_cols, const fx_launch* cfg) {
  fx_launch c = cfg ? *cfg : fx_launch{0, 0, 0, 0};
  const bool all_default = !c.block && !c.ept && !c.vec_bytes && !c.split;
  const bool half = elem == 2;
  const int cus = device_cus();
  fx_launch d;
  switch (kind) {
    case FX_R_ACCU: case FX_R_NORM: d = fx_launch{512, half ? 1 : 2, 16, 2 * cus}; break;
    case FX_R_COLSUM: d = fx_launch{256, half ? 1 : 2, 16, n_cols >= cus ? 1 : 0}; break;
    case FX_R_ROWSUM: d = fx_launch{256, 2, elem, 64}; break;
    default:
      // two vectors per thread fill an interpreter pass for 4- and 8-byte
      // types; they pay off once there are enough elements to keep the chip
      // busy with fewer threads (training trees: 1.073x the best against
      // 1.096x for one vector everywhere)
      d = elem >= 4 && n_rows * n_cols >= ((int64_t)1 << 20) ? fx_launch{256, 2, 16, 0}
                                                            : fx_launch{64, 1, 16, 0};
      break;
  }
  if (!c.block) c.block = d.block;
  if (!c.ept) c.ept = d.ept;
  if (!c.vec_bytes) c.vec_bytes = d.vec_bytes;
  if (all_default) c.split = d.split;
  return c;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

ws_layout workspace_for(int kind, int64_t n_rows, int64_t n_cols, const launch& L, int) {
  ws_layout W;
  if (kind == FX_R_ACCU || kind == FX_R_NORM || kind == FX_R_DOT) {
    if (L.split > 1) {
      W.counter_bytes = 256;
      W.partial_bytes = (size_t)L.split * 8;
    }
  } else if (kind == FX_R_COLSUM) {
    if (L.split > 1) {
      W.counter_bytes = round256((size_t)n_cols * 4);
      W.partial_bytes = (size_t)n_cols * L.split * 8;
    }
  } else if (kind == FX_R_ROWSUM) {
    if (L.split > 1) {
      // counters for the worst case of one element per vector
      W.counter_bytes = round256((size_t)ceil_div(n_rows, L.block) * 4);
      W.partial_bytes = (size_t)n_rows * L.split * 8;
    }
  }
  return W;
}

}  // namespace fx

using namespace fx;

static int elem_size(fx_dtype dt) {
  switch (dt) {
    case FX_F32: case FX_U32: return 4;
    case FX_F64: return 8;
    case FX_BF16: case FX_F16: return 2;
  }
  return 0;
}

extern "C" {

const char* fx_version(void) { return "fx 0.1 (gfx950)"; }

const char* fx_last_error(void) { return last_error().c_str(); }

int fx_synchronize(void* stream) {
  return hip_check(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "hipStreamSynchronize");
}

size_t fx_workspace_bytes(int kind, fx_dtype dt, fx_shape shape, const fx_launch* cfg) {
  const int elem = elem_size(dt);
  if (!elem || shape.n_rows < 0 || shape.n_cols < 0 || check_launch(cfg)) return 0;
  if (kind < FX_R_ACCU || kind > FX_R_DOT) return 0;
  launch L = resolve(kind, elem, shape.n_rows, shape.n_cols, cfg, true);
  size_t b = workspace_for(kind, shape.n_rows, shape.n_cols, L, 16 / elem).total();
  // the same call may evaluate a run-time tape, whose defaults differ:
  // enough for both
  if (kind != FX_R_DOT) {
    const fx_launch t = tape_launch(kind, elem, shape.n_rows, shape.n_cols, cfg);
    launch T = resolve(kind, elem, shape.n_rows, shape.n_cols, &t, true);
    b = std::max(b, workspace_for(kind, shape.n_rows, shape.n_cols, T, 16 / elem).total());
  }
  return b;
}

int fx_resolve_launch(int kind, fx_dtype dt, fx_shape shape, const fx_launch* cfg,
                      fx_launch* out) {
  const int elem = elem_size(dt);
  if (!elem) return fail(FX_E_DTYPE, "unknown dtype %d", (int)dt);
  if (!out || shape.n_rows < 0 || shape.n_cols < 0) return fail(FX_E_ARG, "bad arguments");
  if (kind < 0 || kind > FX_R_DOT) return fail(FX_E_ARG, "unknown kind %d", kind);
  if (int rc = check_launch(cfg)) return rc;
  launch L = resolve(kind, elem, shape.n_rows, shape.n_cols, cfg, true);
  *out = fx_launch{L.block, L.ept, L.vec_bytes, L.split};
  return FX_OK;
}

}  // extern "C"
