// Learned launch-configuration model: a two-layer perceptron
//   x -> standardise -> h = relu(W1 x + b1) -> logits = W2 h + b2
// whose logits are split into one softmax head per launch knob (block, EPT,
// vector width, split), trained with softmax cross-entropy against the
// exhaustive autotuner's best configuration and Adam.  FP32 throughout, plain
// FMA arithmetic (the layers are 25x64 and 64x12: far too small for matrix
// cores to matter).
//
// Kernels:
//   k_mlp_rows    one block per batch row: forward, loss, dlogits, dh (the
//                 batch's rows optionally gathered through an index list)
//   k_mlp_params  one thread per parameter: gradient summed over the batch
//                 in row order (deterministic), then the Adam update
//   k_mlp_predict one block per row: forward and per-head argmax
// Parameters are one flat array: W1 [H x F] row-major, b1 [H], W2 [C x H],
// b2 [C], C = sum of head sizes.
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "fx_kernels.hpp"

namespace fx {

constexpr int kMlpMaxF = 64, kMlpMaxH = 256, kMlpMaxC = 64, kMlpMaxHeads = 8;

struct mlp_dims {
  int F, H, C, n_heads;
  int head_off[kMlpMaxHeads + 1];
  __host__ __device__ int W1() const { return 0; }
  __host__ __device__ int b1() const { return H * F; }
  __host__ __device__ int W2() const { return H * F + H; }
  __host__ __device__ int b2() const { return H * F + H + C * H; }
  __host__ __device__ int n_params() const { return H * F + H + C * H + C; }
};

// Forward of one row in a block of >= max(H, C) threads; xn, h in LDS.
__device__ void mlp_row_forward(const mlp_dims& d, const float* __restrict__ x,
                                const float* __restrict__ mean, const float* __restrict__ stdv,
                                const float* __restrict__ P, float* xn, float* h, float* logit) {
  const int t = threadIdx.x;
  if (t < d.F) xn[t] = (x[t] - mean[t]) / stdv[t];
  __syncthreads();
  if (t < d.H) {
    float a = P[d.b1() + t];
    const float* w = P + d.W1() + t * d.F;
    for (int f = 0; f < d.F; ++f) a = fmaf(w[f], xn[f], a);
    h[t] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (t < d.C) {
    float a = P[d.b2() + t];
    const float* w = P + d.W2() + t * d.H;
    for (int j = 0; j < d.H; ++j) a = fmaf(w[j], h[j], a);
    logit[t] = a;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_rows(mlp_dims d, const float* __restrict__ X,
                                                const int32_t* __restrict__ labels,
                                                const int32_t* __restrict__ rows, int B,
                                                const float* __restrict__ mean,
                                                const float* __restrict__ stdv,
                                                const float* __restrict__ P, float* __restrict__ XN,
                                                float* __restrict__ Hs, float* __restrict__ DL,
                                                float* __restrict__ DH, float* __restrict__ row_loss) {
  __shared__ float xn[kMlpMaxF], h[kMlpMaxH], logit[kMlpMaxC], dl[kMlpMaxC];
  __shared__ float head_loss[kMlpMaxHeads];
  const int b = blockIdx.x, t = threadIdx.x;
  const size_t r = rows ? (size_t)rows[b] : (size_t)b;  // batch row b is data row r
  mlp_row_forward(d, X + r * d.F, mean, stdv, P, xn, h, logit);
  // per-head softmax cross-entropy: loss = log sum exp(logits) - logit[y];
  // dlogits = (softmax - onehot(y)) / B
  if (t < d.n_heads) {
    const int o = d.head_off[t], k = d.head_off[t + 1] - o;
    float m = logit[o];
    for (int c = 1; c < k; ++c) m = fmaxf(m, logit[o + c]);
    float z = 0.f;
    for (int c = 0; c < k; ++c) z += expf(logit[o + c] - m);
    const int y = min(max(labels[r * d.n_heads + t], 0), k - 1);
    for (int c = 0; c < k; ++c) {
      const float p = expf(logit[o + c] - m) / z;
      dl[o + c] = (p - (c == y ? 1.f : 0.f)) / (float)B;
    }
    head_loss[t] = logf(z) + m - logit[o + y];
  }
  __syncthreads();
  if (t == 0) {
    float L = 0.f;
    for (int q = 0; q < d.n_heads; ++q) L += head_loss[q];
    row_loss[b] = L;
  }
  if (t < d.F) XN[(size_t)b * d.F + t] = xn[t];
  if (t < d.H) {
    // dh_j = relu'(h_j) * sum_c W2[c, j] dl_c
    float g = 0.f;
    for (int c = 0; c < d.C; ++c) g = fmaf(P[d.W2() + c * d.H + t], dl[c], g);
    Hs[(size_t)b * d.H + t] = h[t];
    DH[(size_t)b * d.H + t] = h[t] > 0.f ? g : 0.f;
  }
  if (t < d.C) DL[(size_t)b * d.C + t] = dl[t];
}

// One thread per parameter: gradient over the batch in row order, then Adam.
// With lr == 0 the gradient is only written to `grad` (no update).
__global__ __launch_bounds__(256) void k_mlp_params(mlp_dims d, int B, const float* __restrict__ XN,
                                                  const float* __restrict__ Hs,
                                                  const float* __restrict__ DL,
                                                  const float* __restrict__ DH, float* __restrict__ P,
                                                  float* __restrict__ M, float* __restrict__ V,
                                                  float* __restrict__ grad, float lr, float beta1,
                                                  float beta2, float eps, float c1, float c2,
                                                  const float* __restrict__ row_loss,
                                                  float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && loss) {
    float L = 0.f;
    for (int b = 0; b < B; ++b) L += row_loss[b];
    *loss = L / (float)B;
  }
  if (i >= d.n_params()) return;
  float g = 0.f;
  if (i < d.b1()) {  // W1[j, f]
    const int j = i / d.F, f = i % d.F;
    for (int b = 0; b < B; ++b) g = fmaf(DH[(size_t)b * d.H + j], XN[(size_t)b * d.F + f], g);
  } else if (i < d.W2()) {  // b1[j]
    const int j = i - d.b1();
    for (int b = 0; b < B; ++b) g += DH[(size_t)b * d.H + j];
  } else if (i < d.b2()) {  // W2[c, j]
    const int c = (i - d.W2()) / d.H, j = (i - d.W2()) % d.H;
    for (int b = 0; b < B; ++b) g = fmaf(DL[(size_t)b * d.C + c], Hs[(size_t)b * d.H + j], g);
  } else {  // b2[c]
    const int c = i - d.b2();
    for (int b = 0; b < B; ++b) g += DL[(size_t)b * d.C + c];
  }
  if (grad) grad[i] = g;
  if (lr == 0.f) return;
  const float m = beta1 * M[i] + (1.f - beta1) * g;
  const float v = beta2 * V[i] + (1.f - beta2) * g * g;
  M[i] = m;
  V[i] = v;
  P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_forward(mlp_dims d, const float* __restrict__ X,
                                                   const float* __restrict__ mean,
                                                   const float* __restrict__ stdv,
                                                   const float* __restrict__ P,
                                                   float* __restrict__ logits,
                                                   int32_t* __restrict__ choice) {
  __shared__ float xn[kMlpMaxF], h[kMlpMaxH], logit[kMlpMaxC];
  const int b = blockIdx.x, t = threadIdx.x;
  mlp_row_forward(d, X + (size_t)b * d.F, mean, stdv, P, xn, h, logit);
  if (logits && t < d.C) logits[(size_t)b * d.C + t] = logit[t];
  if (choice && t < d.n_heads) {
    const int o = d.head_off[t], k = d.head_off[t + 1] - o;
    int best = 0;
    for (int c = 1; c < k; ++c)
      if (logit[o + c] > logit[o + best]) best = c;
    choice[(size_t)b * d.n_heads + t] = best;
  }
}

}  // namespace fx

using namespace fx;

struct fx_model {
  mlp_dims d;
  float* dP = nullptr;   // params, Adam moments, standardisation
  float* dM = nullptr;
  float* dV = nullptr;
  float* dMean = nullptr;
  float* dStd = nullptr;
  float* scratch = nullptr;  // XN, Hs, DL, DH, row_loss for `cap` rows
  int cap = 0;
  int32_t* perm = nullptr;  // fx_model_train's visiting order, `perm_cap` entries
  size_t perm_cap = 0;
  long step = 0;
  // Host twin for single queries.  Training updates the parameters on the
  // device only and marks the twin stale; it is refreshed (after the device
  // has finished) before anything reads it.  `version` counts every change
  // of the parameters or the standardisation, so cached picks can tell.
  mutable std::mutex twin_mu;
  mutable bool twin_stale = false;
  mutable std::vector<float> hP;
  std::vector<float> hMean, hStd;
  std::atomic<long> version{0};
};

namespace fx {
long model_version(const fx_model* m) { return m ? m->version.load() : 0; }
}  // namespace fx

// Bring the host twin of the parameters up to date (caller holds twin_mu).
static int refresh_twin(const fx_model* m) {
  if (!m->twin_stale) return FX_OK;
  if (int rc = hip_check(hipDeviceSynchronize(), "model twin refresh")) return rc;
  if (int rc = hip_check(hipMemcpy(m->hP.data(), m->dP, m->d.n_params() * sizeof(float),
                                   hipMemcpyDeviceToHost), "model twin refresh"))
    return rc;
  m->twin_stale = false;
  return FX_OK;
}

// Release paths cannot report errors: a failed hipFree here only means the
// context is already gone.
static void model_free(fx_model* m) {
  (void)hipFree(m->dP);
  (void)hipFree(m->dM);
  (void)hipFree(m->dV);
  (void)hipFree(m->dMean);
  (void)hipFree(m->dStd);
  (void)hipFree(m->scratch);
  (void)hipFree(m->perm);
}

static int ensure_scratch(fx_model* m, int B) {
  if (B <= m->cap) return FX_OK;
  (void)hipFree(m->scratch);
  m->scratch = nullptr;
  const mlp_dims& d = m->d;
  const size_t per_row = (size_t)d.F + 2 * d.H + d.C + 1;
  if (int rc = hip_check(hipMalloc((void**)&m->scratch, per_row * B * sizeof(float)), "hipMalloc")) {
    m->cap = 0;
    return rc;
  }
  m->cap = B;
  return FX_OK;
}

extern "C" {

int fx_model_create(int32_t n_features, int32_t hidden, const int32_t* head_sizes, int32_t n_heads,
                    fx_model** out) {
  if (!out || !head_sizes) return fail(FX_E_ARG, "NULL argument");
  *out = nullptr;
  if (n_features <= 0 || n_features > kMlpMaxF || hidden <= 0 || hidden > kMlpMaxH ||
      n_heads <= 0 || n_heads > kMlpMaxHeads)
    return fail(FX_E_ARG, "model dimensions out of range (F <= %d, H <= %d, heads <= %d)", kMlpMaxF,
                kMlpMaxH, kMlpMaxHeads);
  mlp_dims d{};
  d.F = n_features;
  d.H = hidden;
  d.n_heads = n_heads;
  d.head_off[0] = 0;
  for (int q = 0; q < n_heads; ++q) {
    if (head_sizes[q] < 2) return fail(FX_E_ARG, "head %d needs at least two classes", q);
    d.head_off[q + 1] = d.head_off[q] + head_sizes[q];
  }
  d.C = d.head_off[n_heads];
  if (d.C > kMlpMaxC) return fail(FX_E_ARG, "too many classes (%d)", d.C);
  fx_model* m = new (std::nothrow) fx_model;
  if (!m) return fail(FX_E_ARG, "out of host memory");
  m->d = d;
  const size_t np = d.n_params();
  hipError_t e = hipSuccess;
  auto alloc = [&](float** p, size_t n) {
    if (e == hipSuccess) e = hipMalloc((void**)p, n * sizeof(float));
  };
  alloc(&m->dP, np);
  alloc(&m->dM, np);
  alloc(&m->dV, np);
  alloc(&m->dMean, d.F);
  alloc(&m->dStd, d.F);
  if (e == hipSuccess) e = hipMemset(m->dP, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->dM, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->dV, 0, np * sizeof(float));
  m->hP.assign(np, 0.f);
  m->hMean.assign(d.F, 0.f);
  m->hStd.assign(d.F, 1.f);
  if (e == hipSuccess)
    e = hipMemcpy(m->dMean, m->hMean.data(), d.F * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->dStd, m->hStd.data(), d.F * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    int rc = hip_check(e, "fx_model_create");
    model_free(m);
    delete m;
    return rc;
  }
  *out = m;
  return FX_OK;
}

int32_t fx_model_num_params(const fx_model* m) { return m ? m->d.n_params() : 0; }

int fx_model_set(fx_model* m, const float* params, const float* mean, const float* stdv) {
  if (!m) return fail(FX_E_ARG, "NULL model");
  const mlp_dims& d = m->d;
  if (stdv)
    for (int f = 0; f < d.F; ++f)
      if (!(stdv[f] > 0.f)) return fail(FX_E_ARG, "standard deviation %d is not positive", f);
  std::lock_guard<std::mutex> g(m->twin_mu);
  // only the arrays passed are written; the others keep their current values
  // on the device (the host twin of the parameters may be stale then, and is
  // refreshed when next read)
  hipError_t e = hipSuccess;
  if (params) {
    e = hipDeviceSynchronize();  // queued training steps finish before the overwrite
    m->hP.assign(params, params + d.n_params());
    m->twin_stale = false;
    if (e == hipSuccess)
      e = hipMemcpy(m->dP, m->hP.data(), d.n_params() * sizeof(float), hipMemcpyHostToDevice);
    // a new starting point resets Adam
    if (e == hipSuccess) e = hipMemset(m->dM, 0, d.n_params() * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->dV, 0, d.n_params() * sizeof(float));
    m->step = 0;
  }
  if (mean) {
    m->hMean.assign(mean, mean + d.F);
    if (e == hipSuccess)
      e = hipMemcpy(m->dMean, m->hMean.data(), d.F * sizeof(float), hipMemcpyHostToDevice);
  }
  if (stdv) {
    m->hStd.assign(stdv, stdv + d.F);
    if (e == hipSuccess)
      e = hipMemcpy(m->dStd, m->hStd.data(), d.F * sizeof(float), hipMemcpyHostToDevice);
  }
  m->version++;
  return hip_check(e, "fx_model_set");
}

int fx_model_get(fx_model* m, float* params, float* mean, float* stdv) {
  if (!m) return fail(FX_E_ARG, "NULL model");
  const mlp_dims& d = m->d;
  std::lock_guard<std::mutex> g(m->twin_mu);
  m->twin_stale = true;  // read the device copy even if nothing was trained
  if (int rc = refresh_twin(m)) return rc;
  if (params) memcpy(params, m->hP.data(), d.n_params() * sizeof(float));
  if (mean) memcpy(mean, m->hMean.data(), d.F * sizeof(float));
  if (stdv) memcpy(stdv, m->hStd.data(), d.F * sizeof(float));
  return FX_OK;
}

// Gradient (lr = 0) or one Adam step over a batch of B rows in device memory.
// `rows` (device, may be NULL) lists the B data rows of the batch.
static int model_step(fx_model* m, const float* X, const int32_t* labels, const int32_t* rows,
                      int32_t B, float lr, float beta1, float beta2, float eps, float* d_loss,
                      float* d_grad, hipStream_t st) {
  if (!m || !X || !labels || B <= 0) return fail(FX_E_ARG, "bad arguments");
  if (int rc = ensure_scratch(m, B)) return rc;
  const mlp_dims& d = m->d;
  float* XN = m->scratch;
  float* Hs = XN + (size_t)B * d.F;
  float* DL = Hs + (size_t)B * d.H;
  float* DH = DL + (size_t)B * d.C;
  float* RL = DH + (size_t)B * d.H;
  const int threads = std::max(64, ((std::max(d.H, std::max(d.F, d.C)) + 63) / 64) * 64);
  hipLaunchKernelGGL(k_mlp_rows, dim3(B), dim3(threads), 0, st, d, X, labels, rows, B, m->dMean,
                     m->dStd, m->dP, XN, Hs, DL, DH, RL);
  double c1 = 1.0, c2 = 1.0;
  if (lr != 0.f) {
    m->step += 1;
    c1 = 1.0 - pow((double)beta1, (double)m->step);
    c2 = 1.0 - pow((double)beta2, (double)m->step);
  }
  const int np = d.n_params();
  hipLaunchKernelGGL(k_mlp_params, dim3((np + 255) / 256), dim3(256), 0, st, d, (int)B, XN, Hs, DL,
                     DH, m->dP, m->dM, m->dV, d_grad, lr, beta1, beta2, eps, (float)c1, (float)c2,
                     RL, d_loss);
  if (lr != 0.f) {  // the parameters change on the device
    std::lock_guard<std::mutex> g(m->twin_mu);
    m->twin_stale = true;
    m->version++;
  }
  return hip_check(hipGetLastError(), "k_mlp launch");
}

int fx_model_train_step(fx_model* m, const float* d_X, const int32_t* d_labels, int32_t batch,
                        float lr, float* d_loss, void* stream) {
  if (!(lr > 0.f)) return fail(FX_E_ARG, "learning rate must be positive");
  return model_step(m, d_X, d_labels, nullptr, batch, lr, 0.9f, 0.999f, 1e-8f, d_loss, nullptr,
                    S(stream));
}

int fx_model_train(fx_model* m, const float* d_X, const int32_t* d_labels, int32_t n,
                   int32_t epochs, int32_t batch, float lr, const int32_t* perm,
                   float* d_losses, void* stream) {
  if (!m || !d_X || !d_labels || n <= 0 || epochs < 0 || batch <= 0)
    return fail(FX_E_ARG, "bad arguments");
  if (!(lr > 0.f)) return fail(FX_E_ARG, "learning rate must be positive");
  if (epochs == 0) return FX_OK;
  const size_t total = (size_t)epochs * n;
  if (perm) {  // every epoch's order must be a permutation of 0..n-1
    std::vector<uint8_t> seen(n);
    for (int32_t e = 0; e < epochs; ++e) {
      std::fill(seen.begin(), seen.end(), 0);
      for (int32_t i = 0; i < n; ++i) {
        const int32_t r = perm[(size_t)e * n + i];
        if (r < 0 || r >= n || seen[r]) return fail(FX_E_ARG, "epoch %d order is not a permutation", e);
        seen[r] = 1;
      }
    }
  }
  hipStream_t st = S(stream);
  if (total > m->perm_cap) {
    (void)hipFree(m->perm);
    m->perm = nullptr;
    m->perm_cap = 0;
    if (int rc = hip_check(hipMalloc((void**)&m->perm, total * sizeof(int32_t)), "hipMalloc"))
      return rc;
    m->perm_cap = total;
  }
  std::vector<int32_t> natural;
  const int32_t* src = perm;
  if (!src) {
    natural.resize(total);
    for (size_t i = 0; i < total; ++i) natural[i] = (int32_t)(i % (size_t)n);
    src = natural.data();
  }
  // The order buffer belongs to the model: the copy is queued behind the
  // stream's earlier work, and waited for before the host array can go.
  if (int rc = hip_check(hipMemcpyAsync(m->perm, src, total * sizeof(int32_t),
                                        hipMemcpyHostToDevice, st), "hipMemcpyAsync"))
    return rc;
  if (int rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize")) return rc;
  for (int32_t e = 0; e < epochs; ++e)
    for (int32_t s = 0; s < n; s += batch) {
      const int32_t b = std::min(batch, n - s);
      const bool last = s + b >= n;
      if (int rc = model_step(m, d_X, d_labels, m->perm + (size_t)e * n + s, b, lr, 0.9f, 0.999f,
                              1e-8f, last && d_losses ? d_losses + e : nullptr, nullptr, st))
        return rc;
    }
  return FX_OK;
}

int fx_model_grad(fx_model* m, const float* d_X, const int32_t* d_labels, int32_t batch,
                  float* d_grad, float* d_loss, void* stream) {
  if (!d_grad) return fail(FX_E_ARG, "NULL gradient output");
  return model_step(m, d_X, d_labels, nullptr, batch, 0.f, 0.9f, 0.999f, 1e-8f, d_loss, d_grad,
                    S(stream));
}

int fx_model_forward(const fx_model* m, const float* d_X, int32_t batch, float* d_logits,
                     int32_t* d_choice, void* stream) {
  if (!m || !d_X || batch < 0 || (!d_logits && !d_choice)) return fail(FX_E_ARG, "bad arguments");
  if (batch == 0) return FX_OK;
  const mlp_dims& d = m->d;
  const int threads = std::max(64, ((std::max(d.H, std::max(d.F, d.C)) + 63) / 64) * 64);
  hipLaunchKernelGGL(k_mlp_forward, dim3(batch), dim3(threads), 0, S(stream), d, d_X, m->dMean,
                     m->dStd, m->dP, d_logits, d_choice);
  return hip_check(hipGetLastError(), "k_mlp_forward launch");
}

// Host twin of the predict kernel for one feature row (no GPU involved): the
// same arithmetic in the same order, FP32 with fused multiply-adds.
int fx_model_choose(const fx_model* m, const float* x, int32_t* choice) {
  if (!m || !x || !choice) return fail(FX_E_ARG, "NULL argument");
  const mlp_dims& d = m->d;
  std::lock_guard<std::mutex> g(m->twin_mu);
  if (int rc = refresh_twin(m)) return rc;
  const float* P = m->hP.data();
  float xn[kMlpMaxF], h[kMlpMaxH], logit[kMlpMaxC];
  for (int f = 0; f < d.F; ++f) xn[f] = (x[f] - m->hMean[f]) / m->hStd[f];
  for (int j = 0; j < d.H; ++j) {
    float a = P[d.b1() + j];
    for (int f = 0; f < d.F; ++f) a = fmaf(P[d.W1() + j * d.F + f], xn[f], a);
    h[j] = a > 0.f ? a : 0.f;
  }
  for (int c = 0; c < d.C; ++c) {
    float a = P[d.b2() + c];
    for (int j = 0; j < d.H; ++j) a = fmaf(P[d.W2() + c * d.H + j], h[j], a);
    logit[c] = a;
  }
  for (int q = 0; q < d.n_heads; ++q) {
    const int o = d.head_off[q], k = d.head_off[q + 1] - o;
    int best = 0;
    for (int c = 1; c < k; ++c)
      if (logit[o + c] > logit[o + best]) best = c;
    choice[q] = best;
  }
  return FX_OK;
}

void fx_model_destroy(fx_model* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();  // queued work may still use the buffers
  model_free(m);
  delete m;
}

}  // extern "C"
