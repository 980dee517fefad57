// Screener network (fp32): 32 -> 128 -> 128 -> 4, ReLU, sigmoid output, binary
// cross-entropy, Adam; plus the feature construction from node profiles.  The network
// orders the screening of child subregions; it never decides a flag.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/nep.h"
#include "common.h"

namespace nep {

constexpr int MIN = 32, MH = 128, MOUT = 4;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MIN * MH, OFF_W2 = OFF_B1 + MH, OFF_B2 = OFF_W2 + MH * MH,
              OFF_W3 = OFF_B2 + MH, OFF_B3 = OFF_W3 + MH * MOUT, NPARAM = OFF_B3 + MOUT;

// Z[b][o] = act(sum_i A[row(b)][i] W[i][o] + bias[o]); one block per sample, one
// thread per output; the sample's input row is staged in LDS.
__global__ __launch_bounds__(128) void dense_fwd_kernel(const float* __restrict__ A, int in,
                                                        const int* __restrict__ idx, const float* __restrict__ W,
                                                        const float* __restrict__ bias, int out,
                                                        float* __restrict__ Z, int relu) {
  __shared__ float a[MH];
  const int b = blockIdx.x, o = threadIdx.x;
  const long long row = idx ? idx[b] : b;
  for (int i = threadIdx.x; i < in; i += blockDim.x) a[i] = A[row * in + i];
  __syncthreads();
  if (o >= out) return;
  float acc = bias[o];
  for (int i = 0; i < in; ++i) acc += a[i] * W[i * out + o];
  Z[(long long)b * out + o] = relu ? fmaxf(acc, 0.f) : acc;
}

// dz = (sigmoid(z) - y) / (B * 4); per-block partial of the mean BCE loss
__global__ __launch_bounds__(256) void bce_grad_kernel(const float* __restrict__ logits, const float* __restrict__ Y,
                                                       const int* __restrict__ idx, int B,
                                                       float* __restrict__ dz, float* __restrict__ part) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (e < B * MOUT) {
    const int b = e / MOUT, k = e % MOUT;
    const long long row = idx ? idx[b] : b;
    const float z = logits[e], y = Y[row * MOUT + k];
    const float p = 1.f / (1.f + expf(-z));
    dz[e] = (p - y) / (float)(B * MOUT);
    l = fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)));
  }
  l = wave_sum(l);
  __shared__ float r[4];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = r[0] + r[1] + r[2] + r[3];
}

// dA[b][i] = [act[b][i] > 0] * sum_o dZ[b][o] W[i][o]  (ReLU derivative of the input)
__global__ __launch_bounds__(128) void dense_bwd_in_kernel(const float* __restrict__ dZ, int out,
                                                           const float* __restrict__ W, int in,
                                                           const float* __restrict__ act, float* __restrict__ dA) {
  __shared__ float d[MH];
  const int b = blockIdx.x, i = threadIdx.x;
  for (int o = threadIdx.x; o < out; o += blockDim.x) d[o] = dZ[(long long)b * out + o];
  __syncthreads();
  if (i >= in) return;
  float acc = 0.f;
  for (int o = 0; o < out; ++o) acc += d[o] * W[i * out + o];
  dA[(long long)b * in + i] = act[(long long)b * in + i] > 0.f ? acc : 0.f;
}

// dW[i][o] = sum_b A[row(b)][i] dZ[b][o] (samples in order), block i = in gives db
__global__ __launch_bounds__(128) void dense_bwd_w_kernel(const float* __restrict__ A, int in,
                                                          const int* __restrict__ idx, const float* __restrict__ dZ,
                                                          int out, int B, float* __restrict__ dW,
                                                          float* __restrict__ db) {
  const int i = blockIdx.x, o = threadIdx.x;
  if (o >= out) return;
  float acc = 0.f;
  if (i < in) {
    for (int b = 0; b < B; ++b) {
      const long long row = idx ? idx[b] : b;
      acc += A[row * in + i] * dZ[(long long)b * out + o];
    }
    dW[i * out + o] = acc;
  } else {
    for (int b = 0; b < B; ++b) acc += dZ[(long long)b * out + o];
    db[o] = acc;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void sigmoid_kernel(const float* __restrict__ z, float* __restrict__ p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 1.f / (1.f + expf(-z[i]));
}

// raw[r][j] = log10(profile[r][j]) (profiles are positive norms; 0 -> -300)
__global__ __launch_bounds__(256) void log_profile_kernel(const double* __restrict__ prof, long long total,
                                                          float* __restrict__ raw) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const double v = prof[e];
  raw[e] = (float)(v > 0 ? log10(v) : -300.0);
}

// column mean and standard deviation over the listed rows (one block per column)
__global__ __launch_bounds__(256) void column_stats_kernel(const float* __restrict__ raw, int ncol,
                                                           const int* __restrict__ rows, int nrows,
                                                           float* __restrict__ mean, float* __restrict__ sd) {
  const int j = blockIdx.x;
  double s = 0, s2 = 0;
  for (int r = threadIdx.x; r < nrows; r += 256) {
    const double v = raw[(long long)rows[r] * ncol + j];
    s += v;
    s2 += v * v;
  }
  s = wave_sum(s);
  s2 = wave_sum(s2);
  __shared__ double a[4], c[4];
  if ((threadIdx.x & 63) == 0) { a[threadIdx.x >> 6] = s; c[threadIdx.x >> 6] = s2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mu = (a[0] + a[1] + a[2] + a[3]) / nrows;
    const double var = (c[0] + c[1] + c[2] + c[3]) / nrows - mu * mu;
    mean[j] = (float)mu;
    sd[j] = (float)(var > 1e-12 ? sqrt(var) : 1.0);
  }
}

__global__ __launch_bounds__(256) void standardize_kernel(float* __restrict__ raw, long long total, int ncol,
                                                          const float* __restrict__ mean,
                                                          const float* __restrict__ sd) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int j = (int)(e % ncol);
  raw[e] = (raw[e] - mean[j]) / sd[j];
}

}  // namespace nep

using namespace nep;

// workspace: Z1, Z2 (B x 128), Z3, dZ3 (B x 4), dA2, dA1 (B x 128), loss partials
static size_t work_floats(int B) { return (size_t)B * (4 * MH + 2 * MOUT) + (size_t)(B * MOUT + 255) / 256 + 1; }

extern "C" int nep_mlp_param_count(void) { return NPARAM; }
extern "C" size_t nep_mlp_workspace_floats(int B) { return B > 0 ? work_floats(B) : 0; }

static nep_status fwd(const float* P, const float* X, const int* idx, int B, float* w, hipStream_t st) {
  float* Z1 = w;
  float* Z2 = Z1 + (size_t)B * MH;
  float* Z3 = Z2 + (size_t)B * MH;
  dense_fwd_kernel<<<B, 128, 0, st>>>(X, MIN, idx, P + OFF_W1, P + OFF_B1, MH, Z1, 1);
  dense_fwd_kernel<<<B, 128, 0, st>>>(Z1, MH, nullptr, P + OFF_W2, P + OFF_B2, MH, Z2, 1);
  dense_fwd_kernel<<<B, 128, 0, st>>>(Z2, MH, nullptr, P + OFF_W3, P + OFF_B3, MOUT, Z3, 0);
  return hipGetLastError() == hipSuccess ? NEP_OK : NEP_ERR_HIP;
}

extern "C" nep_status nep_mlp_forward(const float* params, const float* X, const int32_t* idx, int B, float* probs,
                                      float* work, hipStream_t st) {
  if (!params || !X || !probs || !work || B < 1) return NEP_ERR_ARG;
  nep_status r = fwd(params, X, idx, B, work, st);
  if (r != NEP_OK) return r;
  const float* Z3 = work + (size_t)2 * B * MH;
  sigmoid_kernel<<<(B * MOUT + 255) / 256, 256, 0, st>>>(Z3, probs, B * MOUT);
  return hipGetLastError() == hipSuccess ? NEP_OK : NEP_ERR_HIP;
}

// ---------------------------------------------------------------- forward without allocation
// The activations of nep_mlp_forward_noalloc live in a file-scope device array (one copy
// per GPU, held until the process ends).  Host code never uses the array's name as an
// address: its device address is looked up once per device with hipGetSymbolAddress and
// that pointer is what the kernels receive.
static __device__ __align__(256) float scratch[(size_t)NEP_MLP_NOALLOC_MAX_B * (2 * MH + MOUT)];

static constexpr int MAX_DEVICES = 64;
static float* g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mu;

static nep_status scratch_of_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return NEP_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return NEP_ERR_HIP;
    }
    g_scratch[dev] = static_cast<float*>(p);
  }
  *out = g_scratch[dev];
  return NEP_OK;
}

extern "C" nep_status nep_mlp_forward_noalloc(const float* params, const float* X, const int32_t* idx, int B,
                                              float* probs, hipStream_t st) {
  if (!params || !X || !probs || B < 1) return NEP_ERR_ARG;
  if (B > NEP_MLP_NOALLOC_MAX_B) return NEP_ERR_CAPACITY;
  float* w = nullptr;
  nep_status r = scratch_of_current_device(&w);
  if (r != NEP_OK) return r;
  // every activation is written before it is read: nothing in the array needs clearing
  r = fwd(params, X, idx, B, w, st);
  if (r != NEP_OK) return r;
  sigmoid_kernel<<<(B * MOUT + 255) / 256, 256, 0, st>>>(w + (size_t)2 * B * MH, probs, B * MOUT);
  return hipGetLastError() == hipSuccess ? NEP_OK : NEP_ERR_HIP;
}

extern "C" nep_status nep_mlp_grad(const float* params, const float* X, const float* Y, const int32_t* idx, int B,
                                   float* grad, float* loss, float* work, hipStream_t st) {
  if (!params || !X || !Y || !grad || !work || B < 1) return NEP_ERR_ARG;
  nep_status r = fwd(params, X, idx, B, work, st);
  if (r != NEP_OK) return r;
  float* Z1 = work;
  float* Z2 = Z1 + (size_t)B * MH;
  float* Z3 = Z2 + (size_t)B * MH;
  float* dZ3 = Z3 + (size_t)B * MOUT;
  float* dA2 = dZ3 + (size_t)B * MOUT;
  float* dA1 = dA2 + (size_t)B * MH;
  float* part = dA1 + (size_t)B * MH;
  const int nblk = (B * MOUT + 255) / 256;
  bce_grad_kernel<<<nblk, 256, 0, st>>>(Z3, Y, idx, B, dZ3, part);
  // layer 3: dW3 = Z2^T dZ3, db3; dA2 = dZ3 W3^T masked by Z2 > 0
  dense_bwd_w_kernel<<<MH + 1, 128, 0, st>>>(Z2, MH, nullptr, dZ3, MOUT, B, grad + OFF_W3, grad + OFF_B3);
  dense_bwd_in_kernel<<<B, 128, 0, st>>>(dZ3, MOUT, params + OFF_W3, MH, Z2, dA2);
  // layer 2
  dense_bwd_w_kernel<<<MH + 1, 128, 0, st>>>(Z1, MH, nullptr, dA2, MH, B, grad + OFF_W2, grad + OFF_B2);
  dense_bwd_in_kernel<<<B, 128, 0, st>>>(dA2, MH, params + OFF_W2, MH, Z1, dA1);
  // layer 1 (input rows gathered through idx)
  dense_bwd_w_kernel<<<MIN + 1, 128, 0, st>>>(X, MIN, idx, dA1, MH, B, grad + OFF_W1, grad + OFF_B1);
  if (hipGetLastError() != hipSuccess) return NEP_ERR_HIP;
  if (loss) {
    // mean loss = (sum of the block partials, in block order) / (B * 4); synchronises
    float h[64];
    if (nblk > 64) return NEP_ERR_CAPACITY;
    if (hipMemcpyAsync(h, part, sizeof(float) * nblk, hipMemcpyDeviceToHost, st) != hipSuccess) return NEP_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return NEP_ERR_HIP;
    double sum = 0;
    for (int i = 0; i < nblk; ++i) sum += h[i];
    *loss = (float)(sum / (B * MOUT));
  }
  return NEP_OK;
}

extern "C" nep_status nep_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                                   float beta1, float beta2, float eps, hipStream_t st) {
  if (!params || !grad || !m || !v || step < 1) return NEP_ERR_ARG;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  adam_kernel<<<(NPARAM + 255) / 256, 256, 0, st>>>(params, grad, m, v, NPARAM, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? NEP_OK : NEP_ERR_HIP;
}

extern "C" nep_status nep_mlp_features(const double* profiles, int rows, int ncol, const int32_t* stat_rows,
                                       int nstat, float* mean, float* sd, float* X, hipStream_t st) {
  if (!profiles || !X || !mean || !sd || rows < 1 || ncol < 1) return NEP_ERR_ARG;
  const long long total = (long long)rows * ncol;
  const unsigned g = (unsigned)((total + 255) / 256);
  log_profile_kernel<<<g, 256, 0, st>>>(profiles, total, X);
  if (stat_rows && nstat > 0) column_stats_kernel<<<ncol, 256, 0, st>>>(X, ncol, stat_rows, nstat, mean, sd);
  standardize_kernel<<<g, 256, 0, st>>>(X, total, ncol, mean, sd);
  return hipGetLastError() == hipSuccess ? NEP_OK : NEP_ERR_HIP;
}
