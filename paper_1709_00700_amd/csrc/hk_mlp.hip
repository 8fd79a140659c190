// Learned cost model kernels: a 12 -> 64 -> 64 -> 1 ReLU network in FP32
// predicting ln(run time) of a (query, variant) pair, with its forward pass,
// mean-squared-error gradient and Adam update. These are tiny dense layers,
// so they run on the vector ALUs: one wavefront evaluates one sample with
// one lane per hidden unit; weights sit in LDS (W2 also transposed so that
// both passes read it without bank conflicts); lanes exchange activations
// with readlane broadcasts.
//
// Flat parameter layout (5,057 floats): W1 [64x12] | b1 [64] | W2 [64x64] |
// b2 [64] | W3 [64] | b3 [1].
#include <hip/hip_runtime.h>

#include "hawk_device.h"
#include "hawk_mlp.h"

#define NI MLP_IN
#define NH MLP_HIDDEN
#define OFF_W1 0
#define OFF_B1 (NH * NI)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH)

struct MlpShared {
  float w1[NH * NI];
  float w2[NH * NH];    // w2[j * NH + i] = W2[j][i]
  float w2t[NH * NH];   // w2t[i * NH + j] = W2[j][i]
  float mu[NI], isd[NI];
};

__device__ __forceinline__ void mlp_stage(MlpShared& S, const float* __restrict__ p, const float* __restrict__ mu,
                                          const float* __restrict__ sd) {
  for (int i = threadIdx.x; i < NH * NI; i += blockDim.x) S.w1[i] = p[OFF_W1 + i];
  for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) {
    const float w = p[OFF_W2 + i];
    S.w2[i] = w;
    S.w2t[(i % NH) * NH + i / NH] = w;
  }
  if (threadIdx.x < NI) {
    S.mu[threadIdx.x] = mu[threadIdx.x];
    S.isd[threadIdx.x] = 1.0f / sd[threadIdx.x];
  }
  __syncthreads();
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// forward pass of one sample by one wave; lane j = hidden unit j
struct MlpAct { float xn[NI]; float z1, h1, z2, h2, yhat; };

__device__ __forceinline__ void mlp_sample(const MlpShared& S, const float* __restrict__ p,
                                           const float* __restrict__ x, MlpAct& a) {
  const int j = __lane_id();
#pragma unroll
  for (int k = 0; k < NI; ++k) a.xn[k] = (x[k] - S.mu[k]) * S.isd[k];
  float z1 = p[OFF_B1 + j];
#pragma unroll
  for (int k = 0; k < NI; ++k) z1 = fmaf(S.w1[j * NI + k], a.xn[k], z1);
  a.z1 = z1;
  a.h1 = fmaxf(z1, 0.0f);
  float z2 = p[OFF_B2 + j];
#pragma unroll 16
  for (int i = 0; i < NH; ++i) z2 = fmaf(S.w2t[i * NH + j], __shfl(a.h1, i, WAVE), z2);
  a.z2 = z2;
  a.h2 = fmaxf(z2, 0.0f);
  a.yhat = wave_sum(p[OFF_W3 + j] * a.h2) + p[OFF_B3];
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ p, const float* __restrict__ mu,
                                                     const float* __restrict__ sd, const float* __restrict__ X,
                                                     int64_t m, float* __restrict__ out) {
  __shared__ MlpShared S;
  mlp_stage(S, p, mu, sd);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
  for (int64_t s = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; s < m; s += waves) {
    MlpAct a;
    mlp_sample(S, p, X + s * NI, a);
    if (__lane_id() == 0) out[s] = a.yhat;
  }
}

// Gradient of mean((yhat - y)^2) over m_total samples; wave w handles samples
// [w*per, (w+1)*per) of this launch and writes its partial gradient row.
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ p, const float* __restrict__ mu,
                                                  const float* __restrict__ sd, const float* __restrict__ X,
                                                  const float* __restrict__ y, const int32_t* __restrict__ idx,
                                                  int64_t m, int64_t per, float scale, float* __restrict__ partial,
                                                  float* __restrict__ partial_loss) {
  __shared__ MlpShared S;
  mlp_stage(S, p, mu, sd);
  const int j = __lane_id();
  const int64_t w = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE;
  float gw1[NI], gw2[NH];
#pragma unroll
  for (int k = 0; k < NI; ++k) gw1[k] = 0.f;
#pragma unroll
  for (int i = 0; i < NH; ++i) gw2[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
  const float w3 = p[OFF_W3 + j];
  const int64_t s0 = w * per, s1 = s0 + per < m ? s0 + per : m;
  for (int64_t t = s0; t < s1; ++t) {
    const int64_t s = idx ? idx[t] : t;
    MlpAct a;
    mlp_sample(S, p, X + s * NI, a);
    const float err = a.yhat - y[s];
    lsum += err * err;
    const float d3 = scale * err;          // dL/dyhat, scale = 2 / m_total
    gw3 = fmaf(d3, a.h2, gw3);
    gb3 += d3;
    const float d2 = a.z2 > 0.f ? d3 * w3 : 0.f;   // dL/dz2 of unit j
    gb2 += d2;
#pragma unroll
    for (int i = 0; i < NH; ++i) gw2[i] = fmaf(d2, __shfl(a.h1, i, WAVE), gw2[i]);
    float d1 = 0.f;                         // dL/dz1 of unit j: sum over k of W2[k][j] d2_k
#pragma unroll 16
    for (int k = 0; k < NH; ++k) d1 = fmaf(S.w2[k * NH + j], __shfl(d2, k, WAVE), d1);
    d1 = a.z1 > 0.f ? d1 : 0.f;
    gb1 += d1;
#pragma unroll
    for (int k = 0; k < NI; ++k) gw1[k] = fmaf(d1, a.xn[k], gw1[k]);
  }
  float* row = partial + w * MLP_NPARAMS;
#pragma unroll
  for (int k = 0; k < NI; ++k) row[OFF_W1 + j * NI + k] = gw1[k];
  row[OFF_B1 + j] = gb1;
#pragma unroll
  for (int i = 0; i < NH; ++i) row[OFF_W2 + j * NH + i] = gw2[i];
  row[OFF_B2 + j] = gb2;
  row[OFF_W3 + j] = gw3;
  if (j == 0) {
    row[OFF_B3] = gb3;
    partial_loss[w] = lsum;
  }
}

// fixed-order sum of the per-wave partial rows (deterministic gradient)
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ partial, int64_t rows,
                                                    float* __restrict__ grad, const float* __restrict__ partial_loss,
                                                    float* __restrict__ loss, float loss_scale) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < MLP_NPARAMS) {
    float acc = 0.f;
    for (int64_t r = 0; r < rows; ++r) acc += partial[r * MLP_NPARAMS + q];
    grad[q] = acc;
  }
  if (q == 0 && loss) {
    float l = 0.f;
    for (int64_t r = 0; r < rows; ++r) l += partial_loss[r];
    *loss = l * loss_scale;
  }
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                                              float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  // bias-corrected moments: c1 = 1 - b1^t, c2 = 1 - b2^t
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// argmin over each row of predictions (one wave per row): index of the
// smallest value, the first one on ties
__global__ void __launch_bounds__(256) k_argmin_rows(const float* __restrict__ v, int64_t rows, int64_t cols,
                                                     int32_t* __restrict__ out) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
  for (int64_t r = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; r < rows; r += waves) {
    float best = INFINITY;
    int32_t bi = 0x7fffffff;
    for (int64_t c = __lane_id(); c < cols; c += WAVE) {
      const float x = v[r * cols + c];
      if (x < best) {
        best = x;
        bi = static_cast<int32_t>(c);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ob = __shfl_xor(best, o, WAVE);
      const int32_t oi = __shfl_xor(bi, o, WAVE);
      if (ob < best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (__lane_id() == 0) out[r] = bi == 0x7fffffff ? 0 : bi;
  }
}

hipError_t hk_mlp_forward(hipStream_t st, const float* p, const float* mu, const float* sd, const float* X, int64_t m,
                          float* out) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(hk_grid_for(m, 4, 4096)), dim3(256), 0, st, p, mu, sd, X, m, out);
  return hipGetLastError();
}

int64_t hk_mlp_grad_rows(int64_t m) { return hk_grid_for(m, 16, 256) * 4; }

hipError_t hk_mlp_grad(hipStream_t st, const float* p, const float* mu, const float* sd, const float* X, const float* y,
                       const int32_t* idx, int64_t m, float* partial, float* partial_loss, int64_t partial_cap_rows,
                       float* grad, float* loss) {
  const int64_t rows = hk_mlp_grad_rows(m);   // waves, 4 per block
  if (rows > partial_cap_rows) return hipErrorInvalidValue;  // scratch too small for this batch
  const int64_t per = (m + rows - 1) / rows;
  const float scale = m > 0 ? 2.0f / static_cast<float>(m) : 0.f;
  hipLaunchKernelGGL(k_mlp_grad, dim3(rows / 4), dim3(256), 0, st, p, mu, sd, X, y, idx, m, per, scale, partial,
                     partial_loss);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAMS + 255) / 256), dim3(256), 0, st, partial, rows, grad,
                     partial_loss, loss, m > 0 ? 1.0f / static_cast<float>(m) : 0.f);
  return hipGetLastError();
}

hipError_t hk_adam(hipStream_t st, float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1,
                   float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m1, m2, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t hk_argmin_rows(hipStream_t st, const float* v, int64_t rows, int64_t cols, int32_t* out) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_argmin_rows, dim3(hk_grid_for(rows, 4, 4096)), dim3(256), 0, st, v, rows, cols, out);
  return hipGetLastError();
}
