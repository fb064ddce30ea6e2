// mlp.hip -- the penalty controller network (a project addition: the paper
// fixes beta by hand-set rules, Sec.3.1 and Sec.3.2) and its training kernels.
//
// Network: f (8) -> tanh(W1 f + b1) (64) -> tanh(W2 h1 + b2) (64) -> o = W3 h2 + b3,
// output y = ymax tanh(o), read as the natural log of the multiplier for beta.
// Parameters, FP32: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
// Loss: 1/(2B) sum_b (y_b - t_b)^2.
//
// One 64-wide wavefront per workgroup; lane i owns hidden unit i in both layers
// and keeps the gradient rows of its unit in registers.  Each workgroup walks a
// contiguous slice of the batch; the per-workgroup gradients are summed in a
// fixed order by a second kernel, so results are deterministic.
#include "rac_internal.h"

namespace rac {
namespace {

constexpr int IN = RAC_MLP_IN, HD = RAC_MLP_HIDDEN, NP = RAC_MLP_NPARAM;
constexpr int OFF_B1 = HD * IN, OFF_W2 = OFF_B1 + HD, OFF_B2 = OFF_W2 + HD * HD,
              OFF_W3 = OFF_B2 + HD, OFF_B3 = OFF_W3 + HD;

__device__ __forceinline__ float wsum(float v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(64) k_mlp_forward(const float* __restrict__ w,
                                                    const float* __restrict__ feats, int64_t batch,
                                                    float ymax, float* __restrict__ y) {
  __shared__ float f[IN];
  __shared__ float h1[HD];
  const int i = threadIdx.x;
  for (int64_t bi = blockIdx.x; bi < batch; bi += gridDim.x) {
    if (i < IN) f[i] = feats[bi * IN + i];
    __syncthreads();
    float s = w[OFF_B1 + i];
    for (int k = 0; k < IN; ++k) s += w[i * IN + k] * f[k];
    h1[i] = tanhf(s);
    __syncthreads();
    s = w[OFF_B2 + i];
    for (int k = 0; k < HD; ++k) s += w[OFF_W2 + i * HD + k] * h1[k];
    const float h2 = tanhf(s);
    const float o = wsum(w[OFF_W3 + i] * h2) + w[OFF_B3];
    if (i == 0) y[bi] = ymax * tanhf(o);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64) k_mlp_grad_part(const float* __restrict__ w,
                                                      const float* __restrict__ feats,
                                                      const float* __restrict__ target, int64_t batch,
                                                      float ymax, float* __restrict__ part,
                                                      float* __restrict__ loss_part) {
  __shared__ float W2s[HD * HD];
  __shared__ float f[IN];
  __shared__ float h1[HD];
  __shared__ float d2s[HD];
  const int i = threadIdx.x;
  for (int e = i; e < HD * HD; e += 64) W2s[e] = w[OFF_W2 + e];
  float W1r[IN];
#pragma unroll
  for (int k = 0; k < IN; ++k) W1r[k] = w[i * IN + k];
  const float b1 = w[OFF_B1 + i], b2 = w[OFF_B2 + i], W3i = w[OFF_W3 + i], b3 = w[OFF_B3];
  float gW1[IN], gW2[HD];
#pragma unroll
  for (int k = 0; k < IN; ++k) gW1[k] = 0.f;
#pragma unroll
  for (int k = 0; k < HD; ++k) gW2[k] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f, gb3 = 0.f, loss = 0.f;
  const int64_t lo = (int64_t)blockIdx.x * batch / gridDim.x;
  const int64_t hi = (int64_t)(blockIdx.x + 1) * batch / gridDim.x;
  const float invB = 1.0f / (float)batch;
  __syncthreads();
  for (int64_t bi = lo; bi < hi; ++bi) {
    if (i < IN) f[i] = feats[bi * IN + i];
    __syncthreads();
    float s = b1;
#pragma unroll
    for (int k = 0; k < IN; ++k) s += W1r[k] * f[k];
    const float a1 = tanhf(s);
    h1[i] = a1;
    __syncthreads();
    s = b2;
#pragma unroll 8
    for (int k = 0; k < HD; ++k) s += W2s[i * HD + k] * h1[k];
    const float a2 = tanhf(s);
    const float o = wsum(W3i * a2) + b3;
    const float th = tanhf(o);
    const float e = ymax * th - target[bi];
    loss += 0.5f * e * e;
    const float dout = e * ymax * (1.f - th * th) * invB;
    gb3 += dout;
    gW3 += dout * a2;
    const float d2 = dout * W3i * (1.f - a2 * a2);
    d2s[i] = d2;
    gb2 += d2;
#pragma unroll
    for (int k = 0; k < HD; ++k) gW2[k] += d2 * h1[k];
    __syncthreads();
    float t = 0.f;
#pragma unroll 8
    for (int j = 0; j < HD; ++j) t += W2s[j * HD + i] * d2s[j];
    const float d1 = t * (1.f - a1 * a1);
    gb1 += d1;
#pragma unroll
    for (int k = 0; k < IN; ++k) gW1[k] += d1 * f[k];
    __syncthreads();
  }
  float* P = part + (int64_t)blockIdx.x * NP;
#pragma unroll
  for (int k = 0; k < IN; ++k) P[i * IN + k] = gW1[k];
  P[OFF_B1 + i] = gb1;
#pragma unroll
  for (int k = 0; k < HD; ++k) P[OFF_W2 + i * HD + k] = gW2[k];
  P[OFF_B2 + i] = gb2;
  P[OFF_W3 + i] = gW3;
  if (i == 0) {
    P[OFF_B3] = gb3;
    loss_part[blockIdx.x] = loss;
  }
}

__global__ void __launch_bounds__(256) k_mlp_grad_sum(const float* __restrict__ part, int nparts,
                                                      float* __restrict__ grad,
                                                      float* __restrict__ loss_part,
                                                      int64_t batch) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < NP) {
    float s = 0.f;
    for (int q = 0; q < nparts; ++q) s += part[(int64_t)q * NP + e];
    grad[e] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float l = 0.f;
    for (int q = 0; q < nparts; ++q) l += loss_part[q];
    loss_part[nparts] = l / (float)batch;
  }
}

__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  float c1, float c2, float lr, float b1, float b2,
                                                  float eps) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= NP) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  w[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

hipError_t launch_mlp_forward(const float* w, const float* feats, int64_t batch, float ymax, float* y,
                              hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  int64_t blocks = batch < 8192 ? batch : 8192;
  k_mlp_forward<<<(unsigned)blocks, 64, 0, st>>>(w, feats, batch, ymax, y);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* w, const float* feats, const float* target,
                                int64_t batch, float ymax, float* grad, float* partial_grad,
                                float* loss_part, int nparts, hipStream_t st) {
  k_mlp_grad_part<<<(unsigned)nparts, 64, 0, st>>>(w, feats, target, batch, ymax, partial_grad,
                                                   loss_part);
  k_mlp_grad_sum<<<(unsigned)((NP + 255) / 256), 256, 0, st>>>(partial_grad, nparts, grad, loss_part,
                                                               batch);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int64_t t, float lr, float b1,
                           float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  k_mlp_adam<<<(unsigned)((NP + 255) / 256), 256, 0, st>>>(w, g, m, v, c1, c2, lr, b1, b2, eps);
  return hipGetLastError();
}

}  // namespace rac
