// mlp.hip - training of the warm-start MLP (8 -> 32 -> 32 -> 1, tanh, tanh, logistic).
//
// One workgroup of 256 threads runs the whole training: each step draws a minibatch
// with a counter-based generator (splitmix64 of seed, step and slot), runs forward and
// backward per sample (one thread per sample), reduces the parameter gradients over
// the batch from LDS and applies an Adam update. With grad_out set it computes the
// loss and gradient of one batch (the given rows, in order) and changes nothing.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tn {

constexpr int kMF = 8, kMH1 = 32, kMH2 = 32;
constexpr int kMP = kMF * kMH1 + kMH1 + kMH1 * kMH2 + kMH2 + kMH2 + 1;
static_assert(kMP == kMlpParams, "parameter count");

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ __launch_bounds__(256) void mlp_train_kernel(float *w, float *adam_m, float *adam_v, const float *X,
                                                        const float *Y, long long nrows, int steps, int batch,
                                                        float lr, unsigned long long seed, long long t0,
                                                        float *loss_out, float *grad_out) {
  __shared__ float sw[kMP], sm[kMP], sv[kMP], gacc[kMP];
  __shared__ float Xb[kMlpBatch * kMF], H1[kMlpBatch * kMH1], H2[kMlpBatch * kMH2];
  __shared__ float G1[kMlpBatch * kMH1], G2[kMlpBatch * kMH2], g3[kMlpBatch];
  __shared__ float red[4];
  const int tid = threadIdx.x;
  for (int e = tid; e < kMP; e += 256) { sw[e] = w[e]; sm[e] = adam_m[e]; sv[e] = adam_v[e]; }
  __syncthreads();
  const float *W1 = sw, *b1 = W1 + kMF * kMH1, *W2 = b1 + kMH1, *b2 = W2 + kMH1 * kMH2, *W3 = b2 + kMH2, *b3 = W3 + kMH2;
  float last_loss = 0.0f;
  for (int step = 0; step < steps; ++step) {
    float lpart = 0.0f;
    if (tid < batch) {
      long long idx = tid;
      if (!grad_out) idx = (long long)(splitmix64(seed ^ splitmix64((unsigned long long)(t0 + step) * 1024ull + tid)) >> 1) % nrows;
      float x[kMF], h1[kMH1], h2[kMH2];
#pragma unroll
      for (int a = 0; a < kMF; ++a) { x[a] = X[idx * kMF + a]; Xb[tid * kMF + a] = x[a]; }
#pragma unroll
      for (int j = 0; j < kMH1; ++j) {
        float z = b1[j];
#pragma unroll
        for (int a = 0; a < kMF; ++a) z += x[a] * W1[a * kMH1 + j];
        h1[j] = tanhf(z);
        H1[tid * kMH1 + j] = h1[j];
      }
#pragma unroll
      for (int j = 0; j < kMH2; ++j) {
        float z = b2[j];
#pragma unroll
        for (int a = 0; a < kMH1; ++a) z += h1[a] * W2[a * kMH2 + j];
        h2[j] = tanhf(z);
        H2[tid * kMH2 + j] = h2[j];
      }
      float z3 = b3[0];
#pragma unroll
      for (int a = 0; a < kMH2; ++a) z3 += h2[a] * W3[a];
      const float out = 1.0f / (1.0f + expf(-z3));
      const float r = out - Y[idx];
      lpart = r * r;
      const float gz3 = 2.0f * r / float(batch) * out * (1.0f - out);
      g3[tid] = gz3;
      float gz2[kMH2];
#pragma unroll
      for (int j = 0; j < kMH2; ++j) {
        gz2[j] = gz3 * W3[j] * (1.0f - h2[j] * h2[j]);
        G2[tid * kMH2 + j] = gz2[j];
      }
#pragma unroll
      for (int a = 0; a < kMH1; ++a) {
        float gh = 0.0f;
#pragma unroll
        for (int j = 0; j < kMH2; ++j) gh += gz2[j] * W2[a * kMH2 + j];
        G1[tid * kMH1 + a] = gh * (1.0f - h1[a] * h1[a]);
      }
    }
    // loss (block sum)
    for (int o = 32; o >= 1; o >>= 1) lpart += __shfl_xor(lpart, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = lpart;
    __syncthreads();
    last_loss = (red[0] + red[1] + red[2] + red[3]) / float(batch);
    // parameter gradients: sums over the batch
    for (int q = tid; q < kMP; q += 256) {
      float g = 0.0f;
      if (q < kMF * kMH1) {
        const int a = q / kMH1, j = q % kMH1;
        for (int t = 0; t < batch; ++t) g += Xb[t * kMF + a] * G1[t * kMH1 + j];
      } else if (q < kMF * kMH1 + kMH1) {
        const int j = q - kMF * kMH1;
        for (int t = 0; t < batch; ++t) g += G1[t * kMH1 + j];
      } else if (q < kMF * kMH1 + kMH1 + kMH1 * kMH2) {
        const int r = q - kMF * kMH1 - kMH1, a = r / kMH2, j = r % kMH2;
        for (int t = 0; t < batch; ++t) g += H1[t * kMH1 + a] * G2[t * kMH2 + j];
      } else if (q < kMF * kMH1 + kMH1 + kMH1 * kMH2 + kMH2) {
        const int j = q - kMF * kMH1 - kMH1 - kMH1 * kMH2;
        for (int t = 0; t < batch; ++t) g += G2[t * kMH2 + j];
      } else if (q < kMP - 1) {
        const int j = q - (kMP - 1 - kMH2);
        for (int t = 0; t < batch; ++t) g += H2[t * kMH2 + j] * g3[t];
      } else {
        for (int t = 0; t < batch; ++t) g += g3[t];
      }
      gacc[q] = g;
    }
    __syncthreads();
    if (grad_out) break;
    // Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction
    const float tt = float(t0 + step + 1);
    const float c1 = 1.0f - powf(0.9f, tt), c2 = 1.0f - powf(0.999f, tt);
    for (int q = tid; q < kMP; q += 256) {
      const float g = gacc[q];
      sm[q] = 0.9f * sm[q] + 0.1f * g;
      sv[q] = 0.999f * sv[q] + 0.001f * g * g;
      sw[q] -= lr * (sm[q] / c1) / (sqrtf(sv[q] / c2) + 1e-8f);
    }
    __syncthreads();
  }
  if (grad_out) {
    for (int q = tid; q < kMP; q += 256) grad_out[q] = gacc[q];
  } else {
    for (int q = tid; q < kMP; q += 256) { w[q] = sw[q]; adam_m[q] = sm[q]; adam_v[q] = sv[q]; }
  }
  if (tid == 0) loss_out[0] = last_loss;
}

hipError_t launch_mlp_train(float *w, float *m, float *v, const float *X, const float *Y, long long nrows, int steps,
                            int batch, float lr, unsigned long long seed, long long t0, float *loss_out,
                            float *grad_out, hipStream_t stream) {
  hipLaunchKernelGGL(mlp_train_kernel, dim3(1), dim3(256), 0, stream, w, m, v, X, Y, nrows, steps, batch, lr, seed,
                     t0, loss_out, grad_out);
  return hipGetLastError();
}

}  // namespace tn
