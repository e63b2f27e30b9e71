// Training and inference kernels of the learned bucket classifier: forward
// probabilities, forward + backward (mean softmax cross-entropy gradient,
// reduced in a fixed order), and Adam on FP32 master parameters with BF16
// working copies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_internal.hpp"
#include "sfft_mlp.hpp"

namespace sfft {

constexpr int kTile = 128;  // rows per work-group in the gradient kernel

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void __launch_bounds__(kWG) mlp_forward_kernel(const uint16_t* __restrict__ w,
                                                          const float* __restrict__ x, int64_t n,
                                                          float* __restrict__ prob) {
  __shared__ float W[kMlpParams];
  mlp_load(w, W);
  for (int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x; r < n; r += (int64_t)gridDim.x * kWG) {
    float xi[kMlpIn];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) xi[i] = bf16_round(x[r * kMlpIn + i]);
    prob[r] = mlp_prob(W, xi);
  }
}

// Gradient of the mean softmax cross-entropy over `rows` rows.  Row q of the
// batch is row q of x when seed == 0, else a row drawn by a counter-based hash
// of (seed, step, q).  Work-group g takes the tiles of kTile rows g, g + G, ...
// in order: forward per row (one thread per row), then the parameter gradients
// as sums over the tile's rows in LDS, added to per-thread accumulators (each
// thread owns fixed parameters).  The group's sums go to row g of `part`
// (kMlpPartStride floats: the parameters, then the loss sum); mlp_reduce_kernel
// adds the rows in order, so the result does not depend on timing.
constexpr int kN1 = kMlpH * kMlpIn + kMlpH;    // W1, b1 (contiguous from kW1)
constexpr int kN2 = kMlpH * kMlpH + kMlpH;     // W2, b2 (from kW2)
constexpr int kN3 = kMlpOut * kMlpH + kMlpOut; // W3, b3 (from kW3)
constexpr int kE1 = (kN1 + kWG - 1) / kWG, kE2 = (kN2 + kWG - 1) / kWG,
              kE3 = (kN3 + kWG - 1) / kWG;

__global__ void __launch_bounds__(kWG) mlp_grad_kernel(const uint16_t* __restrict__ w,
                                                       const float* __restrict__ x,
                                                       const uint8_t* __restrict__ y, int64_t n,
                                                       int64_t rows, uint64_t seed, uint64_t step,
                                                       float* __restrict__ part) {
  __shared__ float W[kMlpParams];
  // rows padded by one word so that one row per lane spreads over the banks
  __shared__ float H1[kTile][kMlpH + 1];  // h1, later dL/da1
  __shared__ float H2[kTile][kMlpH + 1];  // h2, later dL/da2
  __shared__ float X[kTile][kMlpIn];
  __shared__ float DZ[kTile][kMlpOut];
  __shared__ float red[kWG];
  mlp_load(w, W);
  const int tid = threadIdx.x;
  const float inv_rows = 1.f / (float)rows;
  float a1[kE1], a2[kE2], a3[kE3];
#pragma unroll
  for (int e = 0; e < kE1; ++e) a1[e] = 0.f;
#pragma unroll
  for (int e = 0; e < kE2; ++e) a2[e] = 0.f;
#pragma unroll
  for (int e = 0; e < kE3; ++e) a3[e] = 0.f;
  float lsum = 0.f;
  const int64_t ntiles = (rows + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kTile;
    const int nt = (int)min<int64_t>(kTile, rows - base);
    if (tid < kTile) {
      if (tid < nt) {
        const int64_t q = base + tid;
        const int64_t r = seed ? (int64_t)(splitmix64(seed ^ (step << 32) ^ (uint64_t)q) %
                                           (uint64_t)n)
                               : q;
        float xi[kMlpIn];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) {
          xi[i] = bf16_round(x[r * kMlpIn + i]);
          X[tid][i] = xi[i];
        }
        for (int o = 0; o < kMlpH; ++o) {
          float a = W[kB1 + o];
#pragma unroll
          for (int i = 0; i < kMlpIn; ++i) a += W[kW1 + o * kMlpIn + i] * xi[i];
          H1[tid][o] = a > 0.f ? a : 0.f;
        }
        float z0 = W[kB3], z1 = W[kB3 + 1];
        for (int o = 0; o < kMlpH; ++o) {
          float a = W[kB2 + o];
          for (int i = 0; i < kMlpH; ++i) a += W[kW2 + o * kMlpH + i] * H1[tid][i];
          const float h = a > 0.f ? a : 0.f;
          H2[tid][o] = h;
          z0 += W[kW3 + o] * h;
          z1 += W[kW3 + kMlpH + o] * h;
        }
        // loss = logsumexp(z) - z[label], finite however far apart the logits are
        const float zm = fmaxf(z0, z1);
        const float e0 = expf(z0 - zm), e1 = expf(z1 - zm);
        const float den = e0 + e1;
        const int lab = y[r] ? 1 : 0;
        lsum += zm + logf(den) - (lab ? z1 : z0);
        DZ[tid][0] = (e0 / den - (lab == 0 ? 1.f : 0.f)) * inv_rows;
        DZ[tid][1] = (e1 / den - (lab == 1 ? 1.f : 0.f)) * inv_rows;
      } else {
        for (int i = 0; i < kMlpIn; ++i) X[tid][i] = 0.f;
        for (int o = 0; o < kMlpH; ++o) H1[tid][o] = H2[tid][o] = 0.f;
        DZ[tid][0] = DZ[tid][1] = 0.f;
      }
    }
    __syncthreads();
    // dW3 = DZ^T H2, db3 = sum DZ
#pragma unroll
    for (int e = 0; e < kE3; ++e) {
      const int q = tid + e * kWG;
      if (q < kN3) {
        float g = 0.f;
        if (q < kMlpOut * kMlpH) {
          const int c = q / kMlpH, o = q - c * kMlpH;
          for (int s = 0; s < kTile; ++s) g += DZ[s][c] * H2[s][o];
        } else {
          const int c = q - kMlpOut * kMlpH;
          for (int s = 0; s < kTile; ++s) g += DZ[s][c];
        }
        a3[e] += g;
      }
    }
    __syncthreads();
    // dL/da2 = (DZ W3) * [h2 > 0], in place of H2
    for (int q = tid; q < kTile * kMlpH; q += kWG) {
      const int s = q / kMlpH, o = q - s * kMlpH;
      const float d = DZ[s][0] * W[kW3 + o] + DZ[s][1] * W[kW3 + kMlpH + o];
      H2[s][o] = H2[s][o] > 0.f ? d : 0.f;
    }
    __syncthreads();
    // dW2 = dA2^T H1, db2 = sum dA2
#pragma unroll
    for (int e = 0; e < kE2; ++e) {
      const int q = tid + e * kWG;
      if (q < kN2) {
        float g = 0.f;
        if (q < kMlpH * kMlpH) {
          const int o = q / kMlpH, i = q - o * kMlpH;
          for (int s = 0; s < kTile; ++s) g += H2[s][o] * H1[s][i];
        } else {
          const int o = q - kMlpH * kMlpH;
          for (int s = 0; s < kTile; ++s) g += H2[s][o];
        }
        a2[e] += g;
      }
    }
    // dL/da1 = (dA2 W2) * [h1 > 0]; computed into registers, then written over H1
    constexpr int PER = kTile * kMlpH / kWG;
    float d1[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * kWG;
      const int s = q / kMlpH, i = q - s * kMlpH;
      float d = 0.f;
      for (int o = 0; o < kMlpH; ++o) d += H2[s][o] * W[kW2 + o * kMlpH + i];
      d1[e] = H1[s][i] > 0.f ? d : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * kWG;
      H1[q / kMlpH][q % kMlpH] = d1[e];
    }
    __syncthreads();
    // dW1 = dA1^T X, db1 = sum dA1
#pragma unroll
    for (int e = 0; e < kE1; ++e) {
      const int q = tid + e * kWG;
      if (q < kN1) {
        float g = 0.f;
        if (q < kMlpH * kMlpIn) {
          const int o = q / kMlpIn, i = q - o * kMlpIn;
          for (int s = 0; s < kTile; ++s) g += H1[s][o] * X[s][i];
        } else {
          const int o = q - kMlpH * kMlpIn;
          for (int s = 0; s < kTile; ++s) g += H1[s][o];
        }
        a1[e] += g;
      }
    }
    __syncthreads();  // the next tile overwrites X, H1, H2, DZ
  }
  red[tid] = lsum;
  __syncthreads();
  for (int off = kWG / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  float* pg = part + (size_t)blockIdx.x * kMlpPartStride;
  if (tid == 0) pg[kMlpParams] = red[0];
#pragma unroll
  for (int e = 0; e < kE1; ++e)
    if (tid + e * kWG < kN1) pg[kW1 + tid + e * kWG] = a1[e];
#pragma unroll
  for (int e = 0; e < kE2; ++e)
    if (tid + e * kWG < kN2) pg[kW2 + tid + e * kWG] = a2[e];
#pragma unroll
  for (int e = 0; e < kE3; ++e)
    if (tid + e * kWG < kN3) pg[kW3 + tid + e * kWG] = a3[e];
}

// grad[q] = sum over the groups' rows of part in group order; loss = mean row loss.
__global__ void mlp_reduce_kernel(const float* __restrict__ part, int groups, float inv_rows,
                                  float* __restrict__ grad, float* __restrict__ loss) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q <= kMlpParams;
       q += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int g = 0; g < groups; ++g) s += part[(size_t)g * kMlpPartStride + q];
    if (q < kMlpParams)
      grad[q] = s;
    else
      loss[0] = s * inv_rows;
  }
}

__global__ void mlp_fill_kernel(float* __restrict__ a, int n, float v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = v;
}

__global__ void mlp_init_master_kernel(const uint16_t* __restrict__ w, float* __restrict__ master,
                                       float* __restrict__ m, float* __restrict__ v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    master[i] = bf16_to_f32(w[i]);
    m[i] = 0.f;
    v[i] = 0.f;
  }
}

// Adam step t (1-based) on FP32 masters; BF16 working copy written to w.
__global__ void mlp_adam_kernel(float* __restrict__ master, float* __restrict__ m,
                                float* __restrict__ v, const float* __restrict__ g,
                                uint16_t* __restrict__ w, int n, float lr, float bc1, float bc2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    const float wi = master[i] - upd;
    master[i] = wi;
    w[i] = f32_to_bf16(wi);
  }
}

__global__ void mlp_accum_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                 float scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] += src[0] * scale;
}

// ------------------------------------------------------------ launchers -----
int launch_mlp_forward(const void* w, const float* x, int64_t n, float* prob, void* stream) {
  const int64_t blocks = (n + kWG - 1) / kWG;
  const int grid = (int)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(kWG), 0, (hipStream_t)stream,
                     (const uint16_t*)w, x, n, prob);
  return (int)hipGetLastError();
}

int launch_mlp_grad(const void* w, const float* x, const uint8_t* y, int64_t n, int64_t rows,
                    uint64_t seed, uint64_t step, float* part, float* grad, float* loss,
                    void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t ntiles = (rows + kTile - 1) / kTile;
  const int groups = (int)(ntiles < kMlpGradGroups ? ntiles : kMlpGradGroups);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(groups), dim3(kWG), 0, s, (const uint16_t*)w, x, y,
                     n, rows, seed, step, part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 256) / 256), dim3(256), 0, s,
                     (const float*)part, groups, 1.f / (float)rows, grad, loss);
  return (int)hipGetLastError();
}

int launch_mlp_init(const void* w, float* master, float* m, float* v, void* stream) {
  hipLaunchKernelGGL(mlp_init_master_kernel, dim3(20), dim3(256), 0, (hipStream_t)stream,
                     (const uint16_t*)w, master, m, v, kMlpParams);
  return (int)hipGetLastError();
}

int launch_mlp_adam(float* master, float* m, float* v, const float* g, void* w, float lr,
                    float bc1, float bc2, void* stream) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(20), dim3(256), 0, (hipStream_t)stream, master, m, v,
                     g, (uint16_t*)w, kMlpParams, lr, bc1, bc2);
  return (int)hipGetLastError();
}

int launch_mlp_accum(const float* src, float* dst, float scale, void* stream) {
  hipLaunchKernelGGL(mlp_accum_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, src, dst,
                     scale);
  return (int)hipGetLastError();
}

int launch_fill(float* a, int n, float v, void* stream) {
  hipLaunchKernelGGL(mlp_fill_kernel, dim3((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), dim3(256),
                     0, (hipStream_t)stream, a, n, v);
  return (int)hipGetLastError();
}

}  // namespace sfft
