// Image loss and dL/dI for the training step (L1 or L2 against a target).
#include "g4d_common.h"

namespace g4d {
namespace {

__global__ void __launch_bounds__(256) k_image_loss(int kind, uint64_t n, const float* __restrict__ img,
                                                     const float* __restrict__ tgt, float scale,
                                                     float* __restrict__ loss, float* __restrict__ grad) {
  __shared__ float s_part[4];
  float acc = 0.f;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const float d = img[i] - tgt[i];
    if (kind == 1) {
      acc += fabsf(d);
      grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    } else {
      acc = fmaf(d, d, acc);
      grad[i] = 2.f * scale * d;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, scale * (s_part[0] + s_part[1] + s_part[2] + s_part[3]));
}

}  // namespace

void launch_image_loss(int kind, uint64_t n, const float* img, const float* tgt, float scale, float* loss,
                       float* grad, hipStream_t s) {
  if (n == 0) return;
  uint64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_image_loss, dim3((unsigned)g), dim3(256), 0, s, kind, n, img, tgt, scale, loss, grad);
}

}  // namespace g4d
