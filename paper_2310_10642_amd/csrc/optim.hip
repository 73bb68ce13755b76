// The training-step tail around the render: the Adam update of every
// parameter group in one launch (Sec. 4.2 trains with the optimiser settings
// of 3D Gaussian Splatting, i.e. Adam), and the 4D split sampling of
// Sec. 3.3 / 4.4 (new positions drawn from the primitive's full 4D Gaussian).
#include "shade.h"

namespace g4d {
namespace {

using namespace shade;

// Grid-stride over the concatenated groups; a group's slice of the moment
// buffers starts at the previous group's end.
__global__ void __launch_bounds__(256) k_adam(AdamGroups a, uint64_t total, float b1, float b2, float eps,
                                              float inv_bc1, float inv_bc2, float* __restrict__ m,
                                              float* __restrict__ v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    int gi = 0;
#pragma unroll
    for (int k = 0; k < kAdamGroups - 1; ++k) gi += (i >= a.end[k]) ? 1 : 0;
    const uint64_t j = i - (gi ? a.end[gi - 1] : 0);
    const float g = a.grad[gi][j];
    const float mm = fmaf(b1, m[i], (1.f - b1) * g);
    const float vv = fmaf(b2, v[i], (1.f - b2) * g * g);
    m[i] = mm;
    v[i] = vv;
    a.param[gi][j] -= a.lr[gi] * (mm * inv_bc1) / (sqrtf(vv * inv_bc2) + eps);
  }
}

__global__ void __launch_bounds__(256) k_split_sample(RenderParams p, uint64_t count, const int32_t* __restrict__ idx,
                                                      const float4* __restrict__ z, float4* __restrict__ out) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int i = idx[k];
  if (i < 0 || i >= p.n) {  // not a primitive: no read, NaN row
    const float nan = __int_as_float(0x7FC00000);
    out[k] = make_float4(nan, nan, nan, nan);
    return;
  }
  Shape4 sh;
  build_shape<float>(p.q_left[i], p.q_right[i], p.log_scales4[i], sh);
  const float4 mu = p.means4[i], zz = z[k];
  float o[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) o[r] = fmaf(sh.M[r][0], zz.x, fmaf(sh.M[r][1], zz.y, fmaf(sh.M[r][2], zz.z, sh.M[r][3] * zz.w)));
  out[k] = make_float4(mu.x + o[0], mu.y + o[1], mu.z + o[2], mu.w + o[3]);
}

}  // namespace

void launch_adam(const AdamGroups& a, float b1, float b2, float eps, float bc1, float bc2, float* m, float* v,
                 hipStream_t s) {
  const uint64_t total = a.end[kAdamGroups - 1];
  if (total == 0) return;
  uint64_t g = (total + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)g), dim3(256), 0, s, a, total, b1, b2, eps, 1.f / bc1, 1.f / bc2, m, v);
}

void launch_split_sample(const RenderParams& p, uint64_t count, const int32_t* idx, const float* z, float* out,
                         hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_split_sample, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, idx,
                     reinterpret_cast<const float4*>(z), reinterpret_cast<float4*>(out));
}

}  // namespace g4d
