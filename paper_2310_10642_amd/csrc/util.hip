// Small device-side helpers that keep the render and backward enqueue free of
// host-side memory operations: view upload through kernel arguments, fills
// (also of device-counted extents), the instance-arena capacity check and a
// device-counted copy.
#include "g4d_common.h"

namespace g4d {
namespace {

constexpr int kViewChunk = 8;  // views per upload launch (960 bytes of arguments)

struct ViewChunk {
  ViewDev v[kViewChunk];
};

__global__ void k_set_views(ViewChunk chunk, int count, ViewDev* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < count) out[i] = chunk.v[i];
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Zeroes per_item float4 for each of min(*n_dev, max_items) items.
__global__ void k_zero_counted(float4* __restrict__ p, const uint32_t* __restrict__ n_dev, uint32_t per_item,
                               uint64_t max_items) {
  const uint64_t items = min((uint64_t)*n_dev, max_items);
  const uint64_t n = items * per_item;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = z;
}

// An instance total over the arena capacity raises the sticky overflow flag
// and empties the batch, so every later stage sees zero instances. With
// a_tot, a sync-free round's active records and (checked) instances are then
// added to the render's totals.
__global__ void k_cap_check(const unsigned long long* __restrict__ inst64, uint32_t* __restrict__ n_inst,
                            uint32_t* __restrict__ overflow, unsigned long long cap, const uint32_t* __restrict__ a,
                            uint32_t* __restrict__ a_tot, unsigned long long* __restrict__ i_tot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t ni = *n_inst;
  if (*inst64 > cap) {
    *overflow = 1u;
    *n_inst = ni = 0u;
  }
  if (a_tot) {
    *a_tot += *a;
    *i_tot += ni;
  }
}

__global__ void k_copy_pairs(const uint32_t* __restrict__ ka, const uint32_t* __restrict__ va,
                             uint32_t* __restrict__ kb, uint32_t* __restrict__ vb, const uint32_t* __restrict__ n_dev,
                             uint32_t n_max) {
  const uint32_t n = n_dev ? min(*n_dev, n_max) : n_max;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    kb[i] = ka[i];
    vb[i] = va[i];
  }
}

unsigned stride_grid(uint64_t n, unsigned cap) {
  const uint64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

void launch_set_views(const ViewDev* host, int n, ViewDev* dev, hipStream_t s) {
  for (int v0 = 0; v0 < n; v0 += kViewChunk) {
    ViewChunk c{};
    const int cnt = (n - v0) < kViewChunk ? (n - v0) : kViewChunk;
    for (int i = 0; i < cnt; ++i) c.v[i] = host[v0 + i];
    hipLaunchKernelGGL(k_set_views, dim3(1), dim3(64), 0, s, c, cnt, dev + v0);
  }
}

void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(stride_grid(n, 2048)), dim3(256), 0, s, p, n, value);
}

void launch_zero_counted(float* p, const uint32_t* n_dev, uint32_t floats_per_item, uint64_t max_items,
                         hipStream_t s) {
  if (max_items == 0) return;
  const uint32_t per = floats_per_item / 4;
  // two workgroups per CU stream the zeros fastest (14.6 -> 13.0 us for the
  // bench's 82 MB against 2048 workgroups)
  hipLaunchKernelGGL(k_zero_counted, dim3(stride_grid(max_items * per, 512)), dim3(256), 0, s,
                     reinterpret_cast<float4*>(p), n_dev, per, max_items);
}

void launch_cap_check(const uint32_t* inst64, uint32_t* n_inst, uint32_t* overflow, uint64_t cap, hipStream_t s,
                      const uint32_t* a, uint32_t* a_tot, uint32_t* i_tot64) {
  hipLaunchKernelGGL(k_cap_check, dim3(1), dim3(64), 0, s, reinterpret_cast<const unsigned long long*>(inst64),
                     n_inst, overflow, (unsigned long long)cap, a, a_tot,
                     reinterpret_cast<unsigned long long*>(i_tot64));
}

void launch_copy_pairs(const uint32_t* ka, const uint32_t* va, uint32_t* kb, uint32_t* vb, const uint32_t* n_dev,
                       uint32_t n_max, hipStream_t s) {
  if (n_max == 0) return;
  hipLaunchKernelGGL(k_copy_pairs, dim3(stride_grid(n_max, 4096)), dim3(256), 0, s, ka, va, kb, vb, n_dev, n_max);
}

}  // namespace g4d
