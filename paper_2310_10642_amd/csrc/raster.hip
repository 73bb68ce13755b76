// Tile rasteriser: front-to-back alpha blending of Eq. (6) with p_i(t) folded
// into each primitive's opacity (Sec. 3.2), and its backward pass.
//
// One workgroup per 16x16 tile (4 waves, one pixel per lane). The tile's
// primitive list is staged through LDS in batches; every lane evaluates each
// staged primitive for its own pixel, so LDS reads are broadcasts.
//
// The forward pass keeps only the final transmittance and the number of list
// entries up to the last contributor per pixel. The backward pass walks the
// list back to front from there, recovering T_i = T_{i+1} / (1 - a_i), and
// works in two phases per batch of 16 primitives: (1) each lane (pixel)
// writes dL/dpower and a_i T_i for the 16 primitives into LDS; (2) the lanes
// regroup as 16 primitives x 16 pixel columns and accumulate the per-primitive
// sums over the tile's pixels from LDS. No cross-lane reduction is needed per
// fragment; one 16-lane reduction per batch combines the columns, and one
// atomic per value and (tile, primitive) adds the tile's share.
#include "g4d_common.h"

namespace g4d {
namespace {

constexpr int kFwdBatch = 256;
constexpr int kBwdBatch = 16;
constexpr int kGwStride = 256 + 16;  // padded LDS row per primitive (pixels)

// log2 of opacity * exp(power) at offset (dx, dy) from the mean.
// sa = (u, v, A, B), sb = (C, log2 opacity, ., .) with
// A = -log2(e)/2 conic00, B = -log2(e) conic01, C = -log2(e)/2 conic11.
__device__ __forceinline__ float frag_log2(float dx, float dy, float4 sa, float4 sb) {
  return fmaf(dx, fmaf(sa.z, dx, sa.w * dy), fmaf(sb.x * dy, dy, sb.y));
}

__device__ __forceinline__ void stage_record(const Record& r, float4& sa, float4& sb, float4& sc) {
  sa = make_float4(r.a.x, r.a.y, -0.5f * kLog2e * r.b.x, -kLog2e * r.b.y);
  sb = make_float4(-0.5f * kLog2e * r.b.z, __log2f(r.a.w), r.a.z, 0.f);
  sc = make_float4(r.c.x, r.c.y, r.c.z, 0.f);
}

__device__ __forceinline__ int find_view(const ViewDev* views, int n_views, int tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_raster_forward(int n_views, const ViewDev* __restrict__ views,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ ival,
                                                         const Record* __restrict__ recs, float bg0, float bg1,
                                                         float bg2, float* __restrict__ out_rgb,
                                                         float* __restrict__ out_depth, float* __restrict__ out_alpha,
                                                         float* __restrict__ pix_t, uint32_t* __restrict__ pix_last) {
  __shared__ float4 s_a[kFwdBatch], s_b[kFwdBatch], s_c[kFwdBatch];
  const int tile = blockIdx.x;
  const int vi = find_view(views, n_views, tile);
  const ViewDev& vw = views[vi];
  const int lt = tile - vw.tile_base;
  const int tx = lt % vw.tiles_x, ty = lt / vw.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < vw.width && py < vw.height;
  const float fx = px + 0.5f, fy = py + 0.5f;
  const uint2 rg = ranges[tile];
  const int count = (int)(rg.y - rg.x);

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  for (int b0 = 0; b0 < count; b0 += kFwdBatch) {
    if (__syncthreads_count(done) == 256) break;
    const int e = b0 + threadIdx.x;
    if (e < count) {
      const Record r = recs[ival[rg.x + e]];
      float4 sa, sb, sc;
      stage_record(r, sa, sb, sc);
      s_a[threadIdx.x] = sa;
      s_b[threadIdx.x] = sb;
      s_c[threadIdx.x] = sc;
    }
    __syncthreads();
    const int nb = min(kFwdBatch, count - b0);
    if (!done) {
      for (int j = 0; j < nb; ++j) {
        const float4 sa = s_a[j];
        const float4 sb = s_b[j];
        const float p2 = frag_log2(fx - sa.x, fy - sa.y, sa, sb);
        if (p2 < kLog2AlphaMin) continue;
        const float a = fminf(__builtin_amdgcn_exp2f(p2), kAlphaMax);
        const float Tn = fmaf(-a, T, T);
        if (Tn < kTStop) {
          done = true;
          break;
        }
        const float4 sc = s_c[j];
        const float w = a * T;
        C0 = fmaf(w, sc.x, C0);
        C1 = fmaf(w, sc.y, C1);
        C2 = fmaf(w, sc.z, C2);
        D = fmaf(w, sb.z, D);
        T = Tn;
        last = (uint32_t)(b0 + j + 1);
      }
    }
  }
  if (!inside) return;
  const long long hw = (long long)vw.width * vw.height;
  const long long pl = (long long)py * vw.width + px;
  const long long pix = vw.pix_base + pl;
  float* rgb = out_rgb + 3 * vw.pix_base + pl;
  rgb[0] = fmaf(T, bg0, C0);
  rgb[hw] = fmaf(T, bg1, C1);
  rgb[2 * hw] = fmaf(T, bg2, C2);
  if (out_depth) out_depth[pix] = D;
  if (out_alpha) out_alpha[pix] = 1.f - T;
  pix_t[pix] = T;
  pix_last[pix] = last;
}

__global__ void __launch_bounds__(256) k_raster_backward(
    int n_views, const ViewDev* __restrict__ views, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ival,
    const Record* __restrict__ recs, float bg0, float bg1, float bg2, const float* __restrict__ dl_rgb,
    const float* __restrict__ dl_depth, const float* __restrict__ dl_alpha, const float* __restrict__ pix_t,
    const uint32_t* __restrict__ pix_last, float* __restrict__ grad2d) {
  __shared__ float4 s_a[kBwdBatch], s_b[kBwdBatch], s_c[kBwdBatch];
  __shared__ uint32_t s_d[kBwdBatch];
  __shared__ float2 s_gw[kBwdBatch * kGwStride];
  __shared__ float4 s_pix[256];
  __shared__ uint32_t s_max;

  const int tile = blockIdx.x;
  const int vi = find_view(views, n_views, tile);
  const ViewDev& vw = views[vi];
  const int lt = tile - vw.tile_base;
  const int tx = lt % vw.tiles_x, ty = lt / vw.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < vw.width && py < vw.height;
  const float fx = px + 0.5f, fy = py + 0.5f;
  const uint2 rg = ranges[tile];
  const int count = (int)(rg.y - rg.x);

  if (threadIdx.x == 0) s_max = 0u;
  float T = 1.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f;
  uint32_t last = 0;
  if (inside) {
    const long long hw = (long long)vw.width * vw.height;
    const long long pl = (long long)py * vw.width + px;
    const long long pix = vw.pix_base + pl;
    const float* g = dl_rgb + 3 * vw.pix_base + pl;
    gC0 = g[0];
    gC1 = g[hw];
    gC2 = g[2 * hw];
    if (dl_depth) gD = dl_depth[pix];
    if (dl_alpha) gA = dl_alpha[pix];
    T = pix_t[pix];
    last = pix_last[pix];
  }
  s_pix[threadIdx.x] = make_float4(gC0, gC1, gC2, gD);
  __syncthreads();
  if (last) atomicMax(&s_max, last);
  // "behind" accumulators: colour, depth and alpha of everything after the
  // current primitive, normalised by the transmittance after it
  float B0 = bg0, B1 = bg1, B2 = bg2, Bd = 0.f, Ba = 0.f;
  __syncthreads();
  const int max_last = (int)s_max;

  const int j2 = threadIdx.x >> 4;  // phase 2: primitive within the batch
  const int c2 = threadIdx.x & 15;  // phase 2: pixel column
  for (int b0 = ((max_last + kBwdBatch - 1) / kBwdBatch - 1) * kBwdBatch; b0 >= 0; b0 -= kBwdBatch) {
    __syncthreads();
    if (threadIdx.x < kBwdBatch) {
      const int e = b0 + threadIdx.x;
      if (e < count) {
        const uint32_t d = ival[rg.x + e];
        float4 sa, sb, sc;
        stage_record(recs[d], sa, sb, sc);
        s_a[threadIdx.x] = sa;
        s_b[threadIdx.x] = sb;
        s_c[threadIdx.x] = sc;
        s_d[threadIdx.x] = d;
      }
    }
    __syncthreads();
    // ---- phase 1: this lane's pixel, back to front over the batch ----
#pragma unroll 4
    for (int j = kBwdBatch - 1; j >= 0; --j) {
      float g = 0.f, w = 0.f;
      if ((uint32_t)(b0 + j) < last) {
        const float4 sa = s_a[j];
        const float4 sb = s_b[j];
        const float p2 = frag_log2(fx - sa.x, fy - sa.y, sa, sb);
        if (p2 >= kLog2AlphaMin) {
          const float G = __builtin_amdgcn_exp2f(p2);
          const float a = fminf(G, kAlphaMax);
          const float4 sc = s_c[j];
          T = T / (1.f - a);
          w = a * T;
          const float dLda = T * (gC0 * (sc.x - B0) + gC1 * (sc.y - B1) + gC2 * (sc.z - B2) + gD * (sb.z - Bd) +
                                  gA * (1.f - Ba));
          B0 = fmaf(a, sc.x - B0, B0);
          B1 = fmaf(a, sc.y - B1, B1);
          B2 = fmaf(a, sc.z - B2, B2);
          Bd = fmaf(a, sb.z - Bd, Bd);
          Ba = fmaf(a, 1.f - Ba, Ba);
          g = (G < kAlphaMax) ? dLda * G : 0.f;  // dL/dpower
        }
      }
      s_gw[j * kGwStride + threadIdx.x] = make_float2(g, w);
    }
    __syncthreads();
    // ---- phase 2: primitive j2, pixel column c2, rows 0..15 ----
    const int e2 = b0 + j2;
    float Sg = 0.f, Sgy = 0.f, Sgyy = 0.f, Sr = 0.f, Sgc = 0.f, Sb = 0.f, Sd = 0.f;
    float dx = 0.f;
    if (e2 < count) {
      const float4 sa = s_a[j2];
      dx = (float)(tx * kTile + c2) + 0.5f - sa.x;
      const float dy0 = (float)(ty * kTile) + 0.5f - sa.y;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int p = k * 16 + c2;
        const float2 gw = s_gw[j2 * kGwStride + p];
        const float4 pd = s_pix[p];
        const float dy = dy0 + (float)k;
        Sg += gw.x;
        const float gdy = gw.x * dy;
        Sgy += gdy;
        Sgyy = fmaf(gdy, dy, Sgyy);
        Sr = fmaf(gw.y, pd.x, Sr);
        Sgc = fmaf(gw.y, pd.y, Sgc);
        Sb = fmaf(gw.y, pd.z, Sb);
        Sd = fmaf(gw.y, pd.w, Sd);
      }
    }
    float v[10] = {Sg, dx * Sg, Sgy, dx * dx * Sg, dx * Sgy, Sgyy, Sr, Sgc, Sb, Sd};
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
      for (int q = 0; q < 10; ++q) v[q] += __shfl_xor(v[q], off, 16);
    if (c2 == 0 && e2 < count) {
      bool nz = false;
#pragma unroll
      for (int q = 0; q < 10; ++q) nz |= (v[q] != 0.f);
      if (nz) {
        const uint32_t d = s_d[j2];
        const Record r = recs[d];
        const float k0 = r.b.x, k1 = r.b.y, k2 = r.b.z;
        // v: Sg, Sgx, Sgy, Sgxx, Sgxy, Sgyy, w*dL/dr, w*dL/dg, w*dL/db, w*dL/dD
        float* o = grad2d + (size_t)d * 12;
        unsafeAtomicAdd(o + 0, k0 * v[1] + k1 * v[2]);   // dL/du
        unsafeAtomicAdd(o + 1, k1 * v[1] + k2 * v[2]);   // dL/dv
        unsafeAtomicAdd(o + 2, -0.5f * v[3]);            // dL/dconic00
        unsafeAtomicAdd(o + 3, -v[4]);                   // dL/dconic01
        unsafeAtomicAdd(o + 4, -0.5f * v[5]);            // dL/dconic11
        unsafeAtomicAdd(o + 5, v[0] / r.a.w);            // dL/d(opacity p)
        unsafeAtomicAdd(o + 6, v[6]);
        unsafeAtomicAdd(o + 7, v[7]);
        unsafeAtomicAdd(o + 8, v[8]);
        unsafeAtomicAdd(o + 9, v[9]);                    // dL/dz
      }
    }
  }
}

}  // namespace

void launch_raster_forward(int total_tiles, int n_views, const ViewDev* views, const uint2* ranges,
                           const uint32_t* ival, const Record* rec_sorted, const float* bg, float* out_rgb,
                           float* out_depth, float* out_alpha, float* pix_t, uint32_t* pix_last, hipStream_t s) {
  if (total_tiles == 0) return;
  hipLaunchKernelGGL(k_raster_forward, dim3(total_tiles), dim3(256), 0, s, n_views, views, ranges, ival, rec_sorted,
                     bg[0], bg[1], bg[2], out_rgb, out_depth, out_alpha, pix_t, pix_last);
}

void launch_raster_backward(int total_tiles, int n_views, const ViewDev* views, const uint2* ranges,
                            const uint32_t* ival, const Record* rec_sorted, const float* bg, const float* dl_rgb,
                            const float* dl_depth, const float* dl_alpha, const float* pix_t,
                            const uint32_t* pix_last, float* grad2d, hipStream_t s) {
  if (total_tiles == 0) return;
  hipLaunchKernelGGL(k_raster_backward, dim3(total_tiles), dim3(256), 0, s, n_views, views, ranges, ival, rec_sorted,
                     bg[0], bg[1], bg[2], dl_rgb, dl_depth, dl_alpha, pix_t, pix_last, grad2d);
}

}  // namespace g4d
