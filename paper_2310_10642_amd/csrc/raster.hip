// Tile rasteriser: front-to-back alpha blending of Eq. (6) with p_i(t) folded
// into each primitive's opacity (Sec. 3.2), and its backward pass.
//
// One workgroup per 16x16 tile; each of its 4 waves owns an 8x8 quadrant, one
// pixel per lane. The tile's primitive list is staged through LDS in batches.
// While staging, each entry's alpha-floor ellipse (the pixels where
// opacity * exp(power) can reach 1/255) is bounded by a box and tested against
// the four quadrants; every wave then walks only the entries that can touch
// its quadrant, 16 at a time under a wave-uniform bit mask with the entry
// index a constant in each unrolled step (LDS reads at immediate offsets).
// A skipped entry would have failed the 1/255 test at every pixel of the
// quadrant, so the blend is unchanged. The per-fragment body is branch-free:
// skipped and post-stop fragments get alpha 0.
//
// The forward pass keeps only the final transmittance and the number of list
// entries up to the last contributor per pixel. The backward pass walks the
// list back to front from there, recovering T_i = T_{i+1} / (1 - a_i), and
// works in two phases per batch of 12 primitives: (1) each lane (pixel)
// writes dL/dpower and a_i T_i for the batch into LDS; (2) waves 1-3 regroup
// as 12 primitives x 16 pixel columns and accumulate the per-primitive sums
// over the tile's pixels (only over quadrants where the primitive blended),
// while wave 0 stages the next batch.
// A 16-lane DPP reduce-scatter per batch combines the columns, leaving each
// of ten lanes of a primitive's row with one value of its gradient line, and
// those lanes add the tile's share with one FP64 atomic instruction into one
// 128-byte line.
#include <algorithm>
#include <type_traits>

#include "shade.h"

namespace g4d {
namespace {

using shade::sc_fma;

// List entries per backward batch. 12 rather than 16: the per-(primitive,
// pixel) buffers then take 26 KB, the workgroup 31.6 KB of LDS, and with at
// most 96 VGPRs (the launch bound) five workgroups share a CU instead of four;
// the backward is bound by issue stalls more than by its instruction count,
// so the fifth wave per SIMD outweighs the third more barriers per entry. The
// batch's 12 primitives also leave wave 0 free for the staging in phase 2.
constexpr int kBwdBatch = 12;
static_assert(kBwdBatch == 12, "phase 2 maps the batch's primitives onto waves 1-3, four each");
// Backward LDS slots of one primitive's per-pixel values: pixel (row, col) of
// the tile sits at 16 row + (col ^ 8 [(row >> 1) & 1]); the x-halves of rows
// 2-3 of every four are swapped so that a wave's 8x8 quadrant (4 rows per
// half-wave) hits 32 distinct banks when writing, and 16 columns x 2
// primitives (stride 272 = 16 mod 32) do when reading.
constexpr int kGwStride = 256 + 16;
__device__ __forceinline__ int gw_slot(int row, int col) { return 16 * row + (col ^ (((row >> 1) & 1) << 3)); }

// log2 of opacity * exp(power) at offset (dx, dy) from the mean.
// sa = (u, v, A, B), sb = (C, log2 opacity, ., .) with
// A = -log2(e)/2 conic00, B = -log2(e) conic01, C = -log2(e)/2 conic11.
__device__ __forceinline__ float frag_log2(float dx, float dy, float4 sa, float4 sb) {
  return fmaf(dx, fmaf(sa.z, dx, sa.w * dy), fmaf(sb.x * dy, dy, sb.y));
}

// A record whose colour is NaN (its primitive has a non-finite 4DSH
// coefficient) is staged fully transparent: log2 opacity far below the 1/255
// floor at every pixel (finite, so its reciprocal stays finite), colour 0.
constexpr float kHiddenLog2 = -100.f;

__device__ __forceinline__ float staged_log2_opacity(const Record& r) {
  return isnan(r.c.x) ? kHiddenLog2 : __log2f(r.a.w);
}

__device__ __forceinline__ void stage_record(const Record& r, float4& sa, float4& sb, float4& sc) {
  const bool hide = isnan(r.c.x);
  sa = make_float4(r.a.x, r.a.y, -0.5f * kLog2e * r.b.x, -kLog2e * r.b.y);
  sb = make_float4(-0.5f * kLog2e * r.b.z, staged_log2_opacity(r), r.a.z, 0.f);
  sc = hide ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(r.c.x, r.c.y, r.c.z, 0.f);
}

// Whether the record's alpha-floor ellipse (where opacity * exp(power) reaches
// 1/255) meets the 8x8 quadrant q of the tile, whose pixel centres span
// x0 + 8 (q & 1) + [0.5, 7.5], y0 + 8 (q >> 1) + [0.5, 7.5]. In the staged
// form a fragment counts when log2 opacity - Q(dx, dy) >= log2(1/255), with
// Q = A dx^2 + 2 B dx dy + C dy^2 (A = -sa.z, 2B = -sa.w, C = -sb.x), a
// convex quadratic: its minimum over the quadrant is zero when the quadrant
// holds the centre, else it lies on an edge, where Q is a 1D quadratic
// minimised at a clamped point. The bound is loosened (0.1 % + 0.01) so
// rounding never drops a blended pixel.
__device__ __forceinline__ bool quadrant_hit(const float4& sa, const float4& sb, float tile_x0, float tile_y0, int q) {
  const float lim = fmaf(sb.y - kLog2AlphaMin, 1.001f, 0.01f);
  if (!(lim > 0.f)) return false;
  const float A = -sa.z, B = -0.5f * sa.w, C = -sb.x;
  const float ex0 = tile_x0 + 8.f * (q & 1) + 0.5f - sa.x, ex1 = ex0 + 7.f;
  const float ey0 = tile_y0 + 8.f * (q >> 1) + 0.5f - sa.y, ey1 = ey0 + 7.f;
  if (ex0 <= 0.f && ex1 >= 0.f && ey0 <= 0.f && ey1 >= 0.f) return true;
  const auto Q = [&](float dx, float dy) { return fmaf(dx, fmaf(A, dx, 2.f * B * dy), C * dy * dy); };
  const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
  const float ya = __builtin_amdgcn_fmed3f(-B * ex0 * iC, ey0, ey1);
  const float yb = __builtin_amdgcn_fmed3f(-B * ex1 * iC, ey0, ey1);
  const float xa = __builtin_amdgcn_fmed3f(-B * ey0 * iA, ex0, ex1);
  const float xb = __builtin_amdgcn_fmed3f(-B * ey1 * iA, ex0, ex1);
  return fminf(fminf(Q(ex0, ya), Q(ex1, yb)), fminf(Q(xa, ey0), Q(xb, ey1))) <= lim;
}

// stage_record written to LDS in pieces that are whole registers of the loaded
// record (the empty asm statements keep the pieces from being merged into
// wider writes), so a record loaded a batch ahead needs no repacking moves,
// which would wait for the load right after issuing it.
__device__ __forceinline__ void stage_split(const Record& r, float l2o, float4* sa, float4* sb, float4* sc) {
  float2* pa = reinterpret_cast<float2*>(sa);
  pa[0] = make_float2(r.a.x, r.a.y);
  asm volatile("" ::: "memory");
  pa[1] = make_float2(-0.5f * kLog2e * r.b.x, -kLog2e * r.b.y);
  float* pb = reinterpret_cast<float*>(sb);
  pb[0] = -0.5f * kLog2e * r.b.z;
  pb[1] = l2o;
  asm volatile("" ::: "memory");
  pb[2] = r.a.z;
  asm volatile("" ::: "memory");
  pb[3] = 0.f;
  const bool hide = isnan(r.c.x);
  float* pc = reinterpret_cast<float*>(sc);
  pc[0] = hide ? 0.f : r.c.x;
  pc[1] = hide ? 0.f : r.c.y;
  pc[2] = hide ? 0.f : r.c.z;
}

__device__ __forceinline__ int find_view(const ViewDev* views, int n_views, int tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// (the controls used here, row mirrors and quad permutations, read a lane of
// the same row for every lane, so the bound control changes nothing; with it
// set the compiler can fold the move into the add that uses it)
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Reduce-scatter of ten values over each 16-lane row: afterwards lane c holds
// the row sum of value slot(c), slot = 5 (c >> 3) + 3 ((c >> 2) & 1) +
// 2 ((c >> 1) & 1) + (c & 1), on lanes 0-2, 4-5, 8-10, 12-13 (slot -1
// elsewhere). Pairs: row mirror (c <-> 15 - c), half-row mirror, quad
// (c <-> 3 - c), quad (c <-> c ^ 1); each step keeps half of the values.
template <typename V>
__device__ __forceinline__ V row16_reduce_scatter10(const V (&q)[10], int c, int& slot) {
  const bool hi = c & 8, b = c & 4, cc = c & 2, d = c & 1;
  V r[6], s[4], t[2];
#pragma unroll
  for (int i = 0; i < 5; ++i) r[i] = (hi ? q[i + 5] : q[i]) + dpp<0x140>(hi ? q[i] : q[i + 5]);
  r[5] = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) s[i] = (b ? r[i + 3] : r[i]) + dpp<0x141>(b ? r[i] : r[i + 3]);
  s[3] = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) t[i] = (cc ? s[i + 2] : s[i]) + dpp<0x1B>(cc ? s[i] : s[i + 2]);
  const V out = (d ? t[1] : t[0]) + dpp<0xB1>(d ? t[0] : t[1]);
  const int e = 2 * (int)cc + (int)d;
  slot = (e <= (b ? 1 : 2)) ? 5 * (int)hi + 3 * (int)b + e : -1;
  return out;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, 64));
  return v;
}

// Work items of a launch: tile order[i] (or i) for i < n_items. Without a
// queue, workgroup b takes item b; with one, every workgroup of a grid sized
// to stay resident takes items from the counter at *queue (zero at launch)
// until they run out.
__device__ __forceinline__ bool next_item(const uint32_t* __restrict__ order, uint32_t n_items, uint32_t* queue,
                                          uint32_t* s_item, bool first, int& tile) {
  uint32_t item;
  if (queue) {
    __syncthreads();  // the previous item's LDS readers are done
    if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1u);
    __syncthreads();
    item = *s_item;
  } else {
    if (!first) return false;
    item = blockIdx.x;
  }
  if (item >= n_items) return false;
  tile = order ? (int)order[item] : (int)item;
  return true;
}

// DEPTH: whether the depth plane is written (otherwise its sum is compiled
// out). BATCH: list entries staged in LDS at a time (64, 128 or 256).
template <bool DEPTH, int BATCH>
__global__ void __launch_bounds__(256) k_raster_forward(const uint32_t* __restrict__ order, uint32_t n_items,
                                                         uint32_t* queue, int n_views,
                                                         const ViewDev* __restrict__ views,
                                                         const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ ival,
                                                         const Record* __restrict__ recs, float bg0, float bg1,
                                                         float bg2, int channels, bool cull,
                                                         float* __restrict__ out_rgb,
                                                         float* __restrict__ out_depth, float* __restrict__ out_alpha,
                                                         float* __restrict__ pix_t, uint32_t* __restrict__ pix_last) {
  __shared__ float4 s_a[BATCH], s_b[BATCH], s_c[BATCH];
  __shared__ __align__(16) uint8_t s_mask[BATCH];
  __shared__ uint32_t s_item;
  int tile;
  for (bool first = true; next_item(order, n_items, queue, &s_item, first, tile); first = false) {
  const int vi = find_view(views, n_views, tile);
  const ViewDev& vw = views[vi];
  const int lt = tile - vw.tile_base;
  const int tx = lt % vw.tiles_x, ty = lt / vw.tiles_x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = px < vw.width && py < vw.height;
  const float fx = px + 0.5f, fy = py + 0.5f;
  const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
  const uint2 rg = ranges[tile];
  const int count = (int)(rg.y - rg.x);

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  for (int b0 = 0; b0 < count; b0 += BATCH) {
    if (__syncthreads_count(done) == 256) break;
    const int e = b0 + threadIdx.x;
    uint32_t mask = 0u;
    if (threadIdx.x < BATCH && e < count) {
      const Record r = recs[ival[rg.x + e]];
      float4 sa, sb, sc;
      stage_record(r, sa, sb, sc);
      s_a[threadIdx.x] = sa;
      s_b[threadIdx.x] = sb;
      s_c[threadIdx.x] = sc;
      if (cull) {
#pragma unroll
        for (int q = 0; q < 4; ++q) mask |= quadrant_hit(sa, sb, tile_x0, tile_y0, q) ? (1u << q) : 0u;
      } else {
        mask = 0xFu;
      }
    }
    if (threadIdx.x < BATCH) s_mask[threadIdx.x] = (uint8_t)mask;
    __syncthreads();
    if (__all(done)) continue;
    // chunks of 16 entries: a wave-uniform mask of those that can touch this
    // wave's quadrant, walked with constant LDS offsets
    const int nb = min(BATCH, count - b0);
    for (int c0 = 0; c0 < nb; c0 += 16) {
      const uint32_t m = lane < 16 ? (uint32_t)s_mask[c0 + lane] : 0u;
      const uint32_t todo = (uint32_t)__ballot((m >> wave) & 1u);
      // the chunk's first entry as a vector register, so each entry's LDS
      // reads are immediate offsets from it
      int cv;
      asm volatile("v_mov_b32 %0, %1" : "=v"(cv) : "s"(c0));
      const float4* ca = s_a + cv;
      const float4* cb = s_b + cv;
      const float4* cc = s_c + cv;
      uint32_t last_j = 0u;  // 1 + the chunk's last contributing entry (inline constants)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (!((todo >> j) & 1u)) continue;
        const float4 sa = ca[j];
        const float4 sb = cb[j];
        const float p2 = frag_log2(fx - sa.x, fy - sa.y, sa, sb);
        float a = __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(p2), 0.f, kAlphaMax);
        const bool valid = p2 >= kLog2AlphaMin && !done;  // then a >= 1/255 > 0
        a = valid ? a : 0.f;
        const float Tn = fmaf(-a, T, T);
        const bool stop = Tn < kTStop;  // T >= kTStop always, so stop implies a > 0
        done = done || stop;
        a = stop ? 0.f : a;
        const float4 sc = cc[j];
        const float w = a * T;
        C0 = fmaf(w, sc.x, C0);
        C1 = fmaf(w, sc.y, C1);
        C2 = fmaf(w, sc.z, C2);
        if (DEPTH) D = fmaf(w, sb.z, D);
        T = stop ? T : Tn;
        last_j = (valid && !stop) ? (uint32_t)(j + 1) : last_j;  // a > 0, as masks
      }
      last = last_j ? (uint32_t)(b0 + c0) + last_j : last;
      if (__all(done)) break;
    }
  }
  if (inside) {
    const long long hw = (long long)vw.width * vw.height;
    const long long pl = (long long)py * vw.width + px;
    const long long pix = vw.pix_base + pl;
    float* rgb = out_rgb + channels * vw.pix_base + pl;
    rgb[0] = fmaf(T, bg0, C0);
    rgb[hw] = fmaf(T, bg1, C1);
    if (channels == 3) rgb[2 * hw] = fmaf(T, bg2, C2);
    if (DEPTH) out_depth[pix] = D;
    if (out_alpha) out_alpha[pix] = 1.f - T;
    pix_t[pix] = T;
    pix_last[pix] = last;
  }
  }  // items
}

// Whether a record's footprint is so elongated (condition number of its
// conic above ~100: 4 det < 0.04 trace^2) that its gradient must be summed in
// FP64: the short axis's share of dL/dconic is then a small part of much
// larger long-axis terms, which float32 tile sums would lose.
__device__ __forceinline__ bool ill_conditioned(const Record& r) {
  const float tr = r.b.x + r.b.z;
  const float det = fmaf(r.b.x, r.b.z, -r.b.y * r.b.y);
  return det < 0.01f * tr * tr;
}

// Phase 2 of the backward for primitive j2 of the staged batch and pixel
// column c2: its share of the tile sums over the rows of the quadrants where
// it blended, formed into the ten values of its gradient line (before the row
// sum). G is the type of the position moments and of the line (float, or
// double for ill-conditioned footprints); the colour and depth sums stay float.
template <typename G, bool HAS_D>
__device__ __forceinline__ void phase2_line(G (&q)[10], bool live, int j2, int c2, int tx, int ty,
                                            const float4* __restrict__ s_a, const float4* __restrict__ s_b,
                                            const uint32_t* __restrict__ s_act, const float* __restrict__ s_g,
                                            const float* __restrict__ s_w, const float4* __restrict__ s_pix) {
  // Row moments are taken about the tile's middle row (offset m = k - 7.5)
  // and moved to the primitive's centre afterwards: with dy = dc + m,
  // sum g dy = dc Sg + Sgm and sum g dy^2 = dc^2 Sg + 2 dc Sgm + Sgmm.
  G Sg = 0, Sgm = 0, Sgmm = 0;
  float Sr = 0.f, Sgc = 0.f, Sb = 0.f, Sd = 0.f;
  G dx = 0, dc = 0;
  if (live) {
    const float4 sa = s_a[j2];
    dx = (G)(tx * kTile + c2) + (G)0.5 - (G)sa.x;
    dc = (G)(ty * kTile) + (G)8 - (G)sa.y;
    const uint32_t act = (s_act[c2 >> 3] | (s_act[2 + (c2 >> 3)] << 16)) >> j2;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (!((act >> (16 * half)) & 1u)) continue;
#pragma unroll
      for (int k = 8 * half; k < 8 * half + 8; ++k) {
        const int p = k * 16 + c2;
        const int slot = j2 * kGwStride + gw_slot(k, c2);
        const float2 gw = make_float2(s_g[slot], s_w[slot]);
        const float4 pd = s_pix[p];
        const G g = gw.x;
        const G m = (G)k - (G)7.5;
        Sg += g;
        Sgm = sc_fma(g, m, Sgm);
        Sgmm = sc_fma(g, m * m, Sgmm);
        Sr = fmaf(gw.y, pd.x, Sr);
        Sgc = fmaf(gw.y, pd.y, Sgc);
        Sb = fmaf(gw.y, pd.z, Sb);
        if (HAS_D) Sd = fmaf(gw.y, pd.w, Sd);
      }
    }
  }
  const G Sgy = sc_fma(dc, Sg, Sgm);
  const G Sgyy = sc_fma(dc, sc_fma(dc, Sg, (G)2 * Sgm), Sgmm);
  // v: Sg, Sgx, Sgy, Sgxx, Sgxy, Sgyy, w*dL/dr, w*dL/dg, w*dL/db, w*dL/dD
  // This column's share of the primitive's gradient line (the 2D-mean,
  // conic and opacity entries are linear in the moments, so they are formed
  // before the row sum): dL/du, dL/dv, dL/dconic (3), dL/d(opacity p),
  // dL/drgb (3), dL/dz.
  const float4 pa = s_a[j2], pb = s_b[j2];
  const G k0 = live ? (G)pa.z * (G)(-2.f / kLog2e) : (G)0, k1 = live ? (G)pa.w * (G)(-1.f / kLog2e) : (G)0;
  const G k2 = live ? (G)pb.x * (G)(-2.f / kLog2e) : (G)0;
  const G iop = live ? (G)__builtin_amdgcn_exp2f(-pb.y) : (G)0;
  const G Sgx = dx * Sg, Sgxy = dx * Sgy;
  q[0] = sc_fma(k0, Sgx, k1 * Sgy);
  q[1] = sc_fma(k1, Sgx, k2 * Sgy);
  q[2] = (G)-0.5 * dx * Sgx;
  q[3] = -Sgxy;
  q[4] = (G)-0.5 * Sgyy;
  q[5] = Sg * iop;
  q[6] = Sr;
  q[7] = Sgc;
  q[8] = Sb;
  q[9] = HAS_D ? (G)Sd : (G)0;
}

// HAS_D / HAS_A: whether dL/d(depth) and dL/d(alpha) are given (otherwise
// their terms are compiled out). With loss.kind set, dl_rgb is the rendered
// image and the image loss is folded in (LossArgs).
template <bool HAS_D, bool HAS_A>
__global__ void __launch_bounds__(256, 5) k_raster_backward(
    const uint32_t* __restrict__ order, uint32_t n_items, uint32_t* queue, int n_views, const ViewDev* __restrict__ views, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ival,
    const Record* __restrict__ recs, float bg0, float bg1, float bg2, const float* __restrict__ dl_rgb,
    const float* __restrict__ dl_depth, const float* __restrict__ dl_alpha, const float* __restrict__ pix_t,
    const uint32_t* __restrict__ pix_last, double* __restrict__ grad2d, bool mark_blended, bool cull,
    LossArgs loss) {
  __shared__ float4 s_a2[2][kBwdBatch], s_b2[2][kBwdBatch], s_c2[2][kBwdBatch];
  __shared__ uint32_t s_d2[2][kBwdBatch];
  __shared__ uint32_t s_qm2[2][kBwdBatch];
  __shared__ uint32_t s_ill2[2];  // per staged batch: bit j when entry j's footprint is ill-conditioned
  __shared__ uint32_t s_act[4];  // per quadrant: bit j when entry j blended somewhere in it
  __shared__ float s_g[kBwdBatch * kGwStride];   // dL/dpower per (primitive, pixel)
  __shared__ float s_w[kBwdBatch * kGwStride];   // a_i T_i per (primitive, pixel)
  __shared__ float4 s_pix[256];
  __shared__ uint32_t s_max;
  __shared__ uint32_t s_item;
  __shared__ float s_loss[4];

  int tile;
  for (bool first = true; next_item(order, n_items, queue, &s_item, first, tile); first = false) {
  const int vi = find_view(views, n_views, tile);
  const ViewDev& vw = views[vi];
  const int lt = tile - vw.tile_base;
  const int tx = lt % vw.tiles_x, ty = lt / vw.tiles_x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lx = (wave & 1) * 8 + (lane & 7), ly = (wave >> 1) * 8 + (lane >> 3);
  const int p_self = ly * 16 + lx;                  // row-major pixel index within the tile
  const int q_self = gw_slot(ly, lx);               // this pixel's slot in s_g / s_w
  const int px = tx * kTile + lx, py = ty * kTile + ly;
  const bool inside = px < vw.width && py < vw.height;
  const float fx = px + 0.5f, fy = py + 0.5f;
  const float tile_x0 = (float)(tx * kTile), tile_y0 = (float)(ty * kTile);
  const uint2 rg = ranges[tile];
  const int count = (int)(rg.y - rg.x);

  if (threadIdx.x == 0) s_max = 0u;
  float T = 1.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f, lsum = 0.f;
  uint32_t last = 0;
  if (inside) {
    const long long hw = (long long)vw.width * vw.height;
    const long long pl = (long long)py * vw.width + px;
    const long long pix = vw.pix_base + pl;
    const float* g = dl_rgb + 3 * vw.pix_base + pl;
    if (loss.kind) {
      // with a folded loss the rgb input is the rendered image: the loss
      // term and dL/dC of each channel against the target, formed as the
      // image-loss kernel forms them
      const float* tg = loss.target + 3 * vw.pix_base + pl;
      lsum = shade::loss_term(loss.kind, g[0] - tg[0], loss.scale, gC0) +
             shade::loss_term(loss.kind, g[hw] - tg[hw], loss.scale, gC1) +
             shade::loss_term(loss.kind, g[2 * hw] - tg[2 * hw], loss.scale, gC2);
    } else {
      gC0 = g[0];
      gC1 = g[hw];
      gC2 = g[2 * hw];
    }
    if (HAS_D) gD = dl_depth[pix];
    if (HAS_A) gA = dl_alpha[pix];
    T = pix_t[pix];
    last = pix_last[pix];
  }
  s_pix[p_self] = make_float4(gC0, gC1, gC2, gD);
  if (loss.kind) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) s_loss[wave] = lsum;
  }
  const uint32_t wave_last = wave_max_u32(last);
  // batches ending at or before every lane's last contributor need no
  // per-entry list-position test
  const uint32_t wave_first_last = wave_min_u32(last);
  __syncthreads();
  if (lane == 0 && wave_last) atomicMax(&s_max, wave_last);
  // the tile's loss, summed over its pixels
  if (loss.kind && threadIdx.x == 0) loss.part[tile] = s_loss[0] + s_loss[1] + s_loss[2] + s_loss[3];
  // Only the dot product of this pixel's output gradient with the colour,
  // depth and alpha of everything behind the current primitive (normalised by
  // the transmittance after it) enters dL/da; it starts at the background.
  float beta = fmaf(gC0, bg0, fmaf(gC1, bg1, gC2 * bg2));
  __syncthreads();
  const int max_last = (int)s_max;

  const int c2 = threadIdx.x & 15;  // phase 2: pixel column
  const int b_first = ((max_last + kBwdBatch - 1) / kBwdBatch - 1) * kBwdBatch;
  // Staging pipeline (threads < 16): the record of the batch after the one in
  // LDS and the list index of the batch after that are in flight, so no wait
  // covers a load issued in the same batch.
  Record nxt;
  uint32_t nxt_d = 0, nn_d = 0;
  // Run by the whole of wave 0: lanes < 16 stage entry e0 + lane; then four
  // lanes per entry test its quadrants on the staged values (taken from the
  // staging lane by a shuffle) and a ballot gathers the four bits.
  auto stage = [&](int e0, int bb) {
    const int t = (int)threadIdx.x;
    const float l2o = staged_log2_opacity(nxt);
    if (t < kBwdBatch && e0 + t < count) {
      stage_split(nxt, l2o, &s_a2[bb][t], &s_b2[bb][t], &s_c2[bb][t]);
      s_d2[bb][t] = nxt_d;
    }
    const int src = t >> 2;
    float4 qa, qb;
    qa.x = __shfl(nxt.a.x, src, 64);
    qa.y = __shfl(nxt.a.y, src, 64);
    qa.z = -0.5f * kLog2e * __shfl(nxt.b.x, src, 64);
    qa.w = -kLog2e * __shfl(nxt.b.y, src, 64);
    qb.x = -0.5f * kLog2e * __shfl(nxt.b.z, src, 64);
    qb.y = __shfl(l2o, src, 64);
    const bool hit = e0 + src < count && (!cull || quadrant_hit(qa, qb, tile_x0, tile_y0, t & 3));
    const uint64_t bits = __ballot(hit);
    if (t < kBwdBatch) s_qm2[bb][t] = (uint32_t)(bits >> (4 * t)) & 0xFu;
    const uint64_t ill = __ballot(t < kBwdBatch && e0 + t < count && ill_conditioned(nxt));
    if (t == 0) s_ill2[bb] = (uint32_t)ill & 0xFFFFu;
  };
  if (wave == 0 && b_first >= 0) {
    if (threadIdx.x < kBwdBatch && b_first + (int)threadIdx.x < count) {
      nxt_d = ival[rg.x + b_first + threadIdx.x];
      nxt = recs[nxt_d];
    }
    stage(b_first, 0);
    const int e1 = b_first - kBwdBatch + (int)threadIdx.x;
    if (threadIdx.x < kBwdBatch && e1 >= 0) {
      nxt_d = ival[rg.x + e1];
      nxt = recs[nxt_d];
    }
    const int e2n = e1 - kBwdBatch;
    if (threadIdx.x < kBwdBatch && e2n >= 0) nn_d = ival[rg.x + e2n];
  }
  int buf = 0;
  for (int b0 = b_first; b0 >= 0; b0 -= kBwdBatch, buf ^= 1) {
    // the stage buffer's first entry as a vector register, so each entry's
    // LDS reads in phase 1 are immediate offsets from it
    int bv;
    asm volatile("v_mov_b32 %0, %1" : "=v"(bv) : "s"(buf * kBwdBatch));
    const float4* s_a = &s_a2[0][0] + bv;
    const float4* s_b = &s_b2[0][0] + bv;
    const float4* s_c = &s_c2[0][0] + bv;
    const uint32_t* s_d = s_d2[buf];
    const uint32_t* s_qm = s_qm2[buf];
    __syncthreads();
    // ---- phase 1: this lane's pixel, back to front over the batch ----
    // entries that can reach this wave's quadrant before its last contributor
    uint32_t todo;
    {
      const uint32_t qm = lane < kBwdBatch ? s_qm[lane] : 0u;
      todo = (uint32_t)__ballot(((qm >> wave) & 1u) && (uint32_t)(b0 + lane) < wave_last);
    }
    uint32_t blended = 0u;
    // CHECK: test the entry's list position against this lane's last
    // contributor (not needed when the batch ends at or before every lane's)
    auto entry = [&](int j, const float4& sa, const float4& sb, const float4& sc, auto check) {
      const float p2 = frag_log2(fx - sa.x, fy - sa.y, sa, sb);
      const bool valid = (!decltype(check)::value || (uint32_t)(b0 + j) < last) && (p2 >= kLog2AlphaMin);
      if (!__any(valid)) return;
      const float G = __builtin_amdgcn_exp2f(p2);
      const float a = valid ? __builtin_amdgcn_fmed3f(G, 0.f, kAlphaMax) : 0.f;
      T = T * __builtin_amdgcn_rcpf(1.f - a);
      float dot = fmaf(gC0, sc.x, fmaf(gC1, sc.y, gC2 * sc.z));
      if (HAS_D) dot = fmaf(gD, sb.z, dot);
      if (HAS_A) dot += gA;
      const float s = dot - beta;
      beta = fmaf(a, s, beta);
      // dL/dpower = dL/da * a for an unclamped alpha (a = G), zero where the
      // clamp holds; a skipped fragment has a = 0
      const float w = a * T;
      const float g = G < kAlphaMax ? w * s : 0.f;
      s_g[j * kGwStride + q_self] = g;
      s_w[j * kGwStride + q_self] = w;
      blended |= 1u << j;
    };
    // back to front over the set entries; j is a constant in every unrolled
    // step, so the LDS addresses are immediate offsets
    if ((uint32_t)b0 + kBwdBatch <= wave_first_last) {
#pragma unroll
      for (int j = kBwdBatch - 1; j >= 0; --j) {
        if (!((todo >> j) & 1u)) continue;
        entry(j, s_a[j], s_b[j], s_c[j], std::false_type{});
      }
    } else {
#pragma unroll
      for (int j = kBwdBatch - 1; j >= 0; --j) {
        if (!((todo >> j) & 1u)) continue;
        entry(j, s_a[j], s_b[j], s_c[j], std::true_type{});
      }
    }
    if (lane == 0) s_act[wave] = blended;
    __syncthreads();
    // ---- phase 2: primitive j2, pixel column c2, rows of active quadrants ----
    // Waves 1-3 take primitives 4 (w - 1) .. 4 (w - 1) + 3; wave 0, which
    // stages the next batch below, takes none, so the waves reach the next
    // barrier together.
    const int rank = wave - 1;
    const int j2 = 4 * rank + (lane >> 4);
    const bool p2 = wave > 0;  // wave-uniform
    const int e2 = b0 + j2;
    const bool live = p2 && e2 < count;
    int slot_q = -1;
    double val = 0.0;
    uint32_t d_atom = 0u;
    if (p2) {
      // FP64 sums for the waves whose four primitives include an
      // ill-conditioned footprint (wave-uniform)
      if ((s_ill2[buf] >> (4 * rank)) & 0xFu) {
        double q[10];
        phase2_line<double, HAS_D>(q, live, j2, c2, tx, ty, s_a, s_b, s_act, s_g, s_w, s_pix);
        val = row16_reduce_scatter10(q, c2, slot_q);
      } else {
        float q[10];
        phase2_line<float, HAS_D>(q, live, j2, c2, tx, ty, s_a, s_b, s_act, s_g, s_w, s_pix);
        val = (double)row16_reduce_scatter10(q, c2, slot_q);
      }
      // the record blended in this tile: flag it in the gradient line's last
      // float (the same 1 from every tile, so plain stores suffice)
      if (mark_blended && c2 == 15 && live && (((s_act[0] | s_act[1] | s_act[2] | s_act[3]) >> j2) & 1u))
        grad2d[(size_t)s_d[j2] * kGrad2dStride + 15] = 1.0;
      d_atom = s_d[j2];
    }
    // stage the next batch into the other buffer (read by nobody until the
    // next loop-top barrier) and advance the loads, before this batch's atomics
    if (wave == 0 && b0 >= kBwdBatch) {
      stage(b0 - kBwdBatch, buf ^ 1);
      const int e1 = b0 - 2 * kBwdBatch + (int)threadIdx.x;
      if (threadIdx.x < kBwdBatch && e1 >= 0) {
        nxt_d = nn_d;
        nxt = recs[nxt_d];
      }
      const int e2n = e1 - kBwdBatch;
      if (threadIdx.x < kBwdBatch && e2n >= 0) nn_d = ival[rg.x + e2n];
    }
    // ten lanes of the primitive's row each add one value of its gradient
    // line, so a wave's atomics for a primitive share one 128-byte line
    if (live && slot_q >= 0 && val != 0.0)
      unsafeAtomicAdd(grad2d + (size_t)d_atom * kGrad2dStride + slot_q, val);
  }
  }  // items
}

// Workgroups of `kernel` that stay resident on the current device (looked
// up once per kernel and device).
template <typename K>
unsigned resident_grid(K kernel) {
  constexpr int kDevs = 64;
  static unsigned cached[kDevs] = {};
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (dev >= 0 && dev < kDevs && cached[dev]) return cached[dev];
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1 || cus < 1)
    return 1024;
  const unsigned g = (unsigned)(per_cu * cus);
  if (dev >= 0 && dev < kDevs) cached[dev] = g;
  return g;
}

// Grid of a launch over total_tiles items: one workgroup per item, or with
// a queue, `blocks` workgroups (-1: as many as stay resident).
template <typename K>
unsigned item_grid(K kernel, int total_tiles, uint32_t* queue, int blocks, hipStream_t s) {
  unsigned grid = (unsigned)total_tiles;
  if (queue) {
    const unsigned want = blocks > 0 ? (unsigned)blocks : resident_grid(kernel);
    grid = std::min(grid, want);
    launch_fill_u32(queue, 1, 0u, s);
  }
  return grid;
}

template <bool DEPTH, int BATCH>
void launch_fwd(int total_tiles, const uint32_t* order, uint32_t* queue, int blocks, int n_views,
                const ViewDev* views, const uint2* ranges, const uint32_t* ival, const Record* rec_sorted,
                const float* bg, int channels, bool cull, float* out_rgb, float* out_depth, float* out_alpha,
                float* pix_t, uint32_t* pix_last, hipStream_t s) {
  const unsigned grid = item_grid(k_raster_forward<DEPTH, BATCH>, total_tiles, queue, blocks, s);
  hipLaunchKernelGGL((k_raster_forward<DEPTH, BATCH>), dim3(grid), dim3(256), 0, s, order, (uint32_t)total_tiles,
                     queue, n_views, views, ranges, ival, rec_sorted, bg[0], bg[1], bg[2], channels, cull, out_rgb,
                     out_depth, out_alpha, pix_t, pix_last);
}

}  // namespace

void launch_raster_forward(int total_tiles, const uint32_t* order, uint32_t* queue, int blocks, int batch,
                           int n_views, const ViewDev* views, const uint2* ranges, const uint32_t* ival,
                           const Record* rec_sorted, const float* bg, int channels, bool cull, float* out_rgb,
                           float* out_depth, float* out_alpha, float* pix_t, uint32_t* pix_last, hipStream_t s) {
  if (total_tiles == 0) return;
#define G4D_FWD(D, B)                                                                                            \
  launch_fwd<D, B>(total_tiles, order, queue, blocks, n_views, views, ranges, ival, rec_sorted, bg, channels, cull, \
                   out_rgb, out_depth, out_alpha, pix_t, pix_last, s)
  const bool d = out_depth != nullptr;
  if (batch == 64) {
    if (d) G4D_FWD(true, 64); else G4D_FWD(false, 64);
  } else if (batch == 128) {
    if (d) G4D_FWD(true, 128); else G4D_FWD(false, 128);
  } else {
    if (d) G4D_FWD(true, 256); else G4D_FWD(false, 256);
  }
#undef G4D_FWD
}

namespace {
template <bool HD, bool HA>
void launch_bwd(int total_tiles, const uint32_t* order, uint32_t* queue, int blocks, int n_views,
                const ViewDev* views, const uint2* ranges, const uint32_t* ival, const Record* rec_sorted,
                const float* bg, const float* dl_rgb, const float* dl_depth, const float* dl_alpha,
                const float* pix_t, const uint32_t* pix_last, double* grad2d, bool mark_blended, bool cull,
                const LossArgs& loss, hipStream_t s) {
  const unsigned grid = item_grid(k_raster_backward<HD, HA>, total_tiles, queue, blocks, s);
  hipLaunchKernelGGL((k_raster_backward<HD, HA>), dim3(grid), dim3(256), 0, s, order, (uint32_t)total_tiles, queue,
                     n_views, views, ranges, ival, rec_sorted, bg[0], bg[1], bg[2], dl_rgb, dl_depth, dl_alpha, pix_t,
                     pix_last, grad2d, mark_blended, cull, loss);
}
}  // namespace

void launch_raster_backward(int total_tiles, const uint32_t* order, uint32_t* queue, int blocks, int n_views,
                            const ViewDev* views, const uint2* ranges, const uint32_t* ival,
                            const Record* rec_sorted, const float* bg, const float* dl_rgb, const float* dl_depth,
                            const float* dl_alpha, const float* pix_t, const uint32_t* pix_last, double* grad2d,
                            bool mark_blended, bool cull, const LossArgs& loss, hipStream_t s) {
  if (total_tiles == 0) return;
#define G4D_BWD(HD, HA)                                                                                          \
  launch_bwd<HD, HA>(total_tiles, order, queue, blocks, n_views, views, ranges, ival, rec_sorted, bg, dl_rgb,      \
                     dl_depth, dl_alpha, pix_t, pix_last, grad2d, mark_blended, cull, loss, s)
  if (dl_depth && dl_alpha) G4D_BWD(true, true);
  else if (dl_depth) G4D_BWD(true, false);
  else if (dl_alpha) G4D_BWD(false, true);
  else G4D_BWD(false, false);
#undef G4D_BWD
}

}  // namespace g4d
