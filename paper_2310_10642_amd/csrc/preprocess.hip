// Per-primitive stages of the 4D Gaussian render. k_preprocess (one thread
// per primitive, looping over the views of a batch so the parameters are
// read once): 4D covariance Sigma = R S S^T R^T with R = L(q_l) R(q_r)
// (Sec. 3.2, "Representation of 4D Gaussian"), temporal marginal and filter
// (Sec. 3.2 and Sec. 4.2), conditional 3D Gaussian at t (Sec. 3.2), EWA
// projection (Eqs. 3-4), footprint and tile rectangle -- and, for a flow
// render, the image-plane displacement of the conditional mean (Sec. 4.3).
// k_colour: the 4D spherindrical-harmonic colour (Sec. 3.2) of the active
// pairs, written into their depth-ordered records once the gather has placed
// them. The backward is in preprocess_bwd.hip.
#include "shade.h"

namespace g4d {
namespace {

using namespace shade;

__global__ void __launch_bounds__(256) k_preprocess(RenderParams p, uint32_t* __restrict__ act,
                                                    uint32_t* __restrict__ dkey, Record* __restrict__ rec,
                                                    int32_t* __restrict__ slot, float4* __restrict__ cdir) {
  const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (gidx >= p.n) return;
  const float4 mu = p.means4[gidx];
  const float4 ls = p.log_scales4[gidx];
  float inl, inr;
  const float4 ql = normalize4(p.q_left[gidx], inl);
  const float4 qr = normalize4(p.q_right[gidx], inr);
  const float opa = 1.f / (1.f + __expf(-p.opacity_logit[gidx]));
  Shape4 sh;
  build_shape(ql, qr, ls, sh);

  for (int vi = 0; vi < p.n_views; ++vi) {
    const size_t idx = (size_t)vi * p.n + gidx;
    const ViewDev& vw = p.views[vi];
    ViewGeom g;
    bool ok = view_geometry(mu, sh, vw, p.t_cull, p.near_plane, g);
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    if (ok) {
      ok = g.det > 0.f;
      const float mid = 0.5f * (g.a2 + g.c2);
      const float lmax = mid + sqrtf(fmaxf(mid * mid - g.det, 0.f));
      const float rad = ceilf(kSigmaExtent * sqrtf(lmax));
      const float ft = 1.f / kTile;
      x0 = (int)fminf(fmaxf(floorf((g.u - rad) * ft), 0.f), (float)vw.tiles_x);
      x1 = (int)fminf(fmaxf(floorf((g.u + rad) * ft) + 1.f, 0.f), (float)vw.tiles_x);
      y0 = (int)fminf(fmaxf(floorf((g.v - rad) * ft), 0.f), (float)vw.tiles_y);
      y1 = (int)fminf(fmaxf(floorf((g.v + rad) * ft) + 1.f, 0.f), (float)vw.tiles_y);
      // Binning footprint: only tiles that can hold a pixel with
      // opacity * exp(power) >= 1/255, i.e. inside the ellipse
      // 1/2 d^T conic d <= ln(255 opacity); its bounding box has half-widths
      // sqrt(2 K Sigma2d_00), sqrt(2 K Sigma2d_11). Every other tile of the
      // 3-sigma rectangle would skip this primitive at every pixel, so the
      // blend is unchanged. The slack keeps the box conservative under FP32.
      const float K = __logf(255.f * opa * g.pt);
      ok = ok && K > -1e-4f;
      const float Kc = fmaxf(K, 0.f);
      const float hx = sqrtf(2.f * Kc * g.a2) * 1.001f + 0.05f;
      const float hy = sqrtf(2.f * Kc * g.c2) * 1.001f + 0.05f;
      const float bx = (float)vw.tiles_x + 1.f, by = (float)vw.tiles_y + 1.f;
      x0 = max(x0, (int)fminf(fmaxf(floorf((g.u - hx) * ft), -1.f), bx));
      x1 = min(x1, (int)fminf(fmaxf(floorf((g.u + hx) * ft) + 1.f, -1.f), bx));
      y0 = max(y0, (int)fminf(fmaxf(floorf((g.v - hy) * ft), -1.f), by));
      y1 = min(y1, (int)fminf(fmaxf(floorf((g.v + hy) * ft) + 1.f, -1.f), by));
      ok = ok && (x1 > x0) && (y1 > y0) && isfinite(g.u) && isfinite(g.v);
    }
    if (!ok) {
      act[idx] = 0u;
      slot[idx] = -1;
      continue;
    }
    Record r;
    r.a = make_float4(g.u, g.v, g.pc[2], opa * g.pt);
    r.b = make_float4(g.conic[0], g.conic[1], g.conic[2], __uint_as_float((uint32_t)x0 | ((uint32_t)x1 << 16)));
    if (p.flow) {
      // Sec. 4.3: the conditional mean moves by v3 dt / S44 (it is linear in
      // t); its projection moves by f (x' z - x z') / (z z') per axis
      const float s = p.flow_dt / g.s44;
      float dp[3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
        dp[i] = s * (vw.rot[3 * i] * g.v3[0] + vw.rot[3 * i + 1] * g.v3[1] + vw.rot[3 * i + 2] * g.v3[2]);
      const float x = g.pc[0], y = g.pc[1], z = g.pc[2], z1 = z + dp[2];
      const bool front = z1 > p.near_plane;
      const float q = front ? 1.f / (z * z1) : 0.f;
      const float fu = vw.fx * (dp[0] * z - x * dp[2]) * q;
      const float fv = vw.fy * (dp[1] * z - y * dp[2]) * q;
      r.c = make_float4(fu, fv, 0.f, __uint_as_float((uint32_t)y0 | ((uint32_t)y1 << 16)));
      rec[idx] = r;
      act[idx] = 1u;
      dkey[idx] = __float_as_uint(g.pc[2]);
      slot[idx] = -1;
      continue;
    }
    // colour: k_colour fills c.xyz of the record's depth-ordered copy from
    // the view direction and t - mu_t
    r.c = make_float4(0.f, 0.f, 0.f, __uint_as_float((uint32_t)y0 | ((uint32_t)y1 << 16)));
    cdir[idx] = make_float4(g.dir[0], g.dir[1], g.dir[2], g.dt);
    rec[idx] = r;
    act[idx] = 1u;
    dkey[idx] = __float_as_uint(g.pc[2]);  // z > near > 0: bit order = numeric order
    slot[idx] = -1;
  }
}

constexpr int kColourViews = 8;  // views whose loads k_colour issues together

// 4D spherindrical-harmonic colour (Sec. 3.2): a quad of lanes per primitive,
// lane `sub` owning the basis functions lm = 4 sub + i. The block's 64
// primitives' coefficients are contiguous in memory; they are staged through
// LDS with 16-byte loads, and each lane takes its [n][4 sub + i][3] from
// there. Per active view every lane evaluates the basis, weights its four
// functions by the Fourier terms, and a quad sum gives c = max(0, 0.5 + sum).
__global__ void __launch_bounds__(256) k_colour(RenderParams p, const int32_t* __restrict__ slot,
                                                const float4* __restrict__ cdir, Record* __restrict__ rec_sorted) {
  __shared__ __align__(16) float s_k[kColourPrims * kCoeffMax];
  const int nb = (p.sh_degree + 1) * (p.sh_degree + 1);
  const int nt = p.t_order + 1;
  const int K3 = nt * nb * 3;
  const int g0 = blockIdx.x * kColourPrims;
  const int nprim = min(kColourPrims, p.n - g0);
  copy_in(s_k, p.coeffs + (size_t)g0 * K3, nprim * K3);
  __syncthreads();
  const int gidx = g0 + (int)(threadIdx.x >> 2);
  const int sub = threadIdx.x & 3;
  if (gidx >= p.n) return;  // uniform per quad
  const float* kc = s_k + (threadIdx.x >> 2) * K3;
  float k[3][kBasisPerLane][3];
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int i = 0; i < kBasisPerLane; ++i) {
      const int lm = sub * kBasisPerLane + i;
#pragma unroll
      for (int c = 0; c < 3; ++c) k[n][i][c] = (lm < nb && n < nt) ? kc[(n * nb + lm) * 3 + c] : 0.f;
    }
  // views eight at a time: all flags, then the directions of the active
  // ones, are loaded before any is used, so the loads overlap
  for (int v0 = 0; v0 < p.n_views; v0 += kColourViews) {
    int on[kColourViews];
    float4 cds[kColourViews];
#pragma unroll
    for (int w = 0; w < kColourViews; ++w) on[w] = v0 + w < p.n_views ? slot[(size_t)(v0 + w) * p.n + gidx] : -1;
#pragma unroll
    for (int w = 0; w < kColourViews; ++w)
      cds[w] = on[w] >= 0 ? cdir[(size_t)(v0 + w) * p.n + gidx] : make_float4(0.f, 0.f, 1.f, 0.f);
#pragma unroll
    for (int w = 0; w < kColourViews; ++w) {
      if (on[w] < 0) continue;  // uniform per quad
      const float4 cd = cds[w];
      float Y[16], cs[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 16; ++j) Y[j] = 0.f;
      sh_eval(p.sh_degree, cd.x, cd.y, cd.z, Y);
      fourier_terms(p.t_order, cd.w, p.t_period, cs);
      float y[kBasisPerLane];
      own_basis(Y, sub, y);
      float col[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < kBasisPerLane; ++i)
          acc = fmaf(y[i], fmaf(cs[0], k[0][i][c], fmaf(cs[1], k[1][i][c], cs[2] * k[2][i][c])), acc);
        col[c] = quad_sum(acc);
      }
      if (sub == 0) {
        float* o = reinterpret_cast<float*>(&rec_sorted[on[w]].c);
        o[0] = fmaxf(col[0] + kColorOffset, 0.f);
        o[1] = fmaxf(col[1] + kColorOffset, 0.f);
        o[2] = fmaxf(col[2] + kColorOffset, 0.f);
      }
    }
  }
}

}  // namespace

void launch_preprocess(const RenderParams& p, uint32_t* act, uint32_t* dkey, Record* rec, int32_t* slot,
                       float4* cdir, hipStream_t s) {
  if (p.n == 0) return;
  const int bs = 256;
  hipLaunchKernelGGL(k_preprocess, dim3((p.n + bs - 1) / bs), dim3(bs), 0, s, p, act, dkey, rec, slot, cdir);
}

void launch_colour(const RenderParams& p, const int32_t* slot, const float4* cdir, Record* rec_sorted,
                   hipStream_t s) {
  if (p.n == 0 || p.flow) return;
  hipLaunchKernelGGL(k_colour, dim3((unsigned)((p.n + kColourPrims - 1) / kColourPrims)), dim3(256), 0, s, p, slot,
                     cdir, rec_sorted);
}

}  // namespace g4d
