// Backward of the per-primitive stages: from the per-record 2D gradients
// (dL/du, dL/dv, dL/dconic, dL/d(opacity p), dL/drgb, dL/dz) to every 4D
// parameter, summed over the views of a batch.
//
// Three kernels, so that each one reads or writes memory in the order it is
// laid out:
//   pairs:   one thread per active (view, primitive) record: the EWA
//            projection, camera, opacity, temporal-marginal and slice chain
//            (Sec. 3.2, Eqs. 3-4) up to dL/dSigma, dL/dmu and dL/dlogit of
//            that view; the colour gradient is passed on (clamp decided from
//            the record's colour).
//   colour:  a quad of lanes per primitive active in some view, four SH
//            basis functions per lane: 4D spherindrical-harmonic coefficients
//            (Sec. 3.2), read and written once; per active view the gradient
//            to the view direction and to t - mu_t is reduced over the quad
//            and passed on.
//   prims:   one thread per primitive: sums the views, adds the colour part
//            through the slice, then Sigma = M M^T, M = R S, R = L(q_l) R(q_r)
//            and the quaternion normalisation.
// The pairs and prims chains run in FP64 (as the forward geometry does): the
// conditional covariance of a long, thin primitive is a difference of nearly
// equal terms, which float32 would leave with few correct bits.
#include "shade.h"

namespace g4d {
namespace {

using namespace shade;

// pair scratch layout (floats per active record)
constexpr int kGeoFloats = 16;  // G4 upper triangle (10), dL/dmu (4), dL/dlogit, |dL/d(u,v)| (-1: not blended)
constexpr int kColFloats = 8;   // dL/draw (3), t - mu_t, view direction (3), 1/|mu_c - c|
constexpr int kCgFloats = 4;    // dL/dmu_c and dL/d(t - mu_t) through the colour

__global__ void __launch_bounds__(256) k_bwd_pairs(RenderParams p, const uint32_t* n_dev, uint32_t n_max,
                                                    const uint32_t* __restrict__ ids, const Record* __restrict__ recs,
                                                    const double* __restrict__ grad2d, float4* __restrict__ geo,
                                                    float4* __restrict__ colbuf) {
  const uint32_t n = min(*n_dev, n_max);
  const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  const uint32_t id = ids[d];
  const int vi = (int)(id / (uint32_t)p.n);
  const int gidx = (int)(id - (uint32_t)vi * (uint32_t)p.n);
  const float4 mu = p.means4[gidx];
  Shape4T<double> sh;
  build_shape<double>(p.q_left[gidx], p.q_right[gidx], p.log_scales4[gidx], sh);
  const double opa = 1.0 / (1.0 + exp(-(double)p.opacity_logit[gidx]));
  const ViewDev& vw = p.views[vi];
  ViewGeomT<double> g;
  view_geometry<double>(mu, sh, vw, (double)p.t_cull, (double)p.near_plane, g);
  const double* ln = grad2d + (size_t)d * kGrad2dStride;
  const double2 q0 = *reinterpret_cast<const double2*>(ln), q1 = *reinterpret_cast<const double2*>(ln + 2);
  const double2 q2 = *reinterpret_cast<const double2*>(ln + 4), q3 = *reinterpret_cast<const double2*>(ln + 6);
  const double2 q4 = *reinterpret_cast<const double2*>(ln + 8);
  const double gu = q0.x, gv = q0.y, gC0 = q1.x, gC1 = q1.y, gC2 = q2.x, go = q2.y, gdepth = q4.y;
  // last value of the line: 1 when the record blended some pixel (set by the
  // rasteriser's backward when statistics are on)
  const bool blended = ln[15] > 0.5;
  // colour = max(0, raw + 0.5): the clamp passes the gradient where the blended colour is positive
  const float4 rc = recs[d].c;
  const float graw0 = rc.x > 0.f ? (float)q3.x : 0.f;
  const float graw1 = rc.y > 0.f ? (float)q3.y : 0.f;
  const float graw2 = rc.z > 0.f ? (float)q4.x : 0.f;
  colbuf[2 * (size_t)d] = make_float4(graw0, graw1, graw2, (float)g.dt);
  colbuf[2 * (size_t)d + 1] = make_float4((float)g.dir[0], (float)g.dir[1], (float)g.dir[2], (float)g.rinv);

  // ---- opacity * p(t) ----
  const double gpt = go * opa;
  const double glogit = go * g.pt * opa * (1.0 - opa);
  // ---- conic -> Sigma_2d: G_S = -Q G_Q Q ----
  const double C0 = g.conic[0], C1 = g.conic[1], C2 = g.conic[2];
  const double h1 = 0.5 * gC1;
  const double X00 = C0 * gC0 + C1 * h1, X01 = C0 * h1 + C1 * gC2;
  const double X10 = C1 * gC0 + C2 * h1, X11 = C1 * h1 + C2 * gC2;
  const double G00 = -(X00 * C0 + X01 * C1);
  const double G01 = -(X00 * C1 + X01 * C2);
  const double G11 = -(X10 * C1 + X11 * C2);
  // ---- Sigma_2d = T Sc T^T:  g_Sc = T^T G T,  g_T = 2 G T Sc ----
  double GT[2][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    GT[0][k] = G00 * g.T_[0][k] + G01 * g.T_[1][k];
    GT[1][k] = G01 * g.T_[0][k] + G11 * g.T_[1][k];
  }
  double gSc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gSc[i][j] = g.T_[0][i] * GT[0][j] + g.T_[1][i] * GT[1][j];
  double gT[2][3];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      gT[r][k] = 2.0 * (GT[r][0] * g.Sc[0][k] + GT[r][1] * g.Sc[1][k] + GT[r][2] * g.Sc[2][k]);
  // ---- T = J W:  g_J = g_T W^T ----
  double W[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) W[k] = vw.rot[k];
  const double gJ00 = gT[0][0] * W[0] + gT[0][1] * W[1] + gT[0][2] * W[2];
  const double gJ02 = gT[0][0] * W[6] + gT[0][1] * W[7] + gT[0][2] * W[8];
  const double gJ11 = gT[1][0] * W[3] + gT[1][1] * W[4] + gT[1][2] * W[5];
  const double gJ12 = gT[1][0] * W[6] + gT[1][1] * W[7] + gT[1][2] * W[8];
  // ---- camera-space point (x, y, z) ----
  const double fx = vw.fx, fy = vw.fy;
  const double x = g.pc[0], y = g.pc[1], iz = g.iz, iz2 = iz * iz;
  double gx = gu * fx * iz;
  double gy = gv * fy * iz;
  double gz = gdepth - gu * fx * x * iz2 - gv * fy * y * iz2;
  gz += -gJ00 * fx * iz2 - gJ11 * fy * iz2;
  if (g.clx) {
    gz += gJ02 * fx * g.xi * iz2;
  } else {
    gx += -gJ02 * fx * iz2;
    gz += 2.0 * gJ02 * fx * g.xi * iz2;
  }
  if (g.cly) {
    gz += gJ12 * fy * g.eta * iz2;
  } else {
    gy += -gJ12 * fy * iz2;
    gz += 2.0 * gJ12 * fy * g.eta * iz2;
  }
  // p_cam = W mu_c + w
  double gmuc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) gmuc[i] = W[i] * gx + W[3 + i] * gy + W[6 + i] * gz;
  // ---- slice: Sc = Sxyz - v v^T / S44, mu_c = mu_xyz + v lam ----
  const double inv44 = 1.0 / g.s44;
  double Gv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Gv[i] = gSc[i][0] * g.v3[0] + gSc[i][1] * g.v3[1] + gSc[i][2] * g.v3[2];
  const double vGv = g.v3[0] * Gv[0] + g.v3[1] * Gv[1] + g.v3[2] * Gv[2];
  double gv3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) gv3[i] = -2.0 * Gv[i] * inv44 + gmuc[i] * g.lam;
  double gs44 = vGv * inv44 * inv44;
  const double glam = gmuc[0] * g.v3[0] + gmuc[1] * g.v3[1] + gmuc[2] * g.v3[2];
  double gdt = glam * inv44;
  gs44 += -glam * g.lam * inv44;
  // p(t) = exp(-dt^2 / (2 S44))
  gdt += -gpt * g.pt * g.lam;
  gs44 += gpt * g.pt * 0.5 * g.lam * g.lam;
  // upper triangle of the symmetric dL/dSigma: (00 01 02 03 | 11 12 13 22 | 23 33)
  float4* o = geo + 4 * (size_t)d;
  o[0] = make_float4((float)gSc[0][0], (float)(0.5 * (gSc[0][1] + gSc[1][0])), (float)(0.5 * (gSc[0][2] + gSc[2][0])),
                     (float)(0.5 * gv3[0]));
  o[1] = make_float4((float)gSc[1][1], (float)(0.5 * (gSc[1][2] + gSc[2][1])), (float)(0.5 * gv3[1]), (float)gSc[2][2]);
  o[2] = make_float4((float)(0.5 * gv3[2]), (float)gs44, (float)gmuc[0], (float)gmuc[1]);
  o[3] = make_float4((float)gmuc[2], (float)-gdt, (float)glogit, blended ? (float)sqrt(gu * gu + gv * gv) : -1.f);
}

constexpr int kBwdColourViews = 8;  // views whose slots k_bwd_colour loads together

// The primitives active in some view of the call (the preprocess's list), a
// quad of lanes per primitive, lane `sub` owning the basis functions
// lm = 4 sub + i and reading and writing their coefficients and gradients
// straight from and to memory. Per active view it adds its share of
// dL/dcoeffs, and quad sums give the gradients through the view direction
// and through t - mu_t. Each quad walks only its own active views (the k-th
// of them in round k), so a wave takes as many rounds as its busiest
// primitive has active views. A primitive with a non-finite coefficient was
// rendered transparent: it gets zero gradients.
// Three waves per SIMD (at most 168 VGPRs, a few spilled values) rather than
// the two its 178 registers allow: it streams every listed primitive's
// coefficients in and their gradients out.
__global__ void __launch_bounds__(256, 3) k_bwd_colour(RenderParams p, const int32_t* __restrict__ slot,
                                                     const float4* __restrict__ colbuf, float4* __restrict__ cgbuf,
                                                     float* __restrict__ g_coeffs, bool accumulate) {
  const int nb = (p.sh_degree + 1) * (p.sh_degree + 1);
  const int nt = p.t_order + 1;
  const int K3 = nt * nb * 3;
  const uint32_t count = *p.plist_n;
  const int sub = threadIdx.x & 3;
  const uint32_t stride = (gridDim.x * blockDim.x) >> 2;
  for (uint32_t e0 = ((blockIdx.x * blockDim.x) >> 2); e0 < count; e0 += stride) {
    const uint32_t e = e0 + (threadIdx.x >> 2);
    const bool live = e < count;  // uniform per quad
    const int gidx = live ? (int)p.plist[e] : 0;
    float k[3][kBasisPerLane][3], gk[3][kBasisPerLane][3];
    if (live) load_own_coeffs(p.coeffs + (size_t)gidx * K3, sub, nb, nt, k);
    bool finite = true;
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
      for (int i = 0; i < kBasisPerLane; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!live) k[n][i][c] = 0.f;
          finite = finite && isfinite(k[n][i][c]);
          gk[n][i][c] = 0.f;
        }
    const bool bad = quad_any(!finite);
    for (int v0 = 0; v0 < p.n_views; v0 += kBwdColourViews) {
      int ds[kBwdColourViews];
      uint32_t m = 0u;
#pragma unroll
      for (int w = 0; w < kBwdColourViews; ++w) {
        ds[w] = (live && v0 + w < p.n_views) ? slot[(size_t)(v0 + w) * p.n + gidx] : -1;
        m |= (ds[w] >= 0 ? 1u : 0u) << w;
      }
      // rounds: the most active views of a primitive in this wave
      uint32_t rounds = (uint32_t)__popc(m);
#pragma unroll
      for (int off = 4; off < 64; off <<= 1) rounds = max(rounds, (uint32_t)__shfl_xor((int)rounds, off, 64));
      for (uint32_t r = 0; r < rounds; ++r) {
        // this quad's next active view
        const int w = m ? __ffs(m) - 1 : -1;
        m &= m - 1u;
        int d = -1;
#pragma unroll
        for (int ww = 0; ww < kBwdColourViews; ++ww) d = (ww == w) ? ds[ww] : d;
        if (d < 0) continue;  // uniform per quad
        if (bad) {
          if (sub == 0) cgbuf[d] = make_float4(0.f, 0.f, 0.f, 0.f);
          continue;
        }
        const float4 c0v = colbuf[2 * (size_t)d];
        const float4 c1 = colbuf[2 * (size_t)d + 1];
        const float graw[3] = {c0v.x, c0v.y, c0v.z};
        const float dt = c0v.w;
        float Y[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) Y[jj] = 0.f;
        sh_eval(p.sh_degree, c1.x, c1.y, c1.z, Y);
        float y[kBasisPerLane];
        own_basis(Y, sub, y);
        float cs[3], sn[3];
        fourier_terms(p.t_order, dt, p.t_period, cs, sn);
        // kd[n][i] = sum_ch graw_ch k[n][i][ch]; gy[i] = sum_n cs_n kd[n][i]
        float kd[3][kBasisPerLane], gy[kBasisPerLane];
#pragma unroll
        for (int i = 0; i < kBasisPerLane; ++i) {
          gy[i] = 0.f;
#pragma unroll
          for (int n = 0; n < 3; ++n) {
            kd[n][i] = fmaf(graw[0], k[n][i][0], fmaf(graw[1], k[n][i][1], graw[2] * k[n][i][2]));
            gy[i] = fmaf(cs[n], kd[n][i], gy[i]);
#pragma unroll
            for (int c = 0; c < 3; ++c) gk[n][i][c] = fmaf(cs[n] * y[i], graw[c], gk[n][i][c]);
          }
        }
        // gradient of this lane's basis functions in the view direction
        float gY[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) gY[jj] = (sub == jj / kBasisPerLane) ? gy[jj % kBasisPerLane] : 0.f;
        float gdx, gdy, gdz;
        sh_grad(p.sh_degree, c1.x, c1.y, c1.z, gY, gdx, gdy, gdz);
        gdx = quad_sum(gdx);
        gdy = quad_sum(gdy);
        gdz = quad_sum(gdz);
        // d/d(dt) cos(2 pi n dt / T) = -(2 pi n / T) sin(2 pi n dt / T)
        float gdt = 0.f;
#pragma unroll
        for (int n = 1; n < 3; ++n) {
          float gcos = 0.f;
#pragma unroll
          for (int i = 0; i < kBasisPerLane; ++i) gcos = fmaf(y[i], kd[n][i], gcos);
          gcos = quad_sum(gcos);
          gdt = fmaf(gcos, -2.f * kPi * n / p.t_period * sn[n], gdt);
        }
        if (sub == 0) {
          const float dd = gdx * c1.x + gdy * c1.y + gdz * c1.z;
          cgbuf[d] = make_float4((gdx - c1.x * dd) * c1.w, (gdy - c1.y * dd) * c1.w, (gdz - c1.z * dd) * c1.w, gdt);
        }
      }
    }
    if (live) store_own_coeffs(g_coeffs + (size_t)gidx * K3, sub, nb, nt, gk, accumulate);
  }
}

// Zero coefficient gradients of the primitives active in no view of the call
// (the listed ones are written by k_bwd_colour), coalesced over all of them:
// 16-byte stores when a primitive's K3 floats are whole 16-byte pieces.
__global__ void __launch_bounds__(256) k_zero_inactive_coeffs(RenderParams p, float* __restrict__ g_coeffs) {
  const uint32_t K3 = (uint32_t)((p.t_order + 1) * (p.sh_degree + 1) * (p.sh_degree + 1) * 3);
  const bool vec = (K3 & 3u) == 0u && (reinterpret_cast<uintptr_t>(g_coeffs) & 15u) == 0u;
  const uint32_t per = vec ? K3 >> 2 : K3;  // pieces per primitive
  const uint32_t total = (uint32_t)p.n * per;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    if (p.pany[i / per]) continue;
    if (vec) reinterpret_cast<float4*>(g_coeffs)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    else g_coeffs[i] = 0.f;
  }
}

// Three waves per SIMD (at most 168 VGPRs, a few spilled values) rather than
// the two its 174 registers allow: it streams every primitive's parameters in
// and their gradients out.
__global__ void __launch_bounds__(128, 3) k_bwd_prims(RenderParams p, const int32_t* __restrict__ slot,
                                                   const float4* __restrict__ geo, const float4* __restrict__ cgbuf,
                                                   float4* __restrict__ g_means4, float4* __restrict__ g_log_scales4,
                                                   float4* __restrict__ g_q_left, float4* __restrict__ g_q_right,
                                                   float* __restrict__ g_logit, bool accumulate,
                                                   DensifyStats st) {
  const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (gidx >= p.n) return;
  if (!p.pany[gidx]) {
    if (accumulate) return;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    g_means4[gidx] = z;
    g_log_scales4[gidx] = z;
    g_q_left[gidx] = z;
    g_q_right[gidx] = z;
    g_logit[gidx] = 0.f;
    return;
  }
  const float4 mu = p.means4[gidx];
  Shape4T<double> sh;
  build_shape<double>(p.q_left[gidx], p.q_right[gidx], p.log_scales4[gidx], sh);
  const double s44 = sh.S[3][3], inv44 = 1.0 / s44;
  const double v3[3] = {sh.S[0][3], sh.S[1][3], sh.S[2][3]};

  double G4[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) G4[i][j] = 0.0;
  double gmu[4] = {0.0, 0.0, 0.0, 0.0};
  double glogit = 0.0;
  float st_uv = 0.f, st_t = 0.f;
  int st_n = 0;
  for (int vi = 0; vi < p.n_views; ++vi) {
    const int d = slot[(size_t)vi * p.n + gidx];
    if (d < 0) continue;
    const float4 a = geo[4 * (size_t)d], b = geo[4 * (size_t)d + 1], c = geo[4 * (size_t)d + 2];
    const float4 e = geo[4 * (size_t)d + 3];
    G4[0][0] += a.x; G4[0][1] += a.y; G4[0][2] += a.z; G4[0][3] += a.w;
    G4[1][1] += b.x; G4[1][2] += b.y; G4[1][3] += b.z; G4[2][2] += b.w;
    G4[2][3] += c.x; G4[3][3] += c.y;
    gmu[0] += c.z; gmu[1] += c.w; gmu[2] += e.x; gmu[3] += e.y;
    glogit += e.z;
    // colour part through the slice: mu_c = mu_xyz + v lam, lam = (t - mu_t) / S44
    const float4 cg = cgbuf[d];
    const double lam = ((double)p.views[vi].t - (double)mu.w) * inv44;
    const double glam = cg.x * v3[0] + cg.y * v3[1] + cg.z * v3[2];
    gmu[0] += cg.x; gmu[1] += cg.y; gmu[2] += cg.z;
    G4[0][3] += 0.5 * cg.x * lam;
    G4[1][3] += 0.5 * cg.y * lam;
    G4[2][3] += 0.5 * cg.z * lam;
    G4[3][3] += -glam * lam * inv44;
    const double gmt_col = -(glam * inv44 + cg.w);
    gmu[3] += gmt_col;
    if (e.w >= 0.f) {  // blended in this view: densification statistics (Sec. 3.3)
      st_uv += e.w;
      st_t += (float)fabs(e.y + gmt_col);
      ++st_n;
    }
  }
  if (st.blend_count && st_n) {
    st.uv_grad_norm_sum[gidx] += st_uv;
    st.t_grad_abs_sum[gidx] += st_t;
    st.blend_count[gidx] += st_n;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) G4[i][j] = G4[j][i];

  // ---- Sigma = M M^T, M = R S:  g_M = 2 G4 M ----
  double gR[4][4], gs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double gm = 2.0 * (G4[i][0] * sh.M[0][k] + G4[i][1] * sh.M[1][k] + G4[i][2] * sh.M[2][k] +
                               G4[i][3] * sh.M[3][k]);
      gR[i][k] = gm * sh.s[k];
      gs[k] = fma(gm, sh.R[i][k], gs[k]);
    }
  // ---- R = L Rr:  g_L = g_R Rr^T,  g_Rr = L^T g_R ----
  double L[4][4], Rr[4][4], gL[4][4], gRr[4][4];
  isoclinic_left<double>(sh.ql[0], sh.ql[1], sh.ql[2], sh.ql[3], L);
  isoclinic_right<double>(sh.qr[0], sh.qr[1], sh.qr[2], sh.qr[3], Rr);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a = fma(gR[i][k], Rr[j][k], a);
        b = fma(L[k][i], gR[k][j], b);
      }
      gL[i][j] = a;
      gRr[i][j] = b;
    }
  // matrix-entry gradients to quaternion components (sign patterns of the two matrices)
  double gql[4], gqr[4];
  gql[0] = gL[0][0] + gL[1][1] + gL[2][2] + gL[3][3];
  gql[1] = -gL[0][1] + gL[1][0] - gL[2][3] + gL[3][2];
  gql[2] = -gL[0][2] + gL[1][3] + gL[2][0] - gL[3][1];
  gql[3] = -gL[0][3] - gL[1][2] + gL[2][1] + gL[3][0];
  gqr[0] = gRr[0][0] + gRr[1][1] + gRr[2][2] + gRr[3][3];
  gqr[1] = -gRr[0][1] + gRr[1][0] + gRr[2][3] - gRr[3][2];
  gqr[2] = -gRr[0][2] - gRr[1][3] + gRr[2][0] + gRr[3][1];
  gqr[3] = -gRr[0][3] + gRr[1][2] - gRr[2][1] + gRr[3][0];
  // normalisation q_hat = q / |q|
  const double dl = gql[0] * sh.ql[0] + gql[1] * sh.ql[1] + gql[2] * sh.ql[2] + gql[3] * sh.ql[3];
  const double dr = gqr[0] * sh.qr[0] + gqr[1] * sh.qr[1] + gqr[2] * sh.qr[2] + gqr[3] * sh.qr[3];
  float4 o_ql = make_float4((float)((gql[0] - sh.ql[0] * dl) * sh.inl), (float)((gql[1] - sh.ql[1] * dl) * sh.inl),
                            (float)((gql[2] - sh.ql[2] * dl) * sh.inl), (float)((gql[3] - sh.ql[3] * dl) * sh.inl));
  float4 o_qr = make_float4((float)((gqr[0] - sh.qr[0] * dr) * sh.inr), (float)((gqr[1] - sh.qr[1] * dr) * sh.inr),
                            (float)((gqr[2] - sh.qr[2] * dr) * sh.inr), (float)((gqr[3] - sh.qr[3] * dr) * sh.inr));
  float4 o_ls = make_float4((float)(gs[0] * sh.s[0]), (float)(gs[1] * sh.s[1]), (float)(gs[2] * sh.s[2]),
                            (float)(gs[3] * sh.s[3]));
  float4 o_mu = make_float4((float)gmu[0], (float)gmu[1], (float)gmu[2], (float)gmu[3]);
  float o_logit = (float)glogit;
  if (accumulate) {
    const float4 a = g_q_left[gidx], b = g_q_right[gidx], c = g_log_scales4[gidx], d = g_means4[gidx];
    o_ql = make_float4(o_ql.x + a.x, o_ql.y + a.y, o_ql.z + a.z, o_ql.w + a.w);
    o_qr = make_float4(o_qr.x + b.x, o_qr.y + b.y, o_qr.z + b.z, o_qr.w + b.w);
    o_ls = make_float4(o_ls.x + c.x, o_ls.y + c.y, o_ls.z + c.z, o_ls.w + c.w);
    o_mu = make_float4(o_mu.x + d.x, o_mu.y + d.y, o_mu.z + d.z, o_mu.w + d.w);
    o_logit += g_logit[gidx];
  }
  g_q_left[gidx] = o_ql;
  g_q_right[gidx] = o_qr;
  g_log_scales4[gidx] = o_ls;
  g_means4[gidx] = o_mu;
  g_logit[gidx] = o_logit;
}

}  // namespace

size_t preprocess_backward_scratch_floats(size_t n_records) {
  return n_records * (kGeoFloats + kColFloats + kCgFloats);
}

void launch_preprocess_backward(const RenderParams& p, const int32_t* slot, const double* grad2d,
                                const uint32_t* n_records_dev, uint32_t n_records_max, const uint32_t* ids,
                                const Record* recs, float* scratch, float* g_means4, float* g_log_scales4,
                                float* g_q_left, float* g_q_right, float* g_opacity_logit, float* g_coeffs,
                                bool accumulate, const DensifyStats& stats, hipStream_t s) {
  if (p.n == 0) return;
  float4* geo = reinterpret_cast<float4*>(scratch);
  float4* col = reinterpret_cast<float4*>(scratch + (size_t)n_records_max * kGeoFloats);
  float4* cg = reinterpret_cast<float4*>(scratch + (size_t)n_records_max * (kGeoFloats + kColFloats));
  if (n_records_max > 0)
    hipLaunchKernelGGL(k_bwd_pairs, dim3((n_records_max + 255) / 256), dim3(256), 0, s, p, n_records_dev,
                       n_records_max, ids, recs, grad2d, geo, col);
  if (!accumulate) {
    const uint64_t total = (uint64_t)p.n * (p.t_order + 1) * (p.sh_degree + 1) * (p.sh_degree + 1) * 3;
    const uint64_t g = (total + 255) / 256;
    hipLaunchKernelGGL(k_zero_inactive_coeffs, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, s, p, g_coeffs);
  }
  hipLaunchKernelGGL(k_bwd_colour, dim3(list_grid(p.n)), dim3(256), 0, s, p, slot, col, cg, g_coeffs, accumulate);
  hipLaunchKernelGGL(k_bwd_prims, dim3((p.n + 127) / 128), dim3(128), 0, s, p, slot, geo, cg,
                     reinterpret_cast<float4*>(g_means4), reinterpret_cast<float4*>(g_log_scales4),
                     reinterpret_cast<float4*>(g_q_left), reinterpret_cast<float4*>(g_q_right), g_opacity_logit,
                     accumulate, stats);
}

}  // namespace g4d
