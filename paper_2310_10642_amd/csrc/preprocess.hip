// Per-primitive stages of the 4D Gaussian render, forward and backward.
//
// Forward (one thread per primitive, looping over the views of a batch so the
// parameters are read once): 4D covariance Sigma = R S S^T R^T with
// R = L(q_l) R(q_r) (Sec. 3.2, "Representation of 4D Gaussian"), temporal
// marginal and filter (Sec. 3.2 and Sec. 4.2), conditional 3D Gaussian at t
// (Sec. 3.2), EWA projection (Eqs. 3-4), footprint and tile rectangle, and the
// 4D spherindrical-harmonic colour (Sec. 3.2). Backward: the chain rule of
// the same steps from the per-record 2D gradients to every parameter.
#include "g4d_common.h"

namespace g4d {
namespace {

constexpr float kPi = 3.14159265358979323846f;

// Real SH, orthonormal, Condon-Shortley phase kept, index l*l+l+m.
// Constants: sqrt(2) K_l^m Q_l^m with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
// and Q_l^m = P_l^m / (1-z^2)^{m/2}; polynomials valid on the unit sphere.
constexpr float SH_C0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float SH_C1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float SH_C2a = 1.09254843059207907f;  // sqrt(15/(4 pi))
constexpr float SH_C2b = 0.31539156525252005f;  // sqrt(5/(16 pi))
constexpr float SH_C2c = 0.54627421529603959f;  // sqrt(15/(16 pi))
constexpr float SH_C3a = 0.59004358992664352f;  // sqrt(35/(32 pi))
constexpr float SH_C3b = 2.89061144264055405f;  // sqrt(105/(4 pi))
constexpr float SH_C3c = 0.45704579946446573f;  // sqrt(21/(32 pi))
constexpr float SH_C3d = 0.37317633259011540f;  // sqrt(7/(16 pi))
constexpr float SH_C3e = 1.44530572132027738f;  // sqrt(105/(16 pi))

__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float* Y) {
  Y[0] = SH_C0;
  if (deg < 1) return;
  Y[1] = -SH_C1 * y;
  Y[2] = SH_C1 * z;
  Y[3] = -SH_C1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SH_C2a * x * y;
  Y[5] = -SH_C2a * y * z;
  Y[6] = SH_C2b * (3.f * zz - 1.f);
  Y[7] = -SH_C2a * x * z;
  Y[8] = SH_C2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -SH_C3a * y * (3.f * xx - yy);
  Y[10] = SH_C3b * x * y * z;
  Y[11] = -SH_C3c * y * (5.f * zz - 1.f);
  Y[12] = SH_C3d * z * (5.f * zz - 3.f);
  Y[13] = -SH_C3c * x * (5.f * zz - 1.f);
  Y[14] = SH_C3e * z * (xx - yy);
  Y[15] = -SH_C3a * x * (xx - 3.f * yy);
}

// Accumulates sum_k gY[k] * grad Y_k(x, y, z) into (gx, gy, gz).
__device__ __forceinline__ void sh_grad(int deg, float x, float y, float z, const float* gY, float& gx,
                                        float& gy, float& gz) {
  gx = 0.f; gy = 0.f; gz = 0.f;
  if (deg < 1) return;
  gy += -SH_C1 * gY[1];
  gz += SH_C1 * gY[2];
  gx += -SH_C1 * gY[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += SH_C2a * y * gY[4];  gy += SH_C2a * x * gY[4];
  gy += -SH_C2a * z * gY[5]; gz += -SH_C2a * y * gY[5];
  gz += 6.f * SH_C2b * z * gY[6];
  gx += -SH_C2a * z * gY[7]; gz += -SH_C2a * x * gY[7];
  gx += 2.f * SH_C2c * x * gY[8]; gy += -2.f * SH_C2c * y * gY[8];
  if (deg < 3) return;
  gx += -6.f * SH_C3a * x * y * gY[9];
  gy += -3.f * SH_C3a * (xx - yy) * gY[9];
  gx += SH_C3b * y * z * gY[10]; gy += SH_C3b * x * z * gY[10]; gz += SH_C3b * x * y * gY[10];
  gy += -SH_C3c * (5.f * zz - 1.f) * gY[11]; gz += -10.f * SH_C3c * y * z * gY[11];
  gz += SH_C3d * (15.f * zz - 3.f) * gY[12];
  gx += -SH_C3c * (5.f * zz - 1.f) * gY[13]; gz += -10.f * SH_C3c * x * z * gY[13];
  gx += 2.f * SH_C3e * x * z * gY[14]; gy += -2.f * SH_C3e * y * z * gY[14]; gz += SH_C3e * (xx - yy) * gY[14];
  gx += -3.f * SH_C3a * (xx - yy) * gY[15]; gy += 6.f * SH_C3a * x * y * gY[15];
}

// R = L(ql) R(qr) for unit quaternions, the two matrices of Sec. 3.2.
__device__ __forceinline__ void isoclinic_left(float4 q, float L[4][4]) {
  const float a = q.x, b = q.y, c = q.z, d = q.w;
  L[0][0] = a;  L[0][1] = -b; L[0][2] = -c; L[0][3] = -d;
  L[1][0] = b;  L[1][1] = a;  L[1][2] = -d; L[1][3] = c;
  L[2][0] = c;  L[2][1] = d;  L[2][2] = a;  L[2][3] = -b;
  L[3][0] = d;  L[3][1] = -c; L[3][2] = b;  L[3][3] = a;
}
__device__ __forceinline__ void isoclinic_right(float4 q, float Rr[4][4]) {
  const float p = q.x, qq = q.y, r = q.z, s = q.w;
  Rr[0][0] = p;  Rr[0][1] = -qq; Rr[0][2] = -r;  Rr[0][3] = -s;
  Rr[1][0] = qq; Rr[1][1] = p;   Rr[1][2] = s;   Rr[1][3] = -r;
  Rr[2][0] = r;  Rr[2][1] = -s;  Rr[2][2] = p;   Rr[2][3] = qq;
  Rr[3][0] = s;  Rr[3][1] = r;   Rr[3][2] = -qq; Rr[3][3] = p;
}

__device__ __forceinline__ float4 normalize4(float4 q, float& inv_norm) {
  inv_norm = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  return make_float4(q.x * inv_norm, q.y * inv_norm, q.z * inv_norm, q.w * inv_norm);
}

// View-independent part: rotation, scaled rotation M = R S and Sigma = M M^T.
struct Shape4 {
  float R[4][4];
  float s[4];
  float M[4][4];
  float S[4][4];  // symmetric
};

__device__ __forceinline__ void build_shape(float4 ql, float4 qr, float4 ls, Shape4& sh) {
  float L[4][4], Rr[4][4];
  isoclinic_left(ql, L);
  isoclinic_right(qr, Rr);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = fmaf(L[i][k], Rr[k][j], acc);
      sh.R[i][j] = acc;
    }
  sh.s[0] = __expf(ls.x); sh.s[1] = __expf(ls.y); sh.s[2] = __expf(ls.z); sh.s[3] = __expf(ls.w);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh.M[i][k] = sh.R[i][k] * sh.s[k];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i; j < 4; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = fmaf(sh.M[i][k], sh.M[j][k], acc);
      sh.S[i][j] = acc;
      sh.S[j][i] = acc;
    }
}

// Everything one view needs from a primitive, forward.
struct ViewGeom {
  float dt, s44, pt, lam;
  float v3[3];      // Sigma_{xyz,t}
  float muc[3];     // conditional mean
  float Sc[3][3];   // conditional covariance
  float pc[3];      // camera-space mean
  float iz;
  bool clx, cly;    // Jacobian clamps taken
  float xi, eta;
  float T[2][3];    // J W
  float a2, b2, c2, det;
  float conic[3];
  float u, v;
  float dir[3], rinv;
};

// Slice, camera transform and EWA projection. Returns false when culled by
// the temporal filter or the near plane.
__device__ __forceinline__ bool view_geometry(const float4 mu, const Shape4& sh, const ViewDev& vw, float t_cull,
                                              float near_plane, ViewGeom& g) {
  g.dt = vw.t - mu.w;
  g.s44 = sh.S[3][3];
  g.pt = __expf(-0.5f * g.dt * g.dt / g.s44);
  if (!(g.pt >= t_cull)) return false;
  g.lam = g.dt / g.s44;
  g.v3[0] = sh.S[0][3]; g.v3[1] = sh.S[1][3]; g.v3[2] = sh.S[2][3];
  g.muc[0] = fmaf(g.v3[0], g.lam, mu.x);
  g.muc[1] = fmaf(g.v3[1], g.lam, mu.y);
  g.muc[2] = fmaf(g.v3[2], g.lam, mu.z);
  const float inv44 = 1.f / g.s44;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) g.Sc[i][j] = sh.S[i][j] - g.v3[i] * g.v3[j] * inv44;
  const float* W = vw.rot;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    g.pc[i] = fmaf(W[3 * i + 0], g.muc[0], fmaf(W[3 * i + 1], g.muc[1], fmaf(W[3 * i + 2], g.muc[2], vw.trans[i])));
  if (!(g.pc[2] > near_plane)) return false;
  g.iz = 1.f / g.pc[2];
  const float x = g.pc[0], y = g.pc[1];
  g.u = fmaf(vw.fx * x, g.iz, vw.cx);
  g.v = fmaf(vw.fy * y, g.iz, vw.cy);
  const float xz = x * g.iz, yz = y * g.iz;
  g.clx = fabsf(xz) > vw.lim_x;
  g.cly = fabsf(yz) > vw.lim_y;
  g.xi = fminf(fmaxf(xz, -vw.lim_x), vw.lim_x);
  g.eta = fminf(fmaxf(yz, -vw.lim_y), vw.lim_y);
  // J = [[fx/z, 0, -fx xi/z], [0, fy/z, -fy eta/z]]; T = J W
  const float j00 = vw.fx * g.iz, j02 = -vw.fx * g.xi * g.iz;
  const float j11 = vw.fy * g.iz, j12 = -vw.fy * g.eta * g.iz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.T[0][k] = fmaf(j00, W[k], j02 * W[6 + k]);
    g.T[1][k] = fmaf(j11, W[3 + k], j12 * W[6 + k]);
  }
  // Sigma_2d = T Sc T^T
  float TS[2][3];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      TS[r][k] = fmaf(g.T[r][0], g.Sc[0][k], fmaf(g.T[r][1], g.Sc[1][k], g.T[r][2] * g.Sc[2][k]));
  const float s00 = fmaf(TS[0][0], g.T[0][0], fmaf(TS[0][1], g.T[0][1], TS[0][2] * g.T[0][2]));
  const float s01 = fmaf(TS[0][0], g.T[1][0], fmaf(TS[0][1], g.T[1][1], TS[0][2] * g.T[1][2]));
  const float s11 = fmaf(TS[1][0], g.T[1][0], fmaf(TS[1][1], g.T[1][1], TS[1][2] * g.T[1][2]));
  g.a2 = s00 + kLowpass;
  g.b2 = s01;
  g.c2 = s11 + kLowpass;
  {  // a2 c2 - b2^2 without cancellation error (the b2^2 rounding error is recovered by an FMA)
    const float p = g.b2 * g.b2;
    g.det = fmaf(g.a2, g.c2, -p) - fmaf(g.b2, g.b2, -p);
  }
  const float idet = 1.f / g.det;
  g.conic[0] = g.c2 * idet;
  g.conic[1] = -g.b2 * idet;
  g.conic[2] = g.a2 * idet;
  float rx = g.muc[0] - vw.center[0], ry = g.muc[1] - vw.center[1], rz = g.muc[2] - vw.center[2];
  g.rinv = rsqrtf(rx * rx + ry * ry + rz * rz);
  g.dir[0] = rx * g.rinv; g.dir[1] = ry * g.rinv; g.dir[2] = rz * g.rinv;
  return true;
}

__device__ __forceinline__ int fourier_terms(int t_order, float dt, float period, float* cs) {
  const float ph = 2.f * dt / period;  // cos(2 pi n dt / T) = cospi(n * ph)
#pragma unroll
  for (int n = 0; n <= 2; ++n)
    if (n <= t_order) cs[n] = (n == 0) ? 1.f : cospif(n * ph);
  return t_order + 1;
}

__global__ void __launch_bounds__(256) k_preprocess(RenderParams p, uint32_t* __restrict__ act,
                                                    uint32_t* __restrict__ dkey, Record* __restrict__ rec,
                                                    int32_t* __restrict__ slot) {
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
  const int nb = (p.sh_degree + 1) * (p.sh_degree + 1);
  const int K = (p.t_order + 1) * nb;
  const float* kc = p.coeffs + (size_t)gidx * K * 3;

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
    // 4D spherindrical harmonics colour
    float Y[16], cs[3];
    sh_eval(p.sh_degree, g.dir[0], g.dir[1], g.dir[2], Y);
    const int nt = fourier_terms(p.t_order, g.dt, p.t_period, cs);
    float col[3] = {0.f, 0.f, 0.f};
    for (int n = 0; n < nt; ++n) {
      float acc[3] = {0.f, 0.f, 0.f};
      const float* kn = kc + (size_t)n * nb * 3;
      for (int lm = 0; lm < nb; ++lm) {
        acc[0] = fmaf(kn[3 * lm + 0], Y[lm], acc[0]);
        acc[1] = fmaf(kn[3 * lm + 1], Y[lm], acc[1]);
        acc[2] = fmaf(kn[3 * lm + 2], Y[lm], acc[2]);
      }
      col[0] = fmaf(cs[n], acc[0], col[0]);
      col[1] = fmaf(cs[n], acc[1], col[1]);
      col[2] = fmaf(cs[n], acc[2], col[2]);
    }
    Record r;
    r.a = make_float4(g.u, g.v, g.pc[2], opa * g.pt);
    r.b = make_float4(g.conic[0], g.conic[1], g.conic[2], __uint_as_float((uint32_t)x0 | ((uint32_t)x1 << 16)));
    r.c = make_float4(fmaxf(col[0] + kColorOffset, 0.f), fmaxf(col[1] + kColorOffset, 0.f),
                      fmaxf(col[2] + kColorOffset, 0.f), __uint_as_float((uint32_t)y0 | ((uint32_t)y1 << 16)));
    rec[idx] = r;
    act[idx] = 1u;
    dkey[idx] = __float_as_uint(g.pc[2]);  // z > near > 0: bit order = numeric order
    slot[idx] = -1;
  }
}

// ---------------------------------------------------------------------------
// Backward: per primitive, sum over views of the chain rule from the record
// gradients (dL/du, dL/dv, dL/dconic, dL/d(opacity p), dL/drgb, dL/dz).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) k_preprocess_backward(
    RenderParams p, const int32_t* __restrict__ slot, const float* __restrict__ grad2d,
    float4* __restrict__ g_means4, float4* __restrict__ g_log_scales4, float4* __restrict__ g_q_left,
    float4* __restrict__ g_q_right, float* __restrict__ g_logit, float* __restrict__ g_coeffs, bool accumulate) {
  const int gidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (gidx >= p.n) return;
  const int nb = (p.sh_degree + 1) * (p.sh_degree + 1);
  const int K = (p.t_order + 1) * nb;
  float* gk = g_coeffs + (size_t)gidx * K * 3;

  bool any = false;
  for (int vi = 0; vi < p.n_views; ++vi) any |= slot[(size_t)vi * p.n + gidx] >= 0;
  if (!any) {
    if (accumulate) return;
    g_means4[gidx] = make_float4(0.f, 0.f, 0.f, 0.f);
    g_log_scales4[gidx] = make_float4(0.f, 0.f, 0.f, 0.f);
    g_q_left[gidx] = make_float4(0.f, 0.f, 0.f, 0.f);
    g_q_right[gidx] = make_float4(0.f, 0.f, 0.f, 0.f);
    g_logit[gidx] = 0.f;
    for (int f = 0; f < 3 * K; ++f) gk[f] = 0.f;
    return;
  }

  const float4 mu = p.means4[gidx];
  const float4 ls = p.log_scales4[gidx];
  float inl, inr;
  const float4 ql = normalize4(p.q_left[gidx], inl);
  const float4 qr = normalize4(p.q_right[gidx], inr);
  const float opa = 1.f / (1.f + __expf(-p.opacity_logit[gidx]));
  Shape4 sh;
  build_shape(ql, qr, ls, sh);
  const float* kc = p.coeffs + (size_t)gidx * K * 3;

  float G4[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) G4[i][j] = 0.f;
  float gmu[4] = {0.f, 0.f, 0.f, 0.f};
  float glogit = 0.f;
  bool wrote_k = accumulate;

  for (int vi = 0; vi < p.n_views; ++vi) {
    const int d = slot[(size_t)vi * p.n + gidx];
    if (d < 0) continue;
    const ViewDev& vw = p.views[vi];
    ViewGeom g;
    view_geometry(mu, sh, vw, p.t_cull, p.near_plane, g);
    const float* gr = grad2d + (size_t)d * 12;
    const float4 q0 = *reinterpret_cast<const float4*>(gr);
    const float4 q1 = *reinterpret_cast<const float4*>(gr + 4);
    const float4 q2 = *reinterpret_cast<const float4*>(gr + 8);
    const float gu = q0.x, gv = q0.y, gC0 = q0.z, gC1 = q0.w, gC2 = q1.x, go = q1.y;
    const float gcol[3] = {q1.z, q1.w, q2.x};
    const float gdepth = q2.y;

    // ---- colour (Sec. 3.2, 4DSH) ----
    float Y[16], cs[3], sn[3];
    sh_eval(p.sh_degree, g.dir[0], g.dir[1], g.dir[2], Y);
    const int nt = fourier_terms(p.t_order, g.dt, p.t_period, cs);
    const float ph = 2.f * g.dt / p.t_period;
    for (int n = 0; n < nt; ++n) sn[n] = (n == 0) ? 0.f : sinpif(n * ph);
    float raw[3] = {0.f, 0.f, 0.f};
    for (int n = 0; n < nt; ++n) {
      const float* kn = kc + (size_t)n * nb * 3;
      float acc[3] = {0.f, 0.f, 0.f};
      for (int lm = 0; lm < nb; ++lm) {
        acc[0] = fmaf(kn[3 * lm + 0], Y[lm], acc[0]);
        acc[1] = fmaf(kn[3 * lm + 1], Y[lm], acc[1]);
        acc[2] = fmaf(kn[3 * lm + 2], Y[lm], acc[2]);
      }
      raw[0] = fmaf(cs[n], acc[0], raw[0]);
      raw[1] = fmaf(cs[n], acc[1], raw[1]);
      raw[2] = fmaf(cs[n], acc[2], raw[2]);
    }
    float graw[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) graw[c] = (raw[c] + kColorOffset >= 0.f) ? gcol[c] : 0.f;
    float gY[16];
    for (int lm = 0; lm < nb; ++lm) gY[lm] = 0.f;
    float gdt = 0.f;
    for (int n = 0; n < nt; ++n) {
      const float* kn = kc + (size_t)n * nb * 3;
      float* gkn = gk + (size_t)n * nb * 3;
      float gcos = 0.f;
      for (int lm = 0; lm < nb; ++lm) {
        const float kd = fmaf(kn[3 * lm + 0], graw[0], fmaf(kn[3 * lm + 1], graw[1], kn[3 * lm + 2] * graw[2]));
        gY[lm] = fmaf(cs[n], kd, gY[lm]);
        gcos = fmaf(Y[lm], kd, gcos);
        const float b = cs[n] * Y[lm];
        if (wrote_k) {
          gkn[3 * lm + 0] += b * graw[0];
          gkn[3 * lm + 1] += b * graw[1];
          gkn[3 * lm + 2] += b * graw[2];
        } else {
          gkn[3 * lm + 0] = b * graw[0];
          gkn[3 * lm + 1] = b * graw[1];
          gkn[3 * lm + 2] = b * graw[2];
        }
      }
      // d/d(dt) cos(2 pi n dt / T) = -(2 pi n / T) sin(2 pi n dt / T)
      gdt = fmaf(gcos, -2.f * kPi * n / p.t_period * sn[n], gdt);
    }
    wrote_k = true;
    float gdir[3];
    sh_grad(p.sh_degree, g.dir[0], g.dir[1], g.dir[2], gY, gdir[0], gdir[1], gdir[2]);
    const float dd = gdir[0] * g.dir[0] + gdir[1] * g.dir[1] + gdir[2] * g.dir[2];
    float gmuc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) gmuc[i] = (gdir[i] - g.dir[i] * dd) * g.rinv;

    // ---- opacity * p(t) ----
    float gpt = go * opa;
    glogit = fmaf(go * g.pt, opa * (1.f - opa), glogit);

    // ---- conic -> Sigma_2d: G_S = -Q G_Q Q ----
    const float C0 = g.conic[0], C1 = g.conic[1], C2 = g.conic[2];
    const float h1 = 0.5f * gC1;
    const float X00 = C0 * gC0 + C1 * h1, X01 = C0 * h1 + C1 * gC2;
    const float X10 = C1 * gC0 + C2 * h1, X11 = C1 * h1 + C2 * gC2;
    const float G00 = -(X00 * C0 + X01 * C1);
    const float G01 = -(X00 * C1 + X01 * C2);
    const float G11 = -(X10 * C1 + X11 * C2);
    // ---- Sigma_2d = T Sc T^T:  g_Sc = T^T G T,  g_T = 2 G T Sc ----
    float GT[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      GT[0][k] = G00 * g.T[0][k] + G01 * g.T[1][k];
      GT[1][k] = G01 * g.T[0][k] + G11 * g.T[1][k];
    }
    float gSc[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) gSc[i][j] = g.T[0][i] * GT[0][j] + g.T[1][i] * GT[1][j];
    float gT[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gT[r][k] = 2.f * (GT[r][0] * g.Sc[0][k] + GT[r][1] * g.Sc[1][k] + GT[r][2] * g.Sc[2][k]);
    // ---- T = J W:  g_J = g_T W^T ----
    const float* W = vw.rot;
    const float gJ00 = gT[0][0] * W[0] + gT[0][1] * W[1] + gT[0][2] * W[2];
    const float gJ02 = gT[0][0] * W[6] + gT[0][1] * W[7] + gT[0][2] * W[8];
    const float gJ11 = gT[1][0] * W[3] + gT[1][1] * W[4] + gT[1][2] * W[5];
    const float gJ12 = gT[1][0] * W[6] + gT[1][1] * W[7] + gT[1][2] * W[8];
    // ---- camera-space point (x, y, z) ----
    const float x = g.pc[0], y = g.pc[1], iz = g.iz, iz2 = iz * iz;
    float gx = gu * vw.fx * iz;
    float gy = gv * vw.fy * iz;
    float gz = gdepth - gu * vw.fx * x * iz2 - gv * vw.fy * y * iz2;
    gz += -gJ00 * vw.fx * iz2 - gJ11 * vw.fy * iz2;
    if (g.clx) {
      gz += gJ02 * vw.fx * g.xi * iz2;
    } else {
      gx += -gJ02 * vw.fx * iz2;
      gz += 2.f * gJ02 * vw.fx * g.xi * iz2;
    }
    if (g.cly) {
      gz += gJ12 * vw.fy * g.eta * iz2;
    } else {
      gy += -gJ12 * vw.fy * iz2;
      gz += 2.f * gJ12 * vw.fy * g.eta * iz2;
    }
    // p_cam = W mu_c + w
#pragma unroll
    for (int i = 0; i < 3; ++i) gmuc[i] += W[i] * gx + W[3 + i] * gy + W[6 + i] * gz;

    // ---- slice: Sc = Sxyz - v v^T / S44, mu_c = mu_xyz + v lam ----
    const float inv44 = 1.f / g.s44;
    float Gv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Gv[i] = gSc[i][0] * g.v3[0] + gSc[i][1] * g.v3[1] + gSc[i][2] * g.v3[2];
    const float vGv = g.v3[0] * Gv[0] + g.v3[1] * Gv[1] + g.v3[2] * Gv[2];
    float gv3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) gv3[i] = -2.f * Gv[i] * inv44 + gmuc[i] * g.lam;
    float gs44 = vGv * inv44 * inv44;
    const float glam = gmuc[0] * g.v3[0] + gmuc[1] * g.v3[1] + gmuc[2] * g.v3[2];
    gdt += glam * inv44;
    gs44 += -glam * g.lam * inv44;
    // p(t) = exp(-dt^2 / (2 S44))
    gdt += -gpt * g.pt * g.lam;
    gs44 += gpt * g.pt * 0.5f * g.lam * g.lam;

#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j) G4[i][j] += 0.5f * (gSc[i][j] + gSc[j][i]);
      G4[i][3] += 0.5f * gv3[i];
      G4[3][i] += 0.5f * gv3[i];
      gmu[i] += gmuc[i];
    }
    G4[3][3] += gs44;
    gmu[3] += -gdt;
  }

  // ---- Sigma = M M^T, M = R S:  g_M = 2 G4 M ----
  float gR[4][4], gs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float gm = 2.f * (G4[i][0] * sh.M[0][k] + G4[i][1] * sh.M[1][k] + G4[i][2] * sh.M[2][k] +
                              G4[i][3] * sh.M[3][k]);
      gR[i][k] = gm * sh.s[k];
      gs[k] = fmaf(gm, sh.R[i][k], gs[k]);
    }
  // ---- R = L Rr:  g_L = g_R Rr^T,  g_Rr = L^T g_R ----
  float L[4][4], Rr[4][4], gL[4][4], gRr[4][4];
  isoclinic_left(ql, L);
  isoclinic_right(qr, Rr);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float a = 0.f, b = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a = fmaf(gR[i][k], Rr[j][k], a);
        b = fmaf(L[k][i], gR[k][j], b);
      }
      gL[i][j] = a;
      gRr[i][j] = b;
    }
  // matrix-entry gradients to quaternion components (sign patterns of the two matrices)
  float4 gql, gqr;
  gql.x = gL[0][0] + gL[1][1] + gL[2][2] + gL[3][3];
  gql.y = -gL[0][1] + gL[1][0] - gL[2][3] + gL[3][2];
  gql.z = -gL[0][2] + gL[1][3] + gL[2][0] - gL[3][1];
  gql.w = -gL[0][3] - gL[1][2] + gL[2][1] + gL[3][0];
  gqr.x = gRr[0][0] + gRr[1][1] + gRr[2][2] + gRr[3][3];
  gqr.y = -gRr[0][1] + gRr[1][0] + gRr[2][3] - gRr[3][2];
  gqr.z = -gRr[0][2] - gRr[1][3] + gRr[2][0] + gRr[3][1];
  gqr.w = -gRr[0][3] + gRr[1][2] - gRr[2][1] + gRr[3][0];
  // normalisation q_hat = q / |q|
  const float dl = gql.x * ql.x + gql.y * ql.y + gql.z * ql.z + gql.w * ql.w;
  const float dr = gqr.x * qr.x + gqr.y * qr.y + gqr.z * qr.z + gqr.w * qr.w;
  float4 o_ql = make_float4((gql.x - ql.x * dl) * inl, (gql.y - ql.y * dl) * inl, (gql.z - ql.z * dl) * inl,
                            (gql.w - ql.w * dl) * inl);
  float4 o_qr = make_float4((gqr.x - qr.x * dr) * inr, (gqr.y - qr.y * dr) * inr, (gqr.z - qr.z * dr) * inr,
                            (gqr.w - qr.w * dr) * inr);
  float4 o_ls = make_float4(gs[0] * sh.s[0], gs[1] * sh.s[1], gs[2] * sh.s[2], gs[3] * sh.s[3]);
  float4 o_mu = make_float4(gmu[0], gmu[1], gmu[2], gmu[3]);
  if (accumulate) {
    const float4 a = g_q_left[gidx], b = g_q_right[gidx], c = g_log_scales4[gidx], d = g_means4[gidx];
    o_ql = make_float4(o_ql.x + a.x, o_ql.y + a.y, o_ql.z + a.z, o_ql.w + a.w);
    o_qr = make_float4(o_qr.x + b.x, o_qr.y + b.y, o_qr.z + b.z, o_qr.w + b.w);
    o_ls = make_float4(o_ls.x + c.x, o_ls.y + c.y, o_ls.z + c.z, o_ls.w + c.w);
    o_mu = make_float4(o_mu.x + d.x, o_mu.y + d.y, o_mu.z + d.z, o_mu.w + d.w);
    glogit += g_logit[gidx];
  }
  g_q_left[gidx] = o_ql;
  g_q_right[gidx] = o_qr;
  g_log_scales4[gidx] = o_ls;
  g_means4[gidx] = o_mu;
  g_logit[gidx] = glogit;
}

}  // namespace

void launch_preprocess(const RenderParams& p, uint32_t* act, uint32_t* dkey, Record* rec, int32_t* slot,
                       hipStream_t s) {
  if (p.n == 0) return;
  const int bs = 256;
  hipLaunchKernelGGL(k_preprocess, dim3((p.n + bs - 1) / bs), dim3(bs), 0, s, p, act, dkey, rec, slot);
}

void launch_preprocess_backward(const RenderParams& p, const int32_t* slot, const float* grad2d, float* g_means4,
                                float* g_log_scales4, float* g_q_left, float* g_q_right, float* g_opacity_logit,
                                float* g_coeffs, bool accumulate, hipStream_t s) {
  if (p.n == 0) return;
  const int bs = 128;
  hipLaunchKernelGGL(k_preprocess_backward, dim3((p.n + bs - 1) / bs), dim3(bs), 0, s, p, slot, grad2d,
                     reinterpret_cast<float4*>(g_means4), reinterpret_cast<float4*>(g_log_scales4),
                     reinterpret_cast<float4*>(g_q_left), reinterpret_cast<float4*>(g_q_right), g_opacity_logit,
                     g_coeffs, accumulate);
}

}  // namespace g4d
