// Device helpers shared by the forward and backward per-primitive kernels:
// real SH basis and its gradient, the two isoclinic rotation matrices,
// covariance, and the per-view slice + EWA projection.
#pragma once

#include "g4d_common.h"

namespace g4d {
namespace shade {


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

// cos(2 pi n dt / T) and sin(2 pi n dt / T) for n = 0..t_order (<= 2): one
// sincospi, the second order by the double-angle identities.
__device__ __forceinline__ int fourier_terms(int t_order, float dt, float period, float* cs, float* sn = nullptr) {
  const float ph = 2.f * dt / period;  // cos(2 pi n dt / T) = cospi(n * ph)
  float s1 = 0.f, c1 = 1.f;
  if (t_order >= 1) sincospif(ph, &s1, &c1);
  cs[0] = 1.f;
  cs[1] = t_order >= 1 ? c1 : 0.f;
  cs[2] = t_order >= 2 ? fmaf(2.f * c1, c1, -1.f) : 0.f;
  if (sn) {
    sn[0] = 0.f;
    sn[1] = t_order >= 1 ? s1 : 0.f;
    sn[2] = t_order >= 2 ? 2.f * s1 * c1 : 0.f;
  }
  return t_order + 1;
}

// Sum over the four lanes of a DPP quad (quad_perm [1,0,3,2], then [2,3,0,1]).
__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  return v;
}

// The colour kernels give each primitive one quad: lane `sub` owns the basis
// functions lm = 4 sub + i, i < kBasisPerLane, and their coefficients.
constexpr int kBasisPerLane = 4;

// Primitives per 256-thread block in the colour kernels, and the LDS floats
// that stage their coefficients ([(Fourier term) (L+1)^2 + lm][3] each, at
// most 3 x 16 x 3).
constexpr int kColourPrims = 64;
constexpr int kCoeffMax = 3 * 16 * 3;

// Block copies of `count` floats between global memory and LDS (lds 16-byte
// aligned): 16 bytes per thread and step when g is 16-byte aligned, then
// single floats for the tail; single floats throughout otherwise.
__device__ __forceinline__ void copy_in(float* __restrict__ lds, const float* __restrict__ g, int count) {
  const int n4 = (reinterpret_cast<uintptr_t>(g) & 15u) ? 0 : count >> 2;
  for (int i = threadIdx.x; i < n4; i += blockDim.x)
    reinterpret_cast<float4*>(lds)[i] = reinterpret_cast<const float4*>(g)[i];
  for (int i = 4 * n4 + threadIdx.x; i < count; i += blockDim.x) lds[i] = g[i];
}

// g[i] = lds[i] (+ g[i] when accumulate).
__device__ __forceinline__ void copy_out(float* __restrict__ g, const float* __restrict__ lds, int count,
                                         bool accumulate) {
  const int n4 = (reinterpret_cast<uintptr_t>(g) & 15u) ? 0 : count >> 2;
  for (int i = threadIdx.x; i < n4; i += blockDim.x) {
    float4 v = reinterpret_cast<const float4*>(lds)[i];
    if (accumulate) {
      const float4 o = reinterpret_cast<const float4*>(g)[i];
      v.x += o.x; v.y += o.y; v.z += o.z; v.w += o.w;
    }
    reinterpret_cast<float4*>(g)[i] = v;
  }
  for (int i = 4 * n4 + threadIdx.x; i < count; i += blockDim.x) g[i] = accumulate ? g[i] + lds[i] : lds[i];
}

// y[i] = Y[4 sub + i] (selects with constant indices, no register indexing).
__device__ __forceinline__ void own_basis(const float* Y, int sub, float* y) {
#pragma unroll
  for (int i = 0; i < kBasisPerLane; ++i) y[i] = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) y[j % kBasisPerLane] = (sub == j / kBasisPerLane) ? Y[j] : y[j % kBasisPerLane];
}

}  // namespace shade
}  // namespace g4d
