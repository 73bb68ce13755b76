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

// R = L(ql) R(qr) for unit quaternions, the two matrices of Sec. 3.2
// (written once, for float and double).
template <typename T>
__device__ __forceinline__ void isoclinic_left(T a, T b, T c, T d, T L[4][4]) {
  L[0][0] = a;  L[0][1] = -b; L[0][2] = -c; L[0][3] = -d;
  L[1][0] = b;  L[1][1] = a;  L[1][2] = -d; L[1][3] = c;
  L[2][0] = c;  L[2][1] = d;  L[2][2] = a;  L[2][3] = -b;
  L[3][0] = d;  L[3][1] = -c; L[3][2] = b;  L[3][3] = a;
}
template <typename T>
__device__ __forceinline__ void isoclinic_right(T p, T qq, T r, T s, T Rr[4][4]) {
  Rr[0][0] = p;  Rr[0][1] = -qq; Rr[0][2] = -r;  Rr[0][3] = -s;
  Rr[1][0] = qq; Rr[1][1] = p;   Rr[1][2] = s;   Rr[1][3] = -r;
  Rr[2][0] = r;  Rr[2][1] = -s;  Rr[2][2] = p;   Rr[2][3] = qq;
  Rr[3][0] = s;  Rr[3][1] = r;   Rr[3][2] = -qq; Rr[3][3] = p;
}
__device__ __forceinline__ void isoclinic_left(float4 q, float L[4][4]) { isoclinic_left(q.x, q.y, q.z, q.w, L); }
__device__ __forceinline__ void isoclinic_right(float4 q, float Rr[4][4]) { isoclinic_right(q.x, q.y, q.z, q.w, Rr); }

__device__ __forceinline__ float4 normalize4(float4 q, float& inv_norm) {
  inv_norm = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  return make_float4(q.x * inv_norm, q.y * inv_norm, q.z * inv_norm, q.w * inv_norm);
}

// Scalar helpers for the geometry, written once for float and double (the
// per-primitive forward and backward chains run in FP64, see k_preprocess).
__device__ __forceinline__ float sc_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double sc_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float sc_exp(float x) { return __expf(x); }
__device__ __forceinline__ double sc_exp(double x) { return exp(x); }
__device__ __forceinline__ float sc_rsqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double sc_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sc_abs(float x) { return fabsf(x); }
__device__ __forceinline__ double sc_abs(double x) { return fabs(x); }
__device__ __forceinline__ float sc_clamp(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }
__device__ __forceinline__ double sc_clamp(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

// A quaternion normalised in precision T; inv_norm = 1 / |q|.
template <typename T>
__device__ __forceinline__ void normalize_q(float4 q, T out[4], T& inv_norm) {
  const T a = q.x, b = q.y, c = q.z, d = q.w;
  inv_norm = sc_rsqrt(a * a + b * b + c * c + d * d);
  out[0] = a * inv_norm; out[1] = b * inv_norm; out[2] = c * inv_norm; out[3] = d * inv_norm;
}

// View-independent part: unit quaternions, rotation, scaled rotation M = R S
// and Sigma = M M^T.
template <typename T>
struct Shape4T {
  T ql[4], qr[4], inl, inr;
  T R[4][4];
  T s[4];
  T M[4][4];
  T S[4][4];  // symmetric
  T inv44;    // 1 / Sigma_44
};
using Shape4 = Shape4T<float>;

template <typename T>
__device__ __forceinline__ void build_shape(float4 qlf, float4 qrf, float4 ls, Shape4T<T>& sh) {
  normalize_q<T>(qlf, sh.ql, sh.inl);
  normalize_q<T>(qrf, sh.qr, sh.inr);
  T L[4][4], Rr[4][4];
  isoclinic_left<T>(sh.ql[0], sh.ql[1], sh.ql[2], sh.ql[3], L);
  isoclinic_right<T>(sh.qr[0], sh.qr[1], sh.qr[2], sh.qr[3], Rr);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = sc_fma(L[i][k], Rr[k][j], acc);
      sh.R[i][j] = acc;
    }
  sh.s[0] = sc_exp((T)ls.x); sh.s[1] = sc_exp((T)ls.y); sh.s[2] = sc_exp((T)ls.z); sh.s[3] = sc_exp((T)ls.w);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh.M[i][k] = sh.R[i][k] * sh.s[k];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i; j < 4; ++j) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = sc_fma(sh.M[i][k], sh.M[j][k], acc);
      sh.S[i][j] = acc;
      sh.S[j][i] = acc;
    }
  sh.inv44 = (T)1 / sh.S[3][3];
}

// Everything one view needs from a primitive.
template <typename T>
struct ViewGeomT {
  T dt, s44, pt, lam;
  T v3[3];      // Sigma_{xyz,t}
  T muc[3];     // conditional mean
  T Sc[3][3];   // conditional covariance
  T pc[3];      // camera-space mean
  T iz;
  bool clx, cly;  // Jacobian clamps taken
  T xi, eta;
  T T_[2][3];   // J W
  T a2, b2, c2, det;
  T conic[3];
  T u, v;
  T dir[3], rinv;
};

// Jacobian clamp limits on x/z, y/z: 1.3x the half field of view.
__device__ __forceinline__ void clamp_limits(const ViewDev& vw, float& lx, float& ly) {
  lx = vw.lim_x;
  ly = vw.lim_y;
}
__device__ __forceinline__ void clamp_limits(const ViewDev& vw, double& lx, double& ly) {
  lx = vw.lim_x64;
  ly = vw.lim_y64;
}

// Slice, camera transform and EWA projection (Sec. 3.2, Eqs. 3-4) in
// precision T. Returns false when culled by the temporal filter or the near
// plane (then only dt, s44 and pt are set).
template <typename T>
__device__ __forceinline__ bool view_geometry(const float4 mu, const Shape4T<T>& sh, const ViewDev& vw, T t_cull,
                                              T near_plane, ViewGeomT<T>& g) {
  g.dt = (T)vw.t - (T)mu.w;
  g.s44 = sh.S[3][3];
  const T inv44 = sh.inv44;
  g.pt = sc_exp((T)-0.5 * g.dt * g.dt * inv44);
  if (!(g.pt >= t_cull)) return false;
  g.lam = g.dt * inv44;
  g.v3[0] = sh.S[0][3]; g.v3[1] = sh.S[1][3]; g.v3[2] = sh.S[2][3];
  g.muc[0] = sc_fma(g.v3[0], g.lam, (T)mu.x);
  g.muc[1] = sc_fma(g.v3[1], g.lam, (T)mu.y);
  g.muc[2] = sc_fma(g.v3[2], g.lam, (T)mu.z);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) g.Sc[i][j] = sh.S[i][j] - g.v3[i] * g.v3[j] * inv44;
  T W[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) W[k] = vw.rot[k];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    g.pc[i] = sc_fma(W[3 * i + 0], g.muc[0],
                     sc_fma(W[3 * i + 1], g.muc[1], sc_fma(W[3 * i + 2], g.muc[2], (T)vw.trans[i])));
  if (!(g.pc[2] > near_plane)) return false;
  g.iz = (T)1 / g.pc[2];
  const T fx = vw.fx, fy = vw.fy;
  const T x = g.pc[0], y = g.pc[1];
  g.u = sc_fma(fx * x, g.iz, (T)vw.cx);
  g.v = sc_fma(fy * y, g.iz, (T)vw.cy);
  T lim_x, lim_y;
  clamp_limits(vw, lim_x, lim_y);
  const T xz = x * g.iz, yz = y * g.iz;
  g.clx = sc_abs(xz) > lim_x;
  g.cly = sc_abs(yz) > lim_y;
  g.xi = sc_clamp(xz, -lim_x, lim_x);
  g.eta = sc_clamp(yz, -lim_y, lim_y);
  // J = [[fx/z, 0, -fx xi/z], [0, fy/z, -fy eta/z]]; T = J W
  const T j00 = fx * g.iz, j02 = -fx * g.xi * g.iz;
  const T j11 = fy * g.iz, j12 = -fy * g.eta * g.iz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.T_[0][k] = sc_fma(j00, W[k], j02 * W[6 + k]);
    g.T_[1][k] = sc_fma(j11, W[3 + k], j12 * W[6 + k]);
  }
  // Sigma_2d = T Sc T^T
  T TS[2][3];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      TS[r][k] = sc_fma(g.T_[r][0], g.Sc[0][k], sc_fma(g.T_[r][1], g.Sc[1][k], g.T_[r][2] * g.Sc[2][k]));
  const T s00 = sc_fma(TS[0][0], g.T_[0][0], sc_fma(TS[0][1], g.T_[0][1], TS[0][2] * g.T_[0][2]));
  const T s01 = sc_fma(TS[0][0], g.T_[1][0], sc_fma(TS[0][1], g.T_[1][1], TS[0][2] * g.T_[1][2]));
  const T s11 = sc_fma(TS[1][0], g.T_[1][0], sc_fma(TS[1][1], g.T_[1][1], TS[1][2] * g.T_[1][2]));
  const T lowpass = sizeof(T) == 8 ? (T)kLowpass64 : (T)kLowpass;
  g.a2 = s00 + lowpass;
  g.b2 = s01;
  g.c2 = s11 + lowpass;
  {  // a2 c2 - b2^2 without cancellation error (the b2^2 rounding error is recovered by an FMA)
    const T p = g.b2 * g.b2;
    g.det = sc_fma(g.a2, g.c2, -p) - sc_fma(g.b2, g.b2, -p);
  }
  const T idet = (T)1 / g.det;
  g.conic[0] = g.c2 * idet;
  g.conic[1] = -g.b2 * idet;
  g.conic[2] = g.a2 * idet;
  const T rx = g.muc[0] - (T)vw.center[0], ry = g.muc[1] - (T)vw.center[1], rz = g.muc[2] - (T)vw.center[2];
  g.rinv = sc_rsqrt(rx * rx + ry * ry + rz * rz);
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

// Sum over the four lanes of a DPP quad (quad_perm [1,0,3,2], then [2,3,0,1];
// every lane reads within its quad, so the bound control changes nothing, and
// with it set each move folds into its add).
__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
  return v;
}

// The colour kernels give each primitive one quad: lane `sub` owns the basis
// functions lm = 4 sub + i, i < kBasisPerLane, and their coefficients.
constexpr int kBasisPerLane = 4;

// Primitives per 256-thread block in the colour kernels (a quad each).
constexpr int kColourPrims = 64;

// The colour kernels give each listed primitive a quad; lane `sub` owns the
// basis functions lm = 4 sub + i, i < 4, and their coefficients:
// k[n][i][c] = g[(n nb + 4 sub + i) 3 + c] for Fourier term n < nt and
// basis function 4 sub + i < nb (zero elsewhere), g the primitive's
// [nt][nb][3] coefficients. At SH degree 3 (nb = 16) with g 16-byte aligned,
// a lane's 12 floats per term are three 16-byte pieces and the quad reads
// the term's 192 contiguous bytes together.
__device__ __forceinline__ void load_own_coeffs(const float* __restrict__ g, int sub, int nb, int nt,
                                                float (&k)[3][kBasisPerLane][3]) {
  if (nb == 16 && (reinterpret_cast<uintptr_t>(g) & 15u) == 0) {
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
      if (n < nt) {
        const float4* src = reinterpret_cast<const float4*>(g + n * 48 + 12 * sub);
        q0 = src[0];
        q1 = src[1];
        q2 = src[2];
      }
      k[n][0][0] = q0.x; k[n][0][1] = q0.y; k[n][0][2] = q0.z; k[n][1][0] = q0.w;
      k[n][1][1] = q1.x; k[n][1][2] = q1.y; k[n][2][0] = q1.z; k[n][2][1] = q1.w;
      k[n][2][2] = q2.x; k[n][3][0] = q2.y; k[n][3][1] = q2.z; k[n][3][2] = q2.w;
    }
    return;
  }
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int i = 0; i < kBasisPerLane; ++i) {
      const int lm = sub * kBasisPerLane + i;
#pragma unroll
      for (int c = 0; c < 3; ++c) k[n][i][c] = (lm < nb && n < nt) ? g[(n * nb + lm) * 3 + c] : 0.f;
    }
}

// The reverse for a lane's gradients: written to (or, when accumulate, added
// to) their places in g.
__device__ __forceinline__ void store_own_coeffs(float* __restrict__ g, int sub, int nb, int nt,
                                                 const float (&k)[3][kBasisPerLane][3], bool accumulate) {
  if (nb == 16 && (reinterpret_cast<uintptr_t>(g) & 15u) == 0) {
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      if (n >= nt) continue;
      float4* dst = reinterpret_cast<float4*>(g + n * 48 + 12 * sub);
      float4 q0 = make_float4(k[n][0][0], k[n][0][1], k[n][0][2], k[n][1][0]);
      float4 q1 = make_float4(k[n][1][1], k[n][1][2], k[n][2][0], k[n][2][1]);
      float4 q2 = make_float4(k[n][2][2], k[n][3][0], k[n][3][1], k[n][3][2]);
      if (accumulate) {
        const float4 o0 = dst[0], o1 = dst[1], o2 = dst[2];
        q0.x += o0.x; q0.y += o0.y; q0.z += o0.z; q0.w += o0.w;
        q1.x += o1.x; q1.y += o1.y; q1.z += o1.z; q1.w += o1.w;
        q2.x += o2.x; q2.y += o2.y; q2.z += o2.z; q2.w += o2.w;
      }
      dst[0] = q0;
      dst[1] = q1;
      dst[2] = q2;
    }
    return;
  }
#pragma unroll
  for (int n = 0; n < 3; ++n)
#pragma unroll
    for (int i = 0; i < kBasisPerLane; ++i) {
      const int lm = sub * kBasisPerLane + i;
      if (lm >= nb || n >= nt) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float* dst = g + (n * nb + lm) * 3 + c;
        *dst = accumulate ? *dst + k[n][i][c] : k[n][i][c];
      }
    }
}

// Whether b holds on some lane of this lane's quad (all four lanes active).
__device__ __forceinline__ bool quad_any(bool b) {
  const uint64_t m = __ballot(b);
  return ((m >> (threadIdx.x & 60u)) & 0xFull) != 0ull;
}

// y[i] = Y[4 sub + i] (selects with constant indices, no register indexing).
__device__ __forceinline__ void own_basis(const float* Y, int sub, float* y) {
#pragma unroll
  for (int i = 0; i < kBasisPerLane; ++i) y[i] = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) y[j % kBasisPerLane] = (sub == j / kBasisPerLane) ? Y[j] : y[j % kBasisPerLane];
}

// One value's image-loss term and its gradient (the paper supervises with a
// rendering loss only, Sec. 3.3): kind 1 is L1, |d| with gradient
// scale * sign(d); kind 2 is L2, d^2 with gradient 2 scale d; d = img - target.
__device__ __forceinline__ float loss_term(int kind, float d, float scale, float& g) {
  if (kind == 1) {
    g = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    return fabsf(d);
  }
  g = 2.f * scale * d;
  return d * d;
}

}  // namespace shade
}  // namespace g4d
