// Per-primitive stages of the 4D Gaussian render. k_preprocess (one thread
// per primitive, looping over the views of a batch so the parameters are
// read once): 4D covariance Sigma = R S S^T R^T with R = L(q_l) R(q_r)
// (Sec. 3.2, "Representation of 4D Gaussian"), temporal marginal and filter
// (Sec. 3.2 and Sec. 4.2), conditional 3D Gaussian at t (Sec. 3.2), EWA
// projection (Eqs. 3-4), footprint and tile rectangle -- and, for a flow
// render, the image-plane displacement of the conditional mean (Sec. 4.4).
// This geometry is evaluated in FP64 and every value a record holds is
// rounded to FP32 once, so a record differs from the exact value by that
// rounding alone and the cull, near-plane and rectangle decisions are those of
// the exact arithmetic.
// k_colour: the 4D spherindrical-harmonic colour (Sec. 3.2) of the active
// pairs, written into their depth-ordered records once the gather has placed
// them; it reads the coefficients of the primitives active in some view only.
// The backward is in preprocess_bwd.hip.
#include "shade.h"

namespace g4d {
namespace {

using namespace shade;

__device__ __forceinline__ bool finite4(float4 a) {
  return isfinite(a.x) && isfinite(a.y) && isfinite(a.z) && isfinite(a.w);
}

// One thread per primitive, looping over the views of the call (the FP64
// shape is built once); `lanes` adjacent threads may share a primitive's
// views (1 here: the FP64 shape would be built once per lane). The lanes of a
// primitive then agree whether it is active in some view; the first appends
// it to the list that the colour passes walk.
__global__ void __launch_bounds__(256) k_preprocess(RenderParams p, int lanes, uint32_t* __restrict__ act,
                                                    uint32_t* __restrict__ dkey, Record* __restrict__ rec,
                                                    int32_t* __restrict__ slot, float4* __restrict__ cdir) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int gidx = t / lanes, sub = t - gidx * lanes;
  const bool live = gidx < p.n;
  const int gi = live ? gidx : 0;
  const int vpl = (p.n_views + lanes - 1) / lanes;
  const int v0 = min(sub * vpl, p.n_views), v1 = min(v0 + vpl, p.n_views);
  const float4 mu = p.means4[gi];
  const float4 ls = p.log_scales4[gi];
  const float4 qlf = p.q_left[gi];
  const float4 qrf = p.q_right[gi];
  const float logit = p.opacity_logit[gi];
  // a primitive with a non-finite parameter is culled in every view (and counted)
  const bool bad = live && !(finite4(mu) && finite4(ls) && finite4(qlf) && finite4(qrf) && isfinite(logit));
  bool any = false;
  if (bad) {
    for (int vi = v0; vi < v1; ++vi) {
      const size_t idx = (size_t)vi * p.n + gidx;
      act[idx] = 0u;
      slot[idx] = -1;
      if (p.nonfinite) atomicAdd(p.nonfinite + vi, 1u);
    }
  } else if (live) {
    Shape4T<double> sh;
    build_shape<double>(qlf, qrf, ls, sh);
    const double opa = 1.0 / (1.0 + exp(-(double)logit));
    const double t_cull = p.t_cull, near = p.near_plane;
    for (int vi = v0; vi < v1; ++vi) {
      const size_t idx = (size_t)vi * p.n + gidx;
      const ViewDev& vw = p.views[vi];
      // temporal marginal and filter, slice, camera, EWA projection
      ViewGeomT<double> g;
      bool ok = view_geometry<double>(mu, sh, vw, t_cull, near, g);
      int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
      if (ok) {
        // ---- footprint: integer 3-sigma radius, half-open tile rectangle ----
        const double mid = 0.5 * (g.a2 + g.c2);
        const double lmax = mid + sqrt(fmax(mid * mid - g.det, 0.0));
        const double rad = ceil(kSigmaExtent64 * sqrt(lmax));
        const double tx = vw.tiles_x, ty = vw.tiles_y;
        const double ft = 1.0 / kTile;  // a power of two: the product is exact
        x0 = (int)fmin(fmax(floor((g.u - rad) * ft), 0.0), tx);
        x1 = (int)fmin(fmax(floor((g.u + rad) * ft) + 1.0, 0.0), tx);
        y0 = (int)fmin(fmax(floor((g.v - rad) * ft), 0.0), ty);
        y1 = (int)fmin(fmax(floor((g.v + rad) * ft) + 1.0, 0.0), ty);
        ok = g.det > 0.0 && isfinite(g.u) && isfinite(g.v);
        if (p.ellipse_cull) {
          // Binning footprint: only tiles that can hold a pixel with
          // opacity * exp(power) >= 1/255, i.e. inside the ellipse
          // 1/2 d^T conic d <= ln(255 opacity); its bounding box has
          // half-widths sqrt(2 K Sigma2d_00), sqrt(2 K Sigma2d_11). Every other
          // tile of the 3-sigma rectangle would skip this primitive at every
          // pixel, so the blend is unchanged. The box only narrows the exact
          // rectangle, so it is formed in FP32 with slack for that and for the
          // FP32 evaluation of the fragments.
          const float K = __logf(255.f * (float)(opa * g.pt));
          ok = ok && K > -1e-4f;
          const float Kc = fmaxf(K, 0.f);
          const float hx = sqrtf(2.f * Kc * (float)g.a2) * 1.001f + 0.05f;
          const float hy = sqrtf(2.f * Kc * (float)g.c2) * 1.001f + 0.05f;
          const float uf = (float)g.u, vf = (float)g.v, ft = 1.f / kTile;
          const float bx = (float)vw.tiles_x + 1.f, by = (float)vw.tiles_y + 1.f;
          x0 = max(x0, (int)fminf(fmaxf(floorf((uf - hx) * ft), -1.f), bx));
          x1 = min(x1, (int)fminf(fmaxf(floorf((uf + hx) * ft) + 1.f, -1.f), bx));
          y0 = max(y0, (int)fminf(fmaxf(floorf((vf - hy) * ft), -1.f), by));
          y1 = min(y1, (int)fminf(fmaxf(floorf((vf + hy) * ft) + 1.f, -1.f), by));
        }
        ok = ok && (x1 > x0) && (y1 > y0);
      }
      if (!ok) {
        act[idx] = 0u;
        slot[idx] = -1;
        continue;
      }
      any = true;
      const double z = g.pc[2];
      const float zf = (float)z;
      Record r;
      r.a = make_float4((float)g.u, (float)g.v, zf, (float)(opa * g.pt));
      r.b = make_float4((float)g.conic[0], (float)g.conic[1], (float)g.conic[2],
                        __uint_as_float((uint32_t)x0 | ((uint32_t)x1 << 16)));
      const float yr = __uint_as_float((uint32_t)y0 | ((uint32_t)y1 << 16));
      if (p.flow) {
        // Sec. 4.4: the conditional mean moves by v dt' / Sigma_44 (it is
        // linear in t); its projection moves by f (x' z - x z') / (z z') per axis
        const double sc = (double)p.flow_dt * sh.inv44;
        double dp[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          dp[i] = sc * ((double)vw.rot[3 * i] * g.v3[0] + (double)vw.rot[3 * i + 1] * g.v3[1] +
                        (double)vw.rot[3 * i + 2] * g.v3[2]);
        const double z1 = z + dp[2];
        const bool front = z1 > near;
        const double q = front ? 1.0 / (z * z1) : 0.0;
        r.c = make_float4((float)(vw.fx * (dp[0] * z - g.pc[0] * dp[2]) * q),
                          (float)(vw.fy * (dp[1] * z - g.pc[1] * dp[2]) * q), 0.f, yr);
      } else {
        // colour: k_colour fills c.xyz of the record's depth-ordered copy from
        // the view direction and t - mu_t
        r.c = make_float4(0.f, 0.f, 0.f, yr);
        cdir[idx] = make_float4((float)g.dir[0], (float)g.dir[1], (float)g.dir[2], (float)g.dt);
      }
      rec[idx] = r;
      act[idx] = 1u;
      dkey[idx] = __float_as_uint(zf);  // z > near > 0: bit order = numeric order
      slot[idx] = -1;
    }
  }
  // the primitive's lanes agree on "active in some view"; the first records
  // it and appends it to the list (one atomic per wave)
  const int lane = threadIdx.x & 63;
  const int lead = lane - sub;  // lanes of a primitive never straddle a wave (lanes divides 64)
  const uint64_t m = __ballot(any);
  const bool gany = ((m >> lead) & ((lanes >= 64 ? ~0ull : (1ull << lanes) - 1ull))) != 0ull;
  const bool append = live && sub == 0 && gany;
  if (live && sub == 0) p.pany[gidx] = gany ? 1 : 0;
  const uint64_t am = __ballot(append);
  if (am) {
    uint32_t base = 0;
    if (lane == __ffsll((long long)am) - 1) base = atomicAdd(p.plist_n, (uint32_t)__popcll(am));
    base = __shfl(base, __ffsll((long long)am) - 1, 64);
    const uint64_t below = lane ? (am & (~0ull >> (64 - lane))) : 0ull;
    if (append) p.plist[base + (uint32_t)__popcll(below)] = (uint32_t)gidx;
  }
}

constexpr int kColourViews = 8;  // views whose activity flags k_colour loads together

// 4D spherindrical-harmonic colour (Sec. 3.2) of the primitives active in
// some view (the list the preprocess built): a quad of lanes per listed
// primitive, lane `sub` owning the basis functions lm = 4 sub + i and reading
// their coefficients straight from memory (the quad reads the primitive's
// 192-byte Fourier terms together). Each quad walks only its own active
// views, the k-th in round k (a wave takes as many rounds as its busiest
// primitive has active views), with the next view's direction loaded while
// the current one is evaluated. The colour goes into the pair's record in
// (view, primitive) order, before the depth sort moves it (the pass runs
// beside the scans and the depth sort). Per view every lane evaluates the basis,
// weights its four functions by the Fourier terms, and a quad sum gives
// c = max(0, 0.5 + sum). A primitive with a non-finite coefficient gets a
// NaN colour, which the rasterisers read as fully transparent (and the pair
// is counted as culled).
__global__ void __launch_bounds__(256) k_colour(RenderParams p, const uint32_t* __restrict__ act,
                                                const float4* __restrict__ cdir, Record* __restrict__ rec) {
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
    float k[3][kBasisPerLane][3];
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
        }
    const bool bad = quad_any(!finite);
    for (int v0 = 0; v0 < p.n_views; v0 += kColourViews) {
      int ds[kColourViews];
      uint32_t m = 0u;
#pragma unroll
      for (int w = 0; w < kColourViews; ++w) {
        ds[w] = (live && v0 + w < p.n_views && act[(size_t)(v0 + w) * p.n + gidx]) ? 1 : -1;
        m |= (ds[w] >= 0 ? 1u : 0u) << w;
      }
      uint32_t rounds = (uint32_t)__popc(m);
#pragma unroll
      for (int off = 4; off < 64; off <<= 1) rounds = max(rounds, (uint32_t)__shfl_xor((int)rounds, off, 64));
      // the quad's next active view, its record slot and its direction (in flight)
      int w = m ? __ffs(m) - 1 : -1;
      m = m ? m & (m - 1u) : 0u;
      float4 cd = w >= 0 ? cdir[(size_t)(v0 + w) * p.n + gidx] : make_float4(0.f, 0.f, 1.f, 0.f);
      for (uint32_t r = 0; r < rounds; ++r) {
        const int wc = w;
        const float4 cdc = cd;
        w = m ? __ffs(m) - 1 : -1;
        m = m ? m & (m - 1u) : 0u;
        if (w >= 0) cd = cdir[(size_t)(v0 + w) * p.n + gidx];
        if (wc < 0) continue;  // uniform per quad
        float* o = reinterpret_cast<float*>(&rec[(size_t)(v0 + wc) * p.n + gidx].c);
        if (bad) {
          if (sub == 0) {
            const float nan = __int_as_float(0x7FC00000);
            o[0] = nan;
            o[1] = nan;
            o[2] = nan;
            if (p.nonfinite) atomicAdd(p.nonfinite + v0 + wc, 1u);
          }
          continue;
        }
        float Y[16], cs[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) Y[jj] = 0.f;
        sh_eval(p.sh_degree, cdc.x, cdc.y, cdc.z, Y);
        fourier_terms(p.t_order, cdc.w, p.t_period, cs);
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
          o[0] = fmaxf(col[0] + kColorOffset, 0.f);
          o[1] = fmaxf(col[1] + kColorOffset, 0.f);
          o[2] = fmaxf(col[2] + kColorOffset, 0.f);
        }
      }
    }
  }
}

}  // namespace

int preprocess_lanes(int) { return 1; }

void launch_preprocess(const RenderParams& p, uint32_t* act, uint32_t* dkey, Record* rec, int32_t* slot,
                       float4* cdir, hipStream_t s) {
  if (p.n == 0) return;
  const int lanes = preprocess_lanes(p.n_views);
  const uint64_t threads = (uint64_t)p.n * lanes;
  hipLaunchKernelGGL(k_preprocess, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, p, lanes, act, dkey, rec,
                     slot, cdir);
}

// Workgroups of the kernels that walk the active-primitive list (64 listed
// primitives per workgroup and step): one step for up to 2^20 primitives,
// grid-stride beyond.
unsigned list_grid(int n) {
  const unsigned need = (unsigned)((n + kColourPrims - 1) / kColourPrims);
  return need < 1 ? 1 : (need < 16384 ? need : 16384);
}

void launch_colour(const RenderParams& p, const uint32_t* act, const float4* cdir, Record* rec, hipStream_t s) {
  if (p.n == 0 || p.flow) return;
  hipLaunchKernelGGL(k_colour, dim3(list_grid(p.n)), dim3(256), 0, s, p, act, cdir, rec);
}

}  // namespace g4d
