// Binning of active records into 16x16 tiles, ordered by (tile, depth).
//
// The tile rasteriser the paper adapts (Sec. 3.2, last paragraph of
// "Representation of 4D Gaussian") needs, per tile, the primitives whose
// footprint covers it in front-to-back order. This is an LSD radix sort on the
// composite key (global tile, depth, view*n + index), arranged so the low-order
// passes run on the active records before they are duplicated per tile:
//   1. stable 4-pass radix sort of the active records by float depth bits
//      (ties keep (view, index) order from the compaction scan);
//   2. emission of one (tile, record) instance per tile of the record's
//      rectangle that its alpha-floor ellipse reaches, in that order;
//   3. stable radix sort of the instances by global tile id.
// Every pass is stable, so the result equals a stable sort by (tile, depth)
// of the instances emitted in (view, index) order.
#include <utility>
#include "g4d_common.h"

namespace g4d {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTileElems = kThreads * kItems;  // 4096 elements per block tile
static_assert(kTileElems == 4 * 1024, "the scan tile is four waves of 1024 elements");

__device__ __forceinline__ uint32_t dev_n(const uint32_t* n_dev, uint32_t n_max) {
  return n_dev ? min(*n_dev, n_max) : n_max;
}

// A record's footprint for binning: centre, conic, the bound L on
// Q = a dx^2 + 2 b dx dy + c dy^2 below which opacity * exp(-Q/2) reaches
// 1/255 (loosened by 0.1 % + 0.02 so FP32 rounding never drops a blended
// pixel), the ellipse's half-height ymax, the dy of its leftmost point ey
// (the rightmost is at -ey), and its tile rectangle. D = a c - b^2.
struct Footprint {
  float u, v, b, L, D, ia, ymax, ey;
  uint32_t x0, x1, y0, y1;
};

// Footprint and row_span are written with explicit rounding and no
// contraction, so the instance count of a record and its emission agree. The
// square roots are the hardware instruction (within about an ulp; it is the
// same instruction in both kernels, and far inside the spans' slack).
__device__ __forceinline__ Footprint footprint(const Record& r) {
#pragma clang fp contract(off)
  Footprint f;
  f.u = r.a.x;
  f.v = r.a.y;
  const float a = r.b.x, c = r.b.z;
  f.b = r.b.y;
  // 2 ln(255 opacity) = 2 ln2 (log2 opacity - log2(1/255))
  const float L0 = __fmul_rn(2.f * 0.69314718055994531f, __fsub_rn(__log2f(r.a.w), kLog2AlphaMin));
  f.L = __fmaf_rn(L0, 1.001f, 0.02f);
  const float p = __fmul_rn(f.b, f.b);
  f.D = __fsub_rn(__fmaf_rn(a, c, -p), __fmaf_rn(f.b, f.b, -p));  // product error recovered
  f.ia = __builtin_amdgcn_rcpf(a);
  const float iD = __builtin_amdgcn_rcpf(f.D);
  f.ymax = __builtin_amdgcn_sqrtf(fmaxf(__fmul_rn(__fmul_rn(f.L, a), iD), 0.f));
  const float xmax = __builtin_amdgcn_sqrtf(fmaxf(__fmul_rn(__fmul_rn(f.L, c), iD), 0.f));
  f.ey = __fmul_rn(__fmul_rn(f.b, xmax), __builtin_amdgcn_rcpf(c));
  if (!(f.L > 0.f) || !(f.D > 0.f) || !(f.ymax >= 0.f)) f.ymax = -1.f;  // no tile
  f.L = __fmul_rn(a, f.L);                           // kept as a L from here on
  const uint32_t rx = __float_as_uint(r.b.w), ry = __float_as_uint(r.c.w);
  f.x0 = rx & 0xFFFFu;
  f.x1 = rx >> 16;
  f.y0 = ry & 0xFFFFu;
  f.y1 = ry >> 16;
  return f;
}

// Tiles [xa, xb) of tile row ty whose pixel centres the ellipse Q <= L can
// reach, within the rectangle. Over the row's band of pixel-centre rows the
// ellipse's left edge x(dy) = (-b dy - sqrt(a L - D dy^2)) / a is convex and
// its right edge concave, so their extremes over the band sit at the
// leftmost / rightmost points clamped to the band. exact = false: the
// rectangle's whole row.
__device__ __forceinline__ void row_span(const Footprint& f, uint32_t ty, bool exact, uint32_t& xa, uint32_t& xb) {
#pragma clang fp contract(off)
  constexpr float kEps = 0.01f;  // px
  if (!exact) {
    xa = f.x0;
    xb = f.x1;
    return;
  }
  xa = xb = f.x0;
  const float band0 = __fsub_rn((float)(ty * kTile) + (0.5f - kEps), f.v);
  const float band1 = __fsub_rn((float)(ty * kTile) + (15.5f + kEps), f.v);
  const float lo = fmaxf(band0, -f.ymax), hi = fminf(band1, f.ymax);
  if (!(lo <= hi)) return;
  const float dl = fminf(fmaxf(f.ey, lo), hi), dr = fminf(fmaxf(-f.ey, lo), hi);
  const float sl = __builtin_amdgcn_sqrtf(fmaxf(__fsub_rn(f.L, __fmul_rn(f.D, __fmul_rn(dl, dl))), 0.f));
  const float sr = __builtin_amdgcn_sqrtf(fmaxf(__fsub_rn(f.L, __fmul_rn(f.D, __fmul_rn(dr, dr))), 0.f));
  const float left = __fadd_rn(f.u, __fmul_rn(__fsub_rn(-__fmul_rn(f.b, dl), sl), f.ia));
  const float right = __fadd_rn(f.u, __fmul_rn(__fadd_rn(-__fmul_rn(f.b, dr), sr), f.ia));
  // tile tx holds centres 16 tx + [0.5, 15.5]
  const float ta = ceilf(__fmul_rn(__fsub_rn(left, 15.5f + kEps), 1.f / kTile));
  const float tb = floorf(__fmul_rn(__fadd_rn(right, kEps - 0.5f), 1.f / kTile)) + 1.f;
  const float fx0 = (float)f.x0, fx1 = (float)f.x1;
  xa = (uint32_t)fminf(fmaxf(ta, fx0), fx1);
  xb = (uint32_t)fminf(fmaxf(tb, (float)xa), fx1);
}

// Exclusive scan of one value per thread across a 256-thread block.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t base = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t c = s_wave[w];
    base += (w < wave) ? c : 0u;
    total += c;
  }
  __syncthreads();
  return base + x - v;
}

// ---------------------------------------------------------------- scan ----
// The scan's block tile: wave w holds elements [1024 w, 1024 w + 1024) of the
// tile, and lane l the four 16-byte groups 256 j + 4 l (j = 0..3), so every
// load and store instruction of a wave covers 1 KB of consecutive words and
// the element order is (wave, group, lane, word). The arrays are the
// library's own 256-byte-aligned buffers, so a full tile's groups are aligned.
__device__ __forceinline__ size_t scan_group(int j) {
  return (size_t)(threadIdx.x >> 6) * 1024 + (size_t)j * 256 + (size_t)(threadIdx.x & 63) * 4;
}

__device__ __forceinline__ uint4 load_group(const uint32_t* __restrict__ p, size_t e, size_t n, bool full) {
  if (full) return *reinterpret_cast<const uint4*>(p + e);
  return make_uint4(e < n ? p[e] : 0u, e + 1 < n ? p[e + 1] : 0u, e + 2 < n ? p[e + 2] : 0u, e + 3 < n ? p[e + 3] : 0u);
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in, const uint32_t* n_dev,
                                                           uint32_t n_max, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t s_wave[4];
  const uint32_t n = dev_n(n_dev, n_max);
  const size_t base = (size_t)blockIdx.x * kTileElems;
  if (base >= n) return;
  const bool full = base + kTileElems <= n;
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint4 g = load_group(in, base + scan_group(j), n, full);
    acc += g.x + g.y + g.z + g.w;
  }
  uint32_t total;
  block_exclusive_scan(acc, s_wave, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the tile: each block's offset is the sum of the block
// sums before it, added up by the block's own threads (no separate pass over
// the block sums), and the last block writes the total. With ckey, the input
// is a 0/1 flag per element and every flagged element i also lands in the
// compacted arrays: ckey[out[i]] = dkey[i], cval[out[i]] = i (the flagged
// lanes of one store instruction write a short increasing run of positions).
__global__ void __launch_bounds__(kThreads) k_scan_apply(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                          const uint32_t* n_dev, uint32_t n_max,
                                                          const uint32_t* __restrict__ bsum,
                                                          uint32_t* __restrict__ total,
                                                          const uint32_t* __restrict__ dkey,
                                                          uint32_t* __restrict__ ckey, uint32_t* __restrict__ cval) {
  __shared__ uint32_t s_wave[4];
  const uint32_t n = dev_n(n_dev, n_max);
  const uint32_t nb = (n + kTileElems - 1) / kTileElems;
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) *total = 0u;
  if (blockIdx.x >= nb) return;
  uint32_t part = 0;
  for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kThreads) part += bsum[b];
  uint32_t prefix;
  block_exclusive_scan(part, s_wave, prefix);  // contains barriers; prefix = the block sums before this block
  const size_t base = (size_t)blockIdx.x * kTileElems;
  const bool full = base + kTileElems <= n;
  uint4 g[4];
  uint32_t gx[4];  // each group's exclusive offset within the wave
  uint32_t wsum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    g[j] = load_group(in, base + scan_group(j), n, full);
    const uint32_t s = g[j].x + g[j].y + g[j].z + g[j].w;
    const uint32_t inc = wave_inclusive_scan(s);
    gx[j] = wsum + inc - s;
    wsum += __shfl(inc, 63, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_wave[wave] = wsum;
  __syncthreads();
  uint32_t wbase = prefix, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t c = s_wave[w];
    wbase += (w < wave) ? c : 0u;
    tot += c;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t e = base + scan_group(j);
    const uint32_t v[4] = {g[j].x, g[j].y, g[j].z, g[j].w};
    uint32_t o[4];
    uint32_t run = wbase + gx[j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[i] = run;
      run += v[i];
    }
    if (full) {
      *reinterpret_cast<uint4*>(out + e) = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (e + i < n) out[e + i] = o[i];
    }
    if (ckey) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (v[i]) {  // a flagged element lies below n
          ckey[o[i]] = dkey[e + i];
          cval[o[i]] = (uint32_t)(e + i);
        }
      }
    }
  }
  if (blockIdx.x + 1 == nb && threadIdx.x == 0) *total = prefix + tot;
}

// ---------------------------------------------------------- radix sort ----
// Workgroups are dispatched round-robin over the 8 XCDs; the sort's blocks
// take their ranges of tiles in XCD-major order, so the digit runs that
// consecutive ranges write next to each other come from one XCD's L2.
__device__ __forceinline__ uint32_t sort_block() {
  const uint32_t g = gridDim.x;
  return (g & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (g >> 3) + (blockIdx.x >> 3);
}

__device__ __forceinline__ void block_range(uint32_t n, int grid, uint32_t& t0, uint32_t& t1) {
  const uint32_t tiles = (n + kTileElems - 1) / kTileElems;
  const uint32_t tpb = (tiles + grid - 1) / grid;
  t0 = min(sort_block() * tpb, tiles);
  t1 = min(t0 + tpb, tiles);
}

// K: uint32_t, or uint16_t for keys below 2^16 (the tile ids of a round).
template <typename K>
__global__ void __launch_bounds__(kThreads) k_rs_upsweep(const K* __restrict__ keys, const uint32_t* n_dev,
                                                          uint32_t n_max, int shift, int bits,
                                                          uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[4][256];
  const uint32_t n = dev_n(n_dev, n_max);
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < 4; ++w) hist[w][threadIdx.x] = 0u;
  __syncthreads();
  uint32_t t0, t1;
  block_range(n, gridDim.x, t0, t1);
  const uint32_t mask = (1u << bits) - 1u;
  for (uint32_t t = t0; t < t1; ++t) {
    const size_t tb = (size_t)t * kTileElems;
    if (tb + kTileElems <= n) {
      // full tile: 16-byte loads (four, or two of 16-bit keys), all in flight together
      constexpr int kVec = 16 / (int)sizeof(K);
      uint4 q[kItems / kVec];
#pragma unroll
      for (int i = 0; i < kItems / kVec; ++i)
        q[i] = reinterpret_cast<const uint4*>(keys + tb)[i * kThreads + threadIdx.x];
#pragma unroll
      for (int i = 0; i < kItems / kVec; ++i) {
        const uint32_t w[4] = {q[i].x, q[i].y, q[i].z, q[i].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (sizeof(K) == 4) {
            atomicAdd(&hist[wave][(w[j] >> shift) & mask], 1u);
          } else {
            atomicAdd(&hist[wave][((w[j] & 0xFFFFu) >> shift) & mask], 1u);
            atomicAdd(&hist[wave][(w[j] >> (16 + shift)) & mask], 1u);
          }
        }
      }
    } else {
      for (int i = 0; i < kItems; ++i) {
        const size_t idx = tb + (size_t)i * kThreads + threadIdx.x;
        if (idx < n) atomicAdd(&hist[wave][((uint32_t)keys[idx] >> shift) & mask], 1u);
      }
    }
  }
  __syncthreads();
  const uint32_t d = threadIdx.x;
  counts[(size_t)d * gridDim.x + sort_block()] = hist[0][d] + hist[1][d] + hist[2][d] + hist[3][d];
}

// One 256-thread block per digit: exclusive scan of counts[digit][0..grid) in
// place and the digit's total into digit_tot[digit]. Each thread takes eight
// consecutive counts of a 2048-count chunk, so a row of up to 2048 blocks'
// counts is one block-wide scan, and the small workgroup finds a CU beside
// another stream's work.
constexpr int kRowScanPer = 8;
__global__ void __launch_bounds__(kThreads) k_rs_rowscan(uint32_t* __restrict__ counts, int grid,
                                                         uint32_t* __restrict__ digit_tot) {
  __shared__ uint32_t s_wave[4];
  uint32_t* row = counts + (size_t)blockIdx.x * grid;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < grid; c0 += kThreads * kRowScanPer) {
    const int b0 = c0 + (int)threadIdx.x * kRowScanPer;
    uint32_t v[kRowScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kRowScanPer; ++i) {
      v[i] = b0 + i < grid ? row[b0 + i] : 0u;
      sum += v[i];
    }
    uint32_t tot;
    uint32_t ex = carry + block_exclusive_scan(sum, s_wave, tot);  // contains barriers
#pragma unroll
    for (int i = 0; i < kRowScanPer; ++i) {
      if (b0 + i < grid) row[b0 + i] = ex;
      ex += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// LDS of the stable scatter of one digit pass (30.7 KB with 16-bit keys, five
// workgroups per CU; 39.4 KB with 32-bit keys, four).
template <typename K>
struct ScatterShared {
  K k[kTileElems];                        // the tile reordered by digit
  uint32_t v[kTileElems];
  uint32_t wcnt[4][256];                  // per wave and digit: count, then start
  uint32_t run[256];                      // per digit: next output position of the block
  uint32_t tstart[256];                   // per digit: start of its run in the reordered tile
  uint32_t wave[4];
};

// Output positions of the block's digit runs: run[d] = (pairs of smaller
// digits in the whole pass) + (pairs of digit d in earlier blocks), from the
// per-(digit, block) exclusive scan `counts` and the digit totals.
template <typename K>
__device__ __forceinline__ void scatter_begin(ScatterShared<K>& sh, const uint32_t* __restrict__ counts,
                                              const uint32_t* __restrict__ digit_tot, uint32_t grid, uint32_t block) {
  const uint32_t dg = threadIdx.x;
  uint32_t tot;
  const uint32_t base = block_exclusive_scan(digit_tot[dg], sh.wave, tot);
  sh.run[dg] = base + counts[(size_t)dg * grid + block];
}

// Stable scatter of one tile of up to 4096 (key, value) pairs: wave w holds
// pairs [1024 w, 1024 w + 1024) of the tile, 64 at a time, step i in k[i],
// v[i]; the first nvalid pairs of the tile are valid. A lane's rank among
// equal digits comes from a ballot match over the digit bits; the tile is
// reordered by digit in LDS first, so the global writes of each digit run are
// contiguous. Pairs go to run[d] + their rank among the block's pairs of
// digit d so far (bounded by n_out); with ranges (the last pass over the
// whole key) the keys are not written: each key's first and last position
// bound its range instead (a key >= n_ranges, which a consistent sort never
// produces, is skipped).
// FULL: the tile holds kTileElems valid pairs (the validity tests compile out).
template <bool FULL, typename K>
__device__ __forceinline__ void scatter_tile(ScatterShared<K>& sh, uint32_t (&k)[kItems],
                                             const uint32_t (&v)[kItems], uint32_t nvalid, int shift, int bits,
                                             uint32_t n_out, K* __restrict__ keys_out,
                                             uint32_t* __restrict__ vals_out, uint2* __restrict__ ranges,
                                             uint32_t n_ranges) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t mask = (1u << bits) - 1u;
  const uint32_t dg = threadIdx.x;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < 4; ++w) sh.wcnt[w][threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t base = (uint32_t)wave * (kTileElems / 4);
  constexpr bool kPacked = sizeof(K) == 2;
  uint32_t rank[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = FULL || base + (uint32_t)i * 64 + lane < nvalid;
    const uint32_t d = (k[i] >> shift) & mask;
    // the lanes holding the same digit (a lane mask in two halves): per digit
    // bit, a lane keeps the lanes whose bit equals its own. S is the lane's
    // bit b as a whole-word mask, so each step is one compare for the ballot
    // and one three-input bit operation per half. Digits have at most 8
    // bits; bits above `bits` are zero in every lane.
    const uint64_t vb = __ballot(valid);
    uint32_t plo = (uint32_t)vb, phi = (uint32_t)(vb >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int32_t S = (int32_t)(d << (31 - b)) >> 31;
      const uint64_t m = __ballot(S < 0);
      // x & ~(y ^ z): truth table 0x90 with operands (x, y, z)
      plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)m, (uint32_t)S, 0x90);
      phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(m >> 32), (uint32_t)S, 0x90);
    }
    // equal-digit lanes below this one
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
    const uint32_t pre = sh.wcnt[wave][d];
    // a 16-bit key shares its register with its rank (< 4096). The empty asm
    // makes the rank final here: left to itself the compiler defers the sum
    // past the barrier and keeps each step's masks and count live until then
    if (kPacked) {
      k[i] |= (pre + below) << 16;
      asm volatile("" : "+v"(k[i]));
    } else {
      rank[i] = pre + below;
      asm volatile("" : "+v"(rank[i]));
    }
    // every lane of a digit writes the same count; in a full tile without a
    // branch, so the next step's ballots can overlap this step's LDS access
    const uint32_t cnt = pre + (uint32_t)(__popc(plo) + __popc(phi));
    if (FULL) sh.wcnt[wave][d] = cnt;
    else if (valid && below == 0) sh.wcnt[wave][d] = cnt;
  }
  __syncthreads();
  // per digit: tile-local start, then each wave's start inside it
  const uint32_t c0 = sh.wcnt[0][dg], c1 = sh.wcnt[1][dg], c2 = sh.wcnt[2][dg], c3 = sh.wcnt[3][dg];
  const uint32_t ctot = c0 + c1 + c2 + c3;
  uint32_t all;
  const uint32_t ts = block_exclusive_scan(ctot, sh.wave, all);  // contains barriers
  sh.wcnt[0][dg] = ts;
  sh.wcnt[1][dg] = ts + c0;
  sh.wcnt[2][dg] = ts + c0 + c1;
  sh.wcnt[3][dg] = ts + c0 + c1 + c2;
  sh.tstart[dg] = ts;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = FULL || base + (uint32_t)i * 64 + lane < nvalid;
    if (valid) {
      const uint32_t key = kPacked ? (k[i] & 0xFFFFu) : k[i];
      const uint32_t d = (key >> shift) & mask;
      const uint32_t lp = sh.wcnt[wave][d] + (kPacked ? k[i] >> 16 : rank[i]);
      if (lp < (uint32_t)kTileElems) {
        sh.k[lp] = (K)key;
        sh.v[lp] = v[i];
      }
    }
  }
  __syncthreads();
  const uint32_t nt = FULL ? (uint32_t)kTileElems : min(nvalid, (uint32_t)kTileElems);
#pragma unroll 4
  for (int i = 0; i < kItems; ++i) {
    const uint32_t lp = (uint32_t)i * kThreads + threadIdx.x;
    if (lp < nt) {
      const uint32_t key = sh.k[lp];
      const uint32_t d = (key >> shift) & mask;
      const uint32_t p = sh.run[d] + lp - sh.tstart[d];
      if (p < n_out) {  // always true for consistent counts; keeps a ranking fault in bounds
        if (ranges) {
          // the staged tile is ordered by key, so the first and last of each
          // key's run here bound its range
          if (key < n_ranges) {
            if (lp == 0 || sh.k[lp - 1] != key) atomicMin(&ranges[key].x, p);
            if (lp + 1 == nt || sh.k[lp + 1] != key) atomicMax(&ranges[key].y, p + 1);
          }
        } else {
          keys_out[p] = (K)key;
        }
        vals_out[p] = sh.v[lp];
      }
    }
  }
  __syncthreads();
  sh.run[dg] += ctot;
}

// One digit pass over the pairs in memory: each block takes its range of
// 4096-pair tiles in turn.
template <typename K>
__global__ void __launch_bounds__(kThreads) k_rs_downsweep(const K* __restrict__ keys_in,
                                                            const uint32_t* __restrict__ vals_in,
                                                            K* __restrict__ keys_out,
                                                            uint32_t* __restrict__ vals_out, const uint32_t* n_dev,
                                                            uint32_t n_max, int shift, int bits,
                                                            const uint32_t* __restrict__ counts,
                                                            const uint32_t* __restrict__ digit_tot,
                                                            uint2* __restrict__ ranges, uint32_t n_ranges) {
  __shared__ ScatterShared<K> sh;
  const uint32_t n = dev_n(n_dev, n_max);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  scatter_begin(sh, counts, digit_tot, gridDim.x, sort_block());
  uint32_t t0, t1;
  block_range(n, gridDim.x, t0, t1);
  for (uint32_t t = t0; t < t1; ++t) {
    const size_t base = (size_t)t * kTileElems + (size_t)wave * (kTileElems / 4);
    uint32_t k[kItems], v[kItems];
    const uint32_t nvalid = (uint32_t)min((size_t)kTileElems, (size_t)n - (size_t)t * kTileElems);
    if (nvalid == (uint32_t)kTileElems) {
      // a full tile (all but the last): no per-key bounds test
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const size_t idx = base + (size_t)i * 64 + lane;
        k[i] = (uint32_t)keys_in[idx];
        v[i] = vals_in[idx];
      }
      scatter_tile<true>(sh, k, v, nvalid, shift, bits, n, keys_out, vals_out, ranges, n_ranges);
    } else {
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const size_t idx = base + (size_t)i * 64 + lane;
        k[i] = (idx < n) ? (uint32_t)keys_in[idx] : 0u;
        v[i] = (idx < n) ? vals_in[idx] : 0u;
      }
      scatter_tile<false>(sh, k, v, nvalid, shift, bits, n, keys_out, vals_out, ranges, n_ranges);
    }
  }
}

// ------------------------------------------------------------- gather ----
__global__ void __launch_bounds__(kThreads) k_gather(const uint32_t* n_dev, uint32_t n_max,
                                                      const uint32_t* __restrict__ ids, const Record* __restrict__ rec,
                                                      Record* __restrict__ rec_sorted, int32_t* __restrict__ slot,
                                                      uint32_t* __restrict__ tcount, bool exact,
                                                      unsigned long long* __restrict__ inst64) {
  __shared__ uint32_t s_wave[4];
  const uint32_t n = dev_n(n_dev, n_max);
  const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x * blockDim.x >= n) return;
  uint32_t cnt = 0;
  if (d < n) {
    const uint32_t id = ids[d];
    const Record r = rec[id];
    rec_sorted[d] = r;
    slot[id] = (int32_t)d;
    const Footprint f = footprint(r);
    for (uint32_t ty = f.y0; ty < f.y1; ++ty) {
      uint32_t xa, xb;
      row_span(f, ty, exact, xa, xb);
      cnt += xb - xa;
    }
    tcount[d] = cnt;
  }
  uint32_t total;
  block_exclusive_scan(cnt, s_wave, total);
  if (threadIdx.x == 0) atomicAdd(inst64, (unsigned long long)total);
}

// Active records per view from the compaction scan: pos[(v+1) n] - pos[v n].
__global__ void k_view_counts(const uint32_t* __restrict__ pos, int n_views, uint32_t n, const uint32_t* total,
                              uint32_t* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  if (n == 0) {
    out[v] = 0u;
    return;
  }
  const size_t b = (size_t)v * n;
  const uint32_t start = pos[b];
  const uint32_t end = (v + 1 < n_views) ? pos[b + n] : *total;
  out[v] = end - start;
}

// ---------------------------------------------------------------- emit ----
// One block per 64 consecutive records. The block lays out its records'
// tile rows in LDS (first tile, offset of the row's first instance by a block
// scan of the row widths) and, chunk by chunk, an instance -> row map, then
// writes the block's instances coalesced, one per thread in turn. A block
// whose rows do not fit walks each instance's record rows.
constexpr int kEmitRecs = 64;
constexpr int kEmitRows = 1024;
constexpr int kEmitInst = 4096;

// K: the key type, uint16_t when the round's tile ids are below 2^16.
template <typename K>
__global__ void __launch_bounds__(kThreads) k_emit(const uint32_t* n_dev, uint32_t n_max,
                                                    const uint32_t* __restrict__ toff, const uint32_t* total,
                                                    uint32_t cap, const Record* __restrict__ rec_sorted,
                                                    const uint32_t* __restrict__ ids, uint32_t n_prims,
                                                    const ViewDev* __restrict__ views, bool exact,
                                                    K* __restrict__ ikey, uint32_t* __restrict__ ival,
                                                    uint2* __restrict__ ranges_init, uint32_t tiles) {
  __shared__ uint32_t offs[kEmitRecs + 1];
  __shared__ uint32_t s_rbase[kEmitRecs + 1];
  __shared__ uint32_t s_tb[kEmitRecs], s_tw[kEmitRecs];
  __shared__ Footprint s_fp[kEmitRecs];
  __shared__ uint32_t s_row_off[kEmitRows + 1];  // first instance of each row (block-relative)
  __shared__ uint32_t s_row_tile[kEmitRows];     // global tile id of the row's first instance
  __shared__ uint8_t s_row_rec[kEmitRows];       // record of the row (block-relative, < kEmitRecs)
  __shared__ uint16_t s_inst_row[kEmitInst];     // row of each instance of the chunk (< kEmitRows)
  static_assert(kEmitRecs <= 256 && kEmitRows <= 65536, "narrow LDS maps: 21 KB, 7 workgroups per CU");
  __shared__ uint32_t s_wave[4];
  // the tile ranges that the sort's last pass fills start empty
  if (ranges_init)
    for (uint32_t t = blockIdx.x * kThreads + threadIdx.x; t < tiles; t += gridDim.x * kThreads)
      ranges_init[t] = make_uint2(0xFFFFFFFFu, 0u);
  const uint32_t n = dev_n(n_dev, n_max);
  const uint32_t d0 = blockIdx.x * kEmitRecs;
  if (d0 >= n) return;
  const uint32_t nrec = min((uint32_t)kEmitRecs, n - d0);
  const uint32_t tot = *total;
  uint32_t h = 0;
  if (threadIdx.x < kEmitRecs) {
    const uint32_t d = d0 + threadIdx.x;
    offs[threadIdx.x] = d < n ? toff[d] : tot;
    if (threadIdx.x == 0) offs[kEmitRecs] = (d0 + kEmitRecs < n) ? toff[d0 + kEmitRecs] : tot;
    if (d < n) {
      const Footprint f = footprint(rec_sorted[d]);
      s_fp[threadIdx.x] = f;
      h = f.y1 - f.y0;
      const uint32_t v = ids[d] / n_prims;
      s_tb[threadIdx.x] = (uint32_t)views[v].tile_base;
      s_tw[threadIdx.x] = (uint32_t)views[v].tiles_x;
    }
  }
  uint32_t rows;
  const uint32_t rb = block_exclusive_scan(h, s_wave, rows);  // contains barriers
  if (threadIdx.x < kEmitRecs) s_rbase[threadIdx.x] = rb;
  // each record marks its rows with its block-relative index (h = 0 past
  // the last record), so a row finds its record with one LDS read
  if (rows <= (uint32_t)kEmitRows)
    for (uint32_t k = 0; k < h; ++k) s_row_rec[rb + k] = (uint8_t)threadIdx.x;
  __syncthreads();
  const uint32_t lim = min(tot, cap);
  const uint32_t start = offs[0], end = min(offs[kEmitRecs], lim);
  if (rows <= (uint32_t)kEmitRows) {
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < rows; j0 += kThreads) {
      const uint32_t j = j0 + threadIdx.x;
      uint32_t w = 0;
      if (j < rows) {
        const int lo = s_row_rec[j];
        const Footprint& f = s_fp[lo];
        const uint32_t ty = f.y0 + (j - s_rbase[lo]);
        uint32_t xa, xb;
        row_span(f, ty, exact, xa, xb);
        w = xb - xa;
        s_row_tile[j] = s_tb[lo] + ty * s_tw[lo] + xa;
      }
      uint32_t tot_w;
      const uint32_t ex = block_exclusive_scan(w, s_wave, tot_w);  // contains barriers
      if (j < rows) s_row_off[j] = carry + ex;
      carry += tot_w;
    }
    if (threadIdx.x == 0) s_row_off[rows] = carry;
    __syncthreads();
    // the block's instances in chunks of kEmitInst: each chunk's instances
    // are mapped to their rows, then written coalesced, one per thread in turn
    const uint32_t iend = min(end, start + carry);  // equal: the counts come from the same spans
    for (uint32_t c0 = 0; start + c0 < iend; c0 += kEmitInst) {
      const uint32_t c1 = min(carry, c0 + (uint32_t)kEmitInst);
      if (c0) __syncthreads();  // the previous chunk's reads of the map are done
      for (uint32_t j = threadIdx.x; j < rows; j += kThreads) {
        const uint32_t a = max(s_row_off[j], c0), b = min(s_row_off[j + 1], c1);
        for (uint32_t k = a; k < b; ++k) s_inst_row[k - c0] = (uint16_t)j;
      }
      __syncthreads();
      const uint32_t ie = min(iend, start + c1);
      for (uint32_t i = start + c0 + threadIdx.x; i < ie; i += kThreads) {
        const uint32_t k = i - start, j = s_inst_row[k - c0];
        ikey[i] = (K)(s_row_tile[j] + (k - s_row_off[j]));
        ival[i] = d0 + s_row_rec[j];
      }
    }
  } else {
    for (uint32_t i = start + threadIdx.x; i < end; i += kThreads) {
      int lo = 0, hi = (int)nrec - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= i) lo = mid; else hi = mid - 1;
      }
      const Footprint& f = s_fp[lo];
      uint32_t k = i - offs[lo], tile = 0;
      for (uint32_t ty = f.y0; ty < f.y1; ++ty) {
        uint32_t xa, xb;
        row_span(f, ty, exact, xa, xb);
        if (k < xb - xa) {
          tile = ty * s_tw[lo] + xa + k;
          break;
        }
        k -= xb - xa;
      }
      ikey[i] = (K)(s_tb[lo] + tile);
      ival[i] = d0 + (uint32_t)lo;
    }
  }
}

// Ranges filled by the last radix pass: (max, 0) before it, and tiles it did
// not reach (no instances) set to (0, 0) after it.
__global__ void k_ranges_init(uint2* __restrict__ ranges, uint32_t tiles) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles) ranges[t] = make_uint2(0xFFFFFFFFu, 0u);
}

__global__ void k_ranges_fix(uint2* __restrict__ ranges, uint32_t tiles) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tiles) return;
  const uint2 r = ranges[t];
  if (r.x > r.y) ranges[t] = make_uint2(0u, 0u);
}

template <typename K>
__global__ void k_ranges(const uint32_t* n_dev, uint32_t n_max, const K* __restrict__ ikey,
                         uint2* __restrict__ ranges) {
  // four consecutive keys per thread
  const uint32_t n = dev_n(n_dev, n_max);
  const uint32_t i0 = 4u * (blockIdx.x * blockDim.x + threadIdx.x);
  if (i0 >= n) return;
  uint32_t k[6];  // k[0] = key before i0 (or none), k[1..4] = keys i0..i0+3, k[5] = key after
  for (int j = 0; j < 4; ++j) k[1 + j] = (i0 + j < n) ? (uint32_t)ikey[i0 + j] : 0xFFFFFFFFu;
  k[0] = i0 > 0 ? (uint32_t)ikey[i0 - 1] : 0xFFFFFFFFu;
  k[5] = (i0 + 4 < n) ? (uint32_t)ikey[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
  for (int j = 1; j <= 4; ++j) {
    const uint32_t i = i0 + j - 1;
    if (i >= n) break;
    if (i == 0 || k[j - 1] != k[j]) ranges[k[j]].x = i;
    if (i == n - 1 || k[j + 1] != k[j]) ranges[k[j]].y = i + 1;
  }
}

// Block sums (64-bit per thread), one atomic per block.
__global__ void __launch_bounds__(256) k_sum_u32(const uint32_t* __restrict__ in, uint64_t n,
                                                 unsigned long long* out) {
  __shared__ unsigned long long s_part[4];
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long acc = 0;
  for (; i < n; i += (uint64_t)gridDim.x * blockDim.x) acc += in[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tot = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    if (tot) atomicAdd(out, tot);
  }
}

// Longest tile list: max over tiles of end - start, one atomic per block.
__global__ void __launch_bounds__(256) k_range_max(const uint2* __restrict__ ranges, uint32_t tiles, uint32_t* out) {
  __shared__ uint32_t s_part[4];
  uint32_t len = 0;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < tiles; t += gridDim.x * blockDim.x) {
    const uint2 r = ranges[t];
    len = max(len, r.y - r.x);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) len = max(len, (uint32_t)__shfl_xor((int)len, off, 64));
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t m = max(max(s_part[0], s_part[1]), max(s_part[2], s_part[3]));
    if (m) atomicMax(out, m);
  }
}

// Heavy-first tile order: key 255 - floor(16 log2(len + 1)), so that a
// stable sort of the keys lists tiles by decreasing list length in bins of
// ~4.4 %, keeping the natural order within a bin. The same pass empties the
// ranges the last radix pass did not reach (fix, as k_ranges_fix) and raises
// *max_len to the longest list (as k_range_max).
__global__ void __launch_bounds__(256) k_order_keys(uint2* __restrict__ ranges, uint32_t tiles, bool fix,
                                                    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    uint32_t* max_len) {
  __shared__ uint32_t s_part[4];
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t len = 0;
  if (t < tiles) {
    uint2 r = ranges[t];
    if (fix && r.x > r.y) {
      r = make_uint2(0u, 0u);
      ranges[t] = r;
    }
    len = r.y - r.x;
    const uint32_t b = (uint32_t)(16.f * __log2f((float)len + 1.f));
    keys[t] = 255u - min(b, 255u);
    vals[t] = t;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) len = max(len, (uint32_t)__shfl_xor((int)len, off, 64));
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t m = max(max(s_part[0], s_part[1]), max(s_part[2], s_part[3]));
    if (m) atomicMax(max_len, m);
  }
}

inline unsigned grid_for(uint64_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t scan_scratch_words(size_t n_max) { return (n_max + kTileElems - 1) / kTileElems + 1; }

void launch_scan(const uint32_t* in, uint32_t* out, const uint32_t* n_dev, uint32_t n_host, uint32_t n_max,
                 uint32_t* total, uint32_t* scratch, hipStream_t s, const uint32_t* dkey, uint32_t* ckey,
                 uint32_t* cval) {
  const uint32_t cap = n_dev ? n_max : n_host;
  const unsigned nb = grid_for(cap, kTileElems);
  if (nb == 0) {
    launch_fill_u32(total, 1, 0u, s);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, s, in, n_dev, cap, scratch);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kThreads), 0, s, in, out, n_dev, cap, scratch, total, dkey, ckey,
                     cval);
}

size_t radix_scratch_words(int grid) { return (size_t)256 * grid + 256; }

int radix_grid(uint32_t n_max, int max_blocks) {
  const int need = (int)grid_for(n_max, kTileElems);
  return need < 1 ? 1 : (need < max_blocks ? need : max_blocks);
}

int radix_passes(int bit0, int bit1) { return bit1 > bit0 ? (bit1 - bit0 + 7) / 8 : 0; }

// The digit passes, ping-ponging between the two buffer pairs; returns the
// pair that holds the result.
template <typename K>
std::pair<K*, uint32_t*> radix_passes_run(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt,
                                          const uint32_t* n_dev, uint32_t n_max, int bit0, int bit1, int grid,
                                          uint32_t* scratch, hipStream_t s, uint2* last_ranges,
                                          uint32_t n_ranges) {
  K *kin = keys, *kout = keys_alt;
  uint32_t *vin = vals, *vout = vals_alt;
  for (int b = bit0; b < bit1; b += 8) {
    const int bits = (bit1 - b) < 8 ? (bit1 - b) : 8;
    hipLaunchKernelGGL(k_rs_upsweep<K>, dim3(grid), dim3(kThreads), 0, s, kin, n_dev, n_max, b, bits, scratch);
    hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(kThreads), 0, s, scratch, grid, scratch + (size_t)256 * grid);
    hipLaunchKernelGGL(k_rs_downsweep<K>, dim3(grid), dim3(kThreads), 0, s, kin, vin, kout, vout, n_dev, n_max, b,
                       bits, scratch, scratch + (size_t)256 * grid, b + 8 >= bit1 ? last_ranges : nullptr,
                       b + 8 >= bit1 && last_ranges ? n_ranges : 0u);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  return {kin, vin};
}

void radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, const uint32_t* n_dev,
                uint32_t n_max, int bit0, int bit1, int grid, uint32_t* scratch, hipStream_t s, bool copy_back,
                uint2* last_ranges, uint32_t n_ranges) {
  // an odd pass count ends with a copy back so the result is in (keys, vals),
  // unless the caller takes it from (keys_alt, vals_alt)
  const auto out = radix_passes_run(keys, vals, keys_alt, vals_alt, n_dev, n_max, bit0, bit1, grid, scratch, s,
                                    last_ranges, n_ranges);
  if (out.first != keys && copy_back) launch_copy_pairs(out.first, out.second, keys, vals, n_dev, n_max, s);
}

void radix_sort16(uint16_t* keys, uint32_t* vals, uint16_t* keys_alt, uint32_t* vals_alt, const uint32_t* n_dev,
                  uint32_t n_max, int bit0, int bit1, int grid, uint32_t* scratch, hipStream_t s,
                  uint2* last_ranges, uint32_t n_ranges) {
  radix_passes_run(keys, vals, keys_alt, vals_alt, n_dev, n_max, bit0, bit1, grid, scratch, s, last_ranges,
                   n_ranges);
}

void launch_gather(const uint32_t* n_dev, uint32_t n_max, const uint32_t* ids, const Record* rec, Record* rec_sorted,
                   int32_t* slot, uint32_t* tcount, bool exact, uint32_t* inst64, hipStream_t s) {
  if (n_max == 0) return;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n_max, kThreads)), dim3(kThreads), 0, s, n_dev, n_max, ids, rec,
                     rec_sorted, slot, tcount, exact, reinterpret_cast<unsigned long long*>(inst64));
}

void launch_view_counts(const uint32_t* pos, int n_views, uint32_t n, const uint32_t* total, uint32_t* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_view_counts, dim3(grid_for(n_views, 64)), dim3(64), 0, s, pos, n_views, n, total, out);
}

template <typename K>
void emit_keys(const uint32_t* n_dev, uint32_t n_max, const uint32_t* toff, const uint32_t* total, uint32_t cap,
               const Record* rec_sorted, const uint32_t* ids, int n_prims, const ViewDev* views, bool exact, K* ikey,
               uint32_t* ival, uint2* ranges_init, uint32_t tiles, hipStream_t s) {
  if (n_max == 0) {
    if (ranges_init) launch_ranges_init(ranges_init, tiles, s);
    return;
  }
  hipLaunchKernelGGL(k_emit<K>, dim3(grid_for(n_max, kEmitRecs)), dim3(kThreads), 0, s, n_dev, n_max, toff, total,
                     cap, rec_sorted, ids, (uint32_t)n_prims, views, exact, ikey, ival, ranges_init, tiles);
}

void launch_emit(const uint32_t* n_dev, uint32_t n_max, const uint32_t* toff, const uint32_t* total, uint32_t cap,
                 const Record* rec_sorted, const uint32_t* ids, int n_prims, const ViewDev* views, bool exact,
                 uint32_t* ikey, uint32_t* ival, uint2* ranges_init, uint32_t tiles, hipStream_t s) {
  emit_keys(n_dev, n_max, toff, total, cap, rec_sorted, ids, n_prims, views, exact, ikey, ival, ranges_init, tiles,
            s);
}

void launch_emit(const uint32_t* n_dev, uint32_t n_max, const uint32_t* toff, const uint32_t* total, uint32_t cap,
                 const Record* rec_sorted, const uint32_t* ids, int n_prims, const ViewDev* views, bool exact,
                 uint16_t* ikey, uint32_t* ival, uint2* ranges_init, uint32_t tiles, hipStream_t s) {
  emit_keys(n_dev, n_max, toff, total, cap, rec_sorted, ids, n_prims, views, exact, ikey, ival, ranges_init, tiles,
            s);
}

void launch_ranges_init(uint2* ranges, uint32_t tiles, hipStream_t s) {
  if (tiles) hipLaunchKernelGGL(k_ranges_init, dim3(grid_for(tiles, 256)), dim3(256), 0, s, ranges, tiles);
}

void launch_ranges_fix(uint2* ranges, uint32_t tiles, hipStream_t s) {
  if (tiles) hipLaunchKernelGGL(k_ranges_fix, dim3(grid_for(tiles, 256)), dim3(256), 0, s, ranges, tiles);
}

void launch_ranges(const uint32_t* n_dev, uint32_t n_max, const uint32_t* ikey, uint2* ranges, hipStream_t s) {
  if (n_max == 0) return;
  hipLaunchKernelGGL(k_ranges<uint32_t>, dim3(grid_for((n_max + 3) / 4, 256)), dim3(256), 0, s, n_dev, n_max, ikey,
                     ranges);
}

void launch_ranges(const uint32_t* n_dev, uint32_t n_max, const uint16_t* ikey, uint2* ranges, hipStream_t s) {
  if (n_max == 0) return;
  hipLaunchKernelGGL(k_ranges<uint16_t>, dim3(grid_for((n_max + 3) / 4, 256)), dim3(256), 0, s, n_dev, n_max, ikey,
                     ranges);
}

void launch_sum_u32(const uint32_t* in, uint64_t n, unsigned long long* out, hipStream_t s) {
  if (n == 0) return;
  unsigned g = grid_for(n, 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_sum_u32, dim3(g), dim3(256), 0, s, in, n, out);
}

void launch_tile_order(uint2* ranges, uint32_t tiles, bool fix, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                       uint32_t* order, uint32_t* max_len, int sort_blocks, uint32_t* scratch, hipStream_t s) {
  if (tiles == 0) return;
  hipLaunchKernelGGL(k_order_keys, dim3(grid_for(tiles, 256)), dim3(256), 0, s, ranges, tiles, fix, keys, vals,
                     max_len);
  // one 8-bit pass: the result lands in (keys_alt, order), no copy back
  radix_sort(keys, vals, keys_alt, order, nullptr, tiles, 0, 8, radix_grid(tiles, sort_blocks), scratch, s,
             /*copy_back=*/false);
}

void launch_range_max(const uint2* ranges, uint32_t tiles, uint32_t* out, hipStream_t s) {
  if (tiles == 0) return;
  unsigned g = grid_for(tiles, 1024);
  hipLaunchKernelGGL(k_range_max, dim3(g > 256 ? 256 : g), dim3(256), 0, s, ranges, tiles, out);
}

}  // namespace g4d
