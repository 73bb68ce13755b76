// Internal declarations shared by the HIP translation units of libg4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace g4d {

constexpr int kTile = 16;                 // 16x16 pixel tiles
constexpr float kLowpass = 0.3f;          // EWA dilation, px^2
constexpr double kLowpass64 = 0.3;        // the same, for the FP64 forward geometry
constexpr float kFrustumSlack = 1.3f;     // Jacobian clamp, x half-fov
constexpr double kFrustumSlack64 = 1.3;
constexpr double kSigmaExtent64 = 3.0;
constexpr float kSigmaExtent = 3.0f;      // footprint radius in sigmas
constexpr float kAlphaMax = 0.99f;        // alpha clamp
constexpr float kTStop = 1e-4f;           // transmittance stop threshold
constexpr float kColorOffset = 0.5f;
// log2(1/255): fragments with log2(opacity * exp(power)) below this are skipped
constexpr float kLog2AlphaMin = -7.994353436858858f;
constexpr float kLog2e = 1.4426950408889634f;

// One view of a batch, device side.
struct ViewDev {
  int width, height, tiles_x, tiles_y;
  int tile_base;        // first global tile id of this view
  int pad0;
  long long pix_base;   // first pixel of this view in the concatenated planes
  float fx, fy, cx, cy;
  float rot[9];         // world -> camera rotation, row-major
  float trans[3];
  float center[3];      // camera position (world)
  float t;              // render time
  float lim_x, lim_y;   // Jacobian clamp limits on x/z, y/z
  double lim_x64, lim_y64;  // the same limits in FP64: 1.3 (W/2) / fx, 1.3 (H/2) / fy
};

// Doubles per active record in the screen-space gradient buffer: one 128-byte
// line holding dL/du, dL/dv, dL/dconic (3), dL/d(opacity p), dL/drgb (3),
// dL/dz, padding and (last) the blended flag. The tiles' shares are added in
// FP64: a long footprint adds terms of both signs from many tiles, whose
// float32 sum would lose the small total.
constexpr int kGrad2dStride = 16;

// Per active (view, primitive) record used by binning and rasterisation.
// 3 x float4 = 48 bytes:
//   a: u, v, z, opacity * p(t)
//   b: conic00, conic01, conic11, rect x range (x0 | x1 << 16, as float bits)
//   c: r, g, b, rect y range (y0 | y1 << 16, as float bits)
struct Record {
  float4 a, b, c;
};

struct RenderParams {
  int n;                // primitives
  int n_views;
  int sh_degree, t_order;
  float t_period, t_cull, near_plane;
  float bg[3];
  const float4* means4;
  const float4* log_scales4;
  const float4* q_left;
  const float4* q_right;
  const float* opacity_logit;
  const float* coeffs;
  const ViewDev* views;
  int flow;             // 1: records carry the image-plane flow over flow_dt instead of the colour
  float flow_dt;
  // 1 (default): a record's rectangle is cut to the box of its alpha-floor
  // ellipse and records that can never reach alpha 1/255 are culled; 0: the
  // plain 3-sigma rectangle and no opacity cull (the reference footprint rule)
  int ellipse_cull;
  // per-view counters of (view, primitive) pairs culled for a non-finite
  // parameter, indexed by the view within the call (null: not counted)
  uint32_t* nonfinite;
  // written by the preprocess: per primitive, 1 when it is active in some
  // view of the call; the list of those primitives (in no particular order)
  // and its length
  uint8_t* pany;
  uint32_t* plist;
  uint32_t* plist_n;
};

// Per-primitive densification accumulators (all null: off).
struct DensifyStats {
  float* uv_grad_norm_sum;
  float* t_grad_abs_sum;
  int32_t* blend_count;
};

// ---- launchers (preprocess.hip) ----
// cdir: per (view, primitive) scratch [n_views * n] of (view direction, t - mu_t).
void launch_preprocess(const RenderParams& p, uint32_t* act, uint32_t* dkey, Record* rec, int32_t* slot,
                       float4* cdir, hipStream_t s);
// 4DSH colour of every active pair (act[pair] set by the preprocess) into
// rec[pair].c.xyz, pair = view * n + primitive, before the gather orders the
// records by depth; nothing in flow mode.
void launch_colour(const RenderParams& p, const uint32_t* act, const float4* cdir, Record* rec, hipStream_t s);
// ---- launchers (preprocess_bwd.hip) ----
size_t preprocess_backward_scratch_floats(size_t n_records);
// Lanes per primitive in k_preprocess for a call of n_views views.
int preprocess_lanes(int n_views);
// Workgroups of the kernels that walk the active-primitive list of n primitives.
unsigned list_grid(int n);
void launch_preprocess_backward(const RenderParams& p, const int32_t* slot, const double* grad2d,
                                const uint32_t* n_records_dev, uint32_t n_records_max, const uint32_t* ids,
                                const Record* recs, float* scratch, float* g_means4, float* g_log_scales4,
                                float* g_q_left, float* g_q_right, float* g_opacity_logit, float* g_coeffs,
                                bool accumulate, const DensifyStats& stats, hipStream_t s);

// ---- launchers (loss.hip) ----
void launch_image_loss(int kind, uint64_t n, const float* img, const float* tgt, float scale, float* loss,
                       float* grad, hipStream_t s);

// ---- launchers (sort.hip) ----
// Exclusive scan of n u32 (n read from n_dev when non-null, else n_host); writes total to *total.
// With ckey: the input is a 0/1 flag per element, and every flagged element i
// is also compacted: ckey[out[i]] = dkey[i], cval[out[i]] = i.
size_t scan_scratch_words(size_t n_max);
void launch_scan(const uint32_t* in, uint32_t* out, const uint32_t* n_dev, uint32_t n_host, uint32_t n_max,
                 uint32_t* total, uint32_t* scratch, hipStream_t s, const uint32_t* dkey = nullptr,
                 uint32_t* ckey = nullptr, uint32_t* cval = nullptr);
// LSD radix sort of (key, value) pairs on bits [bit0, bit1) in 8-bit passes
// that ping-pong via alt; the result ends in keys/vals, copied back after an
// odd number of passes unless copy_back is false (then it is in the alt pair).
// With last_ranges (n_ranges entries, keys < 2^bit1, bit0 = 0, at least one
// pass, ranges set to (~0u, 0) by launch_ranges_init or the emission) the last
// pass writes no keys: it bounds each key's run in last_ranges[key] instead
// (launch_ranges_fix then empties the unused); a key >= n_ranges is skipped.
size_t radix_scratch_words(int grid);
int radix_grid(uint32_t n_max, int max_blocks);
int radix_passes(int bit0, int bit1);
void radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, const uint32_t* n_dev,
                uint32_t n_max, int bit0, int bit1, int grid, uint32_t* scratch, hipStream_t s,
                bool copy_back = true, uint2* last_ranges = nullptr, uint32_t n_ranges = 0);
// The same with 16-bit keys (bit1 <= 16), without the copy back: after an odd
// number of passes the result is in (keys_alt, vals_alt).
void radix_sort16(uint16_t* keys, uint32_t* vals, uint16_t* keys_alt, uint32_t* vals_alt, const uint32_t* n_dev,
                  uint32_t n_max, int bit0, int bit1, int grid, uint32_t* scratch, hipStream_t s,
                  uint2* last_ranges = nullptr, uint32_t n_ranges = 0);
void launch_ranges_init(uint2* ranges, uint32_t tiles, hipStream_t s);
void launch_ranges_fix(uint2* ranges, uint32_t tiles, hipStream_t s);
// Depth-ordered records, slot map (view*n + index -> depth position), tiles per record,
// and the 64-bit instance total (to detect 32-bit overflow) in inst64[0..1].
// exact: count only the rectangle's tiles the record's alpha-floor ellipse reaches.
void launch_gather(const uint32_t* n_dev, uint32_t n_max, const uint32_t* ids, const Record* rec, Record* rec_sorted,
                   int32_t* slot, uint32_t* tcount, bool exact, uint32_t* inst64, hipStream_t s);
void launch_view_counts(const uint32_t* pos, int n_views, uint32_t n, const uint32_t* total, uint32_t* out,
                        hipStream_t s);
// Instances beyond min(*total, cap) are not written; exact as for launch_gather.
// Keys are 16-bit when the round's tile ids are below 2^16, else 32-bit. With
// ranges_init, the launch also sets ranges_init[0..tiles) to (~0u, 0), the
// start state of the ranges the sort's last pass fills.
void launch_emit(const uint32_t* n_dev, uint32_t n_max, const uint32_t* toff, const uint32_t* total, uint32_t cap,
                 const Record* rec_sorted, const uint32_t* ids, int n_prims, const ViewDev* views, bool exact,
                 uint32_t* ikey, uint32_t* ival, uint2* ranges_init, uint32_t tiles, hipStream_t s);
void launch_emit(const uint32_t* n_dev, uint32_t n_max, const uint32_t* toff, const uint32_t* total, uint32_t cap,
                 const Record* rec_sorted, const uint32_t* ids, int n_prims, const ViewDev* views, bool exact,
                 uint16_t* ikey, uint32_t* ival, uint2* ranges_init, uint32_t tiles, hipStream_t s);
void launch_ranges(const uint32_t* n_dev, uint32_t n_max, const uint32_t* ikey, uint2* ranges, hipStream_t s);
void launch_ranges(const uint32_t* n_dev, uint32_t n_max, const uint16_t* ikey, uint2* ranges, hipStream_t s);

// ---- launchers (raster.hip) ----
// order (nullable): the tiles in the order workgroups take them, e.g.
// heaviest lists first. queue (nullable): a device counter; then `blocks`
// workgroups (-1: as many as stay resident) take tiles from it in that order
// until they run out (zeroed before the launch); otherwise one workgroup per
// tile. batch (forward): list entries staged in LDS at a time, 64, 128 or 256.
// channels: 3 (rgb planes) or 2 (the first two record colour values, e.g. flow).
// cull: waves walk only the entries whose alpha-floor ellipse meets their
// quadrant (false: every entry; same results).
void launch_raster_forward(int total_tiles, const uint32_t* order, uint32_t* queue, int blocks, int batch,
                           int n_views, const ViewDev* views, const uint2* ranges, const uint32_t* ival,
                           const Record* rec_sorted, const float* bg, int channels, bool cull, float* out_rgb,
                           float* out_depth, float* out_alpha, float* pix_t, uint32_t* pix_last, hipStream_t s);
// The image loss folded into the backward rasteriser: with kind (1 = L1,
// 2 = L2) the rgb input is the rendered image, dL/dC is formed from it and
// target as launch_image_loss forms it, and part[tile] (the launch's tile id)
// receives the tile's unscaled loss sum. kind 0: the rgb input is dL/dC.
struct LossArgs {
  int kind;
  const float* target;
  float scale;
  float* part;
};
void launch_raster_backward(int total_tiles, const uint32_t* order, uint32_t* queue, int blocks, int n_views,
                            const ViewDev* views, const uint2* ranges, const uint32_t* ival,
                            const Record* rec_sorted, const float* bg, const float* dl_rgb, const float* dl_depth,
                            const float* dl_alpha, const float* pix_t, const uint32_t* pix_last, double* grad2d,
                            bool mark_blended, bool cull, const LossArgs& loss, hipStream_t s);
// *loss += scale * sum(part[0..n)) (one workgroup, fixed order).
void launch_loss_partials(const float* part, uint32_t n, float scale, float* loss, hipStream_t s);
void launch_sum_u32(const uint32_t* in, uint64_t n, unsigned long long* out, hipStream_t s);
void launch_range_max(const uint2* ranges, uint32_t tiles, uint32_t* out, hipStream_t s);
// Tile ids by decreasing list length (stable within ~4.4 % length bins) into
// order, through the scratch keys, vals and keys_alt. With fix it first
// empties the ranges the last radix pass did not reach (as launch_ranges_fix),
// and it raises *max_len to the longest list (as launch_range_max).
void launch_tile_order(uint2* ranges, uint32_t tiles, bool fix, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                       uint32_t* order, uint32_t* max_len, int sort_blocks, uint32_t* scratch, hipStream_t s);

// ---- launchers (optim.hip) ----
constexpr int kAdamGroups = 6;
struct AdamGroups {
  float* param[kAdamGroups];
  const float* grad[kAdamGroups];
  uint64_t end[kAdamGroups];  // cumulative element counts
  float lr[kAdamGroups];
};
// bc1 = 1 - beta1^step, bc2 = 1 - beta2^step; m, v: [end[5]] moment buffers.
void launch_adam(const AdamGroups& a, float b1, float b2, float eps, float bc1, float bc2, float* m, float* v,
                 hipStream_t s);
// out[k] = mu_i + R_i S_i z[k], i = idx[k]; NaN rows for i outside [0, n).
void launch_split_sample(const RenderParams& p, uint64_t count, const int32_t* idx, const float* z, float* out,
                         hipStream_t s);

// ---- launchers (util.hip) ----
// Views reach the device through kernel arguments, never a host copy.
void launch_set_views(const ViewDev* host, int n, ViewDev* dev, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t value, hipStream_t s);
// Zeroes floats_per_item (a multiple of 4) floats per item for min(*n_dev, max_items) items.
void launch_zero_counted(float* p, const uint32_t* n_dev, uint32_t floats_per_item, uint64_t max_items,
                         hipStream_t s);
// If the 64-bit instance total at inst64 exceeds cap: *overflow = 1 and
// *n_inst = 0. Then, with a_tot: *a_tot += *a and *(uint64*)i_tot64 += *n_inst
// (one thread).
void launch_cap_check(const uint32_t* inst64, uint32_t* n_inst, uint32_t* overflow, uint64_t cap, hipStream_t s,
                      const uint32_t* a = nullptr, uint32_t* a_tot = nullptr, uint32_t* i_tot64 = nullptr);
void launch_copy_pairs(const uint32_t* ka, const uint32_t* va, uint32_t* kb, uint32_t* vb, const uint32_t* n_dev,
                       uint32_t n_max, hipStream_t s);

}  // namespace g4d
