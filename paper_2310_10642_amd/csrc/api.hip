// C ABI of libg4d: context, argument validation, scratch management and the
// enqueue order of the render and backward passes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/g4d.h"
#include "g4d_common.h"

using namespace g4d;

namespace {

struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
};

}  // namespace

struct g4d_ctx {
  g4d_options opts{};
  hipStream_t stream = nullptr;
  // The colour pass runs on a second stream, overlapping the instance
  // emission and tile sort; the rasterisers wait for it.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool side_pending = false;
  int device = 0;
  std::string err;
  bool hip_failed = false;

  // borrowed primitives
  int64_t n = -1;
  const float *means4 = nullptr, *log_scales4 = nullptr, *q_left = nullptr, *q_right = nullptr;
  const float *opacity_logit = nullptr, *coeffs = nullptr;
  DensifyStats densify{nullptr, nullptr, nullptr};  // borrowed accumulators

  // last render
  struct Round {
    int v0, v1;    // views [v0, v1)
    int tiles;     // tiles of those views
    uint32_t A, I; // active records and tile instances
  };
  bool have_render = false;
  int n_views = 0;
  std::vector<ViewDev> views_h;  // every view; tile_base is set per round
  int64_t total_tiles = 0;
  int64_t total_pix = 0;
  std::vector<Round> rounds;
  int bound = -1;                // round whose records and bins are resident
  uint64_t A_total = 0, I_total = 0;
  std::vector<uint32_t> view_active;
  uint32_t active_hint = 0;      // most active records seen in one view (sizes the depth sort's grid)
  // five radix-sort workgroups per CU: the 16-bit downsweep's LDS (30 KB) and
  // registers (83) let five share a CU, and its blocks then fill them at once
  int sort_blocks = 1280;
  int64_t round_pairs = int64_t(1) << 28;
  int64_t round_instances = int64_t(1) << 30;
  bool sync_free = false;          // no host read of device counts inside render/backward
  bool totals_on_device = false;   // the last render was sync-free: its totals are device counters
  bool heavy_first = true;         // rasterise tiles by decreasing list length
  int persistent_blocks = 0;       // rasteriser workgroups taking tiles from a queue (0: one per tile)
  int lds_batch = 256;             // forward rasteriser: list entries staged in LDS at a time
  bool ellipse_cull = true;        // bin and walk by the alpha-floor ellipse, not its rectangle
  bool autotune_pending = false;   // the next uncaptured render tunes the knobs first
  bool flow_mode = false;          // the render in progress blends flow (Sec. 4.4), not colour
  float flow_dt = 0.f;
  bool no_alloc = false;           // a render_noalloc is in progress: scratch never grows
  void* fixed_scratch = nullptr;   // this device's no-allocation scratch (see g4d_render_noalloc)

  DevBuf views_d, act, pos, dkey, rec, slot, ckey, cval, ckey2, cval2, rec_sorted, tcount, toff;
  DevBuf ikey, ival, ikey2, ival2, ranges, pix_t, pix_last, grad2d, scan_scratch, radix_scratch, counters;
  DevBuf bwd_scratch, okey, oval, okey2, oval2, cdir, pany, plist, loss_part;
  uint32_t* counters_h = nullptr;  // pinned

  // stage timing (HIP events on the context's stream)
  bool timing = false;
  struct EvPair {
    hipEvent_t a, b;
    int stage;
  };
  std::vector<EvPair> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open_ev = nullptr;
  hipEvent_t side_open_ev = nullptr;  // the open stage on the side stream
  double stage_ms[G4D_NUM_STAGES] = {};
  int64_t stage_n[G4D_NUM_STAGES] = {};
};

namespace {

// counters layout (uint32 words)
constexpr int kCntA = 0;          // active records
constexpr int kCntI = 1;          // instances
constexpr int kCntInst64 = 2;     // 64-bit instance total (words 2, 3)
constexpr int kCntFrag = 4;       // 64-bit fragment sum (words 4, 5)
constexpr int kCntMaxList = 6;    // longest tile list over the rounds of a render
constexpr int kCntOverflow = 7;   // sticky: a sync-free render exceeded the instance arena
constexpr int kCntViews = 8;      // per-view active counts follow
constexpr int kMaxViews = 4096;
// after the views: a sync-free render's totals over its rounds, active
// records (u32) and instances (64-bit, words +2, +3)
constexpr int kCntTot = kCntViews + kMaxViews;
// then per view: (view, primitive) pairs culled for a non-finite parameter
constexpr int kCntNF = kCntTot + 4;
// then the length of the round's list of primitives active in some view
constexpr int kCntPList = kCntNF + kMaxViews;
constexpr int kCntQueue = kCntPList + 1;  // the rasterisers' tile queue head
constexpr int kCntWords = kCntPList + 4;
constexpr uint32_t kOnDevice = 0xFFFFFFFFu;  // a round count known only on the device
// Tiles per round (unless one view alone has more): tile ids then fit 16
// bits, and the instance sort by tile takes two 8-bit passes.
constexpr int64_t kRoundTiles = int64_t(1) << 16;

// ---- the no-allocation render's scratch ----
// Limits of g4d_render_noalloc: (view, primitive) pairs per round (and
// primitives), tile instances per round, pixels per call, 16x16 tiles per
// round, radix-sort workgroups.
constexpr size_t kNAPairs = size_t(1) << 19;
constexpr size_t kNAInstances = size_t(1) << 22;
constexpr size_t kNAPixels = size_t(1) << 21;
constexpr size_t kNATiles = size_t(1) << 16;
constexpr int kNASortBlocks = 2048;

size_t na_align(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of each scratch buffer of a render at the limits, in carving order
// (the order of g4d_ctx::render_bufs).
void na_sizes(size_t* out) {
  const size_t P = kNAPairs, I = kNAInstances, X = kNAPixels, T = kNATiles;
  const size_t sizes[] = {
      sizeof(ViewDev) * kMaxViews,                                    // views_d
      4 * P, 4 * P, 4 * P, 4 * P, 4 * P, 4 * P, 4 * P, 4 * P,         // act pos dkey slot ckey cval ckey2 cval2
      4 * P, 4 * P,                                                   // tcount toff
      sizeof(Record) * P, sizeof(Record) * P, sizeof(float4) * P,     // rec rec_sorted cdir
      P, 4 * P,                                                       // pany plist (primitives <= P)
      4 * scan_scratch_words(P), 4 * radix_scratch_words(kNASortBlocks),
      4 * I, 4 * I, 4 * I, 4 * I,                                     // ikey ival ikey2 ival2
      8 * T, 4 * T, 4 * T, 4 * T, 4 * T,                              // ranges okey oval okey2 oval2
      4 * X, 4 * X,                                                   // pix_t pix_last
      sizeof(uint32_t) * kCntWords};                                  // counters
  for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i) out[i] = sizes[i];
}
constexpr int kNABufs = 30;

constexpr size_t na_total_bytes() {
  // an upper bound of the carved total (each buffer 256-byte aligned)
  return (sizeof(ViewDev) * kMaxViews + 256) + 12 * (4 * kNAPairs + 256) + 2 * (48 * kNAPairs + 256) +
         (16 * kNAPairs + 256) + (5 * kNAPairs + 512) + (4 * (kNAPairs / 4096 + 2) + 256) + (4 * (256 * kNASortBlocks + 256) + 256) +
         4 * (4 * kNAInstances + 256) + (8 * kNATiles + 256) + 4 * (4 * kNATiles + 256) + 2 * (4 * kNAPixels + 256) +
         (4 * kCntWords + 256);
}

}  // namespace

// The no-allocation render's scratch: one array per GPU, held until the
// process ends. Host code reaches it only through the address that
// hipGetSymbolAddress gives per device (g4d_create), never through its name.
static __device__ __align__(256) unsigned char scratch[na_total_bytes()];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// This device's address of `scratch` (the device is current); null on failure.
void* device_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_dev[device] = ptr;
  }
  return g_scratch_dev[device];
}

g4d_status fail(g4d_ctx* c, g4d_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

g4d_status check_hip(g4d_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return G4D_OK;
  c->hip_failed = true;
  c->err = std::string(what) + ": " + hipGetErrorString(e);
  return G4D_EHIP;
}

#define HIPCHK(c, expr)                                   \
  do {                                                    \
    g4d_status _s = check_hip((c), (expr), #expr);        \
    if (_s != G4D_OK) return _s;                          \
  } while (0)

bool capturing(g4d_ctx* c) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st != hipStreamCaptureStatusNone;
}

// Grows a scratch buffer (25% headroom). Growth synchronises the stream and
// allocates, so it is refused while the stream is being captured.
g4d_status ensure(g4d_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return G4D_OK;
  if (c->no_alloc)
    return fail(c, G4D_ECAPACITY, "the render needs " + std::to_string(bytes) + " bytes of a scratch buffer that "
                                  "holds " + std::to_string(b.cap) + " in the no-allocation render");
  if (capturing(c))
    return fail(c, G4D_ECAPACITY, "a scratch buffer would grow during stream capture; make the same call "
                                  "uncaptured first");
  if (b.ptr) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(b.ptr));
    b.ptr = nullptr;
    b.cap = 0;
  }
  const size_t want = bytes + bytes / 4;
  hipError_t e = hipMalloc(&b.ptr, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.ptr = nullptr;
    return fail(c, G4D_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  b.cap = want;
  return G4D_OK;
}

template <typename T>
T* P(DevBuf& b) { return reinterpret_cast<T*>(b.ptr); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

int ceil_log2(uint32_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

hipEvent_t take_event(g4d_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void stage_begin(g4d_ctx* c) {
  if (!c->timing || capturing(c)) return;
  c->open_ev = take_event(c);
  if (c->open_ev) (void)hipEventRecord(c->open_ev, c->stream);
}

// A stage enqueued on the side stream, timed by its own pair of events.
void side_stage_begin(g4d_ctx* c) {
  if (!c->timing || capturing(c)) return;
  c->side_open_ev = take_event(c);
  if (c->side_open_ev) (void)hipEventRecord(c->side_open_ev, c->side);
}

void side_stage_end(g4d_ctx* c, int stage) {
  if (!c->timing || !c->side_open_ev || capturing(c)) return;
  hipEvent_t e = take_event(c);
  if (!e) return;
  (void)hipEventRecord(e, c->side);
  c->pending.push_back({c->side_open_ev, e, stage});
  c->side_open_ev = nullptr;
}

void stage_end(g4d_ctx* c, int stage) {
  if (!c->timing || !c->open_ev || capturing(c)) return;
  hipEvent_t e = take_event(c);
  if (!e) return;
  (void)hipEventRecord(e, c->stream);
  c->pending.push_back({c->open_ev, e, stage});
  c->open_ev = nullptr;
}

g4d_status collect_times(g4d_ctx* c) {
  if (c->pending.empty()) return G4D_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipStreamSynchronize(c->side));
  for (auto& p : c->pending) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->stage_ms[p.stage] += ms;
    c->stage_n[p.stage] += 1;
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  return G4D_OK;
}

RenderParams make_params(g4d_ctx* c, int n_views) {
  RenderParams p{};
  p.n = (int)c->n;
  p.n_views = n_views;
  p.sh_degree = c->opts.sh_degree;
  p.t_order = c->opts.t_order;
  p.t_period = c->opts.t_period;
  p.t_cull = c->opts.t_cull;
  p.near_plane = c->opts.near_plane;
  for (int i = 0; i < 3; ++i) p.bg[i] = c->opts.bg[i];
  p.means4 = reinterpret_cast<const float4*>(c->means4);
  p.log_scales4 = reinterpret_cast<const float4*>(c->log_scales4);
  p.q_left = reinterpret_cast<const float4*>(c->q_left);
  p.q_right = reinterpret_cast<const float4*>(c->q_right);
  p.opacity_logit = c->opacity_logit;
  p.coeffs = c->coeffs;
  p.views = P<ViewDev>(c->views_d);
  p.flow = c->flow_mode ? 1 : 0;
  p.flow_dt = c->flow_dt;
  p.ellipse_cull = c->ellipse_cull ? 1 : 0;
  p.nonfinite = nullptr;
  p.pany = P<uint8_t>(c->pany);
  p.plist = P<uint32_t>(c->plist);
  p.plist_n = c->counters.ptr ? P<uint32_t>(c->counters) + kCntPList : nullptr;
  return p;
}

// The main stream waits for a colour pass still running on the side stream.
g4d_status join_side(g4d_ctx* c) {
  if (!c->side_pending) return G4D_OK;
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  c->side_pending = false;
  return G4D_OK;
}

// Starts the colour pass of the enqueued pairs on the side stream, after
// everything enqueued so far on the main stream (the preprocess in particular).
g4d_status fork_colour(g4d_ctx* c, const RenderParams& p) {
  if (p.flow || p.n == 0) return G4D_OK;
  HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
  HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  side_stage_begin(c);
  launch_colour(p, P<uint32_t>(c->act), P<float4>(c->cdir), P<Record>(c->rec), c->side);
  side_stage_end(c, G4D_STAGE_COLOUR);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(c->ev_join, c->side));
  c->side_pending = true;
  return G4D_OK;
}

int round_tiles(const g4d_ctx* c, int v0, int v1) {
  int64_t t = 0;
  for (int v = v0; v < v1; ++v) t += (int64_t)c->views_h[v].tiles_x * c->views_h[v].tiles_y;
  return (int)t;
}

// Per-pair stage of one round, views [v0, v1): preprocess every (view,
// primitive) pair, compact the active ones, sort them by depth, gather the
// records in that order and scan their tile counts. Counts stay on the device.
// count: the pairs culled for a non-finite parameter are counted per view
// (a render; not the binning again of a backward).
g4d_status enqueue_pairs(g4d_ctx* c, int v0, int v1, bool count) {
  g4d_status st = join_side(c);  // the last colour pass writes buffers reused below
  if (st) return st;
  c->bound = -1;
  hipStream_t s = c->stream;
  const int nv = v1 - v0;
  std::vector<ViewDev> vr(c->views_h.begin() + v0, c->views_h.begin() + v1);
  int tile_base = 0;
  for (ViewDev& d : vr) {
    d.tile_base = tile_base;
    tile_base += d.tiles_x * d.tiles_y;
  }
  const uint64_t vn = (uint64_t)c->n * nv;
  if ((st = ensure(c, c->views_d, sizeof(ViewDev) * nv))) return st;
  if ((st = ensure(c, c->act, 4 * vn))) return st;
  if ((st = ensure(c, c->pos, 4 * vn))) return st;
  if ((st = ensure(c, c->dkey, 4 * vn))) return st;
  if ((st = ensure(c, c->slot, 4 * vn))) return st;
  if ((st = ensure(c, c->rec, sizeof(Record) * vn))) return st;
  if ((st = ensure(c, c->cdir, sizeof(float4) * vn))) return st;
  if ((st = ensure(c, c->ckey, 4 * vn))) return st;
  if ((st = ensure(c, c->cval, 4 * vn))) return st;
  if ((st = ensure(c, c->ckey2, 4 * vn))) return st;
  if ((st = ensure(c, c->cval2, 4 * vn))) return st;
  if ((st = ensure(c, c->rec_sorted, sizeof(Record) * vn))) return st;
  if ((st = ensure(c, c->tcount, 4 * vn))) return st;
  if ((st = ensure(c, c->toff, 4 * vn))) return st;
  if ((st = ensure(c, c->pany, (size_t)c->n))) return st;
  if ((st = ensure(c, c->plist, 4 * (size_t)c->n))) return st;
  if ((st = ensure(c, c->scan_scratch, 4 * scan_scratch_words(vn)))) return st;
  if ((st = ensure(c, c->radix_scratch, 4 * radix_scratch_words(c->sort_blocks)))) return st;
  RenderParams p = make_params(c, nv);
  uint32_t* cnt = P<uint32_t>(c->counters);
  if (count) p.nonfinite = cnt + kCntNF + v0;

  launch_set_views(vr.data(), nv, P<ViewDev>(c->views_d), s);
  launch_fill_u32(cnt, 4, 0u, s);
  launch_fill_u32(cnt + kCntPList, 1, 0u, s);
  if (count) launch_fill_u32(cnt + kCntNF + v0, (uint64_t)nv, 0u, s);
  // 1. per (view, primitive): cull, slice, project (the colour follows the
  //    gather, on the second stream)
  stage_begin(c);
  launch_preprocess(p, P<uint32_t>(c->act), P<uint32_t>(c->dkey), P<Record>(c->rec), P<int32_t>(c->slot),
                    P<float4>(c->cdir), s);
  stage_end(c, G4D_STAGE_PREPROCESS);
  // the records' colours on the second stream, beside the scans and the
  // depth sort (joined before the gather copies the records)
  if ((st = fork_colour(c, p))) return st;
  // 2. compaction of active records
  stage_begin(c);
  launch_scan(P<uint32_t>(c->act), P<uint32_t>(c->pos), nullptr, (uint32_t)vn, (uint32_t)vn, cnt + kCntA,
              P<uint32_t>(c->scan_scratch), s, P<uint32_t>(c->dkey), P<uint32_t>(c->ckey), P<uint32_t>(c->cval));
  // per-view counts: at the round's place for a sync-free render, which
  // reads them only after its last round
  launch_view_counts(P<uint32_t>(c->pos), nv, (uint32_t)c->n, cnt + kCntA,
                     cnt + kCntViews + (c->totals_on_device ? v0 : 0), s);
  // 3. stable sort by depth; its grid is sized from the active records seen
  // so far (any grid gives the same order: blocks take ranges of the count
  // the device holds)
  const uint64_t est = c->active_hint ? std::min<uint64_t>(vn, (uint64_t)c->active_hint * nv * 5 / 4 + 4096) : vn;
  const int g_depth = radix_grid((uint32_t)est, c->sort_blocks);
  radix_sort(P<uint32_t>(c->ckey), P<uint32_t>(c->cval), P<uint32_t>(c->ckey2), P<uint32_t>(c->cval2), cnt + kCntA,
             (uint32_t)vn, 0, 32, g_depth, P<uint32_t>(c->radix_scratch), s);
  // 4. depth-ordered records, slot map, tiles per record; 5. instance offsets
  if ((st = join_side(c))) return st;
  launch_gather(cnt + kCntA, (uint32_t)vn, P<uint32_t>(c->cval), P<Record>(c->rec), P<Record>(c->rec_sorted),
                P<int32_t>(c->slot), P<uint32_t>(c->tcount), c->ellipse_cull, cnt + kCntInst64, s);
  launch_scan(P<uint32_t>(c->tcount), P<uint32_t>(c->toff), cnt + kCntA, 0, (uint32_t)vn, cnt + kCntI,
              P<uint32_t>(c->scan_scratch), s);
  stage_end(c, G4D_STAGE_BINNING);
  HIPCHK(c, hipGetLastError());
  return G4D_OK;
}

// Reads a round's active count, instance total and per-view counts
// (synchronises the stream).
g4d_status read_pairs(g4d_ctx* c, int v0, int nv, uint32_t& A, uint64_t& inst64) {
  uint32_t* cnt = P<uint32_t>(c->counters);
  const int vb = kCntViews + (c->totals_on_device ? v0 : 0);  // where enqueue_pairs put the view counts
  HIPCHK(c, hipMemcpyAsync(c->counters_h, cnt, sizeof(uint32_t) * (vb + nv), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  A = c->counters_h[kCntA];
  std::memcpy(&inst64, c->counters_h + kCntInst64, sizeof(inst64));
  std::copy(c->counters_h + vb, c->counters_h + vb + nv, c->view_active.begin() + v0);
  for (int v = 0; v < nv; ++v) c->active_hint = std::max(c->active_hint, c->counters_h[vb + v]);
  return G4D_OK;
}

// Views [v0, v0 + k) cut to at most kRoundTiles tiles (at least one view).
int cap_round_tiles(const g4d_ctx* c, int v0, int k) {
  int64_t t = 0;
  for (int j = 0; j < k; ++j) {
    t += (int64_t)c->views_h[v0 + j].tiles_x * c->views_h[v0 + j].tiles_y;
    if (t > kRoundTiles && j > 0) return j;
  }
  return k;
}

uint64_t arena_instances(const g4d_ctx* c) {
  return std::min(std::min(c->ikey.cap, c->ival.cap), std::min(c->ikey2.cap, c->ival2.cap)) / 4;
}

// Per-instance stage of a round whose pairs are binned: emit the (tile,
// record) instances, sort them stably by tile and find each tile's range.
// a_max bounds the active records and cap the instances (the device counts
// decide within those bounds).
g4d_status bin_tiles(g4d_ctx* c, int tiles, uint32_t a_max, uint32_t cap) {
  hipStream_t s = c->stream;
  g4d_status st;
  if ((st = ensure(c, c->ikey, 4 * (size_t)cap))) return st;
  if ((st = ensure(c, c->ival, 4 * (size_t)cap))) return st;
  if ((st = ensure(c, c->ikey2, 4 * (size_t)cap))) return st;
  if ((st = ensure(c, c->ival2, 4 * (size_t)cap))) return st;
  if ((st = ensure(c, c->ranges, sizeof(uint2) * (size_t)tiles))) return st;
  uint32_t* cnt = P<uint32_t>(c->counters);
  // 6. emit (tile, record) instances; 7. stable sort by tile; 8. ranges
  stage_begin(c);
  // the instances are emitted into whichever buffer pair makes the sort's
  // last pass land in (ikey, ival), so no copy follows an odd pass count;
  // that pass writes the tile ranges instead of the keys (one tile: no
  // passes, the ranges come from the emitted keys)
  const int tile_bits = ceil_log2((uint32_t)tiles);
  const int passes = radix_passes(0, tile_bits);
  const bool odd = passes & 1;
  // with sort passes the emission starts the ranges (see launch_emit)
  if (!passes) launch_fill_u32(P<uint32_t>(c->ranges), 2 * (uint64_t)tiles, 0u, s);
  void* ek = (odd ? c->ikey2 : c->ikey).ptr;
  void* ak = (odd ? c->ikey : c->ikey2).ptr;
  uint32_t* ev = P<uint32_t>(odd ? c->ival2 : c->ival);
  uint32_t* av = P<uint32_t>(odd ? c->ival : c->ival2);
  const uint32_t* ids = P<uint32_t>(c->cval);
  const Record* rs = P<Record>(c->rec_sorted);
  const ViewDev* vd = P<ViewDev>(c->views_d);
  // a round of more instances than the last-level cache holds (2^26, ~400 MB
  // of keys and values in flight) sorts faster on three workgroups per CU
  // (768 on 256 CUs: fewer partial cache lines open at once) than on five
  const int g_tile = radix_grid(cap, cap > (1u << 26) ? std::min(c->sort_blocks, 768) : c->sort_blocks);
  uint32_t* rsc = P<uint32_t>(c->radix_scratch);
  uint2* rg = P<uint2>(c->ranges);
  uint2* rg_init = passes ? rg : nullptr;
  // a round's tile ids fit 16 bits unless one view alone has more tiles;
  // 16-bit keys take a quarter off the sort's bytes per instance
  if (tile_bits <= 16) {
    uint16_t *k16 = static_cast<uint16_t*>(ek), *a16 = static_cast<uint16_t*>(ak);
    launch_emit(cnt + kCntA, a_max, P<uint32_t>(c->toff), cnt + kCntI, cap, rs, ids, (int)c->n, vd,
                c->ellipse_cull, k16, ev, rg_init, (uint32_t)tiles, s);
    if (passes) radix_sort16(k16, ev, a16, av, cnt + kCntI, cap, 0, tile_bits, g_tile, rsc, s, rg, (uint32_t)tiles);
    else launch_ranges(cnt + kCntI, cap, k16, rg, s);
  } else {
    uint32_t *k32 = static_cast<uint32_t*>(ek), *a32 = static_cast<uint32_t*>(ak);
    launch_emit(cnt + kCntA, a_max, P<uint32_t>(c->toff), cnt + kCntI, cap, rs, ids, (int)c->n, vd,
                c->ellipse_cull, k32, ev, rg_init, (uint32_t)tiles, s);
    radix_sort(k32, ev, a32, av, cnt + kCntI, cap, 0, tile_bits, g_tile, rsc, s, /*copy_back=*/false, rg,
               (uint32_t)tiles);
  }
  if (c->heavy_first) {
    // workgroups take the tiles with the longest lists first, so the launch
    // does not end on a few heavy tiles (its key pass also fixes the ranges
    // and finds the longest list); the order lands in oval
    for (DevBuf* b : {&c->okey, &c->oval, &c->okey2, &c->oval2})
      if ((st = ensure(c, *b, 4 * (size_t)tiles))) return st;
    launch_tile_order(rg, (uint32_t)tiles, passes > 0, P<uint32_t>(c->okey), P<uint32_t>(c->oval2),
                      P<uint32_t>(c->okey2), P<uint32_t>(c->oval), cnt + kCntMaxList, c->sort_blocks, rsc, s);
  } else {
    if (passes) launch_ranges_fix(rg, (uint32_t)tiles, s);
    launch_range_max(rg, (uint32_t)tiles, cnt + kCntMaxList, s);
  }
  stage_end(c, G4D_STAGE_BINNING);
  HIPCHK(c, hipGetLastError());
  return G4D_OK;
}

g4d_status rasterise_round(g4d_ctx* c, const g4d_ctx::Round& r, float* out_rgb, float* out_depth, float* out_alpha) {
  hipStream_t s = c->stream;
  g4d_status st = join_side(c);  // the records' colours
  if (st) return st;
  // 9. rasterise the round's views into their places in the outputs
  stage_begin(c);
  static const float kZero3[3] = {0.f, 0.f, 0.f};
  launch_raster_forward(r.tiles, c->heavy_first ? P<uint32_t>(c->oval) : nullptr,
                        c->persistent_blocks ? P<uint32_t>(c->counters) + kCntQueue : nullptr, c->persistent_blocks,
                        c->lds_batch, r.v1 - r.v0,
                        P<ViewDev>(c->views_d), P<uint2>(c->ranges), P<uint32_t>(c->ival), P<Record>(c->rec_sorted),
                        c->flow_mode ? kZero3 : c->opts.bg, c->flow_mode ? 2 : 3, c->ellipse_cull, out_rgb,
                        out_depth, out_alpha,
                        P<float>(c->pix_t), P<uint32_t>(c->pix_last), s);
  stage_end(c, G4D_STAGE_RASTER_FWD);
  HIPCHK(c, hipGetLastError());
  return G4D_OK;
}

// Fills a sync-free round's counts from the device (synchronises).
g4d_status resolve_round(g4d_ctx* c, g4d_ctx::Round& r) {
  if (r.A != kOnDevice) return G4D_OK;
  uint32_t A = 0;
  uint64_t inst = 0;
  g4d_status st = read_pairs(c, r.v0, r.v1 - r.v0, A, inst);
  if (st) return st;
  r.A = A;
  r.I = c->counters_h[kCntI];  // zero after an overflow
  return G4D_OK;
}

// The render's scratch buffers in the carving order of na_sizes.
void render_bufs(g4d_ctx* c, DevBuf** b) {
  DevBuf* l[kNABufs] = {&c->views_d, &c->act,  &c->pos,   &c->dkey,  &c->slot,   &c->ckey,         &c->cval,
                        &c->ckey2,   &c->cval2, &c->tcount, &c->toff, &c->rec,    &c->rec_sorted,   &c->cdir,
                        &c->pany,    &c->plist, &c->scan_scratch, &c->radix_scratch, &c->ikey, &c->ival, &c->ikey2, &c->ival2, &c->ranges,
                        &c->okey,    &c->oval,  &c->okey2, &c->oval2, &c->pix_t,  &c->pix_last,     &c->counters};
  for (int i = 0; i < kNABufs; ++i) b[i] = l[i];
}

// Times the render of this batch under the knobs that do not change results
// and keeps the fastest, one knob group at a time with the others at their
// best so far: radix-sort workgroups; tile order x persistent rasteriser
// (queue of resident workgroups or one workgroup per tile); the forward
// rasteriser's LDS batch. Each candidate renders once to size its scratch,
// then twice timed.
g4d_status autotune(g4d_ctx* c, int32_t n_views, const g4d_camera* cams, const float* times, float* rgb, float* dep,
                    float* alp) {
  const bool timing = c->timing;
  c->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  g4d_status st = check_hip(c, hipEventCreate(&e0), "hipEventCreate");
  if (!st) st = check_hip(c, hipEventCreate(&e1), "hipEventCreate");
  // time the render with the knobs as set
  const auto time_it = [&](float& ms) -> g4d_status {
    g4d_status s2;
    if ((s2 = g4d_render(c, n_views, cams, times, rgb, dep, alp))) return s2;
    if ((s2 = check_hip(c, hipEventRecord(e0, c->stream), "hipEventRecord"))) return s2;
    for (int k = 0; k < 2; ++k)
      if ((s2 = g4d_render(c, n_views, cams, times, rgb, dep, alp))) return s2;
    if ((s2 = check_hip(c, hipEventRecord(e1, c->stream), "hipEventRecord"))) return s2;
    if ((s2 = check_hip(c, hipEventSynchronize(e1), "hipEventSynchronize"))) return s2;
    return check_hip(c, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  };
  float best = 0.f;
  bool first = true;
  // candidate -> knobs; keeps the fastest
  const auto pick = [&](int n, const std::function<void(int)>& set) -> g4d_status {
    int best_i = -1;
    float best_here = 0.f;
    for (int i = 0; i < n; ++i) {
      set(i);
      float ms = 0.f;
      const g4d_status s2 = time_it(ms);
      if (s2) return s2;
      if (best_i < 0 || ms < best_here) {
        best_here = ms;
        best_i = i;
      }
    }
    set(best_i);
    if (first || best_here < best) best = best_here;
    first = false;
    return G4D_OK;
  };
  const int blocks[] = {512, 1024, 1280, 2048};
  const int batches[] = {64, 128, 256};
  if (!st) st = pick(4, [&](int i) { c->sort_blocks = blocks[i]; });
  if (!st)
    st = pick(4, [&](int i) {
      c->heavy_first = (i & 1) != 0;
      c->persistent_blocks = (i & 2) ? -1 : 0;
    });
  if (!st) st = pick(3, [&](int i) { c->lds_batch = batches[i]; });
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->timing = timing;
  return st;
}

}  // namespace

extern "C" {

void g4d_default_options(g4d_options* o) {
  if (!o) return;
  o->sh_degree = 3;
  o->t_order = 2;
  o->t_period = 1.0f;
  o->t_cull = 0.05f;
  o->near_plane = 0.2f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
}

g4d_status g4d_create(const g4d_options* opts, void* hip_stream, g4d_ctx** out) {
  if (!opts || !out) return G4D_EINVAL;
  if (opts->sh_degree < 0 || opts->sh_degree > 3 || opts->t_order < 0 || opts->t_order > 2) return G4D_EINVAL;
  if (!(opts->t_period > 0.f) || !std::isfinite(opts->t_period) || !(opts->t_cull >= 0.f) ||
      !(opts->t_cull <= 1.f) || !(opts->near_plane > 0.f) || !std::isfinite(opts->near_plane))
    return G4D_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(opts->bg[i])) return G4D_EINVAL;
  g4d_ctx* c = new g4d_ctx();
  c->opts = *opts;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->side) (void)hipStreamDestroy(c->side);
    delete c;
    return G4D_EHIP;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->counters_h), kCntWords * sizeof(uint32_t),
                    hipHostMallocDefault) != hipSuccess) {
    delete c;
    return G4D_ENOMEM;
  }
  // this device's copy of the no-allocation scratch (looked up once per device)
  c->fixed_scratch = device_scratch(c->device);
  if (!c->fixed_scratch) {
    (void)hipHostFree(c->counters_h);
    (void)hipEventDestroy(c->ev_fork);
    (void)hipEventDestroy(c->ev_join);
    (void)hipStreamDestroy(c->side);
    delete c;
    return G4D_EHIP;
  }
  *out = c;
  return G4D_OK;
}

g4d_status g4d_destroy(g4d_ctx* c) {
  if (!c) return G4D_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  (void)hipStreamSynchronize(c->side);
  DevBuf* bufs[] = {&c->views_d, &c->act, &c->pos, &c->dkey, &c->rec, &c->slot, &c->ckey, &c->cval, &c->ckey2,
                    &c->cval2, &c->rec_sorted, &c->tcount, &c->toff, &c->ikey, &c->ival, &c->ikey2, &c->ival2,
                    &c->ranges, &c->pix_t, &c->pix_last, &c->grad2d, &c->scan_scratch, &c->radix_scratch,
                    &c->counters, &c->bwd_scratch, &c->okey, &c->oval, &c->okey2, &c->oval2, &c->cdir,
                    &c->pany, &c->plist, &c->loss_part};
  for (DevBuf* b : bufs)
    if (b->ptr) (void)hipFree(b->ptr);
  if (c->counters_h) (void)hipHostFree(c->counters_h);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->open_ev) (void)hipEventDestroy(c->open_ev);
  (void)hipEventDestroy(c->ev_fork);
  (void)hipEventDestroy(c->ev_join);
  (void)hipStreamDestroy(c->side);
  delete c;
  return G4D_OK;
}

g4d_status g4d_set_stream(g4d_ctx* c, void* hip_stream) {
  if (!c) return G4D_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return G4D_OK;
}

g4d_status g4d_set_primitives(g4d_ctx* c, int64_t n, const float* means4, const float* log_scales4,
                              const float* q_left, const float* q_right, const float* opacity_logit,
                              const float* coeffs) {
  if (!c) return G4D_EINVAL;
  if (n < 0) return fail(c, G4D_EINVAL, "n must be >= 0");
  if (n > (int64_t)0x7FFFFFFF) return fail(c, G4D_ECAPACITY, "n exceeds 2^31-1");
  if (n > 0) {
    if (!means4 || !log_scales4 || !q_left || !q_right || !opacity_logit || !coeffs)
      return fail(c, G4D_EINVAL, "null parameter pointer");
    if (!aligned16(means4) || !aligned16(log_scales4) || !aligned16(q_left) || !aligned16(q_right))
      return fail(c, G4D_EINVAL, "means4/log_scales4/q_left/q_right must be 16-byte aligned");
    if (!aligned4(opacity_logit) || !aligned4(coeffs)) return fail(c, G4D_EINVAL, "misaligned pointer");
  }
  c->n = n;
  c->active_hint = 0;
  c->means4 = means4;
  c->log_scales4 = log_scales4;
  c->q_left = q_left;
  c->q_right = q_right;
  c->opacity_logit = opacity_logit;
  c->coeffs = coeffs;
  c->densify = DensifyStats{nullptr, nullptr, nullptr};
  c->have_render = false;
  return G4D_OK;
}

static g4d_status render_impl(g4d_ctx* c, int32_t n_views, const g4d_camera* cams, const float* times,
                              float* out_rgb, float* out_depth, float* out_alpha);

g4d_status g4d_render(g4d_ctx* c, int32_t n_views, const g4d_camera* cams, const float* times, float* out_rgb,
                      float* out_depth, float* out_alpha) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (c->n < 0) return fail(c, G4D_ESTATE, "set_primitives was not called");
  if (n_views < 1 || n_views > kMaxViews) return fail(c, G4D_EINVAL, "n_views must be in [1, 4096]");
  if (!cams || !times || !out_rgb) return fail(c, G4D_EINVAL, "null cams/times/out_rgb");
  if (c->autotune_pending && !capturing(c)) {
    c->autotune_pending = false;
    g4d_status st = autotune(c, n_views, cams, times, out_rgb, out_depth, out_alpha);
    if (st) return st;
  }
  c->flow_mode = false;
  return render_impl(c, n_views, cams, times, out_rgb, out_depth, out_alpha);
}

g4d_status g4d_render_flow(g4d_ctx* c, int32_t n_views, const g4d_camera* cams, const float* times, float frame_dt,
                           float* out_flow) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (c->n < 0) return fail(c, G4D_ESTATE, "set_primitives was not called");
  if (n_views < 1 || n_views > kMaxViews) return fail(c, G4D_EINVAL, "n_views must be in [1, 4096]");
  if (!cams || !times || !out_flow) return fail(c, G4D_EINVAL, "null cams/times/out_flow");
  if (!std::isfinite(frame_dt)) return fail(c, G4D_EINVAL, "non-finite frame_dt");
  c->flow_mode = true;
  c->flow_dt = frame_dt;
  const g4d_status st = render_impl(c, n_views, cams, times, out_flow, nullptr, nullptr);
  c->flow_mode = false;
  c->have_render = false;  // the kept records hold flow, not colour: no backward
  return st;
}

g4d_status g4d_render_noalloc(g4d_ctx* c, int32_t n_views, const g4d_camera* cams, const float* times,
                              float* out_rgb, float* out_depth, float* out_alpha) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (c->n < 0) return fail(c, G4D_ESTATE, "set_primitives was not called");
  if (n_views < 1 || n_views > kMaxViews) return fail(c, G4D_EINVAL, "n_views must be in [1, 4096]");
  if (!cams || !times || !out_rgb) return fail(c, G4D_EINVAL, "null cams/times/out_rgb");
  if ((size_t)c->n > kNAPairs)
    return fail(c, G4D_ECAPACITY, "the no-allocation render takes at most " + std::to_string(kNAPairs) + " primitives");
  size_t pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const g4d_camera& cm = cams[v];
    if (cm.width < 1 || cm.height < 1 || cm.width > 16384 || cm.height > 16384)
      return fail(c, G4D_EINVAL, "camera size out of [1, 16384]");
    const size_t tiles = (size_t)((cm.width + kTile - 1) / kTile) * ((cm.height + kTile - 1) / kTile);
    if (tiles > kNATiles)
      return fail(c, G4D_ECAPACITY, "the no-allocation render takes at most " + std::to_string(kNATiles) +
                                        " 16x16 tiles per view");
    pix += (size_t)cm.width * cm.height;
  }
  if (pix > kNAPixels)
    return fail(c, G4D_ECAPACITY, "the no-allocation render takes at most " + std::to_string(kNAPixels) +
                                      " pixels per call");
  size_t sz[kNABufs];
  na_sizes(sz);
  size_t total = 0;
  for (int i = 0; i < kNABufs; ++i) total += na_align(sz[i]);
  if (total > sizeof(scratch)) return fail(c, G4D_ECAPACITY, "no-allocation scratch layout exceeds its array");
  // the render's buffers point into this device's scratch for the call
  DevBuf* bufs[kNABufs];
  DevBuf saved[kNABufs];
  render_bufs(c, bufs);
  char* base = static_cast<char*>(c->fixed_scratch);
  size_t off = 0;
  for (int i = 0; i < kNABufs; ++i) {
    saved[i] = *bufs[i];
    bufs[i]->ptr = base + off;
    bufs[i]->cap = sz[i];
    off += na_align(sz[i]);
  }
  const int64_t round_pairs = c->round_pairs, round_instances = c->round_instances;
  const int sort_blocks = c->sort_blocks;
  const bool timing = c->timing;
  c->round_pairs = std::min<int64_t>(round_pairs, (int64_t)kNAPairs);
  c->round_instances = std::min<int64_t>(round_instances, (int64_t)kNAInstances);
  c->sort_blocks = std::min(sort_blocks, kNASortBlocks);
  c->timing = false;  // stage timing would create events
  c->no_alloc = true;
  c->flow_mode = false;
  // the array keeps the last call's contents: the counters start at zero
  launch_fill_u32(P<uint32_t>(c->counters), kCntWords, 0u, c->stream);
  g4d_status st = check_hip(c, hipGetLastError(), "launch");
  if (!st) st = render_impl(c, n_views, cams, times, out_rgb, out_depth, out_alpha);
  for (int i = 0; i < kNABufs; ++i) *bufs[i] = saved[i];
  c->round_pairs = round_pairs;
  c->round_instances = round_instances;
  c->sort_blocks = sort_blocks;
  c->timing = timing;
  c->no_alloc = false;
  // the render's state lives in the shared scratch: nothing is kept
  c->have_render = false;
  c->bound = -1;
  return st;
}

static g4d_status render_impl(g4d_ctx* c, int32_t n_views, const g4d_camera* cams, const float* times,
                              float* out_rgb, float* out_depth, float* out_alpha) {
  // ---- views (host) ----
  std::vector<ViewDev> vh(n_views);
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const g4d_camera& cm = cams[v];
    if (cm.width < 1 || cm.height < 1 || cm.width > 16384 || cm.height > 16384)
      return fail(c, G4D_EINVAL, "camera size out of [1, 16384]");
    if (!(cm.fx > 0.f) || !(cm.fy > 0.f) || !std::isfinite(cm.fx) || !std::isfinite(cm.fy) || !std::isfinite(cm.cx) ||
        !std::isfinite(cm.cy))
      return fail(c, G4D_EINVAL, "camera intrinsics must be finite with fx, fy > 0");
    for (int i = 0; i < 12; ++i)
      if (!std::isfinite(cm.world_to_cam[i])) return fail(c, G4D_EINVAL, "non-finite world_to_cam");
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(cm.center[i])) return fail(c, G4D_EINVAL, "non-finite camera center");
    if (!std::isfinite(times[v])) return fail(c, G4D_EINVAL, "non-finite time");
    ViewDev& d = vh[v];
    d.width = cm.width;
    d.height = cm.height;
    d.tiles_x = (cm.width + kTile - 1) / kTile;
    d.tiles_y = (cm.height + kTile - 1) / kTile;
    d.tile_base = 0;
    d.pad0 = 0;
    d.pix_base = pix;
    d.fx = cm.fx; d.fy = cm.fy; d.cx = cm.cx; d.cy = cm.cy;
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) d.rot[3 * r + k] = cm.world_to_cam[4 * r + k];
      d.trans[r] = cm.world_to_cam[4 * r + 3];
      d.center[r] = cm.center[r];
    }
    d.t = times[v];
    d.lim_x = kFrustumSlack * (0.5f * (float)cm.width) / cm.fx;
    d.lim_y = kFrustumSlack * (0.5f * (float)cm.height) / cm.fy;
    d.lim_x64 = kFrustumSlack64 * (0.5 * cm.width) / (double)cm.fx;
    d.lim_y64 = kFrustumSlack64 * (0.5 * cm.height) / (double)cm.fy;
    tiles += (int64_t)d.tiles_x * d.tiles_y;
    pix += (int64_t)cm.width * cm.height;
  }
  if (tiles > (int64_t)0x7FFFFFFF) return fail(c, G4D_ECAPACITY, "too many tiles");

  hipStream_t s = c->stream;
  g4d_status st;
  const bool fresh_counters = c->counters.ptr == nullptr;
  if ((st = ensure(c, c->counters, sizeof(uint32_t) * kCntWords))) return st;
  if (fresh_counters) launch_fill_u32(P<uint32_t>(c->counters), kCntViews, 0u, s);  // the overflow flag starts clear
  if ((st = ensure(c, c->pix_t, 4 * pix))) return st;
  if ((st = ensure(c, c->pix_last, 4 * pix))) return st;

  c->have_render = false;
  c->n_views = n_views;
  c->views_h = vh;
  c->total_tiles = tiles;
  c->total_pix = pix;
  c->rounds.clear();
  c->A_total = c->I_total = 0;
  c->view_active.assign(n_views, 0);
  uint32_t* cnt = P<uint32_t>(c->counters);
  launch_fill_u32(cnt + kCntMaxList, 1, 0u, s);

  c->totals_on_device = c->sync_free;
  if (c->sync_free) {
    // Rounds planned from the views alone (pair and tile caps); counts stay
    // on the device and add up there, and the arena keeps its capacity: a
    // round over it raises the overflow flag and renders background only.
    launch_fill_u32(cnt + kCntTot, kCntWords - kCntTot, 0u, s);
    const uint64_t cap = std::min<uint64_t>(std::max<uint64_t>(arena_instances(c), 1), 0xFFFFFFF0ull);
    const int by_pairs =
        (int)std::min<int64_t>(n_views, std::max<int64_t>(1, c->round_pairs / std::max<int64_t>(c->n, 1)));
    for (int v0 = 0; v0 < n_views;) {
      const int k = cap_round_tiles(c, v0, std::min(by_pairs, n_views - v0));
      g4d_ctx::Round r{v0, v0 + k, round_tiles(c, v0, v0 + k), kOnDevice, kOnDevice};
      if ((st = enqueue_pairs(c, v0, v0 + k, true))) return st;
      launch_cap_check(cnt + kCntInst64, cnt + kCntI, cnt + kCntOverflow, cap, s, cnt + kCntA, cnt + kCntTot,
                       cnt + kCntTot + 2);
      if ((st = bin_tiles(c, r.tiles, (uint32_t)((uint64_t)c->n * k), (uint32_t)cap))) return st;
      c->rounds.push_back(r);
      c->bound = (int)c->rounds.size() - 1;
      if ((st = rasterise_round(c, r, out_rgb, out_depth, out_alpha))) return st;
      v0 += k;
    }
    c->have_render = true;
    return G4D_OK;
  }

  // Rounds of consecutive views under the pair and instance caps, and of at
  // most 2^16 tiles (a single larger view aside), so that the instance sort
  // by tile takes two 8-bit passes. The first round takes at most 16 views;
  // each next round's size is predicted from the last one's instances per
  // view; a round over the instance cap is shrunk in proportion and binned
  // again.
  const uint64_t inst_cap = (uint64_t)c->round_instances;
  const int by_pairs = (int)std::min<int64_t>(n_views, std::max<int64_t>(1, c->round_pairs / std::max<int64_t>(c->n, 1)));
  // the first round is kept modest: an over-full attempt costs a preprocess
  int k_next = std::min(by_pairs, 16);
  for (int v0 = 0; v0 < n_views;) {
    const int k0 = std::min(k_next, n_views - v0);
    int k = cap_round_tiles(c, v0, k0);
    uint32_t A = 0;
    uint64_t inst = 0;
    for (;;) {
      if ((st = enqueue_pairs(c, v0, v0 + k, true))) return st;
      if ((st = read_pairs(c, v0, k, A, inst))) return st;
      if (inst <= inst_cap) break;
      if (k == 1)
        return fail(c, G4D_ECAPACITY, "view " + std::to_string(v0) + " alone needs " + std::to_string(inst) +
                                          " tile instances, over the round cap " + std::to_string(inst_cap));
      k = std::max(1, std::min(k - 1, (int)(0.9 * (double)k * (double)inst_cap / (double)inst)));
    }
    g4d_ctx::Round r{v0, v0 + k, round_tiles(c, v0, v0 + k), A, (uint32_t)inst};
    if ((st = bin_tiles(c, r.tiles, r.A, r.I))) return st;
    c->rounds.push_back(r);
    c->bound = (int)c->rounds.size() - 1;
    if ((st = rasterise_round(c, r, out_rgb, out_depth, out_alpha))) return st;
    c->A_total += A;
    c->I_total += inst;
    k_next = inst ? (int)std::min<double>(by_pairs, std::max(1.0, 0.9 * (double)k * (double)inst_cap / (double)inst))
                  : by_pairs;
    v0 += k;
  }
  c->have_render = true;
  return G4D_OK;
}

namespace {

// The image loss folded into a backward (g4d_render_backward_loss); kind 0:
// the rgb input is dL/drgb.
struct LossSpec {
  int kind = 0;
  const float* target = nullptr;
  float scale = 0.f;
  float* loss_out = nullptr;
};

g4d_status backward_impl(g4d_ctx* c, const LossSpec& ls, const float* rgb_in, const float* dL_ddepth,
                         const float* dL_dalpha, float* g_means4, float* g_log_scales4, float* g_q_left,
                         float* g_q_right, float* g_opacity_logit, float* g_coeffs, int32_t flags) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (!c->have_render) return fail(c, G4D_ESTATE, "no render since the last set_primitives");
  if (!rgb_in) return fail(c, G4D_EINVAL, ls.kind ? "img is required" : "dL_drgb is required");
  if (flags & ~G4D_GRAD_ACCUMULATE) return fail(c, G4D_EINVAL, "unknown flags");
  if (c->n > 0) {
    if (!g_means4 || !g_log_scales4 || !g_q_left || !g_q_right || !g_opacity_logit || !g_coeffs)
      return fail(c, G4D_EINVAL, "null gradient pointer");
    if (!aligned16(g_means4) || !aligned16(g_log_scales4) || !aligned16(g_q_left) || !aligned16(g_q_right))
      return fail(c, G4D_EINVAL, "gradient buffers must be 16-byte aligned");
  }
  hipStream_t s = c->stream;
  g4d_status st;
  // Rounds last to first: the last one is still binned after the render.
  bool accumulate = (flags & G4D_GRAD_ACCUMULATE) != 0;
  uint32_t* cnt = P<uint32_t>(c->counters);
  for (int ri = (int)c->rounds.size() - 1; ri >= 0; --ri) {
    const g4d_ctx::Round r = c->rounds[ri];
    const int nv = r.v1 - r.v0;
    if (c->bound != ri) {
      if ((st = enqueue_pairs(c, r.v0, r.v1, false))) return st;
      if (r.A == kOnDevice) {  // a sync-free round: no host read
        const uint64_t cap = std::min<uint64_t>(std::max<uint64_t>(arena_instances(c), 1), 0xFFFFFFF0ull);
        launch_cap_check(cnt + kCntInst64, cnt + kCntI, cnt + kCntOverflow, cap, s);
        if ((st = bin_tiles(c, r.tiles, (uint32_t)((uint64_t)c->n * nv), (uint32_t)cap))) return st;
      } else {
        uint32_t A = 0;
        uint64_t inst = 0;
        if ((st = read_pairs(c, r.v0, nv, A, inst))) return st;
        if (A != r.A || inst != r.I)
          return fail(c, G4D_ESTATE, "binning a round again gave other counts; primitives changed since render");
        if ((st = bin_tiles(c, r.tiles, r.A, r.I))) return st;
      }
      c->bound = ri;
    }
    // records bound: exact for a synchronous round, every pair for a sync-free one
    const uint32_t a_max = r.A == kOnDevice ? (uint32_t)((uint64_t)c->n * nv) : r.A;
    if ((st = ensure(c, c->grad2d, sizeof(double) * kGrad2dStride * (size_t)a_max))) return st;
    if ((st = ensure(c, c->bwd_scratch, sizeof(float) * preprocess_backward_scratch_floats(a_max)))) return st;
    // the gradient lines start at zero (timed with the preprocess backward,
    // which reads them)
    stage_begin(c);
    launch_zero_counted(P<float>(c->grad2d), cnt + kCntA, 2 * kGrad2dStride, a_max, s);
    stage_end(c, G4D_STAGE_PREPROCESS_BWD);
    if ((st = join_side(c))) return st;  // the records' colours of a round binned again
    LossArgs la{ls.kind, ls.target, ls.scale, nullptr};
    if (ls.kind) {
      if ((st = ensure(c, c->loss_part, sizeof(float) * (size_t)r.tiles))) return st;
      la.part = P<float>(c->loss_part);
    }
    stage_begin(c);
    launch_raster_backward(r.tiles, c->heavy_first ? P<uint32_t>(c->oval) : nullptr,
                           c->persistent_blocks ? cnt + kCntQueue : nullptr, c->persistent_blocks, nv,
                           P<ViewDev>(c->views_d),
                           P<uint2>(c->ranges), P<uint32_t>(c->ival),
                           P<Record>(c->rec_sorted), c->opts.bg, rgb_in, dL_ddepth, dL_dalpha, P<float>(c->pix_t),
                           P<uint32_t>(c->pix_last), P<double>(c->grad2d), c->densify.blend_count != nullptr,
                           c->ellipse_cull, la, s);
    stage_end(c, G4D_STAGE_RASTER_BWD);
    if (ls.kind) {
      stage_begin(c);
      launch_loss_partials(la.part, (uint32_t)r.tiles, ls.scale, ls.loss_out, s);
      stage_end(c, G4D_STAGE_LOSS);
    }
    RenderParams p = make_params(c, nv);
    stage_begin(c);
    launch_preprocess_backward(p, P<int32_t>(c->slot), P<double>(c->grad2d), cnt + kCntA, a_max, P<uint32_t>(c->cval),
                               P<Record>(c->rec_sorted), P<float>(c->bwd_scratch), g_means4, g_log_scales4, g_q_left,
                               g_q_right, g_opacity_logit, g_coeffs, accumulate, c->densify, s);
    stage_end(c, G4D_STAGE_PREPROCESS_BWD);
    HIPCHK(c, hipGetLastError());
    accumulate = true;
  }
  return G4D_OK;
}

}  // namespace

g4d_status g4d_render_backward(g4d_ctx* c, const float* dL_drgb, const float* dL_ddepth, const float* dL_dalpha,
                               float* g_means4, float* g_log_scales4, float* g_q_left, float* g_q_right,
                               float* g_opacity_logit, float* g_coeffs, int32_t flags) {
  return backward_impl(c, LossSpec{}, dL_drgb, dL_ddepth, dL_dalpha, g_means4, g_log_scales4, g_q_left, g_q_right,
                       g_opacity_logit, g_coeffs, flags);
}

g4d_status g4d_render_backward_loss(g4d_ctx* c, int32_t kind, const float* img, const float* target, float scale,
                                    float* loss_out, const float* dL_ddepth, const float* dL_dalpha,
                                    float* g_means4, float* g_log_scales4, float* g_q_left, float* g_q_right,
                                    float* g_opacity_logit, float* g_coeffs, int32_t flags) {
  if (!c) return G4D_EINVAL;
  if (kind != G4D_LOSS_L1 && kind != G4D_LOSS_L2) return fail(c, G4D_EINVAL, "unknown loss kind");
  if (!std::isfinite(scale)) return fail(c, G4D_EINVAL, "non-finite scale");
  if (!img || !target || !loss_out) return fail(c, G4D_EINVAL, "null pointer");
  LossSpec ls;
  ls.kind = kind;
  ls.target = target;
  ls.scale = scale;
  ls.loss_out = loss_out;
  return backward_impl(c, ls, img, dL_ddepth, dL_dalpha, g_means4, g_log_scales4, g_q_left, g_q_right,
                       g_opacity_logit, g_coeffs, flags);
}

g4d_status g4d_set_densify_stats(g4d_ctx* c, float* uv_grad_norm_sum, float* t_grad_abs_sum,
                                 int32_t* blend_count) {
  if (!c) return G4D_EINVAL;
  const int nn = (uv_grad_norm_sum != nullptr) + (t_grad_abs_sum != nullptr) + (blend_count != nullptr);
  if (nn != 0 && nn != 3) return fail(c, G4D_EINVAL, "give all three accumulators or none");
  if (nn == 3 && c->n < 0) return fail(c, G4D_ESTATE, "set_primitives was not called");
  if (nn == 3 && (!aligned4(uv_grad_norm_sum) || !aligned4(t_grad_abs_sum) || !aligned4(blend_count)))
    return fail(c, G4D_EINVAL, "misaligned accumulator");
  c->densify = DensifyStats{uv_grad_norm_sum, t_grad_abs_sum, blend_count};
  return G4D_OK;
}

g4d_status g4d_adam_step(g4d_ctx* c, int64_t n, const g4d_adam_options* o, int64_t step, float* const* params,
                         const float* const* grads, float* exp_avg, float* exp_avg_sq) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (!o || !params || !grads) return fail(c, G4D_EINVAL, "null options or pointer table");
  if (n < 0 || step < 1) return fail(c, G4D_EINVAL, "n must be >= 0 and step >= 1");
  if (!(o->beta1 >= 0.f && o->beta1 < 1.f && o->beta2 >= 0.f && o->beta2 < 1.f && o->eps > 0.f &&
        std::isfinite(o->eps)))
    return fail(c, G4D_EINVAL, "need 0 <= beta < 1 and a finite eps > 0");
  const int64_t K3 = 3ll * (c->opts.t_order + 1) * (c->opts.sh_degree + 1) * (c->opts.sh_degree + 1);
  const int64_t width[kAdamGroups] = {4, 4, 4, 4, 1, K3};
  AdamGroups a{};
  uint64_t end = 0;
  for (int g = 0; g < kAdamGroups; ++g) {
    if (!std::isfinite(o->lr[g])) return fail(c, G4D_EINVAL, "non-finite learning rate");
    if (n > 0 && (!params[g] || !grads[g])) return fail(c, G4D_EINVAL, "null parameter or gradient pointer");
    a.param[g] = params[g];
    a.grad[g] = grads[g];
    a.lr[g] = o->lr[g];
    end += (uint64_t)n * (uint64_t)width[g];
    a.end[g] = end;
  }
  if (n > 0 && (!exp_avg || !exp_avg_sq)) return fail(c, G4D_EINVAL, "null moment buffer");
  const double bc1 = 1.0 - std::pow((double)o->beta1, (double)step);
  const double bc2 = 1.0 - std::pow((double)o->beta2, (double)step);
  if (!(bc1 > 0.0) || !(bc2 > 0.0)) return fail(c, G4D_EINVAL, "bias corrections vanish (beta = 0 and step 0?)");
  launch_adam(a, o->beta1, o->beta2, o->eps, (float)bc1, (float)bc2, exp_avg, exp_avg_sq, c->stream);
  HIPCHK(c, hipGetLastError());
  return G4D_OK;
}

g4d_status g4d_split_sample(g4d_ctx* c, int64_t count, const int32_t* idx, const float* z, float* out_means4) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (c->n < 0) return fail(c, G4D_ESTATE, "set_primitives was not called");
  if (count < 0) return fail(c, G4D_EINVAL, "count must be >= 0");
  if (count > 0 && (!idx || !z || !out_means4)) return fail(c, G4D_EINVAL, "null pointer");
  if (count > 0 && (!aligned16(z) || !aligned16(out_means4)))
    return fail(c, G4D_EINVAL, "z and out_means4 must be 16-byte aligned");
  launch_split_sample(make_params(c, 0), (uint64_t)count, idx, z, out_means4, c->stream);
  HIPCHK(c, hipGetLastError());
  return G4D_OK;
}

g4d_status g4d_image_loss(g4d_ctx* c, int32_t kind, int64_t n, const float* img, const float* target, float scale,
                          float* loss_out, float* grad_out) {
  if (!c) return G4D_EINVAL;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (kind != G4D_LOSS_L1 && kind != G4D_LOSS_L2) return fail(c, G4D_EINVAL, "unknown loss kind");
  if (n < 0) return fail(c, G4D_EINVAL, "n must be >= 0");
  if (!std::isfinite(scale)) return fail(c, G4D_EINVAL, "non-finite scale");
  if (n > 0 && (!img || !target || !loss_out || !grad_out)) return fail(c, G4D_EINVAL, "null pointer");
  if (n > 0 && (grad_out == img || grad_out == target)) return fail(c, G4D_EINVAL, "grad_out aliases an input");
  stage_begin(c);
  launch_image_loss(kind, (uint64_t)n, img, target, scale, loss_out, grad_out, c->stream);
  stage_end(c, G4D_STAGE_LOSS);
  HIPCHK(c, hipGetLastError());
  return G4D_OK;
}

g4d_status g4d_stage_times(g4d_ctx* c, double* ms_out, int64_t* launches_out) {
  if (!c || !ms_out || !launches_out) return G4D_EINVAL;
  g4d_status st = collect_times(c);
  if (st) return st;
  for (int i = 0; i < G4D_NUM_STAGES; ++i) {
    ms_out[i] = c->stage_ms[i];
    launches_out[i] = c->stage_n[i];
  }
  return G4D_OK;
}

g4d_status g4d_get_stats(g4d_ctx* c, g4d_stats* out, int64_t* active_per_view) {
  if (!c || !out) return G4D_EINVAL;
  g4d_status st_join = G4D_OK;
  if (c->hip_failed) return fail(c, G4D_EHIP, "context has a failed HIP call; destroy it");
  if (!c->have_render) return fail(c, G4D_ESTATE, "no render");
  uint32_t* cnt = P<uint32_t>(c->counters);
  if (c->totals_on_device) {
    // a sync-free render: totals and per-view counts were added up on the device
    HIPCHK(c, hipMemcpyAsync(c->counters_h + kCntViews, cnt + kCntViews, sizeof(uint32_t) * (kCntWords - kCntViews),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::copy(c->counters_h + kCntViews, c->counters_h + kCntViews + c->n_views, c->view_active.begin());
    c->A_total = c->counters_h[kCntTot];
    std::memcpy(&c->I_total, c->counters_h + kCntTot + 2, sizeof(uint64_t));
  }
  out->n_views = c->n_views;
  out->active_total = (int64_t)c->A_total;
  out->instances = (int64_t)c->I_total;
  out->tiles = c->total_tiles;
  out->rounds = (int64_t)c->rounds.size();
  // longest list, overflow flag, fragment total and non-finite culls need
  // device reads (the colour pass, which counts some of the latter, joined)
  if ((st_join = join_side(c))) return st_join;
  launch_fill_u32(cnt + kCntFrag, 2, 0u, c->stream);
  launch_sum_u32(P<uint32_t>(c->pix_last), (uint64_t)c->total_pix, reinterpret_cast<unsigned long long*>(cnt + kCntFrag),
                 c->stream);
  uint32_t words[4] = {0, 0, 0, 0};
  uint64_t need = 0;
  std::vector<uint32_t> nf((size_t)c->n_views, 0u);
  HIPCHK(c, hipMemcpyAsync(words, cnt + kCntFrag, sizeof(words), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&need, cnt + kCntInst64, sizeof(need), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(nf.data(), cnt + kCntNF, sizeof(uint32_t) * nf.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->culled_nonfinite = 0;
  for (uint32_t x : nf) out->culled_nonfinite += x;
  uint64_t frag = 0;
  std::memcpy(&frag, words, sizeof(frag));
  out->max_tile_list = words[kCntMaxList - kCntFrag];
  out->fragments = (int64_t)frag;
  if (active_per_view)
    for (int v = 0; v < c->n_views; ++v) active_per_view[v] = c->view_active[v];
  if (words[kCntOverflow - kCntFrag]) {
    launch_fill_u32(cnt + kCntOverflow, 1, 0u, c->stream);
    HIPCHK(c, hipGetLastError());
    return fail(c, G4D_ECAPACITY, "a sync-free render since the last get_stats exceeded the instance arena of " +
                                      std::to_string(arena_instances(c)) + " (last render needs " +
                                      std::to_string(need) + "); its outputs are background only");
  }
  return G4D_OK;
}

g4d_status g4d_set_tuning(g4d_ctx* c, int32_t key, int32_t value) {
  if (!c) return G4D_EINVAL;
  if (key == G4D_TUNE_SORT_BLOCKS) {
    if (value < 1 || value > 65536) return fail(c, G4D_EINVAL, "sort blocks out of [1, 65536]");
    c->sort_blocks = value;
    return G4D_OK;
  }
  if (key == G4D_TUNE_STAGE_TIMING) {
    if (value != 0 && value != 1) return fail(c, G4D_EINVAL, "stage timing is 0 or 1");
    g4d_status st = collect_times(c);
    if (st) return st;
    for (int i = 0; i < G4D_NUM_STAGES; ++i) {
      c->stage_ms[i] = 0.0;
      c->stage_n[i] = 0;
    }
    c->timing = value == 1;
    return G4D_OK;
  }
  if (key == G4D_TUNE_AUTOTUNE) {
    if (value != 0 && value != 1) return fail(c, G4D_EINVAL, "autotune is 0 or 1");
    c->autotune_pending = value == 1;
    return G4D_OK;
  }
  if (key == G4D_TUNE_TILE_ORDER) {
    if (value != 0 && value != 1) return fail(c, G4D_EINVAL, "tile order is 0 or 1");
    c->heavy_first = value == 1;
    c->have_render = false;  // the order of the last render's tiles may be missing
    return G4D_OK;
  }
  if (key == G4D_TUNE_ELLIPSE_CULL) {
    if (value != 0 && value != 1) return fail(c, G4D_EINVAL, "ellipse cull is 0 or 1");
    c->ellipse_cull = value == 1;
    c->have_render = false;  // the last render's bins would come out otherwise
    return G4D_OK;
  }
  if (key == G4D_TUNE_PERSISTENT_BLOCKS) {
    if (value < -1) return fail(c, G4D_EINVAL, "persistent blocks is -1, 0 or a workgroup count");
    c->persistent_blocks = value;
    return G4D_OK;
  }
  if (key == G4D_TUNE_LDS_BATCH) {
    if (value != 64 && value != 128 && value != 256) return fail(c, G4D_EINVAL, "LDS batch is 64, 128 or 256");
    c->lds_batch = value;
    return G4D_OK;
  }
  if (key == G4D_TUNE_SYNC_FREE) {
    if (value != 0 && value != 1) return fail(c, G4D_EINVAL, "sync-free is 0 or 1");
    c->sync_free = value == 1;
    return G4D_OK;
  }
  if (key == G4D_TUNE_ARENA_INSTANCES) {
    if (value < 0) return fail(c, G4D_EINVAL, "arena size must be >= 0");
    g4d_status st;
    for (DevBuf* b : {&c->ikey, &c->ival, &c->ikey2, &c->ival2})
      if ((st = ensure(c, *b, 4 * (size_t)value))) return st;
    return G4D_OK;
  }
  if (key == G4D_TUNE_ROUND_PAIRS || key == G4D_TUNE_ROUND_INSTANCES) {
    if (value < 1) return fail(c, G4D_EINVAL, "round caps must be >= 1");
    (key == G4D_TUNE_ROUND_PAIRS ? c->round_pairs : c->round_instances) = value;
    return G4D_OK;
  }
  return fail(c, G4D_EINVAL, "unknown tuning key");
}

g4d_status g4d_get_tuning(g4d_ctx* c, int32_t key, int32_t* value) {
  if (!c || !value) return G4D_EINVAL;
  const auto clamp32 = [](int64_t v) { return (int32_t)std::min<int64_t>(v, 0x7FFFFFFF); };
  switch (key) {
    case G4D_TUNE_SORT_BLOCKS: *value = c->sort_blocks; break;
    case G4D_TUNE_STAGE_TIMING: *value = c->timing ? 1 : 0; break;
    case G4D_TUNE_ROUND_PAIRS: *value = clamp32(c->round_pairs); break;
    case G4D_TUNE_ROUND_INSTANCES: *value = clamp32(c->round_instances); break;
    case G4D_TUNE_SYNC_FREE: *value = c->sync_free ? 1 : 0; break;
    case G4D_TUNE_ELLIPSE_CULL: *value = c->ellipse_cull ? 1 : 0; break;
    case G4D_TUNE_ARENA_INSTANCES: *value = clamp32((int64_t)arena_instances(c)); break;
    case G4D_TUNE_TILE_ORDER: *value = c->heavy_first ? 1 : 0; break;
    case G4D_TUNE_AUTOTUNE: *value = c->autotune_pending ? 1 : 0; break;
    case G4D_TUNE_PERSISTENT_BLOCKS: *value = c->persistent_blocks; break;
    case G4D_TUNE_LDS_BATCH: *value = c->lds_batch; break;
    default: return fail(c, G4D_EINVAL, "unknown tuning key");
  }
  return G4D_OK;
}

const char* g4d_last_error(const g4d_ctx* c) { return c ? c->err.c_str() : "null context"; }

g4d_status g4d_debug_size(g4d_ctx* c, int32_t what, int64_t* bytes) {
  if (!c || !bytes) return G4D_EINVAL;
  if (!c->have_render) return fail(c, G4D_ESTATE, "no render");
  if (c->bound < 0) return fail(c, G4D_ESTATE, "no round is binned");
  g4d_ctx::Round& r = c->rounds[c->bound];
  g4d_status st = resolve_round(c, r);
  if (st) return st;
  switch (what) {
    case G4D_DBG_RECORDS: *bytes = (int64_t)sizeof(Record) * r.A; break;
    case G4D_DBG_IDS: *bytes = 4ll * r.A; break;
    case G4D_DBG_TILE_KEYS: case G4D_DBG_TILE_VALS: *bytes = 4ll * r.I; break;
    case G4D_DBG_RANGES: *bytes = 8ll * r.tiles; break;
    case G4D_DBG_PIX_T: case G4D_DBG_PIX_LAST: *bytes = 4ll * c->total_pix; break;
    case G4D_DBG_GRAD2D: *bytes = 8ll * kGrad2dStride * r.A; break;
    case G4D_DBG_TILE_ORDER:
      if (!c->heavy_first) return fail(c, G4D_ESTATE, "the heavy-first tile order is off");
      *bytes = 4ll * r.tiles;
      break;
    default: return fail(c, G4D_EINVAL, "unknown debug item");
  }
  return G4D_OK;
}

g4d_status g4d_debug_copy(g4d_ctx* c, int32_t what, void* host_dst, int64_t bytes) {
  if (!c || !host_dst) return G4D_EINVAL;
  int64_t want = 0;
  g4d_status st = g4d_debug_size(c, what, &want);
  if (st) return st;
  if (bytes != want) return fail(c, G4D_EINVAL, "size mismatch");
  if (bytes == 0) return G4D_OK;
  if ((st = join_side(c))) return st;
  if (what == G4D_DBG_TILE_KEYS) {
    // the sort's last pass writes the ranges, not the keys: each position
    // gets the tile whose range covers it (0xFFFFFFFF where none does)
    const g4d_ctx::Round& r = c->rounds[c->bound];
    std::vector<uint2> rg((size_t)r.tiles);
    HIPCHK(c, hipMemcpyAsync(rg.data(), c->ranges.ptr, sizeof(uint2) * rg.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint32_t* keys = static_cast<uint32_t*>(host_dst);
    const uint64_t n = (uint64_t)bytes / 4;
    std::fill(keys, keys + n, 0xFFFFFFFFu);
    for (uint32_t t = 0; t < (uint32_t)rg.size(); ++t)
      for (uint64_t p = rg[t].x; p < rg[t].y && p < n; ++p) keys[p] = t;
    return G4D_OK;
  }
  const void* src = nullptr;
  switch (what) {
    case G4D_DBG_RECORDS: src = c->rec_sorted.ptr; break;
    case G4D_DBG_IDS: src = c->cval.ptr; break;
    case G4D_DBG_TILE_VALS: src = c->ival.ptr; break;
    case G4D_DBG_RANGES: src = c->ranges.ptr; break;
    case G4D_DBG_PIX_T: src = c->pix_t.ptr; break;
    case G4D_DBG_PIX_LAST: src = c->pix_last.ptr; break;
    case G4D_DBG_TILE_ORDER: src = c->oval.ptr; break;
    case G4D_DBG_GRAD2D:
      if (c->grad2d.cap < (size_t)bytes) return fail(c, G4D_ESTATE, "no backward");
      src = c->grad2d.ptr;
      break;
  }
  HIPCHK(c, hipMemcpyAsync(host_dst, src, (size_t)bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return G4D_OK;
}

}  // extern "C"
