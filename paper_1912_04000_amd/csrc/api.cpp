// C ABI of libspecdd: argument validation, workspace layout and the wavefront loop.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"

using namespace sdd;



namespace sdd {

static thread_local std::string g_thread_err;
void set_thread_error(const std::string& m) { g_thread_err = m; }
hipStream_t ctx_stream(const sdd_ctx* ctx) { return ctx->stream; }
const char* thread_error() { return g_thread_err.c_str(); }

}  // namespace sdd

namespace {

int fail(sdd_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  set_thread_error(msg);
  return code;
}

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(ctx, SDD_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

constexpr int kDefaultWave = 1 << 20;
constexpr int kDefaultRounds = 1;
// Persistent render: lanes of the one kernel (a multiple of kWG * kXcds; the traversal spill of a
// plan covers at most 2048 workgroups)
constexpr int kPersistDefaultLanes = 1536 * kWG;
constexpr int kPersistMaxLanes = 2048 * kWG;
constexpr uint32_t kPersistTileItems = 64;  // items of one 8 x 8 tile at one sample

// Lanes of a persistent render: as asked, else as many as the device holds at once (the
// kernel's occupancy times the compute units; kPersistDefaultLanes if the runtime cannot tell),
// never more than the work list has items, a multiple of kWG * kXcds.
uint32_t persist_lanes(const sdd_render_params* p, uint64_t total, int device) {
  const uint64_t g = (uint64_t)kWG * kXcds;
  uint64_t L = (uint64_t)p->wave_paths;
  if (!L) {
    const uint64_t resident = (uint64_t)persist_resident_blocks(device) * kWG;
    L = resident >= g ? resident / g * g : (uint64_t)kPersistDefaultLanes;
  }
  L = std::min<uint64_t>(L, (total + g - 1) / g * g);
  L = (L + g - 1) / g * g;
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(L, g), kPersistMaxLanes);
}
// Ray queries (sdd_trace / sdd_shadow) run one migration round before walking in place, so that
// every query also exercises the migration between cell queues.
constexpr int kQueryRounds = 2;
constexpr int kMaxViewsPerStore = 16;

struct ViewBlock {
  ViewDesc v[kMaxViewsPerStore];
};

__global__ void k_store_views(ViewBlock vb, ViewDesc* dst, int first, int count) {
  int i = threadIdx.x;
  if (i < count) dst[first + i] = vb.v[i];
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

enum {
  L_PIX, L_SMP, L_VIEW, L_BETA, L_NEE, L_LACC, L_HIT, L_RAYS, L_SHCNT, L_SHX, L_CAT, L_CATB, L_LSRC, L_LDST, L_LRANK,
  L_QUEUE, L_CCOUNT, L_COFF, L_KSUM, L_KOFF, L_TILES, L_SPILL, L_CTL, L_VIEWS, L_COUNT
};

struct Plan {
  uint32_t W;
  int B, Bp;
  int n_cells;
  int n_views;
  int trace_blocks;
  uint32_t max_tiles;
  uint32_t sub_shift, key_words;  // queue-key sub-ranges (3 x their levels), counter words per key
  size_t off[L_COUNT];
  size_t total;
};

// levels: the queue keys' origin-block levels, < 0 for as many as the grid allows (sub_levels_for)
Plan make_plan(uint32_t W, int B, int n_cells, int n_views, int levels = -1) {
  Plan p;
  p.W = W;
  p.B = B;
  p.Bp = (B + 3) & ~3;
  p.n_cells = n_cells;
  p.sub_shift = 3u * (uint32_t)(levels < 0 ? sub_levels_for(n_cells, W) : levels) + kDirSubBits;
  p.key_words = std::max<uint32_t>(kKeyStride, 1u << p.sub_shift);
  p.n_views = n_views;
  size_t want = ((size_t)2 * W + kWG - 1) / kWG;
  int tb = (int)std::min<size_t>(2048, std::max<size_t>(kXcds, want));
  tb = (tb + kXcds - 1) / kXcds * kXcds;
  p.trace_blocks = tb;
  p.max_tiles = (uint32_t)(((size_t)2 * W + kTile - 1) / kTile + (size_t)n_cells * kDirBins + 8);
  size_t sz[L_COUNT];
  sz[L_PIX] = 4ull * W;
  sz[L_SMP] = 4ull * W;
  sz[L_VIEW] = 4ull * W;
  sz[L_BETA] = 4ull * p.Bp * W;
  sz[L_NEE] = 4ull * p.Bp * W;
  sz[L_LACC] = 4ull * p.Bp * W;
  sz[L_HIT] = 16ull * W;
  sz[L_RAYS] = 64ull * W;
  sz[L_SHCNT] = 4ull * W;
  sz[L_SHX] = 8ull * kMaxCross * W;
  sz[L_CAT] = 4ull * 2 * kCats * W;
  sz[L_CATB] = 4ull * ((2ull * W + 3) / 4);
  sz[L_LSRC] = 8ull * W;
  sz[L_LDST] = 8ull * W;
  sz[L_LRANK] = 8ull * W;
  sz[L_QUEUE] = 8ull * W;
  sz[L_CCOUNT] = 8ull * n_cells * kDirBins * p.key_words;
  sz[L_COFF] = (4ull * n_cells * kDirBins) << p.sub_shift;
  sz[L_KSUM] = 4ull * n_cells * kDirBins;
  sz[L_KOFF] = 4ull * n_cells * kDirBins;
  sz[L_TILES] = 16ull * p.max_tiles;
  sz[L_SPILL] = 4ull * (kMaxStack - kShortStack) * (size_t)tb * kWG;
  sz[L_CTL] = sizeof(Ctl);
  sz[L_VIEWS] = sizeof(ViewDesc) * (size_t)std::max(1, n_views);
  size_t o = 0;
  for (int i = 0; i < L_COUNT; ++i) {
    p.off[i] = o;
    o = a256(o + sz[i]);
  }
  p.total = o;
  return p;
}

// The plan with the most origin-block levels (up to what the grid allows) whose workspace fits in
// `bytes`, else the one with none: the levels only order the rays inside a queue key, so a
// smaller workspace costs traversal coherence, never results.
Plan fit_plan(uint32_t W, int B, int n_cells, int n_views, size_t bytes) {
  for (int L = sub_levels_for(n_cells, W); L > 0; --L) {
    const Plan p = make_plan(W, B, n_cells, n_views, L);
    if (p.total <= bytes) return p;
  }
  return make_plan(W, B, n_cells, n_views, 0);
}

DevWS ws_view(const Plan& p, void* base) {
  uint8_t* b = (uint8_t*)base;
  DevWS w;
  std::memset(&w, 0, sizeof(w));
  w.pix = (uint32_t*)(b + p.off[L_PIX]);
  w.smp = (uint32_t*)(b + p.off[L_SMP]);
  w.view = (uint32_t*)(b + p.off[L_VIEW]);
  w.beta = (float*)(b + p.off[L_BETA]);
  w.nee = (float*)(b + p.off[L_NEE]);
  w.lacc = (float*)(b + p.off[L_LACC]);
  w.hit = (float4*)(b + p.off[L_HIT]);
  w.rays = (float4*)(b + p.off[L_RAYS]);
  w.shcnt = (uint32_t*)(b + p.off[L_SHCNT]);
  w.shx = (float2*)(b + p.off[L_SHX]);
  w.cat = (uint32_t*)(b + p.off[L_CAT]);
  w.catb = (uint8_t*)(b + p.off[L_CATB]);
  w.lsrc = (uint32_t*)(b + p.off[L_LSRC]);
  w.ldst = (uint32_t*)(b + p.off[L_LDST]);
  w.lrank = (uint32_t*)(b + p.off[L_LRANK]);
  w.queue = (uint32_t*)(b + p.off[L_QUEUE]);
  w.ccount = (uint32_t*)(b + p.off[L_CCOUNT]);
  w.coff = (uint32_t*)(b + p.off[L_COFF]);
  w.ksum = (uint32_t*)(b + p.off[L_KSUM]);
  w.koff = (uint32_t*)(b + p.off[L_KOFF]);
  w.tiles = (uint4*)(b + p.off[L_TILES]);
  w.spill = (uint32_t*)(b + p.off[L_SPILL]);
  w.ctl = (Ctl*)(b + p.off[L_CTL]);
  w.views = (ViewDesc*)(b + p.off[L_VIEWS]);
  w.W = p.W;
  w.max_tiles = p.max_tiles;
  w.trace_threads = (uint32_t)p.trace_blocks * kWG;
  w.n_views = p.n_views;
  w.sub_shift = p.sub_shift;
  w.key_words = p.key_words;
  w.Bp = p.Bp;
  return w;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Camera basis in FP64, handed to the kernels as FP32 vectors.
std::string make_view(const sdd_camera& c, ViewDesc* v) {
  if (!finite3(c.eye) || !finite3(c.target) || !finite3(c.up)) return "camera vectors must be finite";
  if (!(c.vfov_deg > 0 && c.vfov_deg < 180)) return "vfov must lie in (0, 180)";
  if (c.width < 1 || c.height < 1 || (int64_t)c.width * c.height > (1ll << 31)) return "bad image size";
  double f[3] = {(double)c.target[0] - c.eye[0], (double)c.target[1] - c.eye[1], (double)c.target[2] - c.eye[2]};
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0)) return "camera target equals eye";
  for (double& x : f) x /= fl;
  double up[3] = {c.up[0], c.up[1], c.up[2]};
  double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 0)) return "camera up is parallel to the view direction";
  for (double& x : r) x /= rl;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  double t = std::tan(c.vfov_deg * M_PI / 360.0);
  double aspect = (double)c.width / c.height;
  std::memset(v, 0, sizeof(*v));
  for (int i = 0; i < 3; ++i) {
    v->eye[i] = c.eye[i];
    v->fwd[i] = (float)f[i];
    v->right[i] = (float)(r[i] * t * aspect);
    v->upv[i] = (float)(u[i] * t);
  }
  v->width = c.width;
  v->height = c.height;
  return "";
}

std::string check_params(const sdd_render_params* p) {
  if (!p) return "params is null";
  if (p->spp < 1) return "spp must be >= 1";
  if (p->max_depth < 1 || p->max_depth > 64) return "max_depth must lie in 1..64";
  if (p->mode != SDD_MODE_PLAIN && p->mode != SDD_MODE_CACHED) return "unknown mode";
  if (p->wave_paths != 0 && (p->wave_paths < 64 || p->wave_paths > (1 << 26))) return "wave_paths out of range";
  if (p->queue_rounds < 0 || p->queue_rounds > 256) return "queue_rounds out of range";
  if (p->first_sample < 0) return "first_sample must be >= 0";
  if (p->cell_order != 0 && p->cell_order != 1) return "cell_order must be 0 or 1";
  if (p->persistent != 0 && p->persistent != 1) return "persistent must be 0 or 1";
  if (p->persistent && p->mode != SDD_MODE_PLAIN) return "persistent rendering is plain mode only";
  if (p->persistent && p->wave_paths > kPersistMaxLanes) return "persistent rendering takes at most 2^19 lanes";
  return "";
}

int scene_ready(sdd_ctx* ctx, const sdd_scene* s) {
  if (!s) return fail(ctx, SDD_ERR_INVALID_ARG, "scene is null");
  if (!s->dev) return fail(ctx, SDD_ERR_NOT_READY, "scene has not been uploaded");
  return SDD_OK;
}

void record(sdd_ctx* ctx, std::vector<std::pair<hipEvent_t, hipEvent_t>>& pool, size_t& used, bool start) {
  if (start) {
    if (used == pool.size()) {
      hipEvent_t a, b;
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      pool.push_back({a, b});
    }
    (void)hipEventRecord(pool[used].first, ctx->stream);
  } else {
    (void)hipEventRecord(pool[used].second, ctx->stream);
    ++used;
  }
}

// Trace every entry produced so far: rounds of (scan, scatter, trace). In every round but the
// last a ray visits one cell and migrates to the next cell's queue; the last round walks the
// remaining rays through their remaining cells in place.
int trace_phase(sdd_ctx* ctx, const Launch& L, const DevScene& S, const DevWS& w, int& gen, int rounds, int cat_par,
                bool timing) {
  for (int r = 0; r < rounds; ++r) {
    const int hops = r == rounds - 1 ? (1 << 30) : 1;
    HIP_TRY(ctx, launch_scan(L, S, w, gen));
    HIP_TRY(ctx, launch_scatter(L, w, gen));
    if (timing) record(ctx, ctx->ev_trace, ctx->ev_used_trace, true);
    HIP_TRY(ctx, launch_trace(L, S, w, gen, hops));
    if (timing) record(ctx, ctx->ev_trace, ctx->ev_used_trace, false);
    ctx->acc.trace_launches++;
    ++gen;
  }
  // the finished rays' category bytes become the lists the shading kernels read
  HIP_TRY(ctx, launch_gather_cats(L, w, cat_par));
  return SDD_OK;
}

int store_views(sdd_ctx* ctx, const std::vector<ViewDesc>& views, const DevWS& w) {
  for (size_t first = 0; first < views.size(); first += kMaxViewsPerStore) {
    ViewBlock vb;
    std::memset(&vb, 0, sizeof(vb));
    int cnt = (int)std::min<size_t>(kMaxViewsPerStore, views.size() - first);
    for (int i = 0; i < cnt; ++i) vb.v[i] = views[first + i];
    hipLaunchKernelGGL(k_store_views, dim3(1), dim3(kMaxViewsPerStore), 0, ctx->stream, vb, w.views, (int)first, cnt);
    HIP_TRY(ctx, hipGetLastError());
  }
  return SDD_OK;
}

// FNV-1a over a byte range (graph keys).
uint64_t fnv(uint64_t h, const void* data, size_t n) {
  const uint8_t* b = (const uint8_t*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Every launch of one render call, in stream order. Statistics are never zeroed here, so the
// sequence can be captured once and replayed.
// One population of paths (render items k0 .. k0 + n, or training paths) through the bounce
// loop. A cached render stops its paths at vertex kCacheDepth and queries the cache there;
// `finish` runs after the last bounce (accumulation into the images, or the gathering of
// training targets).
constexpr int kCacheDepth = 3;

template <typename Finish>
int run_paths(sdd_ctx* ctx, const sdd_scene* scene, const sdd_render_params* p, const Launch& L, const DevScene& S,
              const DevWS& w, uint64_t k0, uint32_t n, int& gen, bool timing, const PathMode& pm,
              const sdd_cache* cache, const PhotonDev* ph, const PhotonDev* gm, int gm_from, Finish finish) {
  const int rounds = p->queue_rounds ? p->queue_rounds : kDefaultRounds;
  const int D = p->max_depth;
  const bool query = cache && pm.purpose == 0 && D >= kCacheDepth;
  HIP_TRY(ctx, launch_fill_u32(ctx->stream, &w.ctl->cat_count[0][0], 2 * 8 * kKeyStride, 0u));
  HIP_TRY(ctx, launch_fill_u32(ctx->stream, (uint32_t*)w.catb, ((size_t)2 * w.W + 3) / 4, 0u));
  if (ph || gm) HIP_TRY(ctx, launch_fill_u32(ctx->stream, w.ctl->ph_heavy, 2, 0u));
  HIP_TRY(ctx, launch_raygen(L, S, w, k0, n, p->seed, gen, pm));
  int rc = trace_phase(ctx, L, S, w, gen, rounds, 1, timing);
  if (rc) return rc;
  for (int d = 1; d <= D + 1; ++d) {
    const bool last = d == D + 1 || (query && d == kCacheDepth);
    if (timing) record(ctx, ctx->ev_shade, ctx->ev_used_shade, true);
    HIP_TRY(ctx, launch_resolve(L, S, w, d));
    if (scene->hdr.env_nonzero) HIP_TRY(ctx, launch_escape(L, S, w, d));
    if (!last) {
      // photon-map radiance at the opaque vertices, before their lobes: the caustic map, or from
      // vertex gm_from on the global map (the opaque shading then skips the direct term)
      const PhotonDev* map = gm && d >= gm_from ? gm : ph;
      if (map) {
        if (timing) record(ctx, ctx->ev_photon, ctx->ev_used_photon, true);
        HIP_TRY(ctx, launch_photon_gather(L, S, w, *map, d));
        if (timing) record(ctx, ctx->ev_photon, ctx->ev_used_photon, false);
        ctx->acc.photon_launches++;
      }
      HIP_TRY(ctx, launch_shade_opaque(L, S, w, d, D, p->seed, gen, pm));
      if (d < D) HIP_TRY(ctx, launch_shade_glass(L, S, w, d, p->seed, gen, pm));
    }
    if (timing) record(ctx, ctx->ev_shade, ctx->ev_used_shade, false);
    ctx->acc.shade_launches++;
    if (last) {
      if (query) {
        if (timing) record(ctx, ctx->ev_query, ctx->ev_used_query, true);
        HIP_TRY(ctx, launch_cache_query(ctx->stream, cache->dev, S, w, d & 1));
        if (timing) record(ctx, ctx->ev_query, ctx->ev_used_query, false);
        ctx->acc.query_launches++;
      }
      rc = finish();
      if (rc) return rc;
      break;
    }
    rc = trace_phase(ctx, L, S, w, gen, rounds, (d + 1) & 1, timing);
    if (rc) return rc;
  }
  return SDD_OK;
}

// Image update at the end of the wavefront of items [k0, k0 + n). Split at the ends of the views'
// sample planes, the wavefront falls into runs in which every pixel of one image occurs at most
// once: each run is one launch of the plain (non-atomic) update, and launches on the stream do
// not overlap. Beyond kMaxRuns runs (many small views) one launch with atomics does it all.
static hipError_t accumulate_wavefront(const Launch& L, const DevScene& S, const DevWS& w,
                                       const std::vector<ViewDesc>& views, uint64_t k0, uint32_t n) {
  constexpr size_t kMaxRuns = 64;
  std::vector<std::pair<uint32_t, uint32_t>> runs;  // (first slot, slots)
  size_t v = 0;
  for (uint64_t a = k0, e = k0 + n; a < e;) {
    while (v + 1 < views.size() && views[v + 1].item_base <= a) ++v;
    const uint64_t P = (uint64_t)views[v].width * views[v].height, base = views[v].item_base;
    if (P == 0) return launch_accumulate(L, S, w, 0, n, false);
    const uint64_t b = std::min(e, base + ((a - base) / P + 1) * P);
    runs.emplace_back((uint32_t)(a - k0), (uint32_t)(b - a));
    a = b;
    if (runs.size() > kMaxRuns) return launch_accumulate(L, S, w, 0, n, false);
  }
  for (const auto& r : runs) {
    const hipError_t e = launch_accumulate(L, S, w, r.first, r.second, true);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int enqueue_frame(sdd_ctx* ctx, const sdd_scene* scene, const std::vector<ViewDesc>& views,
                  const sdd_render_params* p, const Plan& plan, const DevWS& w, uint64_t total, bool timing,
                  sdd_cache* cache = nullptr, const sdd_train_params* tp = nullptr,
                  const PhotonDev* ph = nullptr, const PhotonDev* gm = nullptr, int gm_from = 0) {
  const int B = scene->hdr.n_bins;
  const uint32_t W = plan.W;
  DevScene S = device_view(scene);
  Launch L{ctx->stream, plan.trace_blocks, p->cell_order};
  int rc = store_views(ctx, views, w);
  if (rc) return rc;
  for (auto& v : views) HIP_TRY(ctx, launch_fill_f32(ctx->stream, v.image, (size_t)B * v.width * v.height, 0.0f));
  HIP_TRY(ctx, launch_fill_u32(ctx->stream, (uint32_t*)w.ctl, offsetof(Ctl, st_paths) / 4, 0u));
  if (p->persistent) {
    // one kernel: the work list's chunk counters (the per-XCD tile counters) start at zero above
    if (timing) record(ctx, ctx->ev_trace, ctx->ev_used_trace, true);
    HIP_TRY(ctx, launch_persist(L, S, w, total, p->seed, p->max_depth, W));
    if (timing) record(ctx, ctx->ev_trace, ctx->ev_used_trace, false);
    ctx->acc.trace_launches++;
    ctx->acc.wavefronts++;
    return SDD_OK;
  }
  HIP_TRY(ctx, launch_fill_u32(ctx->stream, w.ccount, 2ull * scene->hdr.n_cells * kDirBins * w.key_words, 0u));
  int gen = 0;
  const PathMode render_mode{0u, 0, nullptr, nullptr, gm ? gm_from : 0};
  uint64_t wavefront = 0;
  for (uint64_t k0 = 0; k0 < total; k0 += W, ++wavefront) {
    const uint32_t n = (uint32_t)std::min<uint64_t>(W, total - k0);
    // A training batch (full-depth paths recording their third vertex, then Adam steps) runs
    // before the wavefronts it is scheduled for, so that they are rendered with the updated
    // cache whatever the wavefront size; it shares the workspace, which the wavefront's ray
    // generation then starts afresh.
    if (cache && tp && tp->train_paths > 0 &&
        (tp->every > 0 ? wavefront % (uint64_t)tp->every == 0 : wavefront == 0)) {
      const uint32_t nt = (uint32_t)tp->train_paths;
      const PathMode train_mode{1u << 24, kCacheDepth, cache->dev.rx, cache->dev.rw};
      rc = run_paths(ctx, scene, p, L, S, w, cache->train_paths_done, nt, gen, timing, train_mode, cache, ph, gm, gm_from,
                     [&]() -> int {
                       if (timing) record(ctx, ctx->ev_train, ctx->ev_used_train, true);
                       HIP_TRY(ctx, launch_cache_gather(ctx->stream, cache->dev, w, nt, B));
                       HIP_TRY(ctx, launch_cache_compact(ctx->stream, cache->dev, nt,
                                                         (uint32_t)tp->steps * (uint32_t)tp->step_records));
                       int r = cache_train_records(ctx, cache, B, tp->steps, tp->step_records);
                       if (timing) record(ctx, ctx->ev_train, ctx->ev_used_train, false);
                       return r;
                     });
      if (rc) return rc;
      cache->train_paths_done += nt;
      ctx->acc.train_batches++;
    }
    rc = run_paths(ctx, scene, p, L, S, w, k0, n, gen, timing, render_mode, cache, ph, gm, gm_from, [&]() -> int {
      if (timing) record(ctx, ctx->ev_shade, ctx->ev_used_shade, true);
      HIP_TRY(ctx, accumulate_wavefront(L, S, w, views, k0, n));
      if (timing) record(ctx, ctx->ev_shade, ctx->ev_used_shade, false);
      return SDD_OK;
    });
    if (rc) return rc;
    ctx->acc.wavefronts++;
  }
  return SDD_OK;
}

int render_views(sdd_ctx* ctx, const sdd_scene* scene, std::vector<ViewDesc>& views, const sdd_render_params* p,
                 void* ws, size_t ws_bytes, const PhotonDev* ph = nullptr, const PhotonDev* gm = nullptr,
                 int gm_from = 0) {
  const int B = scene->hdr.n_bins;
  uint64_t total = 0;
  for (auto& v : views) {
    v.item_base = total;
    if (p->persistent)  // the work list: (8 x 8 tile, sample) items, 64 per tile and sample
      total += (uint64_t)((v.width + 7) / 8) * ((v.height + 7) / 8) * kPersistTileItems * (uint64_t)v.spp;
    else
      total += (uint64_t)v.width * v.height * (uint64_t)v.spp;
  }
  // never more paths in flight than the frame has items
  uint32_t W = (uint32_t)std::min<uint64_t>(p->wave_paths ? (uint64_t)p->wave_paths : (uint64_t)kDefaultWave, total);
  W = std::max<uint32_t>(W, 64);
  if (p->persistent) {
    // the work list is handed out in chunks of 64 items from 32-bit per-XCD counters
    if (total / kPersistTileItems / kXcds >= (1ull << 31))
      return fail(ctx, SDD_ERR_INVALID_ARG, "persistent render too large: at most 2^42 work items");
    W = persist_lanes(p, total, ctx->device);
  }
  Plan plan = fit_plan(W, B, scene->hdr.n_cells, (int)views.size(), ws_bytes);
  if (!ws) return fail(ctx, SDD_ERR_INVALID_ARG, "workspace is null");
  if (ws_bytes < plan.total)
    return fail(ctx, SDD_ERR_WORKSPACE,
                "workspace too small: need " + std::to_string(plan.total) + " bytes, got " + std::to_string(ws_bytes));
  DevWS w = ws_view(plan, ws);
  // Statistics keep accumulating on the device until sdd_finish collects them; a render into a
  // workspace other than the previous one starts them afresh (outside any captured graph).
  if (ctx->last_ctl != w.ctl)
    HIP_TRY(ctx, launch_fill_u32(ctx->stream, (uint32_t*)&w.ctl->st_paths,
                                 (sizeof(Ctl) - offsetof(Ctl, st_paths)) / 4, 0u));
  ctx->last_ctl = w.ctl;
  if (!p->use_graph)
    return enqueue_frame(ctx, scene, views, p, plan, w, total, p->timing != 0, nullptr, nullptr, ph, gm, gm_from);

  // Graph mode: capture the whole launch sequence once, replay it while the call repeats.
  uint64_t key = 1469598103934665603ull;
  key = fnv(key, views.data(), views.size() * sizeof(ViewDesc));
  sdd_render_params kp = *p;
  kp.timing = 0;
  key = fnv(key, &kp, sizeof(kp));
  key = fnv(key, &scene->dev, sizeof(void*));
  key = fnv(key, &scene->hdr, sizeof(scene->hdr));
  key = fnv(key, &ws, sizeof(void*));
  key = fnv(key, &plan.total, sizeof(plan.total));
  const PhotonDev no_map{};
  key = fnv(key, ph ? ph : &no_map, sizeof(PhotonDev));
  key = fnv(key, gm ? gm : &no_map, sizeof(PhotonDev));
  key = fnv(key, &gm_from, sizeof(gm_from));
  if (!(ctx->graph_exec && ctx->graph_key == key)) {
    if (ctx->graph_exec) {
      (void)hipGraphExecDestroy(ctx->graph_exec);
      ctx->graph_exec = nullptr;
    }
    if (ctx->graph) {
      (void)hipGraphDestroy(ctx->graph);
      ctx->graph = nullptr;
    }
    const uint64_t t0 = ctx->acc.trace_launches, s0 = ctx->acc.shade_launches, f0 = ctx->acc.wavefronts;
    const uint64_t g0 = ctx->acc.photon_launches;
    // The caller's stream may be the null stream, which cannot be captured: record the sequence
    // on the context's own stream (nothing runs there), then launch the graph on the caller's.
    if (!ctx->capture_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->capture_stream;
    hipError_t eb = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
      ctx->stream = user;
      return fail(ctx, SDD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(eb));
    }
    int rc = enqueue_frame(ctx, scene, views, p, plan, w, total, false, nullptr, nullptr, ph, gm, gm_from);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
    ctx->stream = user;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(ctx, SDD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    ctx->graph = g;
    HIP_TRY(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
    ctx->graph_key = key;
    ctx->graph_trace_launches = ctx->acc.trace_launches - t0;
    ctx->graph_shade_launches = ctx->acc.shade_launches - s0;
    ctx->graph_wavefronts = ctx->acc.wavefronts - f0;
    ctx->graph_photon_launches = ctx->acc.photon_launches - g0;
    // the capture only recorded the launches; count them when the graph actually runs
    ctx->acc.trace_launches = t0;
    ctx->acc.shade_launches = s0;
    ctx->acc.wavefronts = f0;
    ctx->acc.photon_launches = g0;
  }
  if (p->timing) record(ctx, ctx->ev_graph, ctx->ev_used_graph, true);
  HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
  if (p->timing) record(ctx, ctx->ev_graph, ctx->ev_used_graph, false);
  ctx->acc.trace_launches += ctx->graph_trace_launches;
  ctx->acc.shade_launches += ctx->graph_shade_launches;
  ctx->acc.wavefronts += ctx->graph_wavefronts;
  ctx->acc.photon_launches += ctx->graph_photon_launches;
  ctx->acc.graph_launches++;
  return SDD_OK;
}

// Workspace of sdd_render_noalloc: a device array of the library itself, so that callers that
// cannot allocate device memory can still render. Each device the library runs on holds its own
// copy for the life of the process. Host code must not pass `scratch` itself to a kernel (on the
// host it only names the symbol): its device address is looked up once per device, with that
// device current, and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up on the first call for it).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// ------------------------------------------------------------------------------------------
// caustic photon map: parameters, buffer layout, device view
// ------------------------------------------------------------------------------------------
std::string check_photon_params(const sdd_photon_params* p) {
  if (!p) return "photon params is null";
  if (p->n_photons < 1) return "n_photons must be >= 1";
  if (p->max_depth < 2 || p->max_depth > 64) return "photon max_depth must lie in 2..64";
  if ((double)p->n_photons * (p->max_depth - 1) >= 4294967296.0)
    return "n_photons (max_depth - 1) must stay below 2^32";
  if (!(p->radius > 0.0f) || !std::isfinite(p->radius)) return "radius must be finite > 0";
  if (p->capacity < 1 || p->capacity > (1ll << 28)) return "capacity must lie in 1..2^28";
  if (p->wave_paths != 0 && (p->wave_paths < 64 || p->wave_paths > (1 << 26))) return "wave_paths out of range";
  if (p->queue_rounds < 0 || p->queue_rounds > 256) return "queue_rounds out of range";
  if (p->kind != SDD_PHOTON_CAUSTIC && p->kind != SDD_PHOTON_GLOBAL) return "unknown photon map kind";
  return "";
}

uint32_t glass_triangles(const sdd_scene* s) {
  const SceneHeader& H = s->hdr;
  const uint8_t* img = s->image.data();
  const float* gt = (const float*)(img + H.off_gtris);
  const int32_t* mt = (const int32_t*)(img + H.off_mtype);
  uint32_t n = 0;
  for (int64_t t = 0; t < H.n_tri; ++t) {
    uint32_t m;
    std::memcpy(&m, gt + 12 * t + 7, 4);
    n += mt[m] == SDD_MAT_GLASS;
  }
  return n;
}

// Buffer layout of a map: control words, window thresholds and triangles, records (position,
// direction, flux quads), bucket counts and starts, and the records' positions and directions
// again in bucket order (what the gathering scans).
void photon_layout(sdd_photon_map* m, const sdd_scene* s, const sdd_photon_params* p) {
  m->prm = *p;
  m->B = s->hdr.n_bins;
  m->Bp = (m->B + 3) & ~3;
  m->max_win = std::max<uint32_t>(1, glass_triangles(s));
  // grid cells of the gather radius, about two buckets per record (2^12 .. 2^22)
  int total = 12;
  while (total < 22 && std::ldexp(1.0, total) < 2.0 * (double)p->capacity) ++total;
  const uint32_t nb = 1u << total;
  m->n_buckets = nb;
  const size_t rq = 2 + (size_t)m->Bp / 4;
  size_t o = 0;
  m->off_ctl = o;    o = a256(o + 256);
  m->off_thr = o;    o = a256(o + 4ull * m->max_win);
  m->off_tri = o;    o = a256(o + 4ull * m->max_win);
  m->off_rec = o;    o = a256(o + 16ull * rq * (size_t)p->capacity);
  m->off_bcount = o; o = a256(o + 4ull * nb);
  m->off_bstart = o; o = a256(o + 4ull * (nb + 1));
  m->off_cand = o;   o = a256(o + 16ull * (size_t)p->capacity);
  m->off_bsum = o;   o = a256(o + 4ull * (nb / kPhotonScanChunk + 1));
  m->off_occ = o;    o = a256(o + 4ull * kPhotonOccWords);
  m->off_srec = o;   o = a256(o + 16ull * rq * (size_t)p->capacity);
  m->total = o;
}

PhotonDev photon_dev(const sdd_photon_map* m) {
  PhotonDev P;
  std::memset(&P, 0, sizeof(P));
  uint8_t* b = (uint8_t*)m->buf;
  P.ctl = (uint32_t*)(b + m->off_ctl);
  P.win_thr = (const uint32_t*)(b + m->off_thr);
  P.win_tri = (const uint32_t*)(b + m->off_tri);
  P.rec = (float4*)(b + m->off_rec);
  P.bcount = (uint32_t*)(b + m->off_bcount);
  P.bstart = (uint32_t*)(b + m->off_bstart);
  P.cand = (float4*)(b + m->off_cand);
  P.bsum = (uint32_t*)(b + m->off_bsum);
  P.occ = (uint32_t*)(b + m->off_occ);
  P.srec = (float4*)(b + m->off_srec);
  P.n_win = (uint32_t)m->thr.size();
  P.cap = (uint32_t)m->prm.capacity;
  P.n_buckets = m->n_buckets;
  P.rq = 2 + (uint32_t)m->Bp / 4;
  P.radius = m->prm.radius;
  P.inv_cell = (float)(1.0 / (double)m->prm.radius);
  P.flux_scale = (float)(m->area / (double)m->prm.n_photons);
  P.seed_lo = (uint32_t)m->prm.seed;
  P.seed_hi = (uint32_t)(m->prm.seed >> 32);
  P.max_depth = m->prm.max_depth;
  P.global = m->prm.kind == SDD_PHOTON_GLOBAL ? 1 : 0;
  return P;
}

uint32_t photon_wave(const sdd_photon_params* p) {
  const uint64_t W = p->wave_paths ? (uint64_t)p->wave_paths : (uint64_t)kDefaultWave;
  return (uint32_t)std::max<uint64_t>(64, std::min<uint64_t>(W, (uint64_t)p->n_photons));
}

}  // namespace

extern "C" {

int sdd_scene_create(const sdd_scene_desc* desc, sdd_scene** out) {
  if (!desc || !out) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  sdd_scene* s = new (std::nothrow) sdd_scene();
  if (!s) return fail(nullptr, SDD_ERR_INTERNAL, "out of host memory");
  std::string e;
  try {
    e = build_scene(*desc, s);
  } catch (const std::exception& ex) {
    e = std::string("internal: ") + ex.what();
  }
  if (!e.empty()) {
    delete s;
    return fail(nullptr, e.rfind("internal", 0) == 0 ? SDD_ERR_INTERNAL : SDD_ERR_INVALID_ARG, e);
  }
  *out = s;
  return SDD_OK;
}

void sdd_scene_destroy(sdd_scene* s) { delete s; }

int sdd_scene_get_info(const sdd_scene* s, sdd_scene_info* out) {
  if (!s || !out) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  *out = s->info;
  return SDD_OK;
}

int sdd_scene_device_bytes(const sdd_scene* s, size_t* bytes) {
  if (!s || !bytes) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  *bytes = s->image.size();
  return SDD_OK;
}

int sdd_scene_host_image(const sdd_scene* s, const void** data, size_t* bytes) {
  if (!s || !data || !bytes) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  *data = s->image.data();
  *bytes = s->image.size();
  return SDD_OK;
}

int sdd_create(sdd_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(nullptr, SDD_ERR_HIP, "no HIP device available");
  if (hip_device < 0 || hip_device >= n) return fail(nullptr, SDD_ERR_INVALID_ARG, "device index out of range");
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) return fail(nullptr, SDD_ERR_HIP, hipGetErrorString(e));
  if (hip_device >= kMaxDevices) return fail(nullptr, SDD_ERR_INVALID_ARG, "device index beyond the supported 64");
  // the device's copy of the static render workspace: its address, once per device
  void* scr = nullptr;
  e = scratch_address(hip_device, &scr);
  if (e != hipSuccess) return fail(nullptr, SDD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  sdd_ctx* c = new sdd_ctx();
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  std::memset(&c->acc, 0, sizeof(c->acc));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
  *out = c;
  return SDD_OK;
}

void sdd_destroy(sdd_ctx* c) {
  if (!c) return;
  for (auto& p : c->ev_trace) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto& p : c->ev_shade) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto& p : c->ev_graph) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto& p : c->ev_query) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto& p : c->ev_train) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  for (auto& p : c->ev_photon) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  delete c;
}

int sdd_set_stream(sdd_ctx* c, void* s) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  c->stream = (hipStream_t)s;
  return SDD_OK;
}

int sdd_scene_upload(sdd_ctx* c, sdd_scene* s, void* dev_buf, size_t bytes) {
  if (!c || !s || !dev_buf) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  if (bytes < s->image.size()) return fail(c, SDD_ERR_WORKSPACE, "scene buffer smaller than sdd_scene_device_bytes");
  if (((uintptr_t)dev_buf & 255) != 0) return fail(c, SDD_ERR_INVALID_ARG, "scene buffer must be 256-byte aligned");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(dev_buf, s->image.data(), s->image.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  s->dev = dev_buf;
  s->dev_bytes = bytes;
  s->dev_device = c->device;
  return SDD_OK;
}

// Rewrite the sun or environment rows of a scene: the host image, and the uploaded copy on the
// context stream (waits, as sdd_scene_upload does). Renders enqueued earlier keep the old values.
static int write_scene_rows(sdd_ctx* c, sdd_scene* s, size_t off, const float* row) {
  const SceneHeader& H = s->hdr;
  float* dst = (float*)(s->image.data() + off);
  for (int j = 0; j < H.bins_pad; ++j) dst[j] = j < H.n_bins && row ? row[j] : 0.0f;
  std::memcpy(s->image.data(), &s->hdr, sizeof(SceneHeader));
  if (s->dev) {
    if (s->dev_device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "scene was uploaded on another device");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync((uint8_t*)s->dev + off, dst, (size_t)H.bins_pad * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(s->dev, s->image.data(), sizeof(SceneHeader), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return SDD_OK;
}

int sdd_set_sun(sdd_ctx* c, sdd_scene* s, const float dir_to_sun[3], const float* irradiance) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!s || !dir_to_sun || !irradiance) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  const double l = std::sqrt((double)dir_to_sun[0] * dir_to_sun[0] + (double)dir_to_sun[1] * dir_to_sun[1] +
                             (double)dir_to_sun[2] * dir_to_sun[2]);
  if (!(l > 1e-12) || !std::isfinite(l)) return fail(c, SDD_ERR_INVALID_ARG, "sun direction must be non-zero and finite");
  for (int j = 0; j < s->hdr.n_bins; ++j)
    if (!(irradiance[j] >= 0) || !std::isfinite(irradiance[j]))
      return fail(c, SDD_ERR_INVALID_ARG, "sun irradiance must be finite >= 0");
  for (int a = 0; a < 3; ++a) s->hdr.sun[a] = (float)(dir_to_sun[a] / l);
  return write_scene_rows(c, s, s->hdr.off_sunE, irradiance);
}

int sdd_set_env(sdd_ctx* c, sdd_scene* s, const float* radiance) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!s) return fail(c, SDD_ERR_INVALID_ARG, "scene is null");
  int nz = 0;
  for (int j = 0; radiance && j < s->hdr.n_bins; ++j) {
    if (!(radiance[j] >= 0) || !std::isfinite(radiance[j]))
      return fail(c, SDD_ERR_INVALID_ARG, "env radiance must be finite >= 0");
    nz |= radiance[j] != 0.0f;
  }
  s->hdr.env_nonzero = nz;
  return write_scene_rows(c, s, s->hdr.off_env, radiance);
}

int sdd_workspace_bytes(const sdd_scene* s, const sdd_render_params* p, size_t* bytes) {
  if (!s || !bytes) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, SDD_ERR_INVALID_ARG, e);
  uint32_t W = p->wave_paths ? (uint32_t)p->wave_paths : (uint32_t)kDefaultWave;
  if (p->persistent) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    W = persist_lanes(p, UINT64_MAX / 2, dev);
  }
  *bytes = make_plan(W, s->hdr.n_bins, s->hdr.n_cells, 64).total;
  return SDD_OK;
}

int sdd_render(sdd_ctx* c, const sdd_scene* s, const sdd_camera* cam, const sdd_render_params* p, void* ws,
               size_t ws_bytes, float* image) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!cam || !image) return fail(c, SDD_ERR_INVALID_ARG, "null camera or image");
  std::string e = check_params(p);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (p->mode != SDD_MODE_PLAIN) return fail(c, SDD_ERR_INVALID_ARG, "cached mode requires a configured cache");
  std::vector<ViewDesc> views(1);
  e = make_view(*cam, &views[0]);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  views[0].spp = p->spp;
  views[0].inv_spp = 1.0f / (float)p->spp;
  views[0].image = image;
  views[0].view_id = p->view;
  views[0].first_sample = (uint32_t)p->first_sample;
  HIP_TRY(c, hipSetDevice(c->device));
  return render_views(c, s, views, p, ws, ws_bytes);
}

int sdd_render_noalloc(sdd_ctx* c, const sdd_scene* s, const sdd_camera* cam, const sdd_render_params* p,
                       float* image) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!cam || !image) return fail(c, SDD_ERR_INVALID_ARG, "null camera or image");
  std::string e = check_params(p);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (p->mode != SDD_MODE_PLAIN) return fail(c, SDD_ERR_INVALID_ARG, "sdd_render_noalloc renders in plain mode only");
  // graph instantiation and timing events allocate: not here
  if (p->use_graph || p->timing || p->persistent)
    return fail(c, SDD_ERR_INVALID_ARG, "sdd_render_noalloc takes neither use_graph, timing nor persistent");
  std::vector<ViewDesc> views(1);
  e = make_view(*cam, &views[0]);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  views[0].spp = p->spp;
  views[0].inv_spp = 1.0f / (float)p->spp;
  views[0].image = image;
  views[0].view_id = p->view;
  views[0].first_sample = (uint32_t)p->first_sample;
  const uint64_t total = (uint64_t)cam->width * cam->height * (uint64_t)p->spp;
  const int B = s->hdr.n_bins, nc = s->hdr.n_cells;
  // paths in flight: as asked, else the most (up to the library default) whose workspace fits
  uint64_t W = p->wave_paths ? (uint64_t)p->wave_paths : (uint64_t)kDefaultWave;
  W = std::max<uint64_t>(64, std::min<uint64_t>(W, total));
  if (!p->wave_paths)
    while (W > 64 && fit_plan((uint32_t)W, B, nc, 1, kScratchBytes).total > kScratchBytes)
      W = std::max<uint64_t>(64, W * 3 / 4);
  const size_t need = fit_plan((uint32_t)W, B, nc, 1, kScratchBytes).total;
  if (need > kScratchBytes)
    return fail(c, SDD_ERR_WORKSPACE,
                "sdd_render_noalloc: " + std::to_string(W) + " paths in flight need " + std::to_string(need) +
                    " bytes of workspace, the static workspace holds " + std::to_string(kScratchBytes) +
                    " (fewer wave_paths, bins or cells)");
  HIP_TRY(c, hipSetDevice(c->device));
  void* ws = nullptr;
  HIP_TRY(c, scratch_address(c->device, &ws));
  sdd_render_params q = *p;
  q.wave_paths = (int32_t)W;
  return render_views(c, s, views, &q, ws, kScratchBytes);
}

int sdd_render_batch(sdd_ctx* c, const sdd_scene* s, const sdd_camera* cams, const int32_t* spp, int32_t n_views,
                     const sdd_render_params* p, void* ws, size_t ws_bytes, float* const* images) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!cams || !spp || !images || n_views < 1 || n_views > 64)
    return fail(c, SDD_ERR_INVALID_ARG, "bad view list (1..64 views)");
  std::string e = check_params(p);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (p->mode != SDD_MODE_PLAIN) return fail(c, SDD_ERR_INVALID_ARG, "cached mode requires a configured cache");
  std::vector<ViewDesc> views(n_views);
  for (int v = 0; v < n_views; ++v) {
    e = make_view(cams[v], &views[v]);
    if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, "view " + std::to_string(v) + ": " + e);
    if (spp[v] < 1) return fail(c, SDD_ERR_INVALID_ARG, "spp per view must be >= 1");
    if (!images[v]) return fail(c, SDD_ERR_INVALID_ARG, "null image pointer");
    views[v].spp = spp[v];
    views[v].inv_spp = 1.0f / (float)spp[v];
    views[v].image = images[v];
    views[v].view_id = (uint32_t)v;
    views[v].first_sample = (uint32_t)p->first_sample;
  }
  HIP_TRY(c, hipSetDevice(c->device));
  return render_views(c, s, views, p, ws, ws_bytes);
}

int sdd_render_cached(sdd_ctx* c, const sdd_scene* s, sdd_cache* k, const sdd_camera* cam,
                      const sdd_render_params* p, const sdd_train_params* tp, void* ws, size_t ws_bytes,
                      float* image) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!cam || !image) return fail(c, SDD_ERR_INVALID_ARG, "null camera or image");
  std::string e = check_params(p);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (p->mode != SDD_MODE_CACHED) return fail(c, SDD_ERR_INVALID_ARG, "sdd_render_cached needs mode SDD_MODE_CACHED");
  if (p->use_graph) return fail(c, SDD_ERR_INVALID_ARG, "cached renders are not captured into graphs");
  if (p->max_depth < kCacheDepth) return fail(c, SDD_ERR_INVALID_ARG, "cached mode needs max_depth >= 3");
  if (!k) return fail(c, SDD_ERR_INVALID_ARG, "cache is null");
  if (!k->ready) return fail(c, SDD_ERR_NOT_READY, "cache parameters are not set (sdd_cache_init / set_params)");
  if (k->device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "cache was created on another device");
  if (s->hdr.n_bins > k->cfg.max_bins) return fail(c, SDD_ERR_INVALID_ARG, "scene has more bins than the cache");
  if (s->hdr.n_mat > k->cfg.n_mat) return fail(c, SDD_ERR_INVALID_ARG, "scene has more materials than the cache");
  std::vector<ViewDesc> views(1);
  e = make_view(*cam, &views[0]);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  views[0].spp = p->spp;
  views[0].inv_spp = 1.0f / (float)p->spp;
  views[0].image = image;
  views[0].view_id = p->view;
  views[0].first_sample = (uint32_t)p->first_sample;
  const uint64_t total = (uint64_t)cam->width * cam->height * (uint64_t)p->spp;
  // never more paths in flight than the frame has items, or a training batch has paths
  const uint64_t w_req = p->wave_paths ? (uint64_t)p->wave_paths : (uint64_t)kDefaultWave;
  const uint64_t w_need = std::max<uint64_t>(total, tp && tp->train_paths > 0 ? (uint64_t)tp->train_paths : 0);
  uint32_t W = (uint32_t)std::min<uint64_t>(w_req, w_need);
  W = std::max<uint32_t>(W, 64);
  if (tp && tp->train_paths != 0) {
    if (tp->train_paths < 0 || (uint64_t)tp->train_paths > w_req || tp->train_paths > k->cfg.max_records)
      return fail(c, SDD_ERR_INVALID_ARG, "train_paths must lie in 0..min(wave paths, max_records)");
    if (tp->step_records < kCacheVerts || tp->step_records > k->cfg.max_step)
      return fail(c, SDD_ERR_INVALID_ARG, "step_records must lie in 32..max_step");
    if (tp->steps < 1 || tp->every < 0) return fail(c, SDD_ERR_INVALID_ARG, "steps must be >= 1 and every >= 0");
    if (p->max_depth <= kCacheDepth)
      return fail(c, SDD_ERR_INVALID_ARG, "training paths need max_depth >= 4 (they continue past the cached vertex)");
  }
  Plan plan = make_plan(W, s->hdr.n_bins, s->hdr.n_cells, 1);
  if (!ws) return fail(c, SDD_ERR_INVALID_ARG, "workspace is null");
  if (ws_bytes < plan.total)
    return fail(c, SDD_ERR_WORKSPACE,
                "workspace too small: need " + std::to_string(plan.total) + " bytes, got " + std::to_string(ws_bytes));
  HIP_TRY(c, hipSetDevice(c->device));
  DevWS w = ws_view(plan, ws);
  if (c->last_ctl != w.ctl)
    HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)&w.ctl->st_paths, (sizeof(Ctl) - offsetof(Ctl, st_paths)) / 4, 0u));
  c->last_ctl = w.ctl;
  views[0].item_base = 0;
  return enqueue_frame(c, s, views, p, plan, w, total, p->timing != 0, k, tp);
}

int sdd_query_workspace_bytes(const sdd_scene* s, int64_t n, size_t* bytes) {
  if (!s || !bytes || n < 1) return fail(nullptr, SDD_ERR_INVALID_ARG, "bad argument");
  uint32_t W = (uint32_t)std::min<int64_t>(n, kDefaultWave);
  *bytes = make_plan(std::max<uint32_t>(W, 64), s->hdr.n_bins, s->hdr.n_cells, 1).total;
  return SDD_OK;
}

static int query(sdd_ctx* c, const sdd_scene* s, const float* orig, const float* dir, const int32_t* skip, int64_t n,
                 void* ws, size_t ws_bytes, bool shadow, float* t, int32_t* id, float* u, float* v, float* vis) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!orig || !dir || n < 1 || !ws) return fail(c, SDD_ERR_INVALID_ARG, "bad ray arrays");
  uint32_t W = std::max<uint32_t>(64, (uint32_t)std::min<int64_t>(n, kDefaultWave));
  Plan plan = make_plan(W, s->hdr.n_bins, s->hdr.n_cells, 1);
  if (ws_bytes < plan.total) return fail(c, SDD_ERR_WORKSPACE, "workspace too small for the ray query");
  HIP_TRY(c, hipSetDevice(c->device));
  DevWS w = ws_view(plan, ws);
  DevScene S = device_view(s);
  Launch L{c->stream, plan.trace_blocks};
  HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)w.ctl, sizeof(Ctl) / 4, 0u));
  HIP_TRY(c, launch_fill_u32(c->stream, w.ccount, 2ull * s->hdr.n_cells * kDirBins * w.key_words, 0u));
  c->last_ctl = w.ctl;
  int gen = 0;
  for (int64_t a = 0; a < n; a += W) {
    uint32_t m = (uint32_t)std::min<int64_t>(W, n - a);
    HIP_TRY(c, launch_fill_u32(c->stream, &w.ctl->cat_count[0][0], 2 * 8 * kKeyStride, 0u));
    HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)w.catb, ((size_t)2 * w.W + 3) / 4, 0u));
    HIP_TRY(c, launch_pack_rays(L, S, w, orig + 3 * a, dir + 3 * a, skip ? skip + a : nullptr, m, shadow ? 1 : 0, gen));
    rc = trace_phase(c, L, S, w, gen, kQueryRounds, 0, false);
    if (rc) return rc;
    if (shadow)
      HIP_TRY(c, launch_resolve_vis(L, S, w, m, vis + (size_t)a * s->hdr.n_bins));
    else
      HIP_TRY(c, launch_unpack_hits(L, S, w, m, t + a, id + a, u + a, v + a));
  }
  return SDD_OK;
}

int sdd_trace(sdd_ctx* c, const sdd_scene* s, const float* orig, const float* dir, const int32_t* skip, int64_t n,
              void* ws, size_t ws_bytes, float* t, int32_t* id, float* u, float* v) {
  if (!t || !id || !u || !v) return fail(c, SDD_ERR_INVALID_ARG, "null output array");
  return query(c, s, orig, dir, skip, n, ws, ws_bytes, false, t, id, u, v, nullptr);
}

int sdd_shadow(sdd_ctx* c, const sdd_scene* s, const float* orig, const float* dir, const int32_t* skip, int64_t n,
               void* ws, size_t ws_bytes, float* vis) {
  if (!vis) return fail(c, SDD_ERR_INVALID_ARG, "null output array");
  return query(c, s, orig, dir, skip, n, ws, ws_bytes, true, nullptr, nullptr, nullptr, nullptr, vis);
}

int sdd_philox(sdd_ctx* c, const uint32_t ctr[4], const uint32_t key[2], int64_t n, uint32_t* out) {
  if (!c || !ctr || !key || !out || n < 0) return fail(c, SDD_ERR_INVALID_ARG, "bad argument");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_philox(c->stream, ctr, key, (uint64_t)n, out));
  return SDD_OK;
}

int sdd_spectral_to_srgb(sdd_ctx* c, const float* image, int32_t n_bins, float lmin, float lmax, int64_t n_pixels,
                         float exposure, float* xyz, float* srgb) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!image || (!xyz && !srgb)) return fail(c, SDD_ERR_INVALID_ARG, "null image, or no output");
  if (n_bins < 1 || n_bins > kMaxBins) return fail(c, SDD_ERR_INVALID_ARG, "n_bins must lie in 1..128");
  if (!(lmin > 0.0f) || !(lmax > lmin) || !std::isfinite(lmax)) return fail(c, SDD_ERR_INVALID_ARG, "need 0 < lambda_min < lambda_max");
  if (n_pixels < 1) return fail(c, SDD_ERR_INVALID_ARG, "n_pixels must be >= 1");
  if (!(exposure >= 0.0f) || !std::isfinite(exposure)) return fail(c, SDD_ERR_INVALID_ARG, "exposure must be finite >= 0");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_spectral_to_srgb(c->stream, image, n_bins, lmin, lmax, (uint64_t)n_pixels, exposure, xyz, srgb));
  return SDD_OK;
}

// ------------------------------------------------------------------------------------------
// caustic photon map
// ------------------------------------------------------------------------------------------
int sdd_photon_map_bytes(const sdd_scene* s, const sdd_photon_params* p, size_t* bytes) {
  if (!s || !bytes) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  const std::string e = check_photon_params(p);
  if (!e.empty()) return fail(nullptr, SDD_ERR_INVALID_ARG, e);
  sdd_photon_map m;
  photon_layout(&m, s, p);
  *bytes = m.total;
  return SDD_OK;
}

int sdd_photon_workspace_bytes(const sdd_scene* s, const sdd_photon_params* p, size_t* bytes) {
  if (!s || !bytes) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  const std::string e = check_photon_params(p);
  if (!e.empty()) return fail(nullptr, SDD_ERR_INVALID_ARG, e);
  *bytes = make_plan(photon_wave(p), s->hdr.n_bins, s->hdr.n_cells, 1).total;
  return SDD_OK;
}

int sdd_photon_map_create(sdd_ctx* c, const sdd_scene* s, const sdd_photon_params* p, void* buf, size_t bytes,
                          sdd_photon_map** out) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!s || !buf || !out) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const std::string e = check_photon_params(p);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (((uintptr_t)buf & 255) != 0) return fail(c, SDD_ERR_INVALID_ARG, "photon map buffer must be 256-byte aligned");
  sdd_photon_map* m = new (std::nothrow) sdd_photon_map();
  if (!m) return fail(c, SDD_ERR_INTERNAL, "out of host memory");
  photon_layout(m, s, p);
  if (bytes < m->total) {
    delete m;
    return fail(c, SDD_ERR_WORKSPACE, "photon map buffer smaller than sdd_photon_map_bytes");
  }
  m->buf = buf;
  m->bytes = bytes;
  m->device = c->device;
  *out = m;
  return SDD_OK;
}

void sdd_photon_map_destroy(sdd_photon_map* m) { delete m; }

int sdd_photon_map_build(sdd_ctx* c, const sdd_scene* s, sdd_photon_map* m, void* ws, size_t ws_bytes) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!m) return fail(c, SDD_ERR_INVALID_ARG, "photon map is null");
  if (m->device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "photon map was created on another device");
  if (s->hdr.n_bins != m->B) return fail(c, SDD_ERR_NOT_READY, "scene bins differ from the photon map's");
  if (glass_triangles(s) > m->max_win) return fail(c, SDD_ERR_INVALID_ARG, "scene has more glass than the photon map");
  // the grid's integer cell coordinates must stay far from overflow
  const double inv_cell = 1.0 / (double)m->prm.radius;
  for (int a = 0; a < 3; ++a)
    if (std::max(std::fabs(s->info.grid_lo[a]), std::fabs(s->info.grid_hi[a])) * inv_cell > 1e9)
      return fail(c, SDD_ERR_INVALID_ARG, "photon radius too small for the scene's extent");
  const uint32_t W = photon_wave(&m->prm);
  Plan plan = make_plan(W, m->B, s->hdr.n_cells, 1);
  if (!ws) return fail(c, SDD_ERR_INVALID_ARG, "workspace is null");
  if (ws_bytes < plan.total)
    return fail(c, SDD_ERR_WORKSPACE,
                "workspace too small: need " + std::to_string(plan.total) + " bytes, got " + std::to_string(ws_bytes));
  HIP_TRY(c, hipSetDevice(c->device));
  // Windows: glass triangles with their projected areas on the scene's unit sun direction (FP32
  // as stored), in FP64, and the integer thresholds of the emission choice.
  const SceneHeader& H = s->hdr;
  const float* gt = (const float*)(s->image.data() + H.off_gtris);
  const int32_t* mt = (const int32_t*)(s->image.data() + H.off_mtype);
  const double sx = H.sun[0], sy = H.sun[1], sz = H.sun[2];
  std::vector<double> cdf{0.0};
  // the previous build's copies out of these vectors must be complete before they change
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  m->thr.clear();
  m->tri.clear();
  for (int64_t t = 0; t < H.n_tri; ++t) {
    const float* v = gt + 12 * t;
    uint32_t mat;
    std::memcpy(&mat, v + 7, 4);
    if (mt[mat] != SDD_MAT_GLASS) continue;
    const double ax = (double)v[4] - v[0], ay = (double)v[5] - v[1], az = (double)v[6] - v[2];
    const double bx = (double)v[8] - v[0], by = (double)v[9] - v[1], bz = (double)v[10] - v[2];
    const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const double a = 0.5 * std::fabs(nx * sx + ny * sy + nz * sz);
    if (!(a > 0.0)) continue;
    m->tri.push_back((uint32_t)t);
    cdf.push_back(cdf.back() + a);
  }
  m->area = cdf.back();
  m->thr.resize(m->tri.size());
  for (size_t w = 0; w < m->tri.size(); ++w) m->thr[w] = (uint32_t)std::floor(cdf[w] / m->area * 16777216.0);
  PhotonDev P = photon_dev(m);
  HIP_TRY(c, launch_fill_u32(c->stream, P.ctl, 64, 0u));
  if (!m->tri.empty()) {
    HIP_TRY(c, hipMemcpyAsync((void*)P.win_thr, m->thr.data(), 4 * m->thr.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync((void*)P.win_tri, m->tri.data(), 4 * m->tri.size(), hipMemcpyHostToDevice, c->stream));
    DevWS w = ws_view(plan, ws);
    if (c->last_ctl != w.ctl)
      HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)&w.ctl->st_paths, (sizeof(Ctl) - offsetof(Ctl, st_paths)) / 4, 0u));
    c->last_ctl = w.ctl;
    HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)w.ctl, offsetof(Ctl, st_paths) / 4, 0u));
    HIP_TRY(c, launch_fill_u32(c->stream, w.ccount, 2ull * H.n_cells * kDirBins * w.key_words, 0u));
    DevScene S = device_view(s);
    // the build's traversal launches are short (photons end after a few vertices): a grid of
    // one workgroup per 1024 photons in flight (half a render wavefront's) gives each wave more
    // parts and fewer end-of-launch probes of the exhausted ranges (caustic build of the church,
    // 4 M photons in wavefronts of 2^20: 12.9 -> 11.0 ms; 512 workgroups slowed the global build)
    const int photon_blocks = std::max(kXcds, (int)std::min<uint32_t>(W / 1024, 2048) / kXcds * kXcds);
    Launch L{c->stream, std::min(plan.trace_blocks, photon_blocks)};
    const int rounds = m->prm.queue_rounds ? m->prm.queue_rounds : kDefaultRounds;
    const int D = m->prm.max_depth;
    int gen = 0;
    const uint64_t N = (uint64_t)m->prm.n_photons;
    for (uint64_t k0 = 0; k0 < N; k0 += W) {
      const uint32_t n = (uint32_t)std::min<uint64_t>(W, N - k0);
      HIP_TRY(c, launch_fill_u32(c->stream, &w.ctl->cat_count[0][0], 2 * 8 * kKeyStride, 0u));
      HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)w.catb, ((size_t)2 * w.W + 3) / 4, 0u));
      // emission and the way from the window to the sun
      HIP_TRY(c, launch_photon_gen(L, S, w, P, k0, n, gen));
      rc = trace_phase(c, L, S, w, gen, rounds, 1, false);
      if (rc) return rc;
      HIP_TRY(c, launch_photon_vis(L, S, w, P, 1));
      for (int d = 1; d <= D; ++d) {
        HIP_TRY(c, launch_photon_shade(L, S, w, P, d, gen));
        if (d == D) break;
        rc = trace_phase(c, L, S, w, gen, rounds, (d + 1) & 1, false);
        if (rc) return rc;
      }
    }
  }
  HIP_TRY(c, launch_photon_build(c->stream, P));
  m->built = true;
  return SDD_OK;
}

int sdd_photon_map_info(sdd_ctx* c, sdd_photon_map* m, sdd_photon_info* out) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!m || !out) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->n_buckets = (int32_t)m->n_buckets;
  out->device_bytes = m->total;
  if (!m->built) return SDD_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  uint32_t h[2];
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(h, (uint8_t*)m->buf + m->off_ctl, sizeof(h), hipMemcpyDeviceToHost));
  out->stored = std::min<int64_t>(h[0], m->prm.capacity);
  out->dropped = h[1];
  out->n_windows = (int32_t)m->tri.size();
  out->window_area = m->area;
  return SDD_OK;
}

int sdd_photon_map_records(sdd_ctx* c, sdd_photon_map* m, int64_t n, float* pos, float* dir, float* flux, int64_t* id,
                           int32_t* vertex) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!m || n < 0) return fail(c, SDD_ERR_INVALID_ARG, "bad argument");
  if (!m->built) return fail(c, SDD_ERR_NOT_READY, "photon map has not been built");
  sdd_photon_info info;
  int rc = sdd_photon_map_info(c, m, &info);
  if (rc) return rc;
  if (n > info.stored) return fail(c, SDD_ERR_INVALID_ARG, "more records asked for than the map holds");
  if (n == 0) return SDD_OK;
  const size_t rq = 2 + (size_t)m->Bp / 4;
  std::vector<float> h((size_t)n * rq * 4);
  HIP_TRY(c, hipMemcpy(h.data(), (uint8_t*)m->buf + m->off_rec, h.size() * 4, hipMemcpyDeviceToHost));
  for (int64_t r = 0; r < n; ++r) {
    const float* q = h.data() + (size_t)r * rq * 4;
    uint32_t lo, hi;
    std::memcpy(&lo, q + 3, 4);
    std::memcpy(&hi, q + 7, 4);
    if (pos) for (int a = 0; a < 3; ++a) pos[3 * r + a] = q[a];
    if (dir) for (int a = 0; a < 3; ++a) dir[3 * r + a] = q[4 + a];
    if (flux) for (int j = 0; j < m->B; ++j) flux[(size_t)r * m->B + j] = q[8 + j];
    if (id) id[r] = (int64_t)((uint64_t)lo | ((uint64_t)(hi >> 8) << 32));
    if (vertex) vertex[r] = (int32_t)(hi & 0xFFu);
  }
  return SDD_OK;
}

int sdd_photon_map_load(sdd_ctx* c, sdd_photon_map* m, int64_t n, const float* pos, const float* dir, const float* flux,
                        const int64_t* id, const int32_t* vertex) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!m || n < 0 || n > m->prm.capacity) return fail(c, SDD_ERR_INVALID_ARG, "bad argument (0 <= n <= capacity)");
  if (n > 0 && (!pos || !dir || !flux)) return fail(c, SDD_ERR_INVALID_ARG, "null record arrays");
  const size_t rq = 2 + (size_t)m->Bp / 4;
  std::vector<float> h((size_t)n * rq * 4, 0.0f);
  for (int64_t r = 0; r < n; ++r) {
    float* q = h.data() + (size_t)r * rq * 4;
    for (int a = 0; a < 3; ++a) {
      q[a] = pos[3 * r + a];
      q[4 + a] = dir[3 * r + a];
      if (!std::isfinite(q[a]) || !std::isfinite(q[4 + a]))
        return fail(c, SDD_ERR_INVALID_ARG, "non-finite record position or direction");
    }
    const uint64_t pid = id ? (uint64_t)id[r] : 0;
    const uint32_t lo = (uint32_t)pid, hi = (uint32_t)(vertex ? vertex[r] & 0xFF : 0) | (uint32_t)(pid >> 32) << 8;
    std::memcpy(q + 3, &lo, 4);
    std::memcpy(q + 7, &hi, 4);
    for (int j = 0; j < m->B; ++j) q[8 + j] = flux[(size_t)r * m->B + j];
  }
  const uint32_t ctl[2] = {(uint32_t)n, 0u};
  HIP_TRY(c, hipSetDevice(c->device));
  if (n > 0)
    HIP_TRY(c, hipMemcpyAsync((uint8_t*)m->buf + m->off_rec, h.data(), h.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync((uint8_t*)m->buf + m->off_ctl, ctl, sizeof(ctl), hipMemcpyHostToDevice, c->stream));
  const PhotonDev P = photon_dev(m);
  HIP_TRY(c, launch_photon_build(c->stream, P));
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the host staging above is freed on return
  m->built = true;
  return SDD_OK;
}

int sdd_render_photons(sdd_ctx* c, const sdd_scene* s, const sdd_photon_map* caustic, const sdd_photon_map* global,
                       int32_t global_from, const sdd_camera* cam, const sdd_render_params* p, void* ws,
                       size_t ws_bytes, float* image) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  int rc = scene_ready(c, s);
  if (rc) return rc;
  if (!cam || !image) return fail(c, SDD_ERR_INVALID_ARG, "null camera or image");
  if (!caustic && !global) return fail(c, SDD_ERR_INVALID_ARG, "no photon map");
  std::string e = check_params(p);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (p->mode != SDD_MODE_PLAIN) return fail(c, SDD_ERR_INVALID_ARG, "sdd_render_photons renders in plain mode");
  if (p->persistent) return fail(c, SDD_ERR_INVALID_ARG, "sdd_render_photons does not render persistent");
  for (const sdd_photon_map* m : {caustic, global}) {
    if (!m) continue;
    if (!m->built) return fail(c, SDD_ERR_NOT_READY, "photon map has not been built");
    if (m->device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "photon map was created on another device");
    if (m->B != s->hdr.n_bins) return fail(c, SDD_ERR_NOT_READY, "scene bins differ from the photon map's");
  }
  if (caustic && caustic->prm.kind != SDD_PHOTON_CAUSTIC)
    return fail(c, SDD_ERR_INVALID_ARG, "the caustic map argument holds a global map");
  if (global && global->prm.kind != SDD_PHOTON_GLOBAL)
    return fail(c, SDD_ERR_INVALID_ARG, "the global map argument holds a caustic map");
  if (global && global_from < 1) return fail(c, SDD_ERR_INVALID_ARG, "global_from must be >= 1 with a global map");
  std::vector<ViewDesc> views(1);
  e = make_view(*cam, &views[0]);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  views[0].spp = p->spp;
  views[0].inv_spp = 1.0f / (float)p->spp;
  views[0].image = image;
  views[0].view_id = p->view;
  views[0].first_sample = (uint32_t)p->first_sample;
  HIP_TRY(c, hipSetDevice(c->device));
  PhotonDev Pc, Pg;
  if (caustic) Pc = photon_dev(caustic);
  if (global) Pg = photon_dev(global);
  return render_views(c, s, views, p, ws, ws_bytes, caustic ? &Pc : nullptr, global ? &Pg : nullptr,
                      global ? global_from : 0);
}

int sdd_finish(sdd_ctx* c) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int status = SDD_OK;
  if (c->last_ctl) {
    Ctl h;
    HIP_TRY(c, hipMemcpy(&h, c->last_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    c->acc.paths += h.st_paths;
    c->acc.vertices += h.st_vertices;
    c->acc.ext_rays += h.st_ext;
    c->acc.shadow_rays += h.st_shadow;
    c->acc.cell_visits += h.st_visits;
    c->acc.migrations += h.st_migr;
    c->acc.escapes += h.st_escape;
    c->acc.glass_crossings += h.st_glass;
    c->acc.err_cross_overflow += h.err_cross;
    c->acc.err_nonfinite += h.err_nonfinite;
    c->acc.err_stack += h.err_stack;
    c->acc.node_visits += h.st_nodes;
    c->acc.tri_tests += h.st_tris;
    c->acc.cache_queries += h.st_queries;
    c->acc.photon_vertices += h.st_ph_vertices;
    c->acc.photons_found += h.st_ph_found;
    c->acc.photon_lit_vertices += h.st_ph_lit;
    c->acc.photon_candidates += h.st_ph_cand;
    c->acc.photon_candidates_max = std::max<uint64_t>(c->acc.photon_candidates_max, h.st_ph_cand_max);
    if (h.err_cross) status = fail(c, SDD_ERR_QUEUE_OVERFLOW, "a shadow ray crossed more glass slabs than recorded");
    else if (h.err_nonfinite)
      status = fail(c, SDD_ERR_DEVICE, std::to_string(h.err_nonfinite) + " non-finite radiance values reached the image");
    c->last_ctl = nullptr;
  }
  for (size_t i = 0; i < c->ev_used_trace; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_trace[i].first, c->ev_trace[i].second) == hipSuccess) c->acc.trace_ms += ms;
  }
  for (size_t i = 0; i < c->ev_used_shade; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_shade[i].first, c->ev_shade[i].second) == hipSuccess) c->acc.shade_ms += ms;
  }
  for (size_t i = 0; i < c->ev_used_graph; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_graph[i].first, c->ev_graph[i].second) == hipSuccess) c->acc.graph_ms += ms;
  }
  for (size_t i = 0; i < c->ev_used_query; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_query[i].first, c->ev_query[i].second) == hipSuccess) c->acc.query_ms += ms;
  }
  for (size_t i = 0; i < c->ev_used_train; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_train[i].first, c->ev_train[i].second) == hipSuccess) c->acc.train_ms += ms;
  }
  for (size_t i = 0; i < c->ev_used_photon; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_photon[i].first, c->ev_photon[i].second) == hipSuccess) c->acc.photon_ms += ms;
  }
  c->ev_used_trace = c->ev_used_shade = c->ev_used_graph = c->ev_used_query = c->ev_used_train = 0;
  c->ev_used_photon = 0;
  return status;
}

int sdd_get_stats(sdd_ctx* c, sdd_stats* out) {
  if (!c || !out) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  *out = c->acc;
  return SDD_OK;
}

int sdd_reset_stats(sdd_ctx* c) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  std::memset(&c->acc, 0, sizeof(c->acc));
  return SDD_OK;
}

const char* sdd_last_error(const sdd_ctx* c) { return c ? c->err.c_str() : thread_error(); }

}  // extern "C"
