// Autotuner: cell grid x wavefront size x queue rounds x cell order, measured on short calibration
// renders.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host.h"

extern "C" int sdd_render_batch(sdd_ctx*, const sdd_scene*, const sdd_camera*, const int32_t*, int32_t,
                                const sdd_render_params*, void*, size_t, float* const*);

namespace {

uint64_t fnv(uint64_t h, const void* data, size_t n) {
  const uint8_t* b = (const uint8_t*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t tune_key(const sdd_scene_desc& d, const sdd_camera* views, int n_views, const sdd_render_params& p,
                  const std::string& device) {
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, d.verts, (size_t)d.n_tri * 36);
  h = fnv(h, d.mat, (size_t)d.n_tri * 2);
  h = fnv(h, d.materials, (size_t)d.n_mat * sizeof(sdd_material));
  const size_t tab = (size_t)d.n_mat * d.n_bins * 4;
  h = fnv(h, d.n_tab, tab);
  h = fnv(h, d.k_tab, tab);
  h = fnv(h, d.rho_tab, tab);
  h = fnv(h, &d.n_bins, sizeof(d.n_bins));
  h = fnv(h, &p.max_depth, sizeof(p.max_depth));
  h = fnv(h, views, (size_t)n_views * sizeof(sdd_camera));
  h = fnv(h, device.data(), device.size());
  return h;
}

bool read_cache(const char* path, uint64_t key, sdd_tune_point* out) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024], want[64];
  std::snprintf(want, sizeof(want), "\"key\": \"%016llx\"", (unsigned long long)key);
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    if (!std::strstr(line, want)) continue;
    const char* g = std::strstr(line, "\"grid\": [");
    const char* w = std::strstr(line, "\"wave_paths\": ");
    const char* r = std::strstr(line, "\"queue_rounds\": ");
    const char* s = std::strstr(line, "\"samples_per_s\": ");
    const char* o = std::strstr(line, "\"cell_order\": ");
    const char* pe = std::strstr(line, "\"persistent\": ");
    if (g && w && r && s && o && pe && std::sscanf(o, "\"cell_order\": %d", &out->cell_order) == 1 &&
        std::sscanf(pe, "\"persistent\": %d", &out->persistent) == 1 &&
        std::sscanf(g, "\"grid\": [%d, %d, %d]", &out->grid[0], &out->grid[1], &out->grid[2]) == 3 &&
        std::sscanf(w, "\"wave_paths\": %d", &out->wave_paths) == 1 &&
        std::sscanf(r, "\"queue_rounds\": %d", &out->queue_rounds) == 1 &&
        std::sscanf(s, "\"samples_per_s\": %lf", &out->samples_per_s) == 1)
      found = true;
  }
  std::fclose(f);
  return found;
}

void write_cache(const char* path, uint64_t key, const sdd_tune_point& b, const std::string& device, int n_tried) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\": \"%016llx\", \"device\": \"%s\", \"grid\": [%d, %d, %d], \"wave_paths\": %d, "
               "\"queue_rounds\": %d, \"cell_order\": %d, \"persistent\": %d, \"samples_per_s\": %.6e, "
               "\"candidates\": %d}\n",
               (unsigned long long)key, device.c_str(), b.grid[0], b.grid[1], b.grid[2], b.wave_paths, b.queue_rounds,
               b.cell_order, b.persistent, b.samples_per_s, n_tried);
  std::fclose(f);
}

}  // namespace

extern "C" int sdd_autotune(sdd_ctx* ctx, const sdd_scene_desc* desc, const sdd_camera* views, int32_t n_views,
                            const sdd_render_params* base, const sdd_tune_space* sp, void* scene_buf,
                            size_t scene_bytes, void* workspace, size_t ws_bytes, float* const* images,
                            const char* cache_path, sdd_tune_result* out) {
  if (!ctx || !desc || !views || !base || !sp || !scene_buf || !workspace || !images || !out || n_views < 1) {
    sdd::set_thread_error("sdd_autotune: null or empty argument");
    return SDD_ERR_INVALID_ARG;
  }
  if (sp->n_waves < 1 || sp->n_waves > 8 || sp->n_grids < 1 || sp->n_grids > 8 || sp->n_rounds < 1 ||
      sp->n_rounds > 4 || sp->calib_spp < 1 || sp->reps < 1 || sp->n_orders < 0 || sp->n_orders > 2 ||
      sp->try_persistent < 0 || sp->try_persistent > 1) {
    sdd::set_thread_error("sdd_autotune: search space out of range");
    return SDD_ERR_INVALID_ARG;
  }
  std::memset(out, 0, sizeof(*out));
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  std::string device = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) device = std::string(prop.name) + "/" + prop.gcnArchName;
  const uint64_t key = tune_key(*desc, views, n_views, *base, device);
  if (read_cache(cache_path, key, &out->best)) {
    out->from_cache = 1;
    return SDD_OK;
  }
  uint64_t samples = 0;
  for (int v = 0; v < n_views; ++v) samples += (uint64_t)views[v].width * views[v].height * sp->calib_spp;
  std::vector<int32_t> spp(n_views, sp->calib_spp);
  hipStream_t stream = sdd::ctx_stream(ctx);  // renders go through the public calls on this stream
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SDD_ERR_HIP;
  int rc = SDD_OK;
  double best = -1.0;
  for (int g = 0; g < sp->n_grids && rc == SDD_OK; ++g) {
    sdd_scene_desc d = *desc;
    for (int a = 0; a < 3; ++a) d.grid[a] = sp->grids[g][a];
    sdd_scene* scene = nullptr;
    rc = sdd_scene_create(&d, &scene);
    if (rc) break;
    size_t need = 0;
    sdd_scene_device_bytes(scene, &need);
    if (need > scene_bytes) {
      sdd_scene_destroy(scene);
      continue;
    }
    rc = sdd_scene_upload(ctx, scene, scene_buf, scene_bytes);
    const int n_orders = sp->n_orders ? sp->n_orders : 1;
    const int n_wave_cands = sp->n_waves * sp->n_rounds * n_orders;
    for (int ci = 0; ci < n_wave_cands + sp->try_persistent && rc == SDD_OK; ++ci) {
      sdd_render_params p = *base;
      p.persistent = 0;
      if (ci < n_wave_cands) {  // wavefront size x rounds x cell order
        const int wi = ci / (sp->n_rounds * n_orders), ri = ci % (sp->n_rounds * n_orders);
        p.wave_paths = sp->wave_paths[wi];
        p.queue_rounds = sp->queue_rounds[ri % sp->n_rounds];
        if (sp->n_orders) p.cell_order = sp->cell_orders[ri / sp->n_rounds];
      } else {  // the persistent kernel with its default lanes
        p.persistent = 1;
        p.wave_paths = 0;
      }
      p.use_graph = 0;
      p.timing = 0;
      p.spp = sp->calib_spp;
      size_t wsn = 0;
      if (sdd_workspace_bytes(scene, &p, &wsn) != SDD_OK || wsn > ws_bytes) continue;
      rc = sdd_render_batch(ctx, scene, views, spp.data(), n_views, &p, workspace, ws_bytes, images);  // warm-up
      if (rc) break;
      float best_ms = 1e30f;
      for (int r = 0; r < sp->reps && rc == SDD_OK; ++r) {
        (void)hipEventRecord(e0, stream);
        rc = sdd_render_batch(ctx, scene, views, spp.data(), n_views, &p, workspace, ws_bytes, images);
        (void)hipEventRecord(e1, stream);
        if (rc) break;
        rc = sdd_finish(ctx);
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) best_ms = ms;
      }
      if (rc) break;
      sdd_tune_point pt;
      std::memset(&pt, 0, sizeof(pt));
      for (int a = 0; a < 3; ++a) pt.grid[a] = d.grid[a];
      pt.wave_paths = p.wave_paths;
      pt.queue_rounds = p.queue_rounds;
      pt.cell_order = p.cell_order;
      pt.persistent = p.persistent;
      pt.samples_per_s = samples / (best_ms * 1e-3);
      if (out->n_tried < 128) out->tried[out->n_tried++] = pt;
      if (pt.samples_per_s > best) {
        best = pt.samples_per_s;
        out->best = pt;
      }
    }
    sdd_scene_destroy(scene);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (best < 0) {
    sdd::set_thread_error("sdd_autotune: no candidate fitted the scene buffer and workspace");
    return SDD_ERR_WORKSPACE;
  }
  write_cache(cache_path, key, out->best, device, out->n_tried);
  return SDD_OK;
}
