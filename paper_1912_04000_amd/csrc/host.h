// Host-side objects of libspecdd (not visible through the C ABI).
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "../../include/specdd.h"
#include "internal.h"

struct sdd_scene {
  std::vector<uint8_t> image;   // serialised device image
  sdd::SceneHeader hdr;
  sdd_scene_info info;
  void* dev = nullptr;          // bound device buffer (after sdd_scene_upload)
  size_t dev_bytes = 0;
  int dev_device = -1;
};

struct sdd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  sdd::Ctl* last_ctl = nullptr;     // control block of the last launched work (inside a workspace)
  sdd_stats acc;               // accumulated statistics
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_trace, ev_shade, ev_graph;
  size_t ev_used_trace = 0, ev_used_shade = 0, ev_used_graph = 0;
  int cu_count = 256;
  // captured launch sequence of the last graph-mode render and the key it was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;   // own stream (default priority) used only to record graphs
  uint64_t graph_key = 0;
  uint64_t graph_trace_launches = 0, graph_shade_launches = 0, graph_wavefronts = 0;
  uint64_t graph_photon_launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_query, ev_train, ev_photon;
  size_t ev_used_query = 0, ev_used_train = 0, ev_used_photon = 0;
};

struct sdd_cache {
  sdd_cache_config cfg;
  sdd::CacheDev dev;          // device view (pointers into the caller's buffer)
  float* opt = nullptr;       // device [4]: Adam step count (uint bits), 1/(1-b1^t), 1/(1-b2^t), step active
  void* buf = nullptr;
  size_t bytes = 0;
  int device = -1;
  bool ready = false;         // parameters defined (init / set_params)
  uint64_t train_paths_done = 0;
};

struct sdd_photon_map {
  sdd_photon_params prm;
  int B = 0, Bp = 0;
  uint32_t max_win = 0;        // window slots (the scene's glass triangles)
  uint32_t n_buckets = 0;
  void* buf = nullptr;
  size_t bytes = 0;
  int device = -1;
  size_t off_ctl = 0, off_thr = 0, off_tri = 0, off_rec = 0, off_bcount = 0, off_bstart = 0, off_cand = 0, off_bsum = 0, off_occ = 0, off_srec = 0, total = 0;
  std::vector<uint32_t> thr, tri;  // windows of the last build (kept alive for its copies)
  double area = 0.0;
  bool built = false;
};

namespace sdd {

// Builds the cell-decomposed scene image. Returns an empty string on success, else the reason.
std::string build_scene(const sdd_scene_desc& d, sdd_scene* out);

// Device view of an uploaded scene.
DevScene device_view(const sdd_scene* s);

void set_thread_error(const std::string& msg);
hipStream_t ctx_stream(const sdd_ctx* ctx);
// One training batch over the records held by the cache (cache_api.cpp).
int cache_train_records(sdd_ctx* c, sdd_cache* k, int B, int steps, int step_records);
const char* thread_error();

}  // namespace sdd
