// Host-side objects of libspecdd (not visible through the C ABI).
#pragma once

#include <string>
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

namespace sdd {

// Builds the cell-decomposed scene image. Returns an empty string on success, else the reason.
std::string build_scene(const sdd_scene_desc& d, sdd_scene* out);

// Device view of an uploaded scene.
DevScene device_view(const sdd_scene* s);

void set_thread_error(const std::string& msg);
hipStream_t ctx_stream(const sdd_ctx* ctx);
const char* thread_error();

}  // namespace sdd
