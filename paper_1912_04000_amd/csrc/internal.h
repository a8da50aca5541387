// Internal layout shared by the host runtime and the gfx950 kernels of libspecdd.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <stddef.h>
#include <stdint.h>

namespace sdd {

// ------------------------------------------------------------------------------------------
// Tunables fixed at compile time
// ------------------------------------------------------------------------------------------
constexpr int kWG = 256;            // threads per workgroup of the traversal/shading kernels
constexpr int kTile = 256;          // rays of one queue key handled by one workgroup tile
constexpr int kShortStack = 12;     // traversal stack entries kept in LDS per thread
constexpr int kMaxStack = 72;       // builder caps BVH depth so the stack never exceeds this
constexpr int kWide = 4;            // children per BVH node
constexpr int kMaxCross = 8;        // glass crossings recorded per shadow ray
constexpr int kMaxBins = 128;
constexpr int kPhotonScanChunk = 4096;  // photon-map buckets per workgroup of the bucket scan
constexpr int kPhotonOccWords = 1024;   // occupancy bitmap of the photon map's hashed super-cells
constexpr int kMaxGrid = 64;
constexpr int kLdsCells = 256;      // cell tables up to this size are staged in LDS by the traversal
constexpr int kXcds = 8;            // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kDirBins = 24;        // ray queues per cell: direction octant x dominant axis
// Queue-key counters sit kKeyStride words apart, one 64-byte line each: their atomics are served
// one at a time per line, and the keys that camera or shadow rays share would otherwise crowd
// a few lines.
constexpr int kKeyStride = 16;
// Each queue key counts its rays in sub-ranges, laid out one after the other in the key's queue
// range: first by one of 2^kDirSubBits sub-bins of the ray's direction inside its direction
// class (dir_sub), then by the block of a 2^L x 2^L x 2^L split of the cell that holds the ray's
// origin (blocks in Morton order). The rays of a tile, and of its 64-ray parts, then start close
// together in similar directions and descend the cell's BVH along similar paths. Tiles still
// span the whole key. L is the largest level up to kMaxSubLevels that keeps the sub-ranges of all
// keys within kSubRangeBudget and within the 2W rays a wavefront of W paths can queue
// (sub_levels_for): finer grids, whose keys hold fewer rays, get fewer levels and the counters
// stay small, and short wavefronts (a photon-map build) do not pay for sub-ranges they cannot
// fill. A key's counters are consecutive words of its own counter lines (DevWS::key_words per
// key), so the atomics on a line come from the producers of one key.
constexpr int kMaxSubLevels = 3;
constexpr int kDirSubBits = 2;
constexpr uint64_t kSubRangeBudget = 1ull << 23;
inline int sub_levels_for(int n_cells, uint32_t W) {
  const uint64_t cap = std::min<uint64_t>(kSubRangeBudget, 2ull * W);
  int L = kMaxSubLevels;
  while (L > 0 && ((uint64_t)n_cells * kDirBins << (3 * L + kDirSubBits)) > cap) --L;
  return L;
}
// k_subscan takes a key's 2^(3 L + kDirSubBits) sub-ranges by wave up to 64 (a divisor of 64)
// and by workgroup above (a multiple of kWG), at every level L
constexpr bool sub_ranges_suit_scan() {
  for (int L = 0; L <= kMaxSubLevels; ++L) {
    const int n = 1 << (3 * L + kDirSubBits);
    if (!(n <= 64 ? 64 % n == 0 : n % kWG == 0)) return false;
  }
  return true;
}
static_assert(sub_ranges_suit_scan(), "sub-ranges per key that k_subscan cannot take");
constexpr uint32_t kBlocked = 0xFFFFFFFFu;
constexpr uint32_t kFirstVisit = 0x80000000u;
constexpr uint32_t kShadowBit = 0x80000000u;  // in the ray's slot word
constexpr uint32_t kInvalidCell = 0xFFFFFFFFu;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;  // produced-list entry without destination queue (skipped)
constexpr uint32_t kEmptyChild = 0xFFFFFFFFu;
// Traversal stack entries: an inner node index, or a leaf as flag | count << 27 | first triangle.
constexpr uint32_t kStackLeaf = 0x80000000u;
constexpr uint32_t kStackLeafMaxCount = 15u;
constexpr uint32_t kStackLeafMaxIndex = (1u << 27) - 1u;
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

// Categories of finished rays: the traversal sorts every ray it finishes into one list per
// category so that each shading kernel runs one branch only (no divergence between kinds).
constexpr int kCatOpaque = 0;      // extension ray hit an opaque triangle
constexpr int kCatGlass = 1;       // extension ray hit a glass triangle
constexpr int kCatEscape = 2;      // extension ray left the scene (environment radiance)
constexpr int kCatShadowClear = 3; // shadow ray reached the sun without crossing glass
constexpr int kCatShadowGlass = 4; // shadow ray reached the sun through glass
constexpr int kCats = 5;

// ------------------------------------------------------------------------------------------
// Serialised scene image (one device buffer, offsets in bytes from its start)
// ------------------------------------------------------------------------------------------
struct SceneHeader {
  uint32_t magic, version;
  int32_t n_tri, n_mat, n_bins, n_cells;
  int32_t grid[3];
  int32_t max_depth;
  float lo[3], hi[3];
  float sun[3];
  int32_t env_nonzero;
  uint64_t off_planes, off_cells, off_nodes, off_ctris, off_gtris, off_mtype, off_thick, off_n, off_k, off_rho,
      off_lambda, off_sunE, off_env;
  uint64_t n_nodes, n_refs;
  float lambda_min_nm, lambda_max_nm;
  int32_t max_leaf;
  int32_t bins_pad;    // row stride of the spectral tables: n_bins rounded up to a multiple of 4
  int32_t pad[4];
  // spectral transmittance maps of glass: texture coordinates per triangle (two float4: u0 v0 u1
  // v1 | u2 v2 0 0), map table (texel offset in floats, width, height, 0), texels [h][w][Bp]
  // (internal transmittance at normal incidence), map of each material (-1 none)
  uint64_t off_uv, off_texinfo, off_texel, off_mtex;
  int32_t n_tex;
  int32_t pad2[3];
};
constexpr size_t kHeaderBytes = 512;   // the header's room at the start of the scene image
static_assert(sizeof(SceneHeader) <= kHeaderBytes, "header fits its room");

// Node of a cell BVH: four children, their boxes stored in the parent as 8-bit bounds on a grid of
// the node's own box (64 bytes, two nodes per 128-byte cache line), four 16-byte words:
//   origin.xyz (FP32) | e_x e_y e_z (bytes) ; child word[4] ; lo.x[4] hi.x[4] lo.y[4] hi.y[4]
//   (bytes) ; lo.z[4] hi.z[4] (bytes) 0 0
// bound = origin + q 2^(e - 127); lo rounded down, hi up, so a stored box contains its child.
// word: an inner child's node index (cell-relative, < 2^27), a leaf as count << 27 | first
// cell triangle (count 1..15), or kEmptyChild for no child.
// Cell triangle (48 bytes): (v0, global id) (v1, material id) (v2, 0).
// Global triangle: the same 48-byte record indexed by the triangle id.

// Device view of a scene (built from the device base pointer and the header).
struct DevScene {
  const float4* nodes;
  const float4* ctris;
  const float4* gtris;
  const int4* cells;    // (node base, node count, tri base, tri count)
  const float* planes;  // gx+1 | gy+1 | gz+1
  const int32_t* mtype;
  const float* thick;
  const float* ntab;
  const float* ktab;
  const float* rho;
  const float* lambda;
  const float* sunE;
  const float* env;
  const float4* guv;    // [n_tri][2] texture coordinates (only when n_tex > 0)
  const int4* texinfo;  // [n_tex] (texel offset in floats, width, height, 0)
  const float* texel;   // maps [h][w][Bp]
  const int32_t* mtex;  // [n_mat] map of the material, -1 none
  int32_t n_tex;
  int32_t gx, gy, gz, n_cells;
  float lo[3], hi[3];
  float inv_cs[3];
  float sun[3];
  int32_t n_bins, n_mat, env_nonzero, bins_pad;
};

// Per-view description for raygen and accumulation.
struct ViewDesc {
  float eye[3];
  float fwd[3];     // unit forward
  float right[3];   // right * tan(vfov/2) * W/H
  float upv[3];     // up * tan(vfov/2)
  int32_t width, height;
  int32_t spp;
  float inv_spp;
  uint64_t item_base;  // first global item of this view
  uint64_t image_off;  // float offset of this view's image inside the image arena (batch)
  float* image;        // [B][H][W]
  uint32_t view_id;
  uint32_t first_sample;
};

// Control block (device) -- counters of the wavefront machinery and statistics.
struct Ctl {
  uint32_t list_count[2];   // produced (ray, cell, rank) entries per generation parity
  uint32_t n_queue;         // entries in the cell-sorted queue of the current round
  uint32_t n_tiles;         // tiles of the current round
  uint32_t ph_heavy[2];     // photon gathering: vertices deferred to the wave-wide pass, per bounce parity
  uint32_t pad0[10];        // to the end of the first 64-byte line
  // per-XCD tile counters of the current round (reset by k_scan), one 64-byte line each: every
  // tile taken is an atomic on one of them, and atomics on one line are served one at a time
  uint32_t tile_next[8 * kKeyStride];
  // finished-ray list lengths per bounce parity and category (kCats used), category c at
  // [c * kKeyStride]: one 64-byte line per counter
  uint32_t cat_count[2][8 * kKeyStride];
  // statistics (accumulated until collected)
  unsigned long long st_paths, st_vertices, st_ext, st_shadow, st_visits, st_migr, st_escape, st_glass;
  unsigned long long err_cross, err_nonfinite, err_stack;
  unsigned long long st_nodes, st_tris;  // BVH nodes visited, triangle tests (traversal work)
  unsigned long long st_queries;         // vertices answered by the radiance cache
  unsigned long long st_ph_vertices;     // opaque vertices that gathered from a photon map
  unsigned long long st_ph_found;        // photon records found within the gather radius (summed)
  unsigned long long st_ph_lit;          // gathering vertices that found at least one record
  unsigned long long st_ph_cand;         // bucket entries tested by the gathering (summed)
  unsigned long long st_ph_cand_max;     // most bucket entries tested for one vertex
  unsigned long long pad1[5];            // to a whole number of 64-byte lines
};

// Device view of a workspace.
struct DevWS {
  uint32_t* pix;
  uint32_t* smp;
  uint32_t* view;
  float* beta;       // [W][Bp] path throughput per bin
  float* nee;        // [W][Bp] direct-term weight of the pending shadow ray
  float* lacc;       // [W][Bp] radiance gathered by the path so far
  float4* hit;       // [W] (t, id bits, u, v)
  float4* rays;      // [2W][2]  (o.xyz, skip bits) (d.xyz, slot | shadow bit)
  uint32_t* shcnt;   // [W] glass crossings of the pending shadow ray, kBlocked if blocked
  float2* shx;       // [kMaxCross][W] glass crossings of shadow rays: (material id bits, triangle id bits)
  uint32_t* cat;     // [2][kCats][W] finished-ray lists
  uint8_t* catb;     // [2W] category + 1 of the finished extension (first W) / shadow ray of a slot
  uint32_t* lsrc;    // [2W] produced entries: ray index | first-visit bit
  uint32_t* ldst;    // [2W] destination cell
  uint32_t* lrank;   // [2W] rank inside the destination cell
  uint32_t* queue;   // [2W] cell-sorted entries of the current round
  uint32_t* ccount;  // [2][n_cells * kDirBins * key_words]: sub-range counters, key_words per key
  uint32_t* coff;    // [n_cells * kDirBins << sub_shift]: offset of each sub-range inside its key's range
  uint32_t* ksum;    // [n_cells * kDirBins] rays per key
  uint32_t* koff;    // [n_cells * kDirBins] queue offset of each key's range
  uint4* tiles;      // [max_tiles] (cell, start, count, 0)
  uint32_t* spill;   // [kMaxStack - kShortStack][trace_threads]
  Ctl* ctl;
  ViewDesc* views;   // [n_views]
  uint32_t W;        // path slots
  uint32_t max_tiles;
  uint32_t trace_threads;
  int32_t n_views;
  int32_t Bp;        // row stride of the per-slot spectral rows
  uint32_t sub_shift;  // 3 L + kDirSubBits: sub-ranges per queue key = 1 << sub_shift
  uint32_t key_words;  // counter words per queue key: max(kKeyStride, 1 << sub_shift)
};

// ------------------------------------------------------------------------------------------
// Learned spectral radiance cache
// ------------------------------------------------------------------------------------------
// Network: input 64 = [position grid 2 Lp | direction grid 2 Ld | material embedding 8 |
// wavelength one-blob 8 | zero padding], four 64-wide ReLU layers without biases, one output.
constexpr int kCacheWidth = 64;
constexpr int kCacheFeat = 2;       // features per grid level
constexpr int kCacheMatDim = 8;
constexpr int kCacheBlob = 8;
constexpr int kCacheMaxLevels = 16;
constexpr int kCacheVerts = 32;     // query vertices per wave (the MFMA N dimension)
constexpr int kCacheWaves = 4;      // waves per workgroup of the cache kernels
constexpr int kCacheERow = 72;      // bf16 row stride of the per-wave encoding tile in LDS

// Device view of a cache (masters, optimizer state, packed weights, training buffers).
struct CacheDev {
  float* P;            // FP32 master parameters, flat layout (see sdd_cache_param_count)
  float* M;            // Adam first moments [n_param]
  float* V;            // Adam second moments [n_param]
  float* G;            // gradients [n_param]
  uint32_t* gpos;      // bf16x2 copy of the position grid [Lp][Tp]
  uint32_t* gdir;      // bf16x2 copy of the direction grid [Ld][Td]
  uint4* wf;           // forward MFMA A operands [4 layers][2 mt][4 kb][64 lanes] (8 bf16 each)
  uint4* wb;           // backward (transposed) A operands, same shape
  uint4* w4b;          // output weights as B-operand words [4 kb][2 halves] (8 bf16 each)
  // training buffers
  float4* rx;          // [max_train] record position, material id bits in w
  float4* rw;          // [max_train] record direction toward the previous vertex, valid flag in w
  float* tgt;          // [max_train][max_bins] suffix radiance targets
  uint32_t* ridx;      // [max_train] compacted record slots; ridx[max_train] = count
  uint16_t* hst;       // [4][max_rows/32][64][32] bf16 layer inputs h0..h3 (tile, unit, row)
  uint16_t* dst;       // [4][max_rows/32][64][32] bf16 deltas of layers 1..4
  float* dE;           // [max_step][64] gradient of the encoding (pos | dir | mat)
  float* loss;         // [2] loss sum, rows
  int64_t n_param;
  int64_t o_pos, o_dir, o_mat, o_w[4], o_w4;
  int32_t Lp, Ld, Tp_log2, Td_log2, n_mat, n_in;
  int32_t Npos[kCacheMaxLevels], Ndir[kCacheMaxLevels];
  uint32_t dense_pos, dense_dir;   // bit l: level l is indexed densely
  float lo[3], ext[3];             // position normalisation box (lo, hi - lo)
  int32_t max_bins, max_train, max_step;
  int32_t pad;
};

// Random-number purpose and training record of a path population: rendered paths use purpose 0
// and record nothing; training paths use purpose 1 (bit 24 of the counter's depth word) and
// record their vertex at depth rec_depth.
struct PathMode {
  uint32_t purpose;    // 0 or 1u << 24
  int32_t rec_depth;   // vertex recorded for training, 0 = none
  float4* rec_x;       // [W] (position, material bits)
  float4* rec_w;       // [W] (direction toward the previous vertex, valid)
  int32_t gm_from = 0; // > 0: from this vertex on, opaque vertices take their diffuse light from a
                       // global photon map (gathered before shading): no direct term, mirror lobe only
};

// Device view of a photon map (a caller buffer laid out by the host): the window table of the
// emission, the stored photon records and a hashed uniform grid over them (cells of the gather
// radius, counting-sorted).
struct PhotonDev {
  uint32_t* ctl;              // [0] photons stored (may exceed cap), [1] photons dropped
  const uint32_t* win_thr;    // [n_win] integer thresholds floor(cdf_w / A 2^24)
  const uint32_t* win_tri;    // [n_win] window triangle ids
  float4* rec;                // [cap][rq]: (pos, id lo bits) (dir, vertex | id hi << 8) flux quads
  uint32_t* bcount;           // [n_buckets] photons per bucket, then scatter cursors
  uint32_t* bstart;           // [n_buckets + 1] first entry of each bucket in `cand`
  float4* cand;               // [cap] in bucket order: (pos, index into srec)
  float4* srec;               // [cap][rq] the records again, in bucket order (what a gather reads)
  uint32_t* bsum;             // [n_buckets / kPhotonScanChunk + 1] scan partial sums
  uint32_t* occ;              // [kPhotonOccWords] bit h: some record lies in a super-cell of hash h
  uint32_t n_win, cap, n_buckets, rq;  // rq = 2 + Bp / 4 float4 per record
  float radius, inv_cell;     // gather radius = grid cell size, 1 / radius
  float flux_scale;           // A / N: flux of a photon per unit of sun irradiance
  uint32_t seed_lo, seed_hi;
  int32_t max_depth;
  int32_t global;             // 1: global map (every opaque vertex stores; the diffuse lobe continues)
};

// Host helpers implemented in the kernels' translation unit.
struct Launch {
  hipStream_t stream;
  int trace_blocks;   // workgroups of the persistent traversal grid (multiple of kXcds)
  int cell_order = 0; // tile list order of the queue scan: 0 cell index, 1 fullest cells first
};

hipError_t launch_fill_f32(hipStream_t s, float* p, size_t n, float v);
hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, size_t n, uint32_t v);
hipError_t launch_raygen(const Launch& L, const DevScene& S, const DevWS& w, uint64_t k0, uint32_t n, uint64_t seed,
                         int gen, const PathMode& pm);
hipError_t launch_scan(const Launch& L, const DevScene& S, const DevWS& w, int gen);
hipError_t launch_scatter(const Launch& L, const DevWS& w, int gen);
hipError_t launch_trace(const Launch& L, const DevScene& S, const DevWS& w, int gen, int hops);
hipError_t launch_gather_cats(const Launch& L, const DevWS& w, int par);
hipError_t launch_resolve(const Launch& L, const DevScene& S, const DevWS& w, int depth);
hipError_t launch_escape(const Launch& L, const DevScene& S, const DevWS& w, int depth);
hipError_t launch_shade_opaque(const Launch& L, const DevScene& S, const DevWS& w, int depth, int max_depth,
                               uint64_t seed, int gen, const PathMode& pm);
hipError_t launch_shade_glass(const Launch& L, const DevScene& S, const DevWS& w, int depth, uint64_t seed, int gen,
                              const PathMode& pm);
hipError_t launch_accumulate(const Launch& L, const DevScene& S, const DevWS& w, uint32_t s0, uint32_t n,
                             bool unique);
uint32_t persist_resident_blocks(int device);
hipError_t launch_persist(const Launch& L, const DevScene& S, const DevWS& w, uint64_t total, uint64_t seed,
                          int max_depth, uint32_t lanes);
hipError_t launch_pack_rays(const Launch& L, const DevScene& S, const DevWS& w, const float* orig, const float* dir,
                            const int32_t* skip, uint32_t n, int shadow, int gen);
hipError_t launch_unpack_hits(const Launch& L, const DevScene& S, const DevWS& w, uint32_t n, float* t, int32_t* id,
                              float* u, float* v);
hipError_t launch_resolve_vis(const Launch& L, const DevScene& S, const DevWS& w, uint32_t n, float* vis);
hipError_t launch_philox(hipStream_t s, const uint32_t ctr[4], const uint32_t key[2], uint64_t n, uint32_t* out);
// caustic photon map
hipError_t launch_photon_gen(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, uint64_t k0,
                             uint32_t n, int gen);
hipError_t launch_photon_vis(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, int par);
hipError_t launch_photon_shade(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, int depth,
                               int gen);
hipError_t launch_photon_build(hipStream_t s, const PhotonDev& P);
hipError_t launch_photon_gather(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, int depth);

// colorimetry (color.hip)
hipError_t launch_spectral_to_srgb(hipStream_t s, const float* img, int B, float lmin, float lmax, uint64_t n,
                                   float exposure, float* xyz, float* srgb);

// radiance cache (cache.hip)
hipError_t launch_cache_init(hipStream_t s, const CacheDev& C, uint64_t seed);
hipError_t launch_cache_sync(hipStream_t s, const CacheDev& C);
hipError_t launch_cache_eval(hipStream_t s, const CacheDev& C, const float* x, const float* wo, const int32_t* mat,
                             uint32_t n, int B, float* out);
hipError_t launch_cache_query(hipStream_t s, const CacheDev& C, const DevScene& S, const DevWS& w, int p);
hipError_t launch_cache_load_records(hipStream_t s, const CacheDev& C, const float* x, const float* wo,
                                     const int32_t* mat, const float* t, uint32_t n, int B);
hipError_t launch_cache_gather(hipStream_t s, const CacheDev& C, const DevWS& w, uint32_t n, int B);
hipError_t launch_cache_compact(hipStream_t s, const CacheDev& C, uint32_t n, uint32_t cap);
hipError_t launch_cache_backward(hipStream_t s, const CacheDev& C, int B, uint32_t v0, uint32_t step_max);
hipError_t launch_cache_adam(hipStream_t s, const CacheDev& C, uint32_t v0, uint32_t step_max, float* opt, float lr,
                             float b1, float b2, float eps);

}  // namespace sdd
