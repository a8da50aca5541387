/*
 * specdd -- spectral path tracing over a spatially decomposed triangle scene, for one
 * AMD Instinct MI355X (gfx950).
 *
 * C ABI of libspecdd.so. The paper this follows is Gbikpi-Benissan, Callet, Magoules,
 * "Spectral domain decomposition method for physically-based rendering of Royaumont abbey"
 * (arXiv:1912.04000). Section numbers and equations below refer to it.
 *
 * Conventions
 *  - Every function returns an int status: SDD_OK (0) or a negative SDD_ERR_* code. The
 *    message of the last failure is available from sdd_last_error(ctx) (ctx may be NULL for
 *    calls that take no context). No C++ exception crosses this boundary.
 *  - Memory ownership: the library never allocates device memory. Scene buffers, workspaces,
 *    images and ray/hit arrays are owned by the caller (for example PyTorch tensors); the
 *    library owns only its opaque host handles (each *_create has a matching *_destroy) and
 *    small host staging memory.
 *  - Streams: device work is enqueued on the stream given to sdd_create / sdd_set_stream and
 *    the call returns after enqueueing. sdd_finish() waits for the stream and turns device
 *    error flags into a status; results are valid only after it returns SDD_OK.
 *  - Threading: a context is not re-entrant; distinct contexts are independent.
 *  - Units: lengths in metres (any consistent unit works for geometry; slab thicknesses are
 *    metres because absorption uses the wavelength in metres), wavelengths in nm (vacuum).
 */
#ifndef SPECDD_H
#define SPECDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDD_OK = 0,
  SDD_ERR_INVALID_ARG = -1,    /* argument out of range, null pointer, non-finite input      */
  SDD_ERR_HIP = -2,            /* a HIP runtime call failed                                   */
  SDD_ERR_WORKSPACE = -3,      /* workspace or buffer smaller than the size the library asked */
  SDD_ERR_QUEUE_OVERFLOW = -4, /* device-side capacity exceeded (reported by sdd_finish)      */
  SDD_ERR_NOT_READY = -5,      /* scene not uploaded / spectrum mismatch                      */
  SDD_ERR_INTERNAL = -6,       /* invariant violated inside the library                       */
  SDD_ERR_DEVICE = -7          /* device reported non-finite or inconsistent state            */
};

typedef struct sdd_ctx sdd_ctx;
typedef struct sdd_scene sdd_scene;

enum { SDD_MAT_OPAQUE = 0, SDD_MAT_GLASS = 1 };

/* Material kind. Opaque: Fresnel-split Lambertian, reflectance F(theta) from n + ik (section 3,
 * eq. 1) plus a diffuse lobe (1 - F) rho / pi, where rho stands for the wall "absorption factor"
 * of section 3. Glass: a thin slab of the given thickness on a zero-thickness quad, with
 * incoherent multiple reflection and Beer-Lambert absorption alpha = 4 pi k / lambda (the
 * spectral absorption of window glass, section 3). */
typedef struct {
  int32_t type;        /* SDD_MAT_OPAQUE or SDD_MAT_GLASS */
  float thickness_m;   /* glass slab thickness in metres (ignored for opaque) */
} sdd_material;

/* Scene description: the paper's three actors are objects, lighting and observer (section 1);
 * this struct carries the first two, the observer is an sdd_camera per render.
 * All pointers are HOST memory, read during sdd_scene_create only. */
typedef struct {
  const float* verts;          /* [n_tri][3][3] triangle vertices (FP32)                      */
  const uint16_t* mat;         /* [n_tri] material id of each triangle, < n_mat               */
  int64_t n_tri;               /* >= 1                                                         */
  const sdd_material* materials; /* [n_mat]                                                    */
  int32_t n_mat;               /* 1 .. 65535                                                   */
  const float* n_tab;          /* [n_mat][n_bins] real index n(lambda_j) > 0 (eq. 1)           */
  const float* k_tab;          /* [n_mat][n_bins] extinction k(lambda_j) >= 0 (eq. 1)          */
  const float* rho_tab;        /* [n_mat][n_bins] diffuse albedo in [0,1] (opaque only)        */
  int32_t n_bins;              /* wavelength bins B, 1 .. 128; centres lmin + (j+1/2)(lmax-lmin)/B */
  float lambda_min_nm, lambda_max_nm; /* 0 < lmin < lmax                                       */
  float sun_dir[3];            /* direction TOWARD the sun (plane wave, section 3); normalised */
  const float* sun_irradiance; /* [n_bins] E_j of the directional source (eq. 3), >= 0        */
  const float* env_radiance;   /* [n_bins] radiance of rays that leave the scene, or NULL (0)  */
  int32_t grid[3];             /* cell grid (the paper's sub-domains, section 5), 1 .. 64 each */
} sdd_scene_desc;

/* Statistics of a built scene. */
typedef struct {
  int64_t n_tri, n_refs, n_nodes, n_cells, n_empty_cells;
  int32_t max_depth, max_leaf;
  size_t device_bytes;
  float grid_lo[3], grid_hi[3];
} sdd_scene_info;

/* Build the spatially decomposed scene on the host: the padded scene box is split into
 * grid[0] x grid[1] x grid[2] cells (the sub-models of section 5); each triangle is referenced
 * by every cell its surface overlaps (no geometry is moved between cells at render time), and
 * each cell gets its own BVH. Needs no GPU. Errors: SDD_ERR_INVALID_ARG for a null pointer,
 * non-finite vertex, material id >= n_mat, n <= 0, k < 0, rho outside [0,1], zero sun
 * direction, grid or bin counts out of range. */
int sdd_scene_create(const sdd_scene_desc* desc, sdd_scene** out);
void sdd_scene_destroy(sdd_scene* scene);
int sdd_scene_get_info(const sdd_scene* scene, sdd_scene_info* out);
/* Bytes of device memory the scene needs (one buffer, 256-byte aligned). */
int sdd_scene_device_bytes(const sdd_scene* scene, size_t* bytes);
/* Read-only view of the serialised device image kept on the host (for inspection/tests). */
int sdd_scene_host_image(const sdd_scene* scene, const void** data, size_t* bytes);

/* Context on one HIP device; hip_stream is a hipStream_t (NULL = the null stream). */
int sdd_create(sdd_ctx** out, int hip_device, void* hip_stream);
void sdd_destroy(sdd_ctx* ctx);
int sdd_set_stream(sdd_ctx* ctx, void* hip_stream);

/* Copy the scene image into caller device memory dev_buf (>= sdd_scene_device_bytes) on the
 * context stream and bind the scene to it; dev_buf must stay valid while the scene is used. */
int sdd_scene_upload(sdd_ctx* ctx, sdd_scene* scene, void* dev_buf, size_t bytes);

/* Pinhole observer (section 1: the observer is the camera position and properties). Pixel
 * (x, y) has y = 0 at the top; its sample s is jittered inside the pixel. */
typedef struct {
  float eye[3], target[3], up[3];
  float vfov_deg;              /* vertical field of view, (0, 180) */
  int32_t width, height;       /* >= 1 */
} sdd_camera;

enum { SDD_MODE_PLAIN = 0, SDD_MODE_CACHED = 1 };

typedef struct {
  int32_t spp;                 /* samples per pixel, >= 1 (per-view counts in sdd_render_batch) */
  int32_t max_depth;           /* surface vertices per path D, 1 .. 64                          */
  uint64_t seed;               /* Philox key                                                   */
  int32_t mode;                /* SDD_MODE_PLAIN or SDD_MODE_CACHED                            */
  int32_t wave_paths;          /* paths in flight per wavefront, >= 64 (0 = library default)   */
  int32_t queue_rounds;        /* traversal rounds per wavefront phase (0 = library default 2):
                                  in each round but the last a ray is traversed in one cell and
                                  then migrates to the queue of the next cell along it; in the
                                  last round rays walk their remaining cells in place         */
  uint32_t view;               /* view index used in the RNG counter (sdd_render only)         */
  int32_t timing;              /* 1: time the traversal launches with HIP events (stats)       */
  int32_t first_sample;        /* samples [first_sample, first_sample + spp) of each pixel are
                                  drawn; renders of consecutive sample ranges average exactly
                                  to one longer render (progressive / resumable rendering)    */
  int32_t use_graph;           /* 1: the call's whole launch sequence is captured into a HIP
                                  graph the first time and replayed (one graph launch) while
                                  the same call (scene, views, images, workspace, parameters)
                                  repeats; timing then covers the whole graph               */
} sdd_render_params;

/* Workspace bytes for rendering with these parameters (paths in flight, bins, cells). */
int sdd_workspace_bytes(const sdd_scene* scene, const sdd_render_params* params, size_t* bytes);

/* Render the spectral image of one view: image_dev is device memory [n_bins][height][width]
 * FP32, overwritten with the mean over spp path samples of the spectral radiance. Each sample
 * is a path of up to max_depth surface vertices; at every opaque vertex the direct term of the
 * directional sun (eq. 3) is added through a shadow ray that is stopped by opaque triangles and
 * attenuated by every glass slab it crosses. Rays migrate between cells through device queues
 * (the interface conditions of section 5). */
int sdd_render(sdd_ctx* ctx, const sdd_scene* scene, const sdd_camera* camera, const sdd_render_params* params,
               void* workspace, size_t workspace_bytes, float* image_dev);

/* Render n_views views with uneven resolution and spp in one sequence of wavefronts: the
 * (view, pixel, sample) items of all views are drained by the same launches. images_dev[v]
 * is [n_bins][H_v][W_v]. View v uses RNG view index v. */
int sdd_render_batch(sdd_ctx* ctx, const sdd_scene* scene, const sdd_camera* views, const int32_t* spp_per_view,
                     int32_t n_views, const sdd_render_params* params, void* workspace, size_t workspace_bytes,
                     float* const* images_dev);

/* Workspace bytes for ray queries (sdd_trace / sdd_shadow) of n rays. */
int sdd_query_workspace_bytes(const sdd_scene* scene, int64_t n, size_t* bytes);

/* Closest hit of arbitrary rays through the cell decomposition: device arrays orig/dir
 * [n][3] FP32, skip [n] int32 (triangle id to ignore, -1 none; may be NULL). Outputs (device):
 * t [n] (+inf on miss), id [n] (-1 on miss), u, v [n] with hit point (1-u-v) v0 + u v1 + v v2.
 * The closest hit is the minimum t > 0 over all triangles, equal t -> smaller id. */
int sdd_trace(sdd_ctx* ctx, const sdd_scene* scene, const float* orig, const float* dir, const int32_t* skip,
              int64_t n, void* workspace, size_t workspace_bytes, float* t_out, int32_t* id_out, float* u_out,
              float* v_out);

/* Sun visibility of arbitrary rays: vis_out [n][n_bins] (device) = 0 if an opaque triangle is
 * hit at t > 0, else the product over the glass triangles crossed of their slab transmittance
 * at the crossing angle. */
int sdd_shadow(sdd_ctx* ctx, const sdd_scene* scene, const float* orig, const float* dir, const int32_t* skip,
               int64_t n, void* workspace, size_t workspace_bytes, float* vis_out);

/* Philox4x32-10 outputs for counters (c0 + i, c1, c2, c3), i < n, key (k0, k1): out [n][4]
 * uint32 (device). The generator that drives every random decision of the renderer. */
int sdd_philox(sdd_ctx* ctx, const uint32_t ctr[4], const uint32_t key[2], int64_t n, uint32_t* out_dev);

/* Search space of the autotuner. */
typedef struct {
  int32_t n_waves;             /* wavefront sizes (paths in flight) to try, 1..8            */
  int32_t wave_paths[8];
  int32_t n_grids;             /* cell grids to try, 1..8                                   */
  int32_t grids[8][3];
  int32_t n_rounds;            /* queue_rounds values to try, 1..4                          */
  int32_t queue_rounds[4];
  int32_t calib_spp;           /* samples per pixel of every view in calibration renders    */
  int32_t reps;                /* timed repetitions per candidate (the fastest is kept)     */
} sdd_tune_space;

typedef struct {
  int32_t grid[3];
  int32_t wave_paths;
  int32_t queue_rounds;
  int32_t pad;
  double samples_per_s;
} sdd_tune_point;

typedef struct {
  sdd_tune_point best;         /* fastest candidate                                          */
  int32_t from_cache;          /* 1: taken from the cache file, nothing was measured          */
  int32_t n_tried;             /* candidates measured (skipped ones do not count)            */
  sdd_tune_point tried[128];
} sdd_tune_result;

/* Autotuner: picks the cell grid, wavefront size and queue rounds with the highest throughput
 * on short calibration renders of the given views (calib_spp samples each), timed with HIP
 * events. The scene is rebuilt on the host for every grid and uploaded to scene_buf; grids whose
 * scene does not fit scene_bytes, and wavefront sizes whose workspace does not fit ws_bytes, are
 * skipped. images are the views' output images (overwritten). The result is appended to the
 * JSON-lines file cache_path (may be NULL) under a key made of the scene arrays, bins, depth,
 * views and device name; a later call with the same key returns the cached choice without
 * rendering. */
int sdd_autotune(sdd_ctx* ctx, const sdd_scene_desc* desc, const sdd_camera* views, int32_t n_views,
                 const sdd_render_params* base, const sdd_tune_space* space, void* scene_buf, size_t scene_bytes,
                 void* workspace, size_t ws_bytes, float* const* images, const char* cache_path,
                 sdd_tune_result* out);

/* Wait for the context stream, then report device-side errors (capacity overflow, non-finite
 * values) of the work enqueued since the previous sdd_finish. */
int sdd_finish(sdd_ctx* ctx);

typedef struct {
  uint64_t paths, vertices, ext_rays, shadow_rays, cell_visits, migrations, escapes, glass_crossings;
  uint64_t trace_launches, shade_launches, wavefronts;
  uint64_t err_cross_overflow, err_nonfinite, err_stack;
  uint64_t node_visits, tri_tests; /* BVH nodes visited and triangle tests of the traversal     */
  double trace_ms;             /* HIP-event time of the traversal launches (timing = 1)      */
  double shade_ms;             /* HIP-event time of the shading launches (timing = 1)        */
  uint64_t graph_launches;     /* graph-mode renders replayed                                 */
  double graph_ms;             /* HIP-event time of the graph launches (timing = 1)          */
} sdd_stats;

/* Counters accumulated since the previous sdd_reset_stats (valid after sdd_finish). */
int sdd_get_stats(sdd_ctx* ctx, sdd_stats* out);
int sdd_reset_stats(sdd_ctx* ctx);

/* Message of the last failure on ctx (or of the calling thread when ctx is NULL). */
const char* sdd_last_error(const sdd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPECDD_H */
