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

/* A spectral transmittance map of glass (section 3: the spectral transmittance measured at points
 * of the medieval samples, read through texture coordinates): width x height texels, each the
 * slab's internal transmittance at normal incidence tau0_j in [0, 1] for every bin, HOST array
 * [height][width][n_bins]. At a hit with texture coordinates (s, t) the map is interpolated
 * bilinearly between texel centres ((i + 1/2) / width, (k + 1/2) / height) and repeats with
 * period 1 in s and t; the slab then transmits tau0^(1 / cos theta_t) per pass instead of
 * exp(-4 pi k d / (lambda cos theta_t)) (Beer-Lambert), its faces still reflecting by the
 * Fresnel factor of n + ik. */
typedef struct {
  int32_t width, height;       /* >= 1, width * height <= 2^24                                 */
  const float* tau0;           /* [height][width][n_bins]                                       */
} sdd_texture;

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
  /* optional spectral transmittance maps of glass (n_tex = 0: none, the pointers are ignored) */
  const float* uv;             /* [n_tri][3][2] texture coordinates of each triangle's vertices */
  int32_t n_tex;               /* 0 .. 65535                                                    */
  const sdd_texture* textures; /* [n_tex]                                                       */
  const int32_t* mat_texture;  /* [n_mat] map of each material, -1 none; glass materials only   */
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

/* Change the lighting of a built scene without rebuilding its cells: the directional sun (a plane
 * wave, section 3; its direct term is eq. 3) as the direction TOWARD the sun (normalised here,
 * non-zero and finite) and the irradiance E_j of every bin (host array [n_bins], finite >= 0);
 * or the radiance of rays that leave the scene (host array [n_bins], finite >= 0, or NULL for
 * zero). The scene's host image is updated and, if it was uploaded, its device copy too, on the
 * context stream; the call waits for the copy. Renders enqueued before the call use the old
 * values. Errors: SDD_ERR_INVALID_ARG (null pointer, bad values, scene uploaded on another
 * device), SDD_ERR_HIP. */
int sdd_set_sun(sdd_ctx* ctx, sdd_scene* scene, const float dir_to_sun[3], const float* irradiance);
int sdd_set_env(sdd_ctx* ctx, sdd_scene* scene, const float* radiance);

/* The sun of a date and clock time at a site (section 3: the sun is a plane wave whose spectrum
 * at the ground changes with the hour, through the incidence angle in the atmosphere, and with
 * the date, through the Earth-Sun distance; Rayleigh scattering theory gives the spectrum).
 * Solar declination, equation of time and (r0/r)^2 from Spencer's (1971) series in the day angle
 * 2 pi (d - 1) / 365; the position from the latitude and the hour angle of true solar time;
 * air mass m from Kasten and Young (1989); Rayleigh optical depth of the standard atmosphere
 * tau(l) = 0.008569 l^-4 (1 + 0.0113 l^-2 + 0.00013 l^-4) (l in um, Hansen and Travis 1974)
 * times pressure_ratio; E_j = B(l_j, T) / B(555 nm, T) (r0/r)^2 exp(-tau(l_j) m) at the bin
 * centres while the sun is above the horizon, else 0. */
typedef struct {
  int32_t day_of_year;         /* 1 .. 366                                                     */
  float clock_hours;           /* local clock time, [0, 24]                                    */
  float utc_offset_hours;      /* zone of the clock, [-14, 14] (e.g. 2 for CEST)               */
  float latitude_deg;          /* site, [-90, 90], north positive                              */
  float longitude_deg;         /* site, [-180, 180], east positive                             */
  float scene_x_azimuth_deg;   /* compass azimuth (clockwise from north) of the scene's +x
                                  axis; +z is up and +y = z x x (90: x east, y north)          */
  float temperature_k;         /* blackbody temperature of the sun, 1e3 .. 1e5 (5778)          */
  float pressure_ratio;        /* surface pressure over 1013.25 hPa, [0, 10]                   */
} sdd_daylight;

typedef struct {
  float elevation_deg, azimuth_deg; /* sun above the horizon / compass azimuth                 */
  float air_mass;                   /* relative optical air mass (+inf below the horizon)      */
  float distance_factor;            /* (r0 / r)^2                                              */
} sdd_daylight_info;

/* Host computation (needs no GPU): direction toward the sun in the scene frame (unit) and the
 * irradiance [n_bins] at the bin centres of [lambda_min, lambda_max]; info may be NULL.
 * Errors: SDD_ERR_INVALID_ARG for parameters out of range or null outputs. */
int sdd_daylight_sun(const sdd_daylight* params, int32_t n_bins, float lambda_min_nm, float lambda_max_nm,
                     float dir_to_sun[3], float* irradiance, sdd_daylight_info* info);
/* sdd_daylight_sun for the scene's bins, then sdd_set_sun with the result. */
int sdd_set_daylight(sdd_ctx* ctx, sdd_scene* scene, const sdd_daylight* params, sdd_daylight_info* info);

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
  int32_t queue_rounds;        /* traversal rounds per wavefront phase (0 = library default 1):
                                  every new ray is queued at the cell holding its origin; in
                                  each round but the last a ray is traversed in one cell and
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
  int32_t cell_order;          /* order in which the traversal takes the cells' queued rays
                                  (section 5: the sub-model with the most waiting rays is taken
                                  next): 0 cell index order, 1 fullest cells first (by the octave
                                  of their queued rays, cell index inside an octave; grids of
                                  more than 4096 cells keep index order). Results do not depend
                                  on it.                                                     */
  int32_t persistent;          /* 1: the whole render (every view of a batch) is ONE persistent
                                  kernel: its lanes take (view, 8 x 8 tile, sample) items from a
                                  device work list, each lane carrying one path through all its
                                  vertices (same random numbers and arithmetic, so the same
                                  image up to the order of the float additions into a pixel),
                                  then its next item; wave_paths is then the number of lanes
                                  (rounded up to a multiple of 2048, at most 2^19; 0 = as many
                                  as the device holds at once);
                                  queue_rounds and cell_order are unused. Plain mode only (not
                                  with photon maps, a cache or sdd_render_noalloc).           */
} sdd_render_params;

/* Workspace bytes for rendering with these parameters (paths in flight, bins, cells). The ray
 * queues order the rays of a (cell, direction class) by direction sub-bin and by the block of the
 * cell they start in, up to 8 x 8 x 8 blocks for grids of at most 170 cells; a render given less
 * than this size uses fewer blocks (the most that fit, down to none: about 3.5 KB per cell),
 * which changes the traversal's speed but not the image. */
int sdd_workspace_bytes(const sdd_scene* scene, const sdd_render_params* params, size_t* bytes);

/* Render the spectral image of one view: image_dev is device memory [n_bins][height][width]
 * FP32, overwritten with the mean over spp path samples of the spectral radiance. Each sample
 * is a path of up to max_depth surface vertices; at every opaque vertex the direct term of the
 * directional sun (eq. 3) is added through a shadow ray that is stopped by opaque triangles and
 * attenuated by every glass slab it crosses. Rays migrate between cells through device queues
 * (the interface conditions of section 5). */
int sdd_render(sdd_ctx* ctx, const sdd_scene* scene, const sdd_camera* camera, const sdd_render_params* params,
               void* workspace, size_t workspace_bytes, float* image_dev);

/* sdd_render for callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): the same render, with the workspace taken
 * from a static device array of the library (64 MiB, one per device, held until the process
 * ends) instead of a caller buffer; the library allocates nothing. wave_paths = 0 picks the most
 * paths in flight (up to 2^20) whose workspace fits, the queues' origin blocks (see
 * sdd_workspace_bytes) taking what is left; a wave_paths whose workspace does not fit (about
 * 0.7 KB per path at 40 bins, plus 3.5 KB per cell) is rejected with SDD_ERR_WORKSPACE.
 * Plain mode only; use_graph and timing must be 0 (SDD_ERR_INVALID_ARG). Every call on a device
 * shares that device's array: calls that overlap on one device (other streams or contexts) race,
 * and each context must call sdd_finish before another context's render uses the array. */
int sdd_render_noalloc(sdd_ctx* ctx, const sdd_scene* scene, const sdd_camera* camera,
                       const sdd_render_params* params, float* image_dev);

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
  int32_t n_orders;            /* cell_order values to try, 0..2 (0: the base parameters')  */
  int32_t cell_orders[2];
  int32_t try_persistent;      /* 1: also time the one persistent kernel on every grid       */
} sdd_tune_space;

typedef struct {
  int32_t grid[3];
  int32_t wave_paths;          /* paths in flight; lanes of the kernel when persistent        */
  int32_t queue_rounds;
  int32_t cell_order;
  int32_t persistent;          /* 1: the candidate is the persistent kernel                  */
  int32_t pad;
  double samples_per_s;
} sdd_tune_point;

typedef struct {
  sdd_tune_point best;         /* fastest candidate                                          */
  int32_t from_cache;          /* 1: taken from the cache file, nothing was measured          */
  int32_t n_tried;             /* candidates measured (skipped ones do not count)            */
  sdd_tune_point tried[128];
} sdd_tune_result;

/* Autotuner: picks the cell grid, wavefront size, queue rounds and cell order (or the persistent
 * kernel, when asked to try it) with the highest throughput
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

/* ------------------------------------------------------------------------------------------
 * Learned spectral radiance cache
 *
 * The paper computes the indirect part of global illumination from photon maps (section 4). In
 * the cached mode of this library that role is taken by a small network trained online on the
 * renderer's own paths: a camera path stops at its third surface vertex x (after two bounces)
 * and adds beta_j L(x, w, lambda_j, material) for every bin j, where L is the network's
 * estimate of the radiance leaving x toward the previous vertex. The plain full-depth path is
 * the fallback and the reference.
 *
 * Network: input 64 = [multiresolution hash grid of the position (L_p levels x 2 features, 3D,
 * Mueller et al. 2022) | hash grid of the octahedral map of w (L_d levels x 2, 2D) | material
 * embedding (8) | one-blob encoding of t = (lambda - lambda_min) / (lambda_max - lambda_min)
 * (8 Gaussians of width 1/8) | zero padding], four 64-wide ReLU layers without biases, one
 * output. Level l has resolution N_l = floor(N_min b^l), b = exp((ln N_max - ln N_min)/(L - 1));
 * its vertices are indexed densely when (N_l + 1)^dim <= T, else by
 * (x * 1 xor y * 2654435761 xor z * 805459861) mod T (32-bit unsigned). Matrix products run in
 * bf16 with FP32 accumulation (grids, layer inputs and weights rounded to bf16 to nearest even);
 * FP32 masters are trained with Adam (Kingma & Ba 2015, bias-corrected) on the relative L2 loss
 * mean((y - t)^2 / (y^2 + 0.01)) with the denominator held constant.
 *
 * Flat parameter layout (FP32, the unit of sdd_cache_get/set_params and of the gradients):
 *   pos grid [L_p][T_p][2] | dir grid [L_d][T_d][2] | material [n_mat][8] |
 *   W0 [64][n_in] | W1 [64][64] | W2 [64][64] | W3 [64][64] | w4 [64],
 *   n_in = 2 (L_p + L_d) + 16; W[out][in] acts as h_out = relu(W h_in).
 * ------------------------------------------------------------------------------------------ */
typedef struct sdd_cache sdd_cache;

typedef struct {
  int32_t levels_pos;          /* L_p, 1..16                                                  */
  int32_t log2_table_pos;      /* T_p = 2^t entries per position level, 4..24                 */
  float nmin_pos, nmax_pos;    /* coarsest / finest position resolution, 1 <= nmin <= nmax <= 2^20 */
  int32_t levels_dir;          /* L_d, 1..16, with 2 (L_p + L_d) + 16 <= 64                    */
  int32_t log2_table_dir;      /* T_d, 2..24                                                  */
  float nmin_dir, nmax_dir;
  int32_t n_mat;               /* materials with an embedding row, 1..65535 (>= scene n_mat)  */
  int32_t max_bins;            /* most wavelength bins of a query or a training record, 1..128 */
  int32_t max_records;         /* training records held at once (training paths per batch)   */
  int32_t max_step;            /* records per Adam step, 32 .. max_records                    */
  float lr, beta1, beta2, eps; /* Adam: lr > 0, 0 <= beta < 1, eps > 0                         */
  float box_lo[3], box_hi[3];  /* the position grid spans this box (hi > lo on every axis)    */
} sdd_cache_config;

typedef struct {
  int64_t n_param;             /* FP32 parameters in the flat layout                          */
  size_t device_bytes;         /* bytes of the cache's device buffer                          */
  int32_t n_in;                /* network inputs before padding to 64                         */
  int32_t npos[16], ndir[16];  /* level resolutions N_l                                       */
  uint32_t dense_pos, dense_dir; /* bit l set: level l is indexed densely                     */
  int64_t adam_steps;          /* Adam steps taken since init / set_params                   */
  int64_t train_paths_done;    /* training paths traced by sdd_render_cached so far           */
} sdd_cache_info;

/* Size of the flat parameter vector and of the device buffer of a configuration. */
int sdd_cache_param_count(const sdd_cache_config* cfg, int64_t* n);
int sdd_cache_bytes(const sdd_cache_config* cfg, size_t* bytes);

/* Bind a cache to caller device memory dev_buf (>= sdd_cache_bytes, 256-byte aligned); it
 * must stay valid while the cache is used. The parameters are undefined until sdd_cache_init
 * or sdd_cache_set_params. Errors: SDD_ERR_INVALID_ARG for a configuration out of range,
 * SDD_ERR_WORKSPACE for a small buffer. */
int sdd_cache_create(sdd_ctx* ctx, const sdd_cache_config* cfg, void* dev_buf, size_t bytes, sdd_cache** out);
void sdd_cache_destroy(sdd_cache* cache);
int sdd_cache_get_info(sdd_ctx* ctx, sdd_cache* cache, sdd_cache_info* out);   /* waits */

/* Random initialisation from Philox (grids U(-1e-4, 1e-4), material embedding U(-1, 1),
 * weights Glorot-uniform); clears the Adam state. */
int sdd_cache_init(sdd_ctx* ctx, sdd_cache* cache, uint64_t seed);
/* Copy FP32 parameters (flat layout, n = sdd_cache_param_count) from HOST memory; clears the
 * Adam state. get_params / get_grads copy to HOST memory and wait for the stream. */
int sdd_cache_set_params(sdd_ctx* ctx, sdd_cache* cache, const float* host, int64_t n);
int sdd_cache_get_params(sdd_ctx* ctx, sdd_cache* cache, float* host, int64_t n);
int sdd_cache_get_grads(sdd_ctx* ctx, sdd_cache* cache, float* host, int64_t n);

/* Network output y (before the clamp at zero that the render applies) for n explicit vertices:
 * device arrays x [n][3] (position), wo [n][3] (unit direction toward the previous vertex),
 * mat [n] int32 (< n_mat); out [n][n_bins] FP32, bin j at wavelength parameter
 * t_j = (j + 1/2) / n_bins. n_bins <= max_bins. */
int sdd_cache_eval(sdd_ctx* ctx, sdd_cache* cache, const float* x, const float* wo, const int32_t* mat, int64_t n,
                   int32_t n_bins, float* out);

/* Gradients of the mean relative L2 loss over the n x n_bins rows of explicit records
 * (device arrays as in sdd_cache_eval, target [n][n_bins]), n <= max_step: the gradient buffer
 * is cleared first; read it with sdd_cache_get_grads. sdd_cache_step then applies one Adam step
 * with it (and clears it). */
int sdd_cache_backward(sdd_ctx* ctx, sdd_cache* cache, const float* x, const float* wo, const int32_t* mat,
                       const float* target, int64_t n, int32_t n_bins);
int sdd_cache_step(sdd_ctx* ctx, sdd_cache* cache);
/* Train on n <= max_records explicit records: ceil(n / max_step) Adam steps, step s on records
 * [s max_step, (s + 1) max_step). */
int sdd_cache_train(sdd_ctx* ctx, sdd_cache* cache, const float* x, const float* wo, const int32_t* mat,
                    const float* target, int64_t n, int32_t n_bins);
/* Mean loss over the rows of the backward passes since the previous call (waits; NaN if none). */
int sdd_cache_loss(sdd_ctx* ctx, sdd_cache* cache, double* mean_loss);

/* Online training inside sdd_render_cached. Once per call (every = 0: before the first
 * wavefront) or before wavefronts 0, every, 2 every, ..., train_paths training paths are traced at
 * full depth: path g (counted across calls by the cache) starts
 * at a pixel of the view drawn from Philox counter (g, g >> 32, 2 << 24, view), draws its
 * decisions with purpose 1 (bit 24 of the counter's depth word), restarts its throughput at one
 * at its third vertex and records that vertex; the radiance it then gathers is the record's
 * target for every bin. The records (in path order, at most steps x step_records) feed `steps`
 * Adam steps of step_records records each. train_paths = 0 leaves the cache unchanged. */
typedef struct {
  int32_t train_paths;         /* 0 .. min(max_records, wave_paths)                            */
  int32_t step_records;        /* 32 .. max_step                                               */
  int32_t steps;               /* >= 1                                                         */
  int32_t every;               /* 0: one batch per call; k >= 1: before every k-th wavefront    */
} sdd_train_params;

/* Render in cached mode (params->mode = SDD_MODE_CACHED, max_depth >= 3, use_graph = 0):
 * vertices 1 and 2 of every path are shaded as in sdd_render (the direct sun term included);
 * the continuation from vertex 2 that hits vertex 3 adds beta_j max(y_j, 0) from the cache for
 * every bin and stops; escapes add the environment as before. The scene's bins must not exceed
 * max_bins and its materials n_mat; the position box is the cache's. train may be NULL. */
int sdd_render_cached(sdd_ctx* ctx, const sdd_scene* scene, sdd_cache* cache, const sdd_camera* camera,
                      const sdd_render_params* params, const sdd_train_params* train, void* workspace,
                      size_t workspace_bytes, float* image_dev);

/* Training records of the last batch, slot by slot (HOST outputs, waits): rec_x [n][4] =
 * (position, material id as uint32 bits), rec_w [n][4] = (direction toward the previous vertex,
 * 1 if the slot's path reached its third vertex else 0), target [n][max_bins]. */
int sdd_cache_get_records(sdd_ctx* ctx, sdd_cache* cache, int64_t n, float* rec_x, float* rec_w, float* target);

/* Caustic photon map (section 4: photon maps are filled with the points where photons sent out
 * from the light sources hit the scene, one map serving the caustics; the radiance a surface
 * sends back is split into separate integrals, the caustic one taken from that map).
 * The source is the directional sun of the scene (section 3). Emission: the windows are the
 * scene's glass triangles, with projected areas a_w = |n_w . s| area_w on the unit sun direction
 * s as stored by the scene (FP32); A = sum_w a_w. Photon i (0 <= i < n_photons) draws x from
 * Philox counter (i, i >> 32, 4 << 24, 0) under key (seed, seed >> 32): window w is the last
 * whose threshold floor(2^24 (a_0 + ... + a_{w-1}) / A) does not exceed x.x >> 8; its point on
 * the window has barycentrics (sqrt(u1)(1 - u2), sqrt(u1) u2) with u1, u2 the 24-bit uniforms
 * of x.y, x.z; its flux is E_j A / n_photons, times the slab transmittance of every other glass
 * triangle between the point and the sun (an opaque one stops it). Vertex 1 is that window
 * point, reached along -s. At vertex k a photon draws u0 from counter (i, i >> 32, k | 4 << 24,
 * 0): glass reflects with probability mean R / (mean R + mean T), else transmits straight on
 * (as camera paths do); an opaque vertex first stores the photon when one of its earlier
 * vertices reflected it (glass face or mirror lobe; light only transmitted is direct light),
 * then takes the mirror lobe with probability mean F / (mean F + mean (1 - F) rho) or ends
 * (a diffuse bounce leaves the caustic paths). Vertex max_depth scatters nothing. A stored
 * record holds the vertex position, the photon's direction of arrival, its flux per bin on
 * arrival, the photon index and the vertex number. */
typedef struct sdd_photon_map sdd_photon_map;

/* Kinds of photon map. A global map (section 4: a map for the global illumination) stores every
 * photon at every opaque vertex it reaches, including the first (direct sunlight through the
 * windows), and continues it at an opaque vertex by the mirror lobe (as above) or else by the
 * cosine-weighted diffuse lobe, direction from the vertex's second and third uniforms as for camera
 * paths, weight (1 - F(cos of the new direction)) rho / (1 - P_s): the Fresnel factor of the
 * diffuse lobe is that of the direction the light leaves in (for camera paths the direction
 * toward the viewer), so a photon, which carries light forward, takes it at its new direction. */
enum { SDD_PHOTON_CAUSTIC = 0, SDD_PHOTON_GLOBAL = 1 };

typedef struct {
  int64_t n_photons;           /* photons sent out, >= 1; n_photons (max_depth - 1) < 2^32     */
  int32_t max_depth;           /* vertices of a photon path, 2 .. 64                           */
  float radius;                /* gather radius r > 0 (scene units), also the map's grid cell   */
  uint64_t seed;               /* Philox key of the photon paths                               */
  int64_t capacity;            /* records the map holds, 1 .. 2^28 (further ones are counted as
                                  dropped)                                                     */
  int32_t wave_paths;          /* photons in flight per wavefront, 64 .. 2^26 (0 = 2^20)       */
  int32_t queue_rounds;        /* traversal rounds per phase as in sdd_render_params (0 = 1)   */
  int32_t kind;                /* SDD_PHOTON_CAUSTIC or SDD_PHOTON_GLOBAL                      */
  int32_t pad;
} sdd_photon_params;

typedef struct {
  int64_t stored;              /* records held (<= capacity)                                   */
  int64_t dropped;             /* records that did not fit                                     */
  int32_t n_windows;           /* glass triangles of non-zero projected area                   */
  int32_t n_buckets;           /* hash-grid buckets                                            */
  double window_area;          /* A, the windows' total projected area                         */
  size_t device_bytes;         /* bytes of the map's device buffer                             */
} sdd_photon_info;

/* Device bytes of a map with these parameters for this scene (its bins and glass triangles). */
int sdd_photon_map_bytes(const sdd_scene* scene, const sdd_photon_params* params, size_t* bytes);
/* Workspace bytes of sdd_photon_map_build (photons in flight, bins, cells). */
int sdd_photon_workspace_bytes(const sdd_scene* scene, const sdd_photon_params* params, size_t* bytes);
/* Bind a map to caller device memory dev_buf (>= sdd_photon_map_bytes, 256-byte aligned), valid
 * while the map is used; the map holds nothing until sdd_photon_map_build. Errors:
 * SDD_ERR_INVALID_ARG (parameters out of range), SDD_ERR_WORKSPACE (small buffer). */
int sdd_photon_map_create(sdd_ctx* ctx, const sdd_scene* scene, const sdd_photon_params* params, void* dev_buf,
                          size_t bytes, sdd_photon_map** out);
void sdd_photon_map_destroy(sdd_photon_map* map);
/* Trace the photons of the map's parameters through the scene (same cell queues and traversal
 * as camera paths) on the context stream, store the records, then sort them into the hashed
 * grid the gathering reads. The scene's bins must match the map's; its sun (direction and
 * spectrum) is read now. Errors: SDD_ERR_NOT_READY (scene not uploaded), SDD_ERR_WORKSPACE;
 * sdd_finish reports SDD_ERR_QUEUE_OVERFLOW when a photon's way to the sun crossed more than 8
 * glass slabs. A scene without glass facing the sun gives an empty map. */
int sdd_photon_map_build(sdd_ctx* ctx, const sdd_scene* scene, sdd_photon_map* map, void* workspace,
                         size_t workspace_bytes);
/* Counts of the last build (waits for the stream). */
int sdd_photon_map_info(sdd_ctx* ctx, sdd_photon_map* map, sdd_photon_info* out);
/* The first n records (n <= stored; any order) to HOST arrays (waits): pos [n][3], dir [n][3]
 * (direction of arrival), flux [n][n_bins], id [n] (photon index), vertex [n]. */
int sdd_photon_map_records(sdd_ctx* ctx, sdd_photon_map* map, int64_t n, float* pos, float* dir, float* flux,
                           int64_t* id, int32_t* vertex);
/* Replace the map's records with n <= capacity records from HOST arrays laid out as
 * sdd_photon_map_records returns them (id and vertex may be NULL: stored as 0) and sort them into
 * the grid (waits for the copy): a map saved from an earlier build or computed elsewhere is then
 * gathered as if built here. */
int sdd_photon_map_load(sdd_ctx* ctx, sdd_photon_map* map, int64_t n, const float* pos, const float* dir,
                        const float* flux, const int64_t* id, const int32_t* vertex);
/* sdd_render (plain mode) with photon maps (section 4), either may be NULL but not both. The
 * density estimate of a map at an opaque vertex adds beta_j (1 - F_j) rho_j / pi times the summed
 * flux of the records within distance r whose direction of arrival d has d . n < 0 (n: the normal
 * on the side the path sees), divided by pi r^2, before the vertex's lobe.
 *  - caustic (SDD_PHOTON_CAUSTIC): estimated at every opaque vertex the path shades before
 *    vertex global_from (at all of them without a global map), besides the direct term;
 *  - global (SDD_PHOTON_GLOBAL), from vertex global_from >= 1 on: the estimate is the vertex's
 *    whole diffuse light (no direct term, no caustic map there) and the path goes on only by the
 *    mirror lobe (with probability P_s, weight F / P_s), else ends.
 * use_graph is allowed (the graph reads the maps' current contents). Errors: SDD_ERR_NOT_READY for
 * a map not built or of other bins, SDD_ERR_INVALID_ARG for a map of the wrong kind, no map, or
 * global_from < 1 with a global map. */
int sdd_render_photons(sdd_ctx* ctx, const sdd_scene* scene, const sdd_photon_map* caustic,
                       const sdd_photon_map* global, int32_t global_from, const sdd_camera* camera,
                       const sdd_render_params* params, void* workspace, size_t workspace_bytes, float* image_dev);

/* Colorimetry of a spectral image (section 6 maps the spectral renderings to RGB by colorimetry;
 * section 1: the observer's visual adaptation is a colorimetric matter). image_dev is device
 * memory [n_bins][n_pixels] FP32 (an image [n_bins][H][W] has n_pixels = H W) sampled at the bin
 * centres lambda_min + (j + 1/2)(lambda_max - lambda_min) / n_bins (nm). The CIE 1931 2-degree
 * colour-matching functions come from the multi-lobe analytic fit of Wyman, Sloan and Shirley
 * (JCGT 2013). Outputs (device, either may be NULL but not both):
 *   xyz_dev [3][n_pixels]:  XYZ = exposure sum_j I_j cmf(l_j) / sum_j ybar(l_j)
 *                           (a flat spectrum of radiance 1 gives Y = exposure);
 *   srgb_dev [n_pixels][3]: sRGB (IEC 61966-2-1, D65 white) of XYZ, clamped to [0, 1] and
 *                           encoded with the sRGB transfer function.
 * Enqueued on the context stream. Errors: SDD_ERR_INVALID_ARG (null image or no output,
 * n_bins outside 1..128, 0 < lambda_min < lambda_max violated, n_pixels < 1, exposure not finite
 * >= 0), SDD_ERR_HIP. */
int sdd_spectral_to_srgb(sdd_ctx* ctx, const float* image_dev, int32_t n_bins, float lambda_min_nm,
                         float lambda_max_nm, int64_t n_pixels, float exposure, float* xyz_dev, float* srgb_dev);

/* Wait for the context stream, then report device-side errors of the work enqueued since the
 * previous sdd_finish: SDD_ERR_QUEUE_OVERFLOW when a shadow ray reached the sun through more
 * glass slabs than the kMaxCross = 8 it records (its visibility then misses the extra slabs),
 * else SDD_ERR_DEVICE when non-finite radiance reached an image (it is stored as computed; huge
 * finite inputs can overflow). The counts are in sdd_stats (err_cross_overflow, err_nonfinite).
 * The flags are cleared by the call. */
int sdd_finish(sdd_ctx* ctx);

typedef struct {
  /* glass_crossings: glass slabs crossed by shadow rays (also by rays an opaque triangle blocks
   * later); err_cross_overflow: shadow rays that reached the sun through more slabs than the
   * kMaxCross = 8 recorded ones (sdd_finish reports SDD_ERR_QUEUE_OVERFLOW then) */
  uint64_t paths, vertices, ext_rays, shadow_rays, cell_visits, migrations, escapes, glass_crossings;
  uint64_t trace_launches, shade_launches, wavefronts;
  uint64_t err_cross_overflow, err_nonfinite, err_stack;
  uint64_t node_visits, tri_tests; /* BVH nodes visited and triangle tests of the traversal     */
  double trace_ms;             /* HIP-event time of the traversal launches (timing = 1)      */
  double shade_ms;             /* HIP-event time of the shading launches (timing = 1)        */
  uint64_t graph_launches;     /* graph-mode renders replayed                                 */
  double graph_ms;             /* HIP-event time of the graph launches (timing = 1)          */
  uint64_t cache_queries;      /* path vertices that took their radiance from the cache       */
  uint64_t query_launches;     /* cache-query launches (one per wavefront of a cached render)  */
  uint64_t train_batches;      /* training batches (training paths + Adam steps) run          */
  double query_ms;             /* HIP-event time of the cache-query launches (timing = 1)     */
  double train_ms;             /* HIP-event time of the training-batch finishing steps:
                                  target gathering, compaction and Adam steps (timing = 1)  */
  uint64_t photon_vertices;    /* opaque vertices that gathered from a photon map             */
  uint64_t photons_found;      /* photon records within the gather radius, summed over them   */
  uint64_t photon_lit_vertices; /* of those vertices, the ones that found at least one record  */
  uint64_t photon_candidates;  /* grid entries tested by them (the found ones included)       */
  uint64_t photon_candidates_max; /* most entries tested for one vertex                        */
  uint64_t photon_launches;    /* photon-gather launches                                       */
  double photon_ms;            /* HIP-event time of the photon-gather launches (timing = 1)   */
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
