// C ABI of the learned radiance cache: configuration, device buffer layout, parameter
// transfer, evaluation and training on explicit records.
#include <cmath>
#include <cstring>
#include <string>

#include "host.h"

using namespace sdd;

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

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

enum {
  C_P, C_M, C_V, C_G, C_GPOS, C_GDIR, C_WF, C_WB, C_W4B, C_OPT, C_LOSS, C_RX, C_RW, C_TGT, C_RIDX, C_HST, C_DST, C_DE,
  C_COUNT
};

struct Layout {
  CacheDev d;               // offsets and sizes (pointers unset)
  size_t off[C_COUNT];
  size_t total;
};

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

// Level resolutions N_l = floor(N_min b^l), b = exp((ln N_max - ln N_min) / (L - 1)).
void levels(double nmin, double nmax, int L, int32_t* N) {
  const double b = L > 1 ? std::exp((std::log(nmax) - std::log(nmin)) / (L - 1)) : 1.0;
  for (int l = 0; l < L; ++l) N[l] = (int32_t)std::floor(nmin * std::pow(b, l));
}

std::string layout(const sdd_cache_config* c, Layout* out) {
  if (!c) return "config is null";
  if (c->levels_pos < 1 || c->levels_pos > kCacheMaxLevels) return "levels_pos must lie in 1..16";
  if (c->levels_dir < 1 || c->levels_dir > kCacheMaxLevels) return "levels_dir must lie in 1..16";
  if (2 * (c->levels_pos + c->levels_dir) + kCacheMatDim + kCacheBlob > kCacheWidth)
    return "2 (levels_pos + levels_dir) + 16 must not exceed 64";
  if (c->log2_table_pos < 4 || c->log2_table_pos > 24) return "log2_table_pos must lie in 4..24";
  if (c->log2_table_dir < 2 || c->log2_table_dir > 24) return "log2_table_dir must lie in 2..24";
  if (!(c->nmin_pos >= 1.0f && c->nmax_pos >= c->nmin_pos && c->nmax_pos <= 1048576.0f))
    return "position resolutions must satisfy 1 <= nmin <= nmax <= 2^20";
  if (!(c->nmin_dir >= 1.0f && c->nmax_dir >= c->nmin_dir && c->nmax_dir <= 1048576.0f))
    return "direction resolutions must satisfy 1 <= nmin <= nmax <= 2^20";
  if (c->n_mat < 1 || c->n_mat > 65535) return "n_mat must lie in 1..65535";
  if (c->max_bins < 1 || c->max_bins > kMaxBins) return "max_bins must lie in 1..128";
  if (c->max_records < kCacheVerts || c->max_records > (1 << 24)) return "max_records must lie in 32..2^24";
  if (c->max_step < kCacheVerts || c->max_step > c->max_records) return "max_step must lie in 32..max_records";
  if (!finite_pos(c->lr) || !finite_pos(c->eps)) return "lr and eps must be positive";
  if (!(c->beta1 >= 0.0f && c->beta1 < 1.0f && c->beta2 >= 0.0f && c->beta2 < 1.0f)) return "betas must lie in [0, 1)";
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(c->box_lo[a]) || !std::isfinite(c->box_hi[a]) || !(c->box_hi[a] > c->box_lo[a]))
      return "box_hi must exceed box_lo on every axis";
  Layout L;
  std::memset(&L, 0, sizeof(L));
  CacheDev& d = L.d;
  d.Lp = c->levels_pos;
  d.Ld = c->levels_dir;
  d.Tp_log2 = c->log2_table_pos;
  d.Td_log2 = c->log2_table_dir;
  d.n_mat = c->n_mat;
  d.n_in = 2 * (d.Lp + d.Ld) + kCacheMatDim + kCacheBlob;
  levels(c->nmin_pos, c->nmax_pos, d.Lp, d.Npos);
  levels(c->nmin_dir, c->nmax_dir, d.Ld, d.Ndir);
  const int64_t Tp = 1ll << d.Tp_log2, Td = 1ll << d.Td_log2;
  for (int l = 0; l < d.Lp; ++l) {
    const int64_t s = (int64_t)d.Npos[l] + 1;
    if (s * s * s <= Tp) d.dense_pos |= 1u << l;
  }
  for (int l = 0; l < d.Ld; ++l) {
    const int64_t s = (int64_t)d.Ndir[l] + 1;
    if (s * s <= Td) d.dense_dir |= 1u << l;
  }
  int64_t o = 0;
  d.o_pos = o;
  o += (int64_t)d.Lp * Tp * kCacheFeat;
  d.o_dir = o;
  o += (int64_t)d.Ld * Td * kCacheFeat;
  d.o_mat = o;
  o += (int64_t)d.n_mat * kCacheMatDim;
  d.o_w[0] = o;
  o += (int64_t)kCacheWidth * d.n_in;
  for (int l = 1; l < 4; ++l) {
    d.o_w[l] = o;
    o += (int64_t)kCacheWidth * kCacheWidth;
  }
  d.o_w4 = o;
  o += kCacheWidth;
  d.n_param = o;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = c->box_lo[a];
    d.ext[a] = (float)((double)c->box_hi[a] - (double)c->box_lo[a]);
  }
  d.max_bins = c->max_bins;
  d.max_train = c->max_records;
  d.max_step = c->max_step;
  const size_t n_tiles = (size_t)((c->max_step + kCacheVerts - 1) / kCacheVerts) * c->max_bins;
  size_t sz[C_COUNT];
  sz[C_P] = sz[C_M] = sz[C_V] = sz[C_G] = 4ull * d.n_param;
  sz[C_GPOS] = 4ull * d.Lp * Tp;
  sz[C_GDIR] = 4ull * d.Ld * Td;
  sz[C_WF] = sz[C_WB] = 16ull * 4 * 2 * 4 * 64;
  sz[C_W4B] = 16ull * 8;
  sz[C_OPT] = 16;
  sz[C_LOSS] = 8;
  sz[C_RX] = sz[C_RW] = 16ull * c->max_records;
  sz[C_TGT] = 4ull * c->max_records * c->max_bins;
  sz[C_RIDX] = 4ull * (c->max_records + 1);
  sz[C_HST] = sz[C_DST] = 2ull * 4 * n_tiles * kCacheWidth * 32;
  sz[C_DE] = 4ull * c->max_step * kCacheWidth;
  size_t off = 0;
  for (int i = 0; i < C_COUNT; ++i) {
    L.off[i] = off;
    off = a256(off + sz[i]);
  }
  L.total = off;
  *out = L;
  return "";
}

void bind(sdd_cache* k, const Layout& L, void* buf) {
  uint8_t* b = (uint8_t*)buf;
  k->dev = L.d;
  CacheDev& d = k->dev;
  d.P = (float*)(b + L.off[C_P]);
  d.M = (float*)(b + L.off[C_M]);
  d.V = (float*)(b + L.off[C_V]);
  d.G = (float*)(b + L.off[C_G]);
  d.gpos = (uint32_t*)(b + L.off[C_GPOS]);
  d.gdir = (uint32_t*)(b + L.off[C_GDIR]);
  d.wf = (uint4*)(b + L.off[C_WF]);
  d.wb = (uint4*)(b + L.off[C_WB]);
  d.w4b = (uint4*)(b + L.off[C_W4B]);
  k->opt = (float*)(b + L.off[C_OPT]);
  d.loss = (float*)(b + L.off[C_LOSS]);
  d.rx = (float4*)(b + L.off[C_RX]);
  d.rw = (float4*)(b + L.off[C_RW]);
  d.tgt = (float*)(b + L.off[C_TGT]);
  d.ridx = (uint32_t*)(b + L.off[C_RIDX]);
  d.hst = (uint16_t*)(b + L.off[C_HST]);
  d.dst = (uint16_t*)(b + L.off[C_DST]);
  d.dE = (float*)(b + L.off[C_DE]);
}

int ready(sdd_ctx* c, sdd_cache* k) {
  if (!c) return fail(nullptr, SDD_ERR_INVALID_ARG, "ctx is null");
  if (!k) return fail(c, SDD_ERR_INVALID_ARG, "cache is null");
  if (k->device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "cache was created on another device");
  if (!k->ready) return fail(c, SDD_ERR_NOT_READY, "cache parameters are not set (sdd_cache_init / set_params)");
  HIP_TRY(c, hipSetDevice(c->device));
  return SDD_OK;
}

// Adam state (moments, step count, gradients, loss) cleared, bf16 copies and packed operands rebuilt.
int reset_state(sdd_ctx* c, sdd_cache* k) {
  const CacheDev& d = k->dev;
  HIP_TRY(c, launch_fill_f32(c->stream, d.M, (size_t)d.n_param, 0.0f));
  HIP_TRY(c, launch_fill_f32(c->stream, d.V, (size_t)d.n_param, 0.0f));
  HIP_TRY(c, launch_fill_f32(c->stream, d.G, (size_t)d.n_param, 0.0f));
  HIP_TRY(c, launch_fill_u32(c->stream, (uint32_t*)k->opt, 4, 0u));
  HIP_TRY(c, launch_fill_f32(c->stream, d.loss, 2, 0.0f));
  HIP_TRY(c, launch_cache_sync(c->stream, d));
  return SDD_OK;
}

int check_records(sdd_ctx* c, sdd_cache* k, const float* x, const float* wo, const int32_t* mat, int64_t n,
                  int32_t n_bins, int64_t cap) {
  if (!x || !wo || !mat) return fail(c, SDD_ERR_INVALID_ARG, "null record array");
  if (n < 1 || n > cap) return fail(c, SDD_ERR_INVALID_ARG, "record count out of range (1.." + std::to_string(cap) + ")");
  if (n_bins < 1 || n_bins > k->cfg.max_bins) return fail(c, SDD_ERR_INVALID_ARG, "n_bins must lie in 1..max_bins");
  return SDD_OK;
}

}  // namespace

namespace sdd {

// One training batch on the records already in the cache (ridx / count set): `steps` Adam steps
// over consecutive groups of step_records records.
int cache_train_records(sdd_ctx* c, sdd_cache* k, int B, int steps, int step_records) {
  const CacheDev& d = k->dev;
  for (int s = 0; s < steps; ++s) {
    const uint32_t v0 = (uint32_t)s * (uint32_t)step_records;
    HIP_TRY(c, launch_cache_backward(c->stream, d, B, v0, (uint32_t)step_records));
    HIP_TRY(c, launch_cache_adam(c->stream, d, v0, (uint32_t)step_records, k->opt, k->cfg.lr, k->cfg.beta1,
                                 k->cfg.beta2, k->cfg.eps));
  }
  return SDD_OK;
}

}  // namespace sdd

extern "C" {

int sdd_cache_param_count(const sdd_cache_config* cfg, int64_t* n) {
  if (!n) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  Layout L;
  std::string e = layout(cfg, &L);
  if (!e.empty()) return fail(nullptr, SDD_ERR_INVALID_ARG, e);
  *n = L.d.n_param;
  return SDD_OK;
}

int sdd_cache_bytes(const sdd_cache_config* cfg, size_t* bytes) {
  if (!bytes) return fail(nullptr, SDD_ERR_INVALID_ARG, "null argument");
  Layout L;
  std::string e = layout(cfg, &L);
  if (!e.empty()) return fail(nullptr, SDD_ERR_INVALID_ARG, e);
  *bytes = L.total;
  return SDD_OK;
}

int sdd_cache_create(sdd_ctx* c, const sdd_cache_config* cfg, void* buf, size_t bytes, sdd_cache** out) {
  if (!c || !out) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  Layout L;
  std::string e = layout(cfg, &L);
  if (!e.empty()) return fail(c, SDD_ERR_INVALID_ARG, e);
  if (!buf) return fail(c, SDD_ERR_INVALID_ARG, "cache buffer is null");
  if (((uintptr_t)buf & 255) != 0) return fail(c, SDD_ERR_INVALID_ARG, "cache buffer must be 256-byte aligned");
  if (bytes < L.total)
    return fail(c, SDD_ERR_WORKSPACE,
                "cache buffer too small: need " + std::to_string(L.total) + " bytes, got " + std::to_string(bytes));
  sdd_cache* k = new sdd_cache();
  k->cfg = *cfg;
  k->buf = buf;
  k->bytes = bytes;
  k->device = c->device;
  bind(k, L, buf);
  *out = k;
  return SDD_OK;
}

void sdd_cache_destroy(sdd_cache* k) { delete k; }

int sdd_cache_get_info(sdd_ctx* c, sdd_cache* k, sdd_cache_info* out) {
  if (!c || !k || !out) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  std::memset(out, 0, sizeof(*out));
  const CacheDev& d = k->dev;
  out->n_param = d.n_param;
  Layout L;
  (void)layout(&k->cfg, &L);
  out->device_bytes = L.total;
  out->n_in = d.n_in;
  for (int l = 0; l < d.Lp; ++l) out->npos[l] = d.Npos[l];
  for (int l = 0; l < d.Ld; ++l) out->ndir[l] = d.Ndir[l];
  out->dense_pos = d.dense_pos;
  out->dense_dir = d.dense_dir;
  out->train_paths_done = (int64_t)k->train_paths_done;
  if (k->ready) {
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float opt[4];
    HIP_TRY(c, hipMemcpy(opt, k->opt, sizeof(opt), hipMemcpyDeviceToHost));
    uint32_t t;
    std::memcpy(&t, &opt[0], 4);
    out->adam_steps = t;
  }
  return SDD_OK;
}

int sdd_cache_init(sdd_ctx* c, sdd_cache* k, uint64_t seed) {
  if (!c || !k) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  if (k->device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "cache was created on another device");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_cache_init(c->stream, k->dev, seed));
  k->ready = true;
  return reset_state(c, k);
}

int sdd_cache_set_params(sdd_ctx* c, sdd_cache* k, const float* host, int64_t n) {
  if (!c || !k || !host) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  if (k->device != c->device) return fail(c, SDD_ERR_INVALID_ARG, "cache was created on another device");
  if (n != k->dev.n_param) return fail(c, SDD_ERR_INVALID_ARG, "parameter count mismatch");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return fail(c, SDD_ERR_INVALID_ARG, "parameters must be finite");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(k->dev.P, host, 4ull * n, hipMemcpyHostToDevice, c->stream));
  k->ready = true;
  return reset_state(c, k);
}

static int copy_out(sdd_ctx* c, sdd_cache* k, const float* src, float* host, int64_t n) {
  int rc = ready(c, k);
  if (rc) return rc;
  if (!host || n != k->dev.n_param) return fail(c, SDD_ERR_INVALID_ARG, "bad output (size must equal n_param)");
  HIP_TRY(c, hipMemcpyAsync(host, src, 4ull * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SDD_OK;
}

int sdd_cache_get_params(sdd_ctx* c, sdd_cache* k, float* host, int64_t n) {
  if (!k) return fail(c, SDD_ERR_INVALID_ARG, "cache is null");
  return copy_out(c, k, k->dev.P, host, n);
}

int sdd_cache_get_grads(sdd_ctx* c, sdd_cache* k, float* host, int64_t n) {
  if (!k) return fail(c, SDD_ERR_INVALID_ARG, "cache is null");
  return copy_out(c, k, k->dev.G, host, n);
}

int sdd_cache_eval(sdd_ctx* c, sdd_cache* k, const float* x, const float* wo, const int32_t* mat, int64_t n,
                   int32_t n_bins, float* out) {
  int rc = ready(c, k);
  if (rc) return rc;
  if (!out) return fail(c, SDD_ERR_INVALID_ARG, "output is null");
  rc = check_records(c, k, x, wo, mat, n, n_bins, (int64_t)1 << 30);
  if (rc) return rc;
  HIP_TRY(c, launch_cache_eval(c->stream, k->dev, x, wo, mat, (uint32_t)n, n_bins, out));
  return SDD_OK;
}

int sdd_cache_backward(sdd_ctx* c, sdd_cache* k, const float* x, const float* wo, const int32_t* mat,
                       const float* target, int64_t n, int32_t n_bins) {
  int rc = ready(c, k);
  if (rc) return rc;
  if (!target) return fail(c, SDD_ERR_INVALID_ARG, "target is null");
  rc = check_records(c, k, x, wo, mat, n, n_bins, k->cfg.max_step);
  if (rc) return rc;
  const CacheDev& d = k->dev;
  HIP_TRY(c, launch_fill_f32(c->stream, d.G, (size_t)d.n_param, 0.0f));
  HIP_TRY(c, launch_cache_load_records(c->stream, d, x, wo, mat, target, (uint32_t)n, n_bins));
  HIP_TRY(c, launch_cache_backward(c->stream, d, n_bins, 0u, (uint32_t)k->cfg.max_step));
  return SDD_OK;
}

int sdd_cache_step(sdd_ctx* c, sdd_cache* k) {
  int rc = ready(c, k);
  if (rc) return rc;
  HIP_TRY(c, launch_cache_adam(c->stream, k->dev, 0u, (uint32_t)k->cfg.max_step, k->opt, k->cfg.lr, k->cfg.beta1,
                               k->cfg.beta2, k->cfg.eps));
  return SDD_OK;
}

int sdd_cache_train(sdd_ctx* c, sdd_cache* k, const float* x, const float* wo, const int32_t* mat,
                    const float* target, int64_t n, int32_t n_bins) {
  int rc = ready(c, k);
  if (rc) return rc;
  if (!target) return fail(c, SDD_ERR_INVALID_ARG, "target is null");
  rc = check_records(c, k, x, wo, mat, n, n_bins, k->cfg.max_records);
  if (rc) return rc;
  HIP_TRY(c, launch_cache_load_records(c->stream, k->dev, x, wo, mat, target, (uint32_t)n, n_bins));
  const int steps = (int)((n + k->cfg.max_step - 1) / k->cfg.max_step);
  return cache_train_records(c, k, n_bins, steps, k->cfg.max_step);
}

int sdd_cache_loss(sdd_ctx* c, sdd_cache* k, double* mean_loss) {
  int rc = ready(c, k);
  if (rc) return rc;
  if (!mean_loss) return fail(c, SDD_ERR_INVALID_ARG, "null argument");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  float h[2];
  HIP_TRY(c, hipMemcpy(h, k->dev.loss, sizeof(h), hipMemcpyDeviceToHost));
  *mean_loss = h[1] > 0.0f ? (double)h[0] / (double)h[1] : std::nan("");
  HIP_TRY(c, launch_fill_f32(c->stream, k->dev.loss, 2, 0.0f));
  return SDD_OK;
}

int sdd_cache_get_records(sdd_ctx* c, sdd_cache* k, int64_t n, float* rec_x, float* rec_w, float* target) {
  int rc = ready(c, k);
  if (rc) return rc;
  if (n < 1 || n > k->cfg.max_records || !rec_x || !rec_w || !target)
    return fail(c, SDD_ERR_INVALID_ARG, "bad record request");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(rec_x, k->dev.rx, 16ull * n, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(rec_w, k->dev.rw, 16ull * n, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(target, k->dev.tgt, 4ull * n * k->cfg.max_bins, hipMemcpyDeviceToHost));
  return SDD_OK;
}

}  // extern "C"
