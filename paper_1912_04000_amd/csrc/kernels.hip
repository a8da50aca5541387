// gfx950 kernels of the spectral path tracer.
//
// Wavefront structure (one "phase" traces every ray produced by the previous step):
//   producer (raygen / shade / pack)  -> (ray, queue sub-range, rank in it) entries; a
//              sub-range is a key (start cell, direction class) and the block of the cell that
//              holds the ray's origin
//   k_subscan  sub-range offsets inside their keys, key counts
//   k_scan     one workgroup: per-key offsets and the tile list, cells in index order or
//              fullest first
//   k_scatter  entries -> cell-sorted queue, a key's rays ordered by origin block
//   k_trace    a tile = up to 256 rays of ONE queue key (cell, direction class), handed out in
//              parts of 64, one ray per lane of a wave; the grid's slab planes, the cell table
//              and each lane's short traversal stack live in LDS, the 4-wide BVH nodes and
//              triangles are read from memory (L2). A lane traverses its ray inside the cell's
//              slab interval; rays that leave the cell are re-queued for the next cell (the
//              interface conditions between the paper's sub-domains, section 5) or, in the
//              final round, walk on in place.
//   shade      per-bin spectral shading: complex Fresnel (eq. 1), thin-slab Beer-Lambert glass,
//              next-event estimation toward the directional sun (eq. 3).
// k_persist renders a whole batch in one persistent kernel instead (the same per-path
// arithmetic, one path per lane at a time, no queues).
#include "device_common.h"

namespace sdd {

// Wave-level append of (src, key) entries: one atomic per wave on the list counter and one per
// distinct destination queue key of the wave. The lanes are first grouped by key (ballot +
// mbcnt, no memory traffic), then the group leaders add their group sizes to the per-key
// counters in one atomic instruction, so a wave waits for one atomic round trip however many
// keys it holds. Every lane of the wave must call it.
__device__ void wave_append(bool valid, uint32_t src, uint32_t cell, uint32_t* list_count, uint32_t* cell_count,
                            const DevWS& w, uint32_t* lsrc, uint32_t* ldst, uint32_t* lrank) {
  const uint64_t m = __ballot(valid);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(list_count, (uint32_t)__popcll(m));
  uint32_t my_leader = 0, my_off = 0, gcount = 0;
  bool is_leader = false;
  uint64_t pending = m;
  while (pending) {
    const uint32_t l = (uint32_t)__ffsll((unsigned long long)pending) - 1u;
    const uint32_t c = __builtin_amdgcn_readlane(cell, (int)l);  // l is wave-uniform
    const bool mine = valid && cell == c;
    const uint64_t same = __ballot(mine);
    if (mine) {
      my_leader = l;
      my_off = count_below(same);
    }
    if (lane_id() == l) {
      is_leader = true;
      gcount = (uint32_t)__popcll(same);
    }
    pending &= ~same;
  }
  uint32_t cb = 0;
  if (is_leader) cb = atomicAdd(&cell_count[ctr_word(w, cell)], gcount);
  cb = __shfl(cb, (int)my_leader);
  base = __builtin_amdgcn_readlane(base, (int)leader);
  if (valid) {
    const uint32_t pos = base + count_below(m);
    lsrc[pos] = src;
    ldst[pos] = cell;
    lrank[pos] = cb + my_off;
  }
}

// Rank of each valid lane's entry inside its destination queue sub-range. The lanes of the first
// kRankGroups distinct keys (in lane order) are grouped, one atomic per group, the rest take one
// atomic each: camera and shadow rays share few keys per wave and a group saves them atomics on
// one address, which are served one at a time, while extension rays, spread over many
// sub-ranges, would cost a grouping pass per lane and save nothing. Every lane of the wave must
// call it.
constexpr int kRankGroups = 8;
__device__ uint32_t wave_key_rank(bool valid, uint32_t key, uint32_t* cell_count, const DevWS& w) {
  const uint64_t m = __ballot(valid);
  if (m == 0) return 0;
  // a lane in no group leads its own group of one
  uint32_t my_leader = lane_id(), my_off = 0, gcount = 1;
  bool is_leader = valid;
  uint64_t pending = m;
  for (int g = 0; g < kRankGroups && pending; ++g) {
    const uint32_t l = (uint32_t)__ffsll((unsigned long long)pending) - 1u;
    const uint32_t c = __builtin_amdgcn_readlane(key, (int)l);  // l is wave-uniform
    const bool mine = valid && key == c;
    const uint64_t same = __ballot(mine);
    if (mine) {
      my_leader = l;
      my_off = count_below(same);
      is_leader = lane_id() == l;
      gcount = (uint32_t)__popcll(same);
    }
    pending &= ~same;
  }
  uint32_t cb = 0;
  if (is_leader) cb = atomicAdd(&cell_count[ctr_word(w, key)], gcount);
  cb = __shfl(cb, (int)my_leader);
  return cb + my_off;
}

// Group leaders and in-group offsets of wave_key_rank, without the atomic.
struct KeyGroups {
  uint32_t my_leader, my_off, gcount;
  bool is_leader;
};
__device__ __forceinline__ KeyGroups wave_key_groups(bool valid, uint32_t key) {
  const uint64_t m = __ballot(valid);
  KeyGroups g{lane_id(), 0u, 1u, valid};
  uint64_t pending = m;
  for (int i = 0; i < kRankGroups && pending; ++i) {
    const uint32_t l = (uint32_t)__ffsll((unsigned long long)pending) - 1u;
    const uint32_t c = __builtin_amdgcn_readlane(key, (int)l);  // l is wave-uniform
    const bool mine = valid && key == c;
    const uint64_t same = __ballot(mine);
    if (mine) {
      g.my_leader = l;
      g.my_off = count_below(same);
      g.is_leader = lane_id() == l;
      g.gcount = (uint32_t)__popcll(same);
    }
    pending &= ~same;
  }
  return g;
}

// wave_key_rank of two entries per lane (a vertex's extension and shadow rays): both atomics are
// issued before either result is waited for. Every lane of the wave must call it.
__device__ __forceinline__ void wave_key_rank2(bool v0, uint32_t k0, bool v1, uint32_t k1, uint32_t* cell_count,
                                               const DevWS& w, uint32_t& r0, uint32_t& r1) {
  const KeyGroups g0 = wave_key_groups(v0, k0), g1 = wave_key_groups(v1, k1);
  uint32_t c0 = 0, c1 = 0;
  if (g0.is_leader) c0 = atomicAdd(&cell_count[ctr_word(w, k0)], g0.gcount);
  if (g1.is_leader) c1 = atomicAdd(&cell_count[ctr_word(w, k1)], g1.gcount);
  r0 = __shfl(c0, (int)g0.my_leader) + g0.my_off;
  r1 = __shfl(c1, (int)g1.my_leader) + g1.my_off;
}

// Workgroup-level append of up to two (src, key) entries per lane (all threads of the
// workgroup call it; s_scr holds kWG / 64 words of LDS): the positions in the produced-entry
// list come from one list-counter atomic per workgroup and a prefix over its waves, the ranks
// inside the destination queues from wave_key_rank. Meant for one-shot kernels: inside a loop
// its two barriers cost more than the per-wave list atomics of wave_append they save.
__device__ void block_append2(uint32_t* s_scr, bool v0, uint32_t src0, uint32_t key0, bool v1, uint32_t src1,
                              uint32_t key1, uint32_t* list_count, uint32_t* cell_count, const DevWS& w,
                              uint32_t* lsrc, uint32_t* ldst, uint32_t* lrank) {
  constexpr int kWaves = kWG / 64;
  const uint32_t wv = threadIdx.x >> 6;
  const uint64_t m0 = __ballot(v0), m1 = __ballot(v1);
  const uint32_t c0 = (uint32_t)__popcll(m0);
  if (lane_id() == 0) s_scr[wv] = c0 + (uint32_t)__popcll(m1);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int q = 0; q < kWaves; ++q) tot += s_scr[q];
    uint32_t base = tot ? atomicAdd(list_count, tot) : 0u;
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t x = s_scr[q];
      s_scr[q] = base;
      base += x;
    }
  }
  __syncthreads();
  // each wave reads only its own word, which no thread rewrites before the next call's barrier
  const uint32_t wbase = s_scr[wv];
  const uint32_t r0 = wave_key_rank(v0, key0, cell_count, w);
  const uint32_t r1 = wave_key_rank(v1, key1, cell_count, w);
  if (v0) {
    const uint32_t pos = wbase + count_below(m0);
    lsrc[pos] = src0;
    ldst[pos] = key0;
    lrank[pos] = r0;
  }
  if (v1) {
    const uint32_t pos = wbase + c0 + count_below(m1);
    lsrc[pos] = src1;
    ldst[pos] = key1;
    lrank[pos] = r1;
  }
}

// ==========================================================================================
// cell grid
// ==========================================================================================

__device__ __forceinline__ int locate_axis(const float* pl, int g, float lo, float inv_cs, float p) {
  int i = (int)floorf((p - lo) * inv_cs);
  i = min(max(i, 0), g - 1);
  while (i > 0 && p < pl[i]) --i;
  while (i < g - 1 && p >= pl[i + 1]) ++i;
  return i;
}

// Start cell of a ray: the cell holding its origin, or the cell where it enters the grid box.
// Returns kInvalidCell if the ray misses the grid box entirely. `pl` is the plane table
// (gx+1 | gy+1 | gz+1 entries, in global memory or a copy in LDS). With `blk` given, it receives
// the block of the cell's 2^L x 2^L x 2^L split (L = kMaxSubLevels) that holds the origin or
// entry point, as a Morton index (bit 3l + a: axis a at level l from the finest), which orders
// the rays inside their queue key.
__device__ uint32_t start_cell_pl(const DevScene& S, const float* pl, F3 o, F3 d, uint32_t* blk = nullptr) {
  const float* px = pl;
  const float* py = pl + S.gx + 1;
  const float* pz = pl + S.gx + 1 + S.gy + 1;
  const float lo[3] = {px[0], py[0], pz[0]};
  const float hi[3] = {px[S.gx], py[S.gy], pz[S.gz]};
  const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (oo[a] < lo[a] || oo[a] >= hi[a]) inside = false;
  F3 p = o;
  if (!inside) {
    // entry point into the grid box (slab test with IEEE reciprocals)
    float tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
      if (dd[a] == 0.0f) {
        if (oo[a] < lo[a] || oo[a] > hi[a]) return kInvalidCell;
        continue;
      }
      const float inv = 1.0f / dd[a];
      float t0 = (lo[a] - oo[a]) * inv, t1 = (hi[a] - oo[a]) * inv;
      tn = fmaxf(tn, fminf(t0, t1));
      tf = fminf(tf, fmaxf(t0, t1));
    }
    if (!(tn <= tf) || tf < 0.0f) return kInvalidCell;
    if (tn > 0.0f) p = o + d * tn;
  }
  const int ix = locate_axis(px, S.gx, lo[0], S.inv_cs[0], p.x);
  const int iy = locate_axis(py, S.gy, lo[1], S.inv_cs[1], p.y);
  const int iz = locate_axis(pz, S.gz, lo[2], S.inv_cs[2], p.z);
  if (blk) {
    constexpr float kSplit = (float)(1 << kMaxSubLevels);
    const float lo3[3] = {px[ix], py[iy], pz[iz]}, hi3[3] = {px[ix + 1], py[iy + 1], pz[iz + 1]};
    const float pp[3] = {p.x, p.y, p.z};
    uint32_t m = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float f = (pp[a] - lo3[a]) * kSplit / (hi3[a] - lo3[a]);
      const uint32_t q = (uint32_t)min(max((int)f, 0), (1 << kMaxSubLevels) - 1);
#pragma unroll
      for (int l = 0; l < kMaxSubLevels; ++l) m |= ((q >> l) & 1u) << (3 * l + a);
    }
    *blk = m;
  }
  return (uint32_t)((iz * S.gy + iy) * S.gx + ix);
}

__device__ uint32_t start_cell(const DevScene& S, F3 o, F3 d) { return start_cell_pl(S, S.planes, o, d); }

// Slab interval of a ray inside cell (ix, iy, iz) and the axis through which it leaves, over a
// plane table (gx+1 | gy+1 | gz+1 entries; the traversal keeps a copy in LDS). The shared
// plane of two neighbouring cells is one table entry evaluated with one expression, so the
// exit distance of a cell equals the entry distance of the next exactly. The reciprocal
// direction is finite (see make_pre), so no slab distance is NaN.
__device__ __forceinline__ void cell_interval_pl(const float* pl, int gx, int gy, int ix, int iy, int iz, F3 o, F3 inv,
                                                 float& tn, float& tf, int& axis) {
  const float* px = pl;
  const float* py = pl + gx + 1;
  const float* pz = pl + gx + 1 + gy + 1;
  const float ax = (px[ix] - o.x) * inv.x, bx = (px[ix + 1] - o.x) * inv.x;
  const float ay = (py[iy] - o.y) * inv.y, by = (py[iy + 1] - o.y) * inv.y;
  const float az = (pz[iz] - o.z) * inv.z, bz = (pz[iz + 1] - o.z) * inv.z;
  const float n0 = fminf(ax, bx), f0 = fmaxf(ax, bx);
  const float n1 = fminf(ay, by), f1 = fmaxf(ay, by);
  const float n2 = fminf(az, bz), f2 = fmaxf(az, bz);
  tn = fmaxf(n0, fmaxf(n1, n2));
  axis = 0;
  tf = f0;
  if (f1 < tf) { tf = f1; axis = 1; }
  if (f2 < tf) { tf = f2; axis = 2; }
}

// ==========================================================================================
// spectral optics (hardware reciprocal / square root / exp2: about 1 ulp each, far inside the
// 1e-4 parity bar, against the multi-instruction IEEE expansions)
// ==========================================================================================
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// Unpolarised Fresnel reflectance of air -> n + ik at incidence cosine c:
//   eta^2 = (n + ik)^2, w = sqrt(eta^2 - sin^2) (principal branch),
//   r_s = (c - w)/(c + w), r_p = (eta^2 c - w)/(eta^2 c + w), F = (|r_s|^2 + |r_p|^2)/2.
__device__ __forceinline__ float fresnel(float n, float k, float c) {
  c = fminf(1.0f, fmaxf(0.0f, c));
  const float s2 = 1.0f - c * c;
  const float er = n * n - k * k, ei = 2.0f * n * k;
  const float zr = er - s2, zi = ei;
  const float r = fsqrt(zr * zr + zi * zi);
  float wr = 0.0f, wi = 0.0f;
  if (r > 0.0f) {
    if (zr >= 0.0f) {
      wr = fsqrt(0.5f * (r + zr));
      wi = 0.5f * zi * frcp(wr);
    } else {
      wi = copysignf(fsqrt(0.5f * (r - zr)), zi);
      wr = 0.5f * zi * frcp(wi);
    }
  }
  const float an = c - wr, ad = c + wr;
  const float Rs = (an * an + wi * wi) * frcp(ad * ad + wi * wi);
  const float pr = er * c, pi = ei * c;
  const float bnr = pr - wr, bni = pi - wi, bdr = pr + wr, bdi = pi + wi;
  const float Rp = (bnr * bnr + bni * bni) * frcp(bdr * bdr + bdi * bdi);
  return 0.5f * (Rs + Rp);
}

// Thin slab: incoherent multiple reflection, Beer-Lambert alpha = 4 pi k / lambda over the
// internal path d / cos(theta_t), refraction angle from the real index.
__device__ __forceinline__ void slab(float n, float k, float lambda_nm, float d_m, float c, float& R, float& T) {
  c = fminf(1.0f, fmaxf(0.0f, c));
  const float st = fsqrt(fmaxf(0.0f, 1.0f - c * c));
  const float si = st * frcp(n);
  const float ci = fsqrt(fmaxf(0.0f, 1.0f - si * si));
  const float alpha = 1.2566370614359172e10f * k * frcp(lambda_nm);  // 4 pi k / (lambda_nm 1e-9 m)
  const float tau = fexp(-alpha * d_m * frcp(ci));
  const float R1 = fresnel(n, k, c);
  const float inv_den = frcp(1.0f - R1 * R1 * tau * tau);
  const float q = (1.0f - R1) * (1.0f - R1);
  R = R1 + q * tau * tau * R1 * inv_den;
  T = q * tau * inv_den;
}

// The slab when its internal transmittance at normal incidence tau0 comes from a measured map
// (section 3): tau = tau0^(1 / cos(theta_t)) per pass, faces reflecting by F of n + ik.
__device__ __forceinline__ void slab_tau0(float n, float k, float tau0, float c, float& R, float& T) {
  c = fminf(1.0f, fmaxf(0.0f, c));
  const float st = fsqrt(fmaxf(0.0f, 1.0f - c * c));
  const float si = st * frcp(n);
  const float ci = fsqrt(fmaxf(0.0f, 1.0f - si * si));
  const float tau = tau0 > 0.0f ? __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(tau0) * frcp(ci)) : 0.0f;
  const float R1 = fresnel(n, k, c);
  const float inv_den = frcp(1.0f - R1 * R1 * tau * tau);
  const float q = (1.0f - R1) * (1.0f - R1);
  R = R1 + q * tau * tau * R1 * inv_den;
  T = q * tau * inv_den;
}

// Texture coordinates of a point with barycentrics (bu, bv) on triangle tri.
__device__ __forceinline__ void hit_st(const DevScene& S, uint32_t tri, float bu, float bv, float& s, float& t) {
  const float4 a = S.guv[2 * (size_t)tri], b = S.guv[2 * (size_t)tri + 1];
  const float w0 = 1.0f - bu - bv;
  s = w0 * a.x + bu * a.z + bv * b.x;
  t = w0 * a.y + bu * a.w + bv * b.y;
}

// Map lookup geometry: the four texels around (s, t) (bilinear between texel centres, periodic
// repeat) as float4-row indices of quad 0, and the two weights.
struct TexTap {
  const float4* base;
  uint32_t r00, r10, r01, r11;  // texel index * quads per texel
  float fx, fy;
};
__device__ __forceinline__ TexTap tex_tap(const DevScene& S, int tex, float s, float t) {
  const int4 ti = S.texinfo[tex];  // (texel offset in floats, width, height, 0)
  // one period: s - floor(s) is exact, so the map repeats without any integer overflow
  const float x = (s - floorf(s)) * (float)ti.y - 0.5f, y = (t - floorf(t)) * (float)ti.z - 0.5f;
  const float x0 = floorf(x), y0 = floorf(y);   // in [-1, size - 1]
  const int i0 = x0 < 0.0f ? ti.y - 1 : min((int)x0, ti.y - 1);
  const int k0 = y0 < 0.0f ? ti.z - 1 : min((int)y0, ti.z - 1);
  const int i1 = i0 + 1 == ti.y ? 0 : i0 + 1, k1 = k0 + 1 == ti.z ? 0 : k0 + 1;
  const uint32_t nq = (uint32_t)S.bins_pad / 4;
  TexTap T;
  T.base = (const float4*)(S.texel + ti.x);
  T.r00 = ((uint32_t)k0 * ti.y + i0) * nq;
  T.r10 = ((uint32_t)k0 * ti.y + i1) * nq;
  T.r01 = ((uint32_t)k1 * ti.y + i0) * nq;
  T.r11 = ((uint32_t)k1 * ti.y + i1) * nq;
  T.fx = x - x0;
  T.fy = y - y0;
  return T;
}
// tau0 of the four bins of quad q at the tap
__device__ __forceinline__ float4 tex_quad(const TexTap& T, int q) {
  const float4 a = T.base[T.r00 + q], b = T.base[T.r10 + q], c = T.base[T.r01 + q], d = T.base[T.r11 + q];
  const float w00 = (1.0f - T.fx) * (1.0f - T.fy), w10 = T.fx * (1.0f - T.fy), w01 = (1.0f - T.fx) * T.fy,
              w11 = T.fx * T.fy;
  return make_float4(w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x, w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y,
                     w00 * a.z + w10 * b.z + w01 * c.z + w11 * d.z, w00 * a.w + w10 * b.w + w01 * c.w + w11 * d.w);
}

// ==========================================================================================
// fills / philox test kernel
// ==========================================================================================
__global__ void k_fill_f32(float* p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_philox(uint4 base, uint32_t k0, uint32_t k1, uint64_t n, uint4* out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = philox(make_uint4(base.x + (uint32_t)i, base.y, base.z, base.w), k0, k1);
}

// ==========================================================================================
// ray generation
// ==========================================================================================
// Wave-level push of one value to a list (one atomic per wave); every lane must call it.
__device__ __forceinline__ void wave_push(bool pred, uint32_t val, uint32_t* count, uint32_t* list) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __builtin_amdgcn_readlane(base, (int)leader);
  if (pred) list[base + count_below(m)] = val;
}

__device__ __forceinline__ uint32_t* cat_list(const DevWS& w, int par, int cat) {
  return w.cat + ((size_t)par * kCats + cat) * w.W;
}

// Camera paths. Render items k0 + i map to (view, sample, pixel) in sample-major order. Training
// paths (kTrain) are items of view 0: path g = k0 + i starts at a pixel drawn from the counter
// (g, g >> 32, purpose 2, view) and uses g as its sample index under purpose 1, so that its
// random numbers never coincide with those of a rendered sample.
template <bool kTrain>
__global__ __launch_bounds__(kWG) void k_raygen(DevScene S, DevWS w, uint64_t k0, uint32_t n, uint32_t key0,
                                                uint32_t key1, int gen, PathMode pm) {
  __shared__ float s_planes[3 * (kMaxGrid + 1)];  // the grid's slab planes, for locating the rays
  for (int q = threadIdx.x; q < S.gx + S.gy + S.gz + 3; q += kWG) s_planes[q] = S.planes[q];
  __syncthreads();
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  const bool valid = i < n;
  uint32_t cell = kInvalidCell, qdir = 0, xo = 0;
  if (valid) {
    const uint64_t k = k0 + i;
    int v = 0;
    uint32_t s, pix;
    if (kTrain) {
      const ViewDesc& V0 = w.views[0];
      const uint64_t P = (uint64_t)V0.width * V0.height;
      const uint4 r0 = philox(make_uint4((uint32_t)k, (uint32_t)(k >> 32), 2u << 24, V0.view_id), key0, key1);
      pix = (uint32_t)(r0.x % P);
      s = (uint32_t)k;
      pm.rec_w[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else {
      while (v + 1 < w.n_views && w.views[v + 1].item_base <= k) ++v;
      const ViewDesc& V1 = w.views[v];
      const uint64_t local = k - V1.item_base;
      const uint64_t P = (uint64_t)V1.width * V1.height;
      if ((local >> 32) == 0 && (P >> 32) == 0) {  // 32-bit division where it suffices
        const uint32_t l32 = (uint32_t)local, p32 = (uint32_t)P;
        s = l32 / p32 + V1.first_sample;
        pix = l32 % p32;
      } else {
        s = (uint32_t)(local / P) + V1.first_sample;
        pix = (uint32_t)(local % P);
      }
    }
    const ViewDesc& V = w.views[v];
    const uint32_t px = pix % (uint32_t)V.width, py = pix / (uint32_t)V.width;
    const uint4 rn = philox(make_uint4(pix, s, pm.purpose, V.view_id), key0, key1);
    const float sx = 2.0f * ((float)px + unif24(rn.x)) / (float)V.width - 1.0f;
    const float sy = 1.0f - 2.0f * ((float)py + unif24(rn.y)) / (float)V.height;
    const F3 fw = f3(V.fwd[0], V.fwd[1], V.fwd[2]);
    const F3 rt = f3(V.right[0], V.right[1], V.right[2]);
    const F3 up = f3(V.upv[0], V.upv[1], V.upv[2]);
    const F3 d = norm3(fw + rt * sx + up * sy);
    const F3 o = f3(V.eye[0], V.eye[1], V.eye[2]);
    w.rays[2 * i] = make_float4(o.x, o.y, o.z, __int_as_float(-1));
    w.rays[2 * i + 1] = make_float4(d.x, d.y, d.z, __uint_as_float(i));
    w.pix[i] = pix;
    w.smp[i] = s;
    w.view[i] = (uint32_t)v;
    cell = start_cell_pl(S, s_planes, o, d, &xo);
    qdir = dir_code(d);
  }
  // Throughput rows at one and radiance rows at zero: the workgroup's paths own one contiguous
  // stretch of each row array, written by the whole workgroup in consecutive quads (per-path row
  // loops would address 64 rows, one cache line each, per store instruction).
  {
    const uint32_t i0 = blockIdx.x * kWG, np = min((uint32_t)kWG, n - min(n, i0));
    const uint32_t nq4 = np * (uint32_t)(w.Bp / 4);
    float4* b4 = (float4*)(w.beta + (size_t)i0 * w.Bp);
    float4* l4 = (float4*)(w.lacc + (size_t)i0 * w.Bp);
    for (uint32_t q = threadIdx.x; q < nq4; q += kWG) {
      b4[q] = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
      l4[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  // Path i's entry in the produced list is entry i (the list is empty before ray generation, its
  // only producer): no list-counter atomic, one per workgroup on one cache line. A path whose ray
  // misses the grid leaves an entry marked kNoKey, which the scatter passes over.
  const int p = gen & 1;
  const bool in_grid = valid && cell != kInvalidCell;
  const uint32_t key = in_grid ? qsub(w, cell, qdir, xo) : kNoKey;
  const uint32_t rank = wave_key_rank(in_grid, key, ccount_of(S, w, p), w);
  if (valid) {
    w.lsrc[i] = i | kFirstVisit;
    w.ldst[i] = key;
    w.lrank[i] = rank;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctl->list_count[p] = n;
  // camera rays that miss the grid box escape at once
  if (valid && cell == kInvalidCell && S.env_nonzero) w.catb[i] = (uint8_t)(kCatEscape + 1);
  // n paths, each with its camera ray: counted once, not with an atomic per workgroup on the
  // statistics' cache line
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd(&w.ctl->st_paths, (unsigned long long)n);
    atomicAdd(&w.ctl->st_ext, (unsigned long long)n);
  }
}

// User rays (closest-hit or shadow queries).
__global__ __launch_bounds__(kWG) void k_pack_rays(DevScene S, DevWS w, const float* orig, const float* dir,
                                                   const int32_t* skip, uint32_t n, int shadow, int gen) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  const bool valid = i < n;
  uint32_t cell = kInvalidCell, qdir = 0, xo = 0;
  uint32_t r = 0;
  if (valid) {
    const F3 o = f3(orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]);
    const F3 d = f3(dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]);
    const int sk = skip ? skip[i] : -1;
    r = shadow ? w.W + i : i;
    w.rays[2 * r] = make_float4(o.x, o.y, o.z, __int_as_float(sk));
    w.rays[2 * r + 1] = make_float4(d.x, d.y, d.z, __uint_as_float(shadow ? (i | kShadowBit) : i));
    const bool finite = isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(d.x) && isfinite(d.y) &&
                        isfinite(d.z) && (d.x != 0.0f || d.y != 0.0f || d.z != 0.0f);
    if (finite) cell = start_cell_pl(S, S.planes, o, d, &xo);
    qdir = dir_code(d);
    if (shadow)
      w.shcnt[i] = 0;
    else
      w.hit[i] = make_float4(INFINITY, __uint_as_float(0xFFFFFFFFu), 0.0f, 0.0f);
  }
  const int p = gen & 1;
  __shared__ uint32_t s_app[kWG / 64];
  block_append2(s_app, valid && cell != kInvalidCell, r | kFirstVisit, qsub(w, cell, qdir, xo), false, 0u, 0u,
                &w.ctl->list_count[p], ccount_of(S, w, p), w, w.lsrc, w.ldst, w.lrank);
}

// Hit records hold the FP32 distance and the triangle id; the distance and barycentrics handed
// out are re-evaluated here with the compensated FP32 plane intersection of refine_hit.
__global__ void k_unpack_hits(DevScene S, DevWS w, uint32_t n, float* t, int32_t* id, float* u, float* v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float4 h = w.hit[i];
    const uint32_t tid = __float_as_uint(h.y);
    float th = h.x, bu = 0.0f, bv = 0.0f;
    if (tid != 0xFFFFFFFFu) {
      const float4* g = S.gtris + (size_t)tid * 3;
      const float4 A = g[0], B = g[1], C = g[2], ro = w.rays[2 * i], rd = w.rays[2 * i + 1];
      bu = bv = 1.0f / 3.0f;
      F3 q;
      refine_hit(f3(ro.x, ro.y, ro.z), f3(rd.x, rd.y, rd.z), f3(A.x, A.y, A.z), f3(B.x, B.y, B.z), f3(C.x, C.y, C.z),
                 th, q, bu, bv);
    }
    t[i] = th;
    id[i] = (int32_t)tid;
    u[i] = bu;
    v[i] = bv;
  }
}

// Crossing c of slot s's shadow ray (from its record): material, incidence cosine and, for a
// material with a transmittance map (tx >= 0), the texture coordinates of the crossing point.
__device__ __forceinline__ void crossing_at(const DevScene& S, const DevWS& w, uint32_t s, uint32_t c, F3 o, F3 d,
                                            int& m, float& cosv, int& tx, float& ss, float& tt) {
  const float2 x = w.shx[(size_t)c * w.W + s];
  const uint32_t tri = __float_as_uint(x.y);
  const float4* g = S.gtris + (size_t)tri * 3;
  const float4 A = g[0], B = g[1], C = g[2];
  const F3 v0 = f3(A.x, A.y, A.z), v1 = f3(B.x, B.y, B.z), v2 = f3(C.x, C.y, C.z);
  m = __float_as_int(x.x);
  cosv = fabsf(dot3(d, geo_normal(v0, v1, v2)));
  tx = -1;
  ss = tt = 0.0f;
  if (S.n_tex > 0) {
    tx = S.mtex[m];
    if (tx >= 0) {
      float t = 0.0f, bu = 1.0f / 3.0f, bv = 1.0f / 3.0f;
      F3 qq;
      refine_hit(o, d, v0, v1, v2, t, qq, bu, bv);
      hit_st(S, tri, bu, bv, ss, tt);
    }
  }
}

// Glass crossings of the shadow ray of slot s (at most kMaxCross recorded, material and
// triangle id each): the material and |cos| between the ray and the slab's normal of each, and
// for a material with a transmittance map (tx >= 0) the texture coordinates of the crossing,
// from the crossing triangle re-intersected with the shadow ray.
__device__ __forceinline__ void crossings(const DevScene& S, const DevWS& w, uint32_t s, uint32_t nc, int* mq,
                                          float* cq, int* tx, float* sq, float* tq) {
  const float4 ro = w.rays[2 * ((size_t)w.W + s)], rd = w.rays[2 * ((size_t)w.W + s) + 1];
  const F3 o = f3(ro.x, ro.y, ro.z), d = f3(rd.x, rd.y, rd.z);
#pragma unroll
  for (int q = 0; q < kMaxCross; ++q) {
    mq[q] = 0;
    cq[q] = 1.0f;
    tx[q] = -1;
    sq[q] = tq[q] = 0.0f;
    if ((uint32_t)q < nc) crossing_at(S, w, s, (uint32_t)q, o, d, mq[q], cq[q], tx[q], sq[q], tq[q]);
  }
}

__global__ void k_resolve_vis(DevScene S, DevWS w, uint32_t n, float* vis) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t c = w.shcnt[i];
    const uint32_t nc = c == kBlocked ? 0u : min(c, (uint32_t)kMaxCross);
    int mq[kMaxCross], tx[kMaxCross];
    float cq[kMaxCross], sq[kMaxCross], tq[kMaxCross];
    crossings(S, w, i, nc, mq, cq, tx, sq, tq);
    for (int j = 0; j < S.n_bins; ++j) {
      float V = 0.0f;
      if (c != kBlocked) {
        V = 1.0f;
#pragma unroll
        for (int q = 0; q < kMaxCross; ++q) {
          if ((uint32_t)q < nc) {
            const int m = mq[q];
            float R, T;
            if (tx[q] >= 0) {
              const float4 t4 = tex_quad(tex_tap(S, tx[q], sq[q], tq[q]), j >> 2);
              const float tau0 = (j & 3) == 0 ? t4.x : ((j & 3) == 1 ? t4.y : ((j & 3) == 2 ? t4.z : t4.w));
              slab_tau0(S.ntab[m * S.bins_pad + j], S.ktab[m * S.bins_pad + j], tau0, cq[q], R, T);
            } else {
              slab(S.ntab[m * S.bins_pad + j], S.ktab[m * S.bins_pad + j], S.lambda[j], S.thick[m], cq[q], R, T);
            }
            V *= T;
          }
        }
      }
      vis[(size_t)i * S.n_bins + j] = V;
    }
  }
}

// ==========================================================================================
// queue: scan + scatter
// ==========================================================================================
constexpr int kScanThreads = 1024;
constexpr int kScanLdsKeys = 8192;  // queue keys whose counts are staged in LDS (beyond: read from memory)
constexpr int kScanOrderCells = 4096;  // largest grid whose cells the scan can order fullest first

// Inclusive sums over the workgroup of one value per thread: shuffles within each wave, then the
// wave totals, scanned by the first wave through LDS.
__device__ __forceinline__ void block_scan2(uint32_t& a, uint32_t& b, uint32_t* s_wa, uint32_t* s_wb) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t xa = __shfl_up(a, off), xb = __shfl_up(b, off);
    if (lane >= off) {
      a += xa;
      b += xb;
    }
  }
  if (lane == 63) {
    s_wa[wid] = a;
    s_wb[wid] = b;
  }
  __syncthreads();
  if (wid == 0) {
    constexpr int nw = kScanThreads / 64;
    uint32_t ta = lane < nw ? s_wa[lane] : 0u, tb = lane < nw ? s_wb[lane] : 0u;
#pragma unroll
    for (int off = 1; off < nw; off <<= 1) {
      const uint32_t xa = __shfl_up(ta, off), xb = __shfl_up(tb, off);
      if (lane >= off) {
        ta += xa;
        tb += xb;
      }
    }
    if (lane < nw) {
      s_wa[lane] = ta;
      s_wb[lane] = tb;
    }
  }
  __syncthreads();
  if (wid > 0) {
    a += s_wa[wid - 1];
    b += s_wb[wid - 1];
  }
}

// Order of the cells in the tile list when it is built fullest first: the cells sorted by the
// octave of their queued rays (s_oct: 1 + floor(log2 count), 0 for an empty cell), fullest octave
// first, ascending cell index inside an octave (neighbouring cells of similar load stay together).
// Written to s_perm[0 .. n_cells); the workgroup must call it together. Each octave that holds cells
// costs one pass over the per-thread chunks of cells and one workgroup prefix sum.
__device__ void cell_order_fullest(int n_cells, const uint8_t* s_oct, uint16_t* s_perm, uint32_t* s_hist,
                                   uint32_t* s_wa, uint32_t* s_wb) {
  if (threadIdx.x < 33) s_hist[threadIdx.x] = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < n_cells; c += kScanThreads) atomicAdd(&s_hist[s_oct[c]], 1u);
  __syncthreads();
  const int chunk = (n_cells + kScanThreads - 1) / kScanThreads;
  const int c0 = min(n_cells, (int)threadIdx.x * chunk), c1 = min(n_cells, c0 + chunk);
  uint32_t base = 0;
  for (int o = 32; o >= 0; --o) {
    const uint32_t in_oct = s_hist[o];  // the same for every thread: no divergence at the barriers
    if (in_oct == 0) continue;
    uint32_t f = 0;
    for (int c = c0; c < c1; ++c) f += s_oct[c] == o ? 1u : 0u;
    uint32_t incl = f, unused = 0;
    block_scan2(incl, unused, s_wa, s_wb);
    uint32_t pos = base + incl - f;
    for (int c = c0; c < c1; ++c)
      if (s_oct[c] == o) s_perm[pos++] = (uint16_t)c;
    base += in_oct;
    __syncthreads();  // s_wa / s_wb are rewritten by the next octave's prefix sum
  }
}

// Sub-ranges of the queue keys (runs before k_scan): a key's sub-range counts are summed in queue
// order, giving each sub-range's offset inside its key's range (coff) and the key's count
// (ksum); up to 64 sub-ranges per key one thread each (shuffles inside the wave), more one
// workgroup per key, each thread (1 << sub_shift) / kWG consecutive ones. It also clears the
// other parity's counters, which the next generation's producers count into.
__global__ __launch_bounds__(kWG) void k_subscan(DevScene S, DevWS w, int gen) {
  const int p = gen & 1;
  const uint32_t* cnt = ccount_of(S, w, p);
  uint32_t* other = ccount_of(S, w, p ^ 1);
  const uint32_t nsub = 1u << w.sub_shift;
  if (nsub <= 64) {
    const uint32_t n = (uint32_t)S.n_cells * kDirBins * nsub;
    const uint32_t t = blockIdx.x * kWG + threadIdx.x;
    const uint32_t j = lane_id() & (nsub - 1u);
    const uint32_t x = t < n ? cnt[ctr_word(w, t)] : 0u;
    uint32_t incl = x;
    for (uint32_t off = 1; off < nsub; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if (j >= off) incl += y;
    }
    if (t < n) {
      w.coff[t] = incl - x;
      if (j == nsub - 1u) w.ksum[t >> w.sub_shift] = incl;
      other[ctr_word(w, t)] = 0;
    }
  } else {
    constexpr int kMaxPer = (1 << (3 * kMaxSubLevels + kDirSubBits)) / kWG;
    static_assert(kMaxPer >= 1 && (1 << (3 * kMaxSubLevels + kDirSubBits)) % kWG == 0, "whole sub-ranges per thread");
    __shared__ uint32_t s_w[kWG / 64];
    const uint32_t per = nsub / kWG;  // a power of two, 1 .. kMaxPer
    const uint32_t k0 = blockIdx.x * nsub + threadIdx.x * per;
    uint32_t x[kMaxPer], sum = 0;
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i) {
      x[i] = (uint32_t)i < per ? cnt[ctr_word(w, k0 + i)] : 0u;
      sum += x[i];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if (lane_id() >= (uint32_t)off) incl += y;
    }
    if (lane_id() == 63) s_w[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (uint32_t q = 0; q < (threadIdx.x >> 6); ++q) run += s_w[q];
#pragma unroll
    for (int i = 0; i < kMaxPer; ++i)
      if ((uint32_t)i < per) {
        w.coff[k0 + i] = run;
        run += x[i];
        other[ctr_word(w, k0 + i)] = 0;
      }
    if (threadIdx.x == kWG - 1) w.ksum[blockIdx.x] = run;
  }
}

// One workgroup turns the per-key counts of the produced entries into the key offsets of the
// cell-sorted queue (koff; a key's sub-ranges follow one another inside its range, at coff) and
// the tile list: a tile is up to kTile entries of one key (across its sub-ranges), the tiles
// of a key consecutive, the keys in cell order (order 0) or, for order 1 and grids of at most
// kScanOrderCells cells, with the cells taken fullest first (cell_order_fullest) and the
// direction classes of a cell in ascending order. The traversal hands the tiles out in list order
// over the XCDs' ranges, so the fullest cells are started first and the launch ends on the
// smallest queues (the paper's sub-model with the most waiting rays is taken next, section 5).
__global__ __launch_bounds__(kScanThreads) void k_scan(DevScene S, DevWS w, int gen, int order) {
  __shared__ uint32_t s_cnt[kScanThreads], s_til[kScanThreads], s_key[kScanLdsKeys];
  __shared__ uint32_t s_wa[kScanThreads / 64], s_wb[kScanThreads / 64];
  __shared__ uint16_t s_perm[kScanOrderCells];
  __shared__ uint8_t s_oct[kScanOrderCells];
  __shared__ uint32_t s_hist[33];
  const int p = gen & 1;
  const int nc = S.n_cells * kDirBins;   // queue keys: (cell, direction octant)
  const bool staged = nc <= kScanLdsKeys;
  const bool ordered = order == 1 && S.n_cells <= kScanOrderCells;
  auto count_of = [&](uint32_t k) -> uint32_t { return staged ? s_key[k] : w.ksum[k]; };
  // counts staged in LDS by key
  if (staged) {
    for (int k = threadIdx.x; k < nc; k += kScanThreads) s_key[k] = w.ksum[k];
    __syncthreads();
  }
  if (ordered) {
    for (int c = threadIdx.x; c < S.n_cells; c += kScanThreads) {
      uint32_t t = 0;
      for (int b = 0; b < kDirBins; ++b) t += count_of(c * kDirBins + b);
      s_oct[c] = (uint8_t)(t ? 32u - (uint32_t)__clz(t) : 0u);
    }
    __syncthreads();
    cell_order_fullest(S.n_cells, s_oct, s_perm, s_hist, s_wa, s_wb);
    __syncthreads();
  }
  // position c of the ordered key sequence -> queue key
  auto key_at = [&](int c) -> uint32_t {
    return ordered ? (uint32_t)s_perm[c / kDirBins] * kDirBins + (uint32_t)(c % kDirBins) : (uint32_t)c;
  };
  const int chunk = (nc + kScanThreads - 1) / kScanThreads;
  const int c0 = min(nc, (int)threadIdx.x * chunk), c1 = min(nc, c0 + chunk);
  uint32_t sc = 0, st = 0;
  for (int c = c0; c < c1; ++c) {
    const uint32_t x = count_of(key_at(c));
    sc += x;
    st += (x + kTile - 1) / kTile;
  }
  uint32_t ic = sc, it = st;
  block_scan2(ic, it, s_wa, s_wb);
  s_cnt[threadIdx.x] = ic;
  s_til[threadIdx.x] = it;
  __syncthreads();
  uint32_t run = ic - sc;
  for (int c = c0; c < c1; ++c) {
    const uint32_t k = key_at(c);
    w.koff[k] = run;
    run += count_of(k);
  }
  // Tiles are written by the whole workgroup, each thread a contiguous block of them: the key of
  // its first tile comes from a binary search of the per-thread tile sums and a walk over that
  // chunk's counts, the following tiles from walking on through the keys. One key may hold
  // thousands of tiles (the camera rays of a frame enter a few cells), which a per-key loop
  // would write serially.
  const uint32_t n_tiles = s_til[kScanThreads - 1];
  const uint32_t per = (n_tiles + kScanThreads - 1) / kScanThreads;
  uint32_t t = min(n_tiles, (uint32_t)threadIdx.x * per);
  const uint32_t t_end = min(n_tiles, t + per);
  if (t < t_end) {
    int lo = 0, hi = kScanThreads - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_til[mid] > t)
        hi = mid;
      else
        lo = mid + 1;
    }
    uint32_t tb = lo ? s_til[lo - 1] : 0u, cb = lo ? s_cnt[lo - 1] : 0u;
    int c = lo * chunk;
    uint32_t k = key_at(c), x = count_of(k), nt = (x + kTile - 1) / kTile;
    for (; t < t_end; ++t) {
      // keys with no tile left are passed over; t < n_tiles keeps c below nc
      while (t >= tb + nt && c + 1 < nc) {
        tb += nt;
        cb += x;
        ++c;
        k = key_at(c);
        x = count_of(k);
        nt = (x + kTile - 1) / kTile;
      }
      const uint32_t q = t - tb;
      w.tiles[t] = make_uint4(k, cb + q * kTile, min((uint32_t)kTile, x - q * kTile), 0u);
    }
  }
  if (threadIdx.x == kScanThreads - 1) {
    w.ctl->n_queue = s_cnt[kScanThreads - 1];
    w.ctl->n_tiles = s_til[kScanThreads - 1];
    w.ctl->list_count[p ^ 1] = 0;
  }
  if (threadIdx.x < kXcds) w.ctl->tile_next[threadIdx.x * kKeyStride] = 0;
}

// Each thread moves kPer pairs of entries (2j, 2j + 1) per pass, all their loads issued before
// any store (the lists and the queue are all uint32 memory: a load after a store would wait for
// it); entries marked kNoKey (no ray) are passed over. Opaque shading puts vertex a's extension
// ray at entry 2a and its shadow ray at 2a + 1, so storing the even entries of a wave's pairs in
// one instruction and the odd ones in the next writes the rays of 64 neighbouring vertices per
// instruction, whose ranks in a shared sub-range are consecutive.
__global__ void k_scatter(DevWS w, int gen) {
  constexpr int kPer = 4;
  const uint32_t n = w.ctl->list_count[gen & 1];
  const uint32_t np = (n + 1) / 2;
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint2* src2 = (const uint2*)w.lsrc;
  const uint2* key2 = (const uint2*)w.ldst;
  const uint2* rank2 = (const uint2*)w.lrank;
  for (uint32_t j0 = blockIdx.x * blockDim.x + threadIdx.x; j0 < np; j0 += kPer * stride) {
    uint2 key[kPer], rank[kPer], src[kPer];
    uint32_t base[2 * kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t j = j0 + k * stride;
      key[k] = j < np ? key2[j] : make_uint2(kNoKey, kNoKey);
      rank[k] = j < np ? rank2[j] : make_uint2(0u, 0u);
      src[k] = j < np ? src2[j] : make_uint2(0u, 0u);
      // an odd count leaves the last pair's second entry outside the list
      if (j == np - 1 && (n & 1u)) key[k].y = kNoKey;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      base[2 * k] = key[k].x != kNoKey ? w.koff[key[k].x >> w.sub_shift] + w.coff[key[k].x] : 0u;
      base[2 * k + 1] = key[k].y != kNoKey ? w.koff[key[k].y >> w.sub_shift] + w.coff[key[k].y] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (key[k].x != kNoKey) w.queue[base[2 * k] + rank[k].x] = src[k].x;
      if (key[k].y != kNoKey) w.queue[base[2 * k + 1] + rank[k].y] = src[k].y;
    }
  }
}

// x, opaque to the compiler: an address formed from it is computed where it is used instead of
// being hoisted out of the traversal loop and held in registers across it (the stores of a
// finished ray's records are rare; their addresses held live made the kernel spill).
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// ==========================================================================================
// traversal
// ==========================================================================================
// Per-ray constants of the traversal: origin, reciprocal direction (box and cell slabs) and the
// shear of the watertight test.
struct RayPre {
  F3 o, inv;
  uint32_t k;  // axes of the watertight test's frame: kx | ky << 2 | kz << 4
  float Sx, Sy, Sz;
};

__device__ __forceinline__ float safe_dir(float c) { return fabsf(c) < 1e-18f ? copysignf(1e-18f, c) : c; }

__device__ __forceinline__ RayPre make_pre(F3 o, F3 d) {
  RayPre R;
  R.o = o;
  // hardware reciprocals (1 ulp): the box test's slack covers the extra rounding, the shear
  // constants of the watertight test only need to be the same for every triangle of the ray.
  // A direction component below 1e-18 in magnitude (zero included) is taken as +-1e-18: with an
  // infinite reciprocal a ray lying in a box or cell face would give 0 * inf = NaN in the slab
  // test and miss boxes it touches; the finite reciprocal makes box slabs, cell intervals and
  // cell steps treat it consistently as tilted by 1e-18 (the triangle test keeps the exact d).
  R.inv = f3(frcp(safe_dir(d.x)), frcp(safe_dir(d.y)), frcp(safe_dir(d.z)));
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  const int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (comp(d, kz) < 0.0f) {
    const int t = kx;
    kx = ky;
    ky = t;
  }
  R.k = (uint32_t)kx | (uint32_t)ky << 2 | (uint32_t)kz << 4;
  const float dz = comp(d, kz);
  R.Sz = frcp(dz);
  R.Sx = comp(d, kx) * R.Sz;
  R.Sy = comp(d, ky) * R.Sz;
  return R;
}

// a*b - c*d with Kahan's FMA scheme: relative error at most 2 ulp (Jeannerod, Louvet, Muller,
// Math. Comp. 2013), so the sign is exact and the result is zero exactly when a*b == c*d.
__device__ __forceinline__ float det2_exact_sign(float a, float b, float c, float d) {
#pragma clang fp contract(off)
  const float w = c * d;
  const float e = __builtin_fmaf(-c, d, w);  // w - c*d, exactly
  const float f = __builtin_fmaf(a, b, -w);
  return f + e;
}

// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013): shear the triangle into the
// ray's frame, evaluate the three 2D edge functions (re-evaluated with an exact-sign scheme
// when one is exactly zero, where the original falls back to FP64), inclusive of edges, no
// back-face culling. Returns false or t with barycentrics.
__device__ __forceinline__ bool wt_test(const RayPre& R, F3 v0, F3 v1, F3 v2, float& t, float& bu, float& bv) {
#pragma clang fp contract(off)
  const F3 A = v0 - R.o, B = v1 - R.o, C = v2 - R.o;
  const int kx = (int)(R.k & 3u), ky = (int)((R.k >> 2) & 3u), kz = (int)(R.k >> 4);
  const float Akz = comp(A, kz), Bkz = comp(B, kz), Ckz = comp(C, kz);
  const float Ax = comp(A, kx) - R.Sx * Akz, Ay = comp(A, ky) - R.Sy * Akz;
  const float Bx = comp(B, kx) - R.Sx * Bkz, By = comp(B, ky) - R.Sy * Bkz;
  const float Cx = comp(C, kx) - R.Sx * Ckz, Cy = comp(C, ky) - R.Sy * Ckz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = det2_exact_sign(Cx, By, Cy, Bx);
    V = det2_exact_sign(Ax, Cy, Ay, Cx);
    W = det2_exact_sign(Bx, Ay, By, Ax);
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  } else if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) {
    return false;
  }
  const float det = U + V + W;
  if (det == 0.0f) return false;
  const float T = U * (R.Sz * Akz) + V * (R.Sz * Bkz) + W * (R.Sz * Ckz);
  const float inv = __builtin_amdgcn_rcpf(det);
  t = T * inv;
  bu = V * inv;
  bv = W * inv;
  return true;
}

// The four child boxes of a 4-wide node against [tmin, tmax] (robust slab test, Ize 2013: the far
// distance is scaled by 1 + 2 gamma_5 so that rounding never culls a box the ray touches): the
// entry distance of each hit child and its word, +inf and kEmptyChild for a missed or empty one.
// The node holds its children's bounds as bytes q on a grid origin + q 2^(e - 127) per axis
// (64-byte node, see the scene builder), so a slab distance is a + q b with a = (origin - o) / d
// and b = 2^(e - 127) / d, one FMA per bound (b is exact: a power of two times 1/d). A distance
// carries the subtraction, the product, the 1-ulp reciprocal and the FMA, four roundings, and
// gamma_5 keeps one in reserve.
__device__ __forceinline__ void box4(const RayPre& R, float4 q0, float4 q1, float4 q2, float4 q3, float tmin,
                                     float tmax, float (&t)[kWide], uint32_t (&w)[kWide]) {
  constexpr float kSlop = 1.0f + 2.0f * 5.0f * 5.9604645e-8f / (1.0f - 5.0f * 5.9604645e-8f);
  const uint32_t e = __float_as_uint(q0.w);
  const float bx = __uint_as_float((e & 0xFFu) << 23) * R.inv.x;
  const float by = __uint_as_float(((e >> 8) & 0xFFu) << 23) * R.inv.y;
  const float bz = __uint_as_float(((e >> 16) & 0xFFu) << 23) * R.inv.z;
  const float ax = (q0.x - R.o.x) * R.inv.x, ay = (q0.y - R.o.y) * R.inv.y, az = (q0.z - R.o.z) * R.inv.z;
  // the near and far bound of each axis, chosen once per node by the sign of the ray's direction
  // (a + q b is monotone in q, increasing for b > 0, so the near plane is the low one then and the
  // high one otherwise; b has the sign of the finite reciprocal, never zero)
  const uint32_t LX = __float_as_uint(q2.x), HX = __float_as_uint(q2.y), LY = __float_as_uint(q2.z),
                 HY = __float_as_uint(q2.w), LZ = __float_as_uint(q3.x), HZ = __float_as_uint(q3.y);
  const uint32_t NX = R.inv.x >= 0.0f ? LX : HX, FX = R.inv.x >= 0.0f ? HX : LX;
  const uint32_t NY = R.inv.y >= 0.0f ? LY : HY, FY = R.inv.y >= 0.0f ? HY : LY;
  const uint32_t NZ = R.inv.z >= 0.0f ? LZ : HZ, FZ = R.inv.z >= 0.0f ? HZ : LZ;
  const uint32_t W[4] = {__float_as_uint(q1.x), __float_as_uint(q1.y), __float_as_uint(q1.z), __float_as_uint(q1.w)};
#pragma unroll
  for (int c = 0; c < kWide; ++c) {
    const float xn = __builtin_fmaf((float)((NX >> (8 * c)) & 0xFFu), bx, ax);
    const float xf = __builtin_fmaf((float)((FX >> (8 * c)) & 0xFFu), bx, ax);
    const float yn = __builtin_fmaf((float)((NY >> (8 * c)) & 0xFFu), by, ay);
    const float yf = __builtin_fmaf((float)((FY >> (8 * c)) & 0xFFu), by, ay);
    const float zn = __builtin_fmaf((float)((NZ >> (8 * c)) & 0xFFu), bz, az);
    const float zf = __builtin_fmaf((float)((FZ >> (8 * c)) & 0xFFu), bz, az);
    const float n = fmaxf(fmaxf(xn, yn), fmaxf(zn, tmin));
    const float f = fminf(fminf(xf, yf), zf) * kSlop;
    const bool hit = n <= fminf(f, tmax) && W[c] != kEmptyChild;
    t[c] = hit ? n : INFINITY;
    w[c] = hit ? W[c] : kEmptyChild;
  }
}

// Sorting network on four (distance, word) pairs, ascending distance.
__device__ __forceinline__ void cswap(float (&t)[kWide], uint32_t (&w)[kWide], int a, int b) {
  const bool s = t[b] < t[a];
  const float ta = t[a], tb = t[b];
  const uint32_t wa = w[a], wb = w[b];
  t[a] = s ? tb : ta;
  t[b] = s ? ta : tb;
  w[a] = s ? wb : wa;
  w[b] = s ? wa : wb;
}
__device__ __forceinline__ void sort4(float (&t)[kWide], uint32_t (&w)[kWide]) {
  cswap(t, w, 0, 1);
  cswap(t, w, 2, 3);
  cswap(t, w, 0, 2);
  cswap(t, w, 1, 3);
  cswap(t, w, 1, 2);
}

struct TraceState {
  // closest hit (distance and triangle id; the hit's reader refines both in FP64)
  float tbest;
  uint32_t best_id;
  // shadow
  bool blocked;
  uint32_t ncross;
};

// What one traversal step did, for the work counters.
enum : int { kStepNone = 0, kStepNode = 1, kStepTri = 2, kStepCross = 3 /* a triangle test that crossed glass */ };

// Traverse the BVH of one cell for hits with t > 0, t >= t_lo, t < t_hi. One loop serves both
// ray kinds (lanes of a wave may hold either): a closest-hit ray shrinks its far bound with every
// accepted hit; a shadow ray keeps it, stops at the first opaque hit and records every glass
// crossing. Both hit children that are leaves are tested in one triangle loop.
// One unit of traversal work for one ray in a cell's BVH: either one triangle of a pending leaf
// (watertight test) or one node (both child boxes, robust slab test). A node visit makes the
// nearer hit inner child the next node and pushes the farther one; a hit leaf child becomes the
// pending leaf (a second one is pushed as a leaf entry). Doing one unit per step keeps the
// lanes of a wave on the same kind of work. Returns false when the cell's traversal is
// finished: nothing pending and the stack empty, or a shadow ray blocked by an opaque triangle.
// pend: the pending leaf as count << 27 | next triangle; none pending while the count is 0.
__device__ __forceinline__ bool trav_step(const DevScene& S, const DevWS& w, const RayPre& R, bool shadow, int4 cinfo,
                                          uint32_t* stack_lds,
                                          uint32_t* spill, uint32_t spill_stride, uint32_t skip, float t_lo,
                                          float t_hi, uint32_t slot, TraceState& st, uint32_t& node, int& sp,
                                          uint32_t& pend, int& work) {
  if ((pend >> 27) == 0 && node == kNoNode) {
    if (sp == 0) return false;
    --sp;
    // LDS and global memory are read through pointers of their own address spaces, so the two
    // loads are not merged into one slower generic load
    uint32_t e = ((const __attribute__((address_space(3))) uint32_t*)stack_lds)[min(sp, kShortStack - 1) * kWG];
    if (sp >= kShortStack)
      e = ((const __attribute__((address_space(1))) uint32_t*)spill)[(size_t)(sp - kShortStack) * spill_stride];
    if (e & kStackLeaf) {
      pend = e & ~kStackLeaf;
    } else {
      node = e;
    }
  }
  // One load serves both kinds of step: a triangle (three float4) or a 4-wide node (four), so a
  // wave whose lanes do different kinds of work waits for one memory round trip per step.
  const bool is_tri = (pend >> 27) != 0;
  const uint32_t tri = pend & kStackLeafMaxIndex;
  if (is_tri) pend = pend + 1u - (1u << 27);  // next triangle, one fewer left (indices stay below 2^27)
  const float4* src = is_tri ? S.ctris + ((size_t)cinfo.z + tri) * 3 : S.nodes + ((size_t)cinfo.x + node) * 4;
  const float4 q0 = src[0], q1 = src[1], q2 = src[2];
  float4 q3 = q0;
  if (!is_tri) q3 = src[3];
  // an empty statement that reads every load: they are issued together here instead of the
  // node-only one being moved into the node branch (a second round trip)
  asm volatile("" ::"v"(q0.x), "v"(q1.x), "v"(q2.x), "v"(q3.x));
  if (is_tri) {
    const uint32_t id = __float_as_uint(q0.w);
    if (id == skip) return true;
    work = kStepTri;
    float t, u, v;
    if (!wt_test(R, f3(q0.x, q0.y, q0.z), f3(q1.x, q1.y, q1.z), f3(q2.x, q2.y, q2.z), t, u, v)) return true;
    if (!(t > 0.0f && t >= t_lo && t < t_hi)) return true;
    if (shadow) {
      const int m = (int)__float_as_uint(q1.w);
      if (S.mtype[m] == 0) {
        st.blocked = true;
        return false;
      }
      if (st.ncross < (uint32_t)kMaxCross)
        w.shx[(size_t)st.ncross * w.W + opaque(slot)] = make_float2(__int_as_float(m), __uint_as_float(id));
      st.ncross++;
      work = kStepCross;
    } else if (t < st.tbest || (t == st.tbest && id < st.best_id)) {
      st.tbest = t;
      st.best_id = id;
    }
    return true;
  }
  // node: the four child boxes (robust slab test), hit children sorted by entry distance; the
  // nearest becomes the next node or the pending leaf, the others are pushed farthest first
  work = kStepNode;
  float kt[kWide];
  uint32_t kw[kWide];
  box4(R, q0, q1, q2, q3, fmaxf(t_lo, 0.0f), shadow ? t_hi : st.tbest, kt, kw);
  sort4(kt, kw);
  node = kNoNode;
  if (kw[0] != kEmptyChild) {
    if (kw[0] >> 27)
      pend = kw[0];
    else
      node = kw[0];
  }
#pragma unroll
  for (int c = kWide - 1; c >= 1; --c) {
    if (kw[c] != kEmptyChild) {
      const uint32_t e = (kw[c] >> 27) ? (kStackLeaf | kw[c]) : kw[c];
      if (sp < kShortStack)
        stack_lds[sp * kWG] = e;
      else
        spill[(size_t)(sp - kShortStack) * spill_stride] = e;
      ++sp;
    }
  }
  return true;
}

// Cell index of a packed cell position ix | iy << 6 | iz << 12 (higher bits ignored).
__device__ __forceinline__ uint32_t cpos_cell(const DevScene& S, uint32_t cpos) {
  return (((cpos >> 12) & 63u) * (uint32_t)S.gy + ((cpos >> 6) & 63u)) * (uint32_t)S.gx + (cpos & 63u);
}

// Lane phases of k_trace.
enum : int { kLaneEnter = 1, kLaneTrav = 2, kLaneLeave = 3, kLaneDone = 4 };

// One tile = up to kTile rays of one queue key (cell, direction bin), handed out as kTile / 64
// parts of 64 rays, one part per wave: the 64 lanes of a wave start their part together, one
// ray each (lanes that traverse the same cell in the same direction class fetch the same nodes
// in the same instruction), and a wave whose rays are done takes its next part without waiting
// for the other waves of its workgroup. A lane steps one BVH node or one triangle per loop
// iteration. A ray's cell is traversed inside the cell's half-open slab interval; in every
// round but the last the ray then migrates to the queue of the next cell, in the last round it
// walks on in place. Finished rays write their category byte; migrating rays are appended to
// the next round's lists by the wave once its part is drained. The kernel runs 8 waves per SIMD
// (64 VGPRs, 16 bytes per lane spilled once per thread): the eighth wave hides more fetch latency
// than the spills cost (7.90 against 8.11 ms per launch at 7 waves and 72 VGPRs on the church
// frame).
constexpr uint32_t kTileParts = kTile / 64;

__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(8))) void k_trace(DevScene S, DevWS w, int gen, int hops) {
  __shared__ uint32_t s_stack[kShortStack * kWG];
  __shared__ uint32_t s_rsrc[kWG], s_rkey[kWG];
  // the grid's slab planes, and its cell table when small enough, staged in LDS: a ray entering
  // a cell then waits for LDS instead of a memory round trip
  __shared__ float s_planes[3 * (kMaxGrid + 1)];
  __shared__ int4 s_cells[kLdsCells];
  // the workgroup's work counters: frequent ones summed per wave in scalar registers, rare ones
  // (migrations, escapes, glass crossings, unrecorded crossings) added here by their lanes
  __shared__ uint32_t s_st[7];
  const int n_planes = S.gx + S.gy + S.gz + 3;
  const bool cells_lds = S.n_cells <= kLdsCells;
  for (int q = threadIdx.x; q < n_planes; q += kWG) s_planes[q] = S.planes[q];
  if (cells_lds)
    for (int q = threadIdx.x; q < S.n_cells; q += kWG) s_cells[q] = S.cells[q];
  stats_init(s_st, 7);
  __syncthreads();
  const uint32_t n_parts = w.ctl->n_tiles * kTileParts;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t lane = lane_id();
  const uint32_t gtid = blockIdx.x * kWG + threadIdx.x;
  uint32_t* spill = w.spill + gtid;
  uint32_t* stack = s_stack + threadIdx.x;
  const int np = (gen + 1) & 1;
  uint32_t n_visit = 0, n_nodes = 0, n_tris = 0;
  // Parts are handed out dynamically: each XCD owns a contiguous range of the cell-sorted tiles
  // (its L2 then holds few cells at a time) and its waves take the next part of that range from
  // a counter; a wave whose range is exhausted takes parts from the other XCDs' ranges.
  uint32_t donor = 0;   // how many ranges this wave has exhausted (wave-uniform)
  for (;;) {
    uint32_t t = 0xFFFFFFFFu;
    for (; donor < (uint32_t)kXcds; ++donor) {
      const uint32_t X = (xcd + donor) % kXcds;
      const uint32_t b = (uint32_t)(((uint64_t)n_parts * X) / kXcds);
      const uint32_t e = (uint32_t)(((uint64_t)n_parts * (X + 1)) / kXcds);
      uint32_t q = 0;
      if (lane == 0) q = atomicAdd(&w.ctl->tile_next[X * kKeyStride], 1u);
      q = b + __builtin_amdgcn_readfirstlane(q);
      if (q < e) {
        t = q;
        break;
      }
    }
    if (t == 0xFFFFFFFFu) break;
    const uint4 tile = w.tiles[t / kTileParts];
    const uint32_t r0 = (t % kTileParts) * 64u;
    if (r0 >= tile.z) continue;  // a part past the end of a partly filled tile
    const int tcell = (int)(tile.x / kDirBins);
    const uint32_t tdir = tile.x % kDirBins;
    const int4 tinfo = S.cells[tcell];
    int phase = kLaneDone;
    RayPre R;
    R.o = R.inv = f3(0.0f, 0.0f, 0.0f);
    R.k = 0;
    R.Sx = R.Sy = R.Sz = 0.0f;
    uint32_t slot = 0, skip = 0, node = 0, pend = 0;
    // cell coordinates, cells entered so far and the exit axis of the current cell:
    // ix | iy << 6 | iz << 12 | hops << 18 | axis << 26 (grids are at most 64 per axis, so a
    // ray enters fewer than 256 cells)
    uint32_t cpos = 0;
    bool shadow = false, first = false;
    int sp = 0;
    float t_lo = 0.0f, tf = 0.0f;
    int4 cinfo = make_int4(0, 0, 0, 0);
    TraceState st;
    st.tbest = INFINITY;
    st.best_id = 0xFFFFFFFFu;
    st.blocked = false;
    st.ncross = 0;
    s_rsrc[threadIdx.x] = 0xFFFFFFFFu;
    if (r0 + lane < tile.z) {
      const uint32_t entry = w.queue[tile.y + r0 + lane];
      const uint32_t r = entry & ~kFirstVisit;
      first = (entry & kFirstVisit) != 0;
      const float4 ro = w.rays[2 * r], rd = w.rays[2 * r + 1];
      skip = __float_as_uint(ro.w);
      const uint32_t sw = __float_as_uint(rd.w);
      shadow = (sw & kShadowBit) != 0;
      slot = sw & ~kShadowBit;
      R = make_pre(f3(ro.x, ro.y, ro.z), f3(rd.x, rd.y, rd.z));
      cpos = (uint32_t)(tcell % S.gx) | (uint32_t)((tcell / S.gx) % S.gy) << 6 |
             (uint32_t)(tcell / (S.gx * S.gy)) << 12;
      st.ncross = shadow ? w.shcnt[slot] : 0u;
      phase = kLaneEnter;
    }
    for (;;) {
      if (__ballot(phase != kLaneDone) == 0) break;
      bool fin = false, out_req = false, esc = false;
      int out_cat = -1, work = kStepNone;
      n_visit += (uint32_t)__popcll(__ballot(phase == kLaneEnter));
      if (phase == kLaneEnter) {
        // the cell's slab interval; traversal starts unless the cell is empty or already passed
        float tn;
        const int ix = (int)(cpos & 63u), iy = (int)((cpos >> 6) & 63u), iz = (int)((cpos >> 12) & 63u);
        const int cell = (int)cpos_cell(S, cpos);
        int axis;
        cell_interval_pl(s_planes, S.gx, S.gy, ix, iy, iz, R.o, R.inv, tn, tf, axis);
        cpos = (cpos & ~(3u << 26)) | (uint32_t)axis << 26;
        t_lo = first ? -INFINITY : tn;
        if (cell == tcell) {
          cinfo = tinfo;
        } else if (cells_lds) {
          // LDS and global memory through pointers of their own address spaces (no generic load)
          const __attribute__((address_space(3))) int* c = (const __attribute__((address_space(3))) int*)s_cells + 4 * cell;
          cinfo = make_int4(c[0], c[1], c[2], c[3]);
        } else {
          const __attribute__((address_space(1))) int* c = (const __attribute__((address_space(1))) int*)S.cells + 4 * cell;
          cinfo = make_int4(c[0], c[1], c[2], c[3]);
        }
        if (cinfo.y > 0 && t_lo < tf) {
          if (!shadow) st.tbest = tf;
          node = 0;
          sp = 0;
          pend = 0;
          phase = kLaneTrav;
        } else {
          phase = kLaneLeave;
        }
      }
      if (phase == kLaneTrav) {
        if (!trav_step(S, w, R, shadow, cinfo, stack, spill, w.trace_threads, skip, t_lo, tf, slot, st, node, sp, pend,
                       work)) {
          if (shadow && st.blocked) {
            w.shcnt[opaque(slot)] = kBlocked;
            fin = true;
          } else if (!shadow && st.best_id != 0xFFFFFFFFu) {
            const uint32_t mat = __float_as_uint(S.gtris[(size_t)st.best_id * 3 + 1].w);
            w.hit[opaque(slot)] = make_float4(st.tbest, __uint_as_float(st.best_id), 0.0f, 0.0f);
            out_cat = S.mtype[mat] == 0 ? kCatOpaque : kCatGlass;
            fin = true;
          } else {
            phase = kLaneLeave;
          }
        }
      }
      if (phase == kLaneLeave) {
        // leave through the exit face (Amanatides-Woo step)
        const int axis = (int)((cpos >> 26) & 3u);
        const float dc = comp(R.inv, axis);  // same sign as the direction component
        const int g = axis == 0 ? S.gx : (axis == 1 ? S.gy : S.gz);
        const int ni = (int)((cpos >> (6 * axis)) & 63u) + (dc > 0.0f ? 1 : -1);
        if (ni < 0 || ni >= g || !(tf < INFINITY)) {
          if (!shadow) {
            w.hit[opaque(slot)] = make_float4(INFINITY, __uint_as_float(0xFFFFFFFFu), 0.0f, 0.0f);
            if (S.env_nonzero) out_cat = kCatEscape;
          } else {
            out_cat = st.ncross > 0 ? kCatShadowGlass : kCatShadowClear;
          }
          esc = true;
          fin = true;
        } else {
          cpos = (cpos & ~(63u << (6 * axis))) | ((uint32_t)ni << (6 * axis));
          cpos += 1u << 18;
          first = false;
          if ((int)((cpos >> 18) & 0xFFu) < hops) {
            phase = kLaneEnter;
          } else {
            out_req = true;
            fin = true;
          }
        }
      }
      n_nodes += (uint32_t)__popcll(__ballot(work == kStepNode));
      n_tris += (uint32_t)__popcll(__ballot(work >= kStepTri));
      if (work == kStepCross) atomicAdd(&s_st[3], 1u);
      if (fin) {
        if (out_req) atomicAdd(&s_st[1], 1u);
        if (esc) atomicAdd(&s_st[2], 1u);
        // shadow rays that reach the sun through more slabs than were recorded
        if (shadow && !st.blocked && !out_req && st.ncross > (uint32_t)kMaxCross) atomicAdd(&s_st[4], 1u);
        if (shadow && !st.blocked) w.shcnt[opaque(slot)] = st.ncross;
        // the finished ray's category, by slot: gathered into slot-ordered lists after the trace
        if (out_cat >= 0) w.catb[(shadow ? (size_t)w.W : 0) + opaque(slot)] = (uint8_t)(out_cat + 1);
        if (out_req) {
          s_rsrc[threadIdx.x] = shadow ? w.W + slot : slot;
          s_rkey[threadIdx.x] = qsub(w, cpos_cell(S, cpos), tdir, 0u);
        }
        phase = kLaneDone;
      }
    }
    // the part is drained: append its migrating rays (one wave-aggregated atomic per list)
    const uint32_t rs = s_rsrc[threadIdx.x];
    wave_append(rs != 0xFFFFFFFFu, rs, s_rkey[threadIdx.x], &w.ctl->list_count[np], ccount_of(S, w, np), w,
                w.lsrc, w.ldst, w.lrank);
  }
  // the workgroup's counts, then one global atomic per counter
  stats_add(s_st, 0, n_visit);
  stats_add(s_st, 5, n_nodes);
  stats_add(s_st, 6, n_tris);
  __syncthreads();
  stats_flush(s_st, 0, &w.ctl->st_visits);
  stats_flush(s_st, 1, &w.ctl->st_migr);
  stats_flush(s_st, 2, &w.ctl->st_escape);
  stats_flush(s_st, 3, &w.ctl->st_glass);
  stats_flush(s_st, 4, &w.ctl->err_cross);
  stats_flush(s_st, 5, &w.ctl->st_nodes);
  stats_flush(s_st, 6, &w.ctl->st_tris);
}

// Finished rays carry their category in a byte per ray slot (extension rays in the first W,
// shadow rays in the second W; 0 = none). This pass turns the bytes into the per-category
// lists of one bounce and clears them. A workgroup compacts a chunk of kWG * kGatherPer
// consecutive slots with a prefix sum, so each chunk lands in the lists in ascending slot
// order (the shading kernels then read neighbouring path slots together) at the cost of one
// atomic per category and chunk.
constexpr int kGatherPer = 16;

__global__ __launch_bounds__(kWG) void k_gather_cats(DevWS w, int par) {
  constexpr int kWaves = kWG / 64;
  __shared__ uint32_t s_wsum[kCats][kWaves];
  __shared__ uint32_t s_base[kCats];
  const size_t n = 2 * (size_t)w.W;
  const size_t chunk = (size_t)kWG * kGatherPer;
  const uint32_t lane = lane_id(), wv = threadIdx.x / 64;
  for (size_t c0 = (size_t)blockIdx.x * chunk; c0 < n; c0 += (size_t)gridDim.x * chunk) {
    const size_t i0 = c0 + (size_t)threadIdx.x * kGatherPer;
    uint8_t b[kGatherPer];
    const bool whole = i0 + kGatherPer <= n;
    if (whole) {
      const uint4 v = *(const uint4*)(w.catb + i0);  // the byte lists start 256-byte aligned
      const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < kGatherPer; ++j) b[j] = (uint8_t)(x[j >> 2] >> (8 * (j & 3)));
    } else {
#pragma unroll
      for (int j = 0; j < kGatherPer; ++j) b[j] = i0 + j < n ? w.catb[i0 + j] : (uint8_t)0;
    }
    uint32_t cnt[kCats];
#pragma unroll
    for (int c = 0; c < kCats; ++c) cnt[c] = 0;
#pragma unroll
    for (int j = 0; j < kGatherPer; ++j)
#pragma unroll
      for (int c = 0; c < kCats; ++c) cnt[c] += b[j] == (uint8_t)(c + 1) ? 1u : 0u;
    // exclusive prefix of the counts over the workgroup: within the wave, then over waves
    uint32_t pre[kCats];
#pragma unroll
    for (int c = 0; c < kCats; ++c) {
      uint32_t incl = cnt[c];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
      }
      pre[c] = incl - cnt[c];
      if (lane == 63) s_wsum[c][wv] = incl;
    }
    __syncthreads();
    if (threadIdx.x < kCats) {
      const int c = threadIdx.x;
      uint32_t tot = 0;
      for (int q = 0; q < kWaves; ++q) {
        const uint32_t x = s_wsum[c][q];
        s_wsum[c][q] = tot;
        tot += x;
      }
      s_base[c] = tot ? atomicAdd(&w.ctl->cat_count[par][c * kKeyStride], tot) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kCats; ++c) pre[c] += s_base[c] + s_wsum[c][wv];
#pragma unroll
    for (int j = 0; j < kGatherPer; ++j) {
      if (b[j]) {
        const size_t i = i0 + j;
        const uint32_t slot = (uint32_t)(i < w.W ? i : i - w.W);
#pragma unroll
        for (int c = 0; c < kCats; ++c)
          if (b[j] == (uint8_t)(c + 1)) cat_list(w, par, c)[pre[c]++] = slot;
      }
    }
    if (whole) {
      *(uint4*)(w.catb + i0) = make_uint4(0u, 0u, 0u, 0u);
    } else {
      for (int j = 0; j < kGatherPer; ++j)
        if (i0 + j < n) w.catb[i0 + j] = 0;
    }
    __syncthreads();  // s_wsum / s_base are rewritten by the next chunk
  }
}

// ==========================================================================================
// shading: per-category kernels over the lists the traversal produced. Every path slot keeps
// its spectral rows contiguous ([slot][bin], rows of Bp floats read as float4), because list
// order follows the traversal (cell by cell), not the slot order.
// ==========================================================================================
// Shadow rays that reached the sun (eq. 3 direct term, weight stored when the ray was spawned,
// attenuated by every glass slab crossed). A slot holds one shadow ray at a time, so no two
// threads of this kernel touch the same radiance row.
// row[q] = f(q, row[q]) over the nq quads (4 bins each) of a path's spectral row, C quads at a
// time, every load of a chunk (the row's quads and whatever tables f reads) issued before the
// chunk's stores: rows and tables are all float memory, so a load that followed a store in
// program order could not be issued before it and would wait a full memory round trip.
template <int C, class F>
__device__ __forceinline__ void row_update(float4* row, int nq, F f) {
  for (int q0 = 0; q0 < nq; q0 += C) {
    float4 v[C];
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (q0 + q < nq) v[q] = f(q0 + q, row[q0 + q]);
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (q0 + q < nq) row[q0 + q] = v[q];
  }
}

// dst[q] = f(q) over nq quads, C at a time, every load of a chunk (whatever f reads) issued before
// the chunk's stores; with store false nothing is written (f still runs, in quad order).
template <int C, class F>
__device__ __forceinline__ void row_write(float4* dst, int nq, bool store, F f) {
  for (int q0 = 0; q0 < nq; q0 += C) {
    float4 v[C];
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (q0 + q < nq) v[q] = f(q0 + q);
    if (store) {
#pragma unroll
      for (int q = 0; q < C; ++q)
        if (q0 + q < nq) dst[q0 + q] = v[q];
    }
  }
}

// The direct term of slot s's shadow ray that reached the sun, into its radiance row: the weight
// stored when the ray was spawned, times the transmittance of the nc glass slabs it crossed (none:
// nc = 0), each slab's from its material, crossing angle and, with a transmittance map, the map
// at the crossing point.
__device__ __forceinline__ void add_direct(const DevScene& S, const DevWS& w, uint32_t s, uint32_t nc) {
  const int Bp = w.Bp, nq = Bp / 4;
  const float4* e = (const float4*)(w.nee + (size_t)s * Bp);
  if (nc == 0) {
    row_update<12>((float4*)(w.lacc + (size_t)s * Bp), nq, [&](int q, float4 l) {
      const float4 a = e[q];
      return make_float4(l.x + a.x, l.y + a.y, l.z + a.z, l.w + a.w);
    });
    return;
  }
  int mq[kMaxCross], tx[kMaxCross];
  float cq[kMaxCross], sq[kMaxCross], tq[kMaxCross];
  crossings(S, w, s, nc, mq, cq, tx, sq, tq);
  const float4* lam = (const float4*)S.lambda;
  row_update<12>((float4*)(w.lacc + (size_t)s * Bp), nq, [&](int q, float4 l) {
    float4 V = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    const float4 la = lam[q];
#pragma unroll
    for (int c = 0; c < kMaxCross; ++c) {
      if ((uint32_t)c < nc) {
        const int m = mq[c];
        const float4 nn = ((const float4*)(S.ntab + m * Bp))[q], kk = ((const float4*)(S.ktab + m * Bp))[q];
        float R0, T0, R1, T1, R2, T2, R3, T3;
        if (tx[c] >= 0) {
          const float4 t4 = tex_quad(tex_tap(S, tx[c], sq[c], tq[c]), q);
          slab_tau0(nn.x, kk.x, t4.x, cq[c], R0, T0);
          slab_tau0(nn.y, kk.y, t4.y, cq[c], R1, T1);
          slab_tau0(nn.z, kk.z, t4.z, cq[c], R2, T2);
          slab_tau0(nn.w, kk.w, t4.w, cq[c], R3, T3);
        } else {
          slab(nn.x, kk.x, la.x, S.thick[m], cq[c], R0, T0);
          slab(nn.y, kk.y, la.y, S.thick[m], cq[c], R1, T1);
          slab(nn.z, kk.z, la.z, S.thick[m], cq[c], R2, T2);
          slab(nn.w, kk.w, la.w, S.thick[m], cq[c], R3, T3);
        }
        V.x *= T0;
        V.y *= T1;
        V.z *= T2;
        V.w *= T3;
      }
    }
    const float4 a = e[q];
    return make_float4(l.x + a.x * V.x, l.y + a.y * V.y, l.z + a.z * V.z, l.w + a.w * V.w);
  });
}

// add_direct for the persistent kernel, in few registers: the weight row is multiplied by one
// crossed slab's transmittance at a time (crossing order), then added to the radiance row.
__device__ __forceinline__ void add_direct_seq(const DevScene& S, const DevWS& w, uint32_t s, uint32_t nc) {
  const int Bp = w.Bp, nq = Bp / 4;
  float4* e = (float4*)(w.nee + (size_t)s * Bp);
  const float4 ro = w.rays[2 * ((size_t)w.W + s)], rd = w.rays[2 * ((size_t)w.W + s) + 1];
  const F3 o = f3(ro.x, ro.y, ro.z), d = f3(rd.x, rd.y, rd.z);
  const float4* lam = (const float4*)S.lambda;
  for (uint32_t c = 0; c < nc; ++c) {
    int m, tx;
    float cq, ss, tt;
    crossing_at(S, w, s, c, o, d, m, cq, tx, ss, tt);
    TexTap tap;
    tap.base = nullptr;
    tap.r00 = tap.r10 = tap.r01 = tap.r11 = 0;
    tap.fx = tap.fy = 0.0f;
    if (tx >= 0) tap = tex_tap(S, tx, ss, tt);
    const float4* nt = (const float4*)(S.ntab + m * Bp);
    const float4* kt = (const float4*)(S.ktab + m * Bp);
    const float th = S.thick[m];
    row_update<2>(e, nq, [&](int q, float4 a) {
      const float4 nn = nt[q], kk = kt[q], la = lam[q];
      float R0, T0, R1, T1, R2, T2, R3, T3;
      if (tx >= 0) {
        const float4 t4 = tex_quad(tap, q);
        slab_tau0(nn.x, kk.x, t4.x, cq, R0, T0);
        slab_tau0(nn.y, kk.y, t4.y, cq, R1, T1);
        slab_tau0(nn.z, kk.z, t4.z, cq, R2, T2);
        slab_tau0(nn.w, kk.w, t4.w, cq, R3, T3);
      } else {
        slab(nn.x, kk.x, la.x, th, cq, R0, T0);
        slab(nn.y, kk.y, la.y, th, cq, R1, T1);
        slab(nn.z, kk.z, la.z, th, cq, R2, T2);
        slab(nn.w, kk.w, la.w, th, cq, R3, T3);
      }
      return make_float4(a.x * T0, a.y * T1, a.z * T2, a.w * T3);
    });
  }
  row_update<4>((float4*)(w.lacc + (size_t)s * Bp), nq, [&](int q, float4 l) {
    const float4 a = e[q];
    return make_float4(l.x + a.x, l.y + a.y, l.z + a.z, l.w + a.w);
  });
}

__global__ __launch_bounds__(kWG) void k_resolve(DevScene S, DevWS w, int depth) {
  const int p = depth & 1;
  const uint32_t n_clear = w.ctl->cat_count[p][kCatShadowClear * kKeyStride];
  const uint32_t n_glass = w.ctl->cat_count[p][kCatShadowGlass * kKeyStride];
  if (blockIdx.x == 0 && threadIdx.x < kCats) w.ctl->cat_count[p ^ 1][threadIdx.x * kKeyStride] = 0;  // next bounce
  const uint32_t n = n_clear + n_glass;
  for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    if (i < n_clear) {
      add_direct(S, w, cat_list(w, p, kCatShadowClear)[i], 0u);
    } else {
      const uint32_t s = cat_list(w, p, kCatShadowGlass)[i - n_clear];
      add_direct(S, w, s, min(w.shcnt[s], (uint32_t)kMaxCross));
    }
  }
}

// Extension rays that left the scene pick up the environment radiance. Launched after
// k_resolve: the same slot may also have had a shadow ray resolved there.
__global__ __launch_bounds__(kWG) void k_escape(DevScene S, DevWS w, int depth) {
  const int p = depth & 1;
  const uint32_t n = w.ctl->cat_count[p][kCatEscape * kKeyStride];
  const int Bp = w.Bp, nq = Bp / 4;
  const float4* env = (const float4*)S.env;
  for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    const uint32_t s = cat_list(w, p, kCatEscape)[i];
    const float4* b4 = (const float4*)(w.beta + (size_t)s * Bp);
    row_update<12>((float4*)(w.lacc + (size_t)s * Bp), nq, [&](int q, float4 l) {
      const float4 a = b4[q], e = env[q];
      return make_float4(l.x + a.x * e.x, l.y + a.y * e.y, l.z + a.z * e.z, l.w + a.w * e.w);
    });
  }
}

// Opaque vertex: direct term toward the sun through a shadow ray (eq. 3), then the
// Fresnel-split lobe choice (mirror with probability mean F, else cosine-weighted diffuse).
// Records a training vertex: position, direction toward the previous vertex, material; the
// path's throughput restarts at one and its gathered radiance at zero, so that what the path
// gathers from here on is the radiance leaving this vertex toward the previous one.
__device__ __forceinline__ void record_vertex(const PathMode& pm, const DevWS& w, uint32_t s, const Vertex& V) {
  pm.rec_x[s] = make_float4(V.p.x, V.p.y, V.p.z, __uint_as_float((uint32_t)V.m));
  pm.rec_w[s] = make_float4(-V.d.x, -V.d.y, -V.d.z, 1.0f);
  float4* b4 = (float4*)(w.beta + (size_t)s * w.Bp);
  float4* l4 = (float4*)(w.lacc + (size_t)s * w.Bp);
  for (int q = 0; q < w.Bp / 4; ++q) {
    b4[q] = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    l4[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

// NQ > 0: the spectral rows have exactly NQ float4 quads (compile time), so the bin loops unroll
// and their loads issue together; NQ = 0 handles any bin count.
// Spectral tables of the templated shading kernels (kLds): n, k and ρ of every material (n_mat
// rows of Bp floats each), then the sun's spectrum, staged in dynamic LDS when they take at most
// kShadeLdsFloats; otherwise read from memory.
constexpr int kShadeLdsFloats = 8192;

template <int NQ, bool kLds>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2))) void k_shade_opaque(DevScene S, DevWS w, int depth, int max_depth, uint32_t key0,
                                                      uint32_t key1, int gen, PathMode pm) {
  __shared__ uint32_t s_st[3];
  __shared__ float s_planes[3 * (kMaxGrid + 1)];  // the grid's slab planes, for locating new rays
  extern __shared__ float4 s_tab4[];
  // Fresnel factors of the templated kernels, one column per thread: kept here rather than in
  // registers between the lobe choice and the throughput update
  __shared__ float s_F[NQ > 0 ? 4 * NQ : 1][kWG];
  const int B = S.n_bins, Bp = w.Bp, nq = NQ > 0 ? NQ : Bp / 4;
  stats_init(s_st, 3);
  for (int q = threadIdx.x; q < S.gx + S.gy + S.gz + 3; q += kWG) s_planes[q] = S.planes[q];
  if constexpr (kLds) {
    float* s_tab = (float*)s_tab4;
    const int mb = S.n_mat * Bp;
    for (int q = threadIdx.x; q < 3 * mb + Bp; q += kWG)
      s_tab[q] = q < mb ? S.ntab[q] : q < 2 * mb ? S.ktab[q - mb] : q < 3 * mb ? S.rho[q - 2 * mb] : S.sunE[q - 3 * mb];
  }
  __syncthreads();
  const int p = depth & 1;
  const uint32_t n = w.ctl->cat_count[p][kCatOpaque * kKeyStride];
  const uint32_t* list = cat_list(w, p, kCatOpaque);
  const size_t W = w.W;
  const int gp = gen & 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctl->list_count[gp] = 2 * n;
  const uint32_t n_iter = (n + kWG - 1) / kWG * kWG;
  for (uint32_t a = blockIdx.x * kWG + threadIdx.x; a < n_iter; a += gridDim.x * kWG) {
    const bool valid = a < n;
    uint32_t s = 0, ext_cell = kInvalidCell, sh_cell = kInvalidCell, ext_dir = 0, sh_dir = 0, ext_xo = 0, sh_xo = 0;
    bool has_sh = false, has_ext = false;
    if (valid) {
      s = list[a];
      const Vertex V = load_vertex(S, w, s);
      if (depth == pm.rec_depth) record_vertex(pm, w, s, V);
      const uint4 rn = philox(make_uint4(w.pix[s], w.smp[s], (uint32_t)depth | pm.purpose, w.views[w.view[s]].view_id),
                              key0, key1);
      const float u0 = unif24(rn.x), u1 = unif24(rn.y), u2 = unif24(rn.z);
      float4* b4 = (float4*)(w.beta + (size_t)s * Bp);
      float4* e4 = (float4*)(w.nee + (size_t)s * Bp);
      const F3 ws = f3(S.sun[0], S.sun[1], S.sun[2]);
      const float cs = dot_exact_sign(V.n, ws);
      // from vertex gm_from on a global photon map supplies the diffuse light, direct light included
      const bool gm = pm.gm_from > 0 && depth >= pm.gm_from;
      const bool nee = !gm && cs > 0.0f;
      const float kn = cs * (1.0f / 3.14159265358979f);
      float a_sum = 0.0f, b_sum = 0.0f;
      bool cont = false, mirror = false;
      float inv_p = 0.0f;
      // lobe choice from the band means of F and (1 - F) rho
      auto choose = [&]() {
        const float am = a_sum / (float)B, bm = b_sum / (float)B;
        cont = depth < max_depth && am + bm > 0.0f;
        if (cont) {
          const float Ps = am / (am + bm);
          mirror = u0 < Ps;
          inv_p = mirror ? 1.0f / Ps : 1.0f / (1.0f - Ps);
          cont = mirror || !gm;  // with a global map the diffuse lobe's light was gathered
        }
      };
      if constexpr (NQ > 0) {
        // The vertex's β row is read before any row is written and the tables come from LDS; the
        // direct term and the throughput update then work from registers. (Rows are float memory
        // like the tables, so a load that followed a store in program order would wait for it.)
        const float4 *nt, *kt, *rt, *E4;
        if constexpr (kLds) {
          const int mb = S.n_mat * Bp / 4;
          nt = s_tab4 + V.m * Bp / 4;
          kt = nt + mb;
          rt = nt + 2 * mb;
          E4 = s_tab4 + 3 * mb;
        } else {
          nt = (const float4*)(S.ntab + V.m * Bp);
          kt = (const float4*)(S.ktab + V.m * Bp);
          rt = (const float4*)(S.rho + V.m * Bp);
          E4 = (const float4*)S.sunE;
        }
        float Dk[4 * NQ];
        float4 bq[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          bq[q] = b4[q];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const float4 nn = nt[q], kk = kt[q], rr = rt[q];
          const float n4[4] = {nn.x, nn.y, nn.z, nn.w}, k4[4] = {kk.x, kk.y, kk.z, kk.w},
                      r4[4] = {rr.x, rr.y, rr.z, rr.w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float F = fresnel(n4[c], k4[c], V.cos_o);
            s_F[4 * q + c][threadIdx.x] = F;
            Dk[4 * q + c] = (1.0f - F) * r4[c];
            if (q < NQ - 1 || 4 * q + c < B) {  // padding bins sit in the last quad only
              a_sum += F;
              b_sum += Dk[4 * q + c];
            }
          }
        }
        choose();
        if (nee) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const float* D = Dk + 4 * q;
            const float4 EE = E4[q];
            e4[q] = make_float4(bq[q].x * D[0] * kn * EE.x, bq[q].y * D[1] * kn * EE.y,
                                bq[q].z * D[2] * kn * EE.z, bq[q].w * D[3] * kn * EE.w);
          }
        }
        if (cont) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const float* D = Dk + 4 * q;
            float G[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) G[c] = mirror ? s_F[4 * q + c][threadIdx.x] : D[c];
            float4 bb = bq[q];
            bb.x *= G[0] * inv_p;
            bb.y *= G[1] * inv_p;
            bb.z *= G[2] * inv_p;
            bb.w *= G[3] * inv_p;
            b4[q] = bb;
          }
        }
      } else {
        const float4* nt = (const float4*)(S.ntab + V.m * Bp);
        const float4* kt = (const float4*)(S.ktab + V.m * Bp);
        const float4* rt = (const float4*)(S.rho + V.m * Bp);
        const float4* E4 = (const float4*)S.sunE;
        // eight quads at a time: their tables, β and sun spectrum are read before their NEE quads
        // are stored, and likewise for the throughput update (each chunk is one memory round
        // trip; at 80 bins 8 measured faster than 4 and 10)
        row_write<8>(e4, nq, nee, [&](int q) {
          const float4 nn = nt[q], kk = kt[q], rr = rt[q];
          const float F[4] = {fresnel(nn.x, kk.x, V.cos_o), fresnel(nn.y, kk.y, V.cos_o),
                              fresnel(nn.z, kk.z, V.cos_o), fresnel(nn.w, kk.w, V.cos_o)};
          const float rho[4] = {rr.x, rr.y, rr.z, rr.w};
          float dif[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            dif[c] = (1.0f - F[c]) * rho[c];
            if (4 * q + c < B) {
              a_sum += F[c];
              b_sum += dif[c];
            }
          }
          float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          if (nee) {
            const float4 bb = b4[q], EE = E4[q];
            out = make_float4(bb.x * dif[0] * kn * EE.x, bb.y * dif[1] * kn * EE.y, bb.z * dif[2] * kn * EE.z,
                              bb.w * dif[3] * kn * EE.w);
          }
          return out;
        });
        choose();
        if (cont)
          row_update<8>(b4, nq, [&](int q, float4 bb) {
            const float4 nn = nt[q], kk = kt[q], rr = rt[q];
            const float F0 = fresnel(nn.x, kk.x, V.cos_o), F1 = fresnel(nn.y, kk.y, V.cos_o),
                        F2 = fresnel(nn.z, kk.z, V.cos_o), F3v = fresnel(nn.w, kk.w, V.cos_o);
            bb.x *= (mirror ? F0 : (1.0f - F0) * rr.x) * inv_p;
            bb.y *= (mirror ? F1 : (1.0f - F1) * rr.y) * inv_p;
            bb.z *= (mirror ? F2 : (1.0f - F2) * rr.z) * inv_p;
            bb.w *= (mirror ? F3v : (1.0f - F3v) * rr.w) * inv_p;
            return bb;
          });
      }
      if (nee) {
        has_sh = true;
        const F3 so = V.p + V.n * V.eps;
        w.rays[2 * (W + s)] = make_float4(so.x, so.y, so.z, __uint_as_float(V.id));
        w.rays[2 * (W + s) + 1] = make_float4(ws.x, ws.y, ws.z, __uint_as_float(s | kShadowBit));
        w.shcnt[s] = 0;
        sh_cell = start_cell_pl(S, s_planes, so, ws, &sh_xo);
        sh_dir = dir_code(ws);
      }
      if (cont) {
        F3 nd;
        if (mirror) {
          nd = V.d - V.ng * (2.0f * V.dn);
        } else {
          float sn, cn;
          sincosf(2.0f * 3.14159265358979f * u1, &sn, &cn);
          const float rr = sqrtf(u2);
          const float lx = rr * cn, ly = rr * sn, lz = sqrtf(fmaxf(0.0f, 1.0f - u2));
          // orthonormal basis around n (Duff et al., JCGT 2017)
          const F3 nrm = V.n;
          const float sg = copysignf(1.0f, nrm.z);
          const float aa = -1.0f / (sg + nrm.z);
          const float bb = nrm.x * nrm.y * aa;
          const F3 t1 = f3(1.0f + sg * nrm.x * nrm.x * aa, sg * bb, -sg * nrm.x);
          const F3 t2 = f3(bb, sg + nrm.y * nrm.y * aa, -nrm.y);
          nd = t1 * lx + t2 * ly + nrm * lz;
        }
        const F3 no = V.p + V.n * V.eps;
        has_ext = true;
        w.rays[2 * s] = make_float4(no.x, no.y, no.z, __uint_as_float(V.id));
        w.rays[2 * s + 1] = make_float4(nd.x, nd.y, nd.z, __uint_as_float(s));
        ext_cell = start_cell_pl(S, s_planes, no, nd, &ext_xo);
        ext_dir = dir_code(nd);
        if (ext_cell == kInvalidCell) w.hit[s] = make_float4(INFINITY, __uint_as_float(0xFFFFFFFFu), 0.0f, 0.0f);
      }
    }
    // Vertex a's new rays take produced-list entries 2a (extension) and 2a + 1 (shadow), an entry
    // without a ray marked kNoKey: no list-counter atomic, which every wave of the launch would
    // queue on (atomics on one cache line are served one at a time). The list is empty when
    // opaque shading starts: the scan of the last traversal round cleared it, and that round
    // walks its rays to the end instead of queuing migrations. Its length is set to 2n above;
    // glass shading, launched next, writes its entries after these.
    {
      const bool ve = has_ext && ext_cell != kInvalidCell, vs = has_sh && sh_cell != kInvalidCell;
      const uint32_t ke = ve ? qsub(w, ext_cell, ext_dir, ext_xo) : kNoKey;
      const uint32_t ks = vs ? qsub(w, sh_cell, sh_dir, sh_xo) : kNoKey;
      uint32_t* cc = ccount_of(S, w, gp);
      uint32_t re, rs;
      wave_key_rank2(ve, ke, vs, ks, cc, w, re, rs);
      if (valid) {
        ((uint2*)w.lsrc)[a] = make_uint2(s | kFirstVisit, ((uint32_t)W + s) | kFirstVisit);
        ((uint2*)w.ldst)[a] = make_uint2(ke, ks);
        ((uint2*)w.lrank)[a] = make_uint2(re, rs);
      }
    }
    // rays that miss the grid box finish at once
    if (has_sh && sh_cell == kInvalidCell) w.catb[(size_t)W + s] = (uint8_t)(kCatShadowClear + 1);
    if (has_ext && ext_cell == kInvalidCell && S.env_nonzero) w.catb[s] = (uint8_t)(kCatEscape + 1);
    stats_add_ballot(s_st, 0, valid);
    stats_add_ballot(s_st, 1, has_sh);
    stats_add_ballot(s_st, 2, has_ext);
  }
  __syncthreads();
  stats_flush(s_st, 0, &w.ctl->st_vertices);
  stats_flush(s_st, 1, &w.ctl->st_shadow);
  stats_flush(s_st, 2, &w.ctl->st_ext);
}

// Glass vertex: thin slab, reflect with probability mean R / (mean R + mean T), else transmit
// straight through (no lateral shift); no direct term at glass.
__global__ __launch_bounds__(kWG) void k_shade_glass(DevScene S, DevWS w, int depth, uint32_t key0, uint32_t key1,
                                                     int gen, PathMode pm) {
  __shared__ uint32_t s_st[1];
  __shared__ float s_planes[3 * (kMaxGrid + 1)];  // the grid's slab planes, for locating new rays
  stats_init(s_st, 1);
  for (int q = threadIdx.x; q < S.gx + S.gy + S.gz + 3; q += kWG) s_planes[q] = S.planes[q];
  __syncthreads();
  const int p = depth & 1;
  const uint32_t n = w.ctl->cat_count[p][kCatGlass * kKeyStride];
  const uint32_t* list = cat_list(w, p, kCatGlass);
  const int B = S.n_bins, Bp = w.Bp;
  const int gp = gen & 1;
  // vertex a's new ray takes produced-list entry base + a, after the 2 n_opaque entries of opaque
  // shading (launched before this kernel in the same bounce); no list-counter atomic
  const uint32_t base = 2 * w.ctl->cat_count[p][kCatOpaque * kKeyStride];
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctl->list_count[gp] = base + n;
  const uint32_t n_iter = (n + kWG - 1) / kWG * kWG;
  for (uint32_t a = blockIdx.x * kWG + threadIdx.x; a < n_iter; a += gridDim.x * kWG) {
    const bool valid = a < n;
    uint32_t s = 0, ext_cell = kInvalidCell, ext_dir = 0, ext_xo = 0;
    if (valid) {
      s = list[a];
      const Vertex V = load_vertex(S, w, s);
      if (depth == pm.rec_depth) record_vertex(pm, w, s, V);
      const uint4 rn = philox(make_uint4(w.pix[s], w.smp[s], (uint32_t)depth | pm.purpose, w.views[w.view[s]].view_id),
                              key0, key1);
      const float u0 = unif24(rn.x);
      const float4* nt = (const float4*)(S.ntab + V.m * Bp);
      const float4* kt = (const float4*)(S.ktab + V.m * Bp);
      const float4* lam = (const float4*)S.lambda;
      const float th = S.thick[V.m];
      // the glass's transmittance map at the hit's texture coordinates, if it has one
      const int tx = S.n_tex > 0 ? S.mtex[V.m] : -1;
      TexTap tap;
      tap.base = nullptr;
      tap.r00 = tap.r10 = tap.r01 = tap.r11 = 0;
      tap.fx = tap.fy = 0.0f;
      if (tx >= 0) {
        float ss, tt;
        hit_st(S, V.id, V.bu, V.bv, ss, tt);
        tap = tex_tap(S, tx, ss, tt);
      }
      // slab R and T of the four bins of quad q (padding bins hold benign table values)
      auto slab4 = [&](int q, float (&R)[4], float (&T)[4]) {
        const float4 nn = nt[q], kk = kt[q], la = lam[q];
        if (tx >= 0) {
          const float4 t4 = tex_quad(tap, q);
          slab_tau0(nn.x, kk.x, t4.x, V.cos_o, R[0], T[0]);
          slab_tau0(nn.y, kk.y, t4.y, V.cos_o, R[1], T[1]);
          slab_tau0(nn.z, kk.z, t4.z, V.cos_o, R[2], T[2]);
          slab_tau0(nn.w, kk.w, t4.w, V.cos_o, R[3], T[3]);
        } else {
          slab(nn.x, kk.x, la.x, th, V.cos_o, R[0], T[0]);
          slab(nn.y, kk.y, la.y, th, V.cos_o, R[1], T[1]);
          slab(nn.z, kk.z, la.z, th, V.cos_o, R[2], T[2]);
          slab(nn.w, kk.w, la.w, th, V.cos_o, R[3], T[3]);
        }
      };
      float mr = 0.0f, mt = 0.0f;
#pragma unroll 4
      for (int q = 0; q < Bp / 4; ++q) {
        float R[4], T[4];
        slab4(q, R, T);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (4 * q + c < B) {
            mr += R[c];
            mt += T[c];
          }
      }
      const float Pr = mr / (mr + mt);
      const bool refl = u0 < Pr;
      const float inv_p = refl ? 1.0f / Pr : 1.0f / (1.0f - Pr);
      row_update<12>((float4*)(w.beta + (size_t)s * Bp), Bp / 4, [&](int q, float4 b) {
        float R[4], T[4];
        slab4(q, R, T);
        return make_float4(b.x * ((refl ? R[0] : T[0]) * inv_p), b.y * ((refl ? R[1] : T[1]) * inv_p),
                           b.z * ((refl ? R[2] : T[2]) * inv_p), b.w * ((refl ? R[3] : T[3]) * inv_p));
      });
      const F3 nd = refl ? V.d - V.ng * (2.0f * V.dn) : V.d;
      const F3 no = refl ? V.p + V.n * V.eps : V.p - V.n * V.eps;
      w.rays[2 * s] = make_float4(no.x, no.y, no.z, __uint_as_float(V.id));
      w.rays[2 * s + 1] = make_float4(nd.x, nd.y, nd.z, __uint_as_float(s));
      ext_cell = start_cell_pl(S, s_planes, no, nd, &ext_xo);
      ext_dir = dir_code(nd);
      if (ext_cell == kInvalidCell) w.hit[s] = make_float4(INFINITY, __uint_as_float(0xFFFFFFFFu), 0.0f, 0.0f);
    }
    {
      const bool ve = valid && ext_cell != kInvalidCell;
      const uint32_t ke = ve ? qsub(w, ext_cell, ext_dir, ext_xo) : kNoKey;
      const uint32_t re = wave_key_rank(ve, ke, ccount_of(S, w, gp), w);
      if (valid) {
        w.lsrc[base + a] = s | kFirstVisit;
        w.ldst[base + a] = ke;
        w.lrank[base + a] = re;
      }
    }
    if (valid && ext_cell == kInvalidCell && S.env_nonzero) w.catb[s] = (uint8_t)(kCatEscape + 1);
    stats_add_ballot(s_st, 0, valid);
  }
  __syncthreads();
  stats_flush(s_st, 0, &w.ctl->st_vertices);
  if (threadIdx.x == 0 && s_st[0]) atomicAdd(&w.ctl->st_ext, (unsigned long long)s_st[0]);
}

// End of a wavefront: every path's gathered radiance, divided by the view's spp, into its
// pixel of the spectral image [B][H][W]. Slots are visited in order, so a wave adds to
// consecutive pixels of one bin plane at a time. Slots s0 .. s0 + n - 1; kUnique: no pixel
// receives two of them, so plain loads and stores replace the atomics.
template <bool kUnique>
__global__ __launch_bounds__(kWG) void k_accumulate(DevScene S, DevWS w, uint32_t s0, uint32_t n) {
  const int B = S.n_bins, Bp = w.Bp;
  uint32_t n_bad = 0;  // bins of this thread's paths whose radiance is not finite
  for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    const uint32_t s = s0 + i;
    const ViewDesc& V = w.views[w.view[s]];
    const size_t plane = (size_t)V.width * V.height;
    float* img = V.image + w.pix[s];
    // 48 bins of the slot's row (and, kUnique, of its pixel) are loaded before the first store
    // or atomic of them: the image and the rows are both float memory, so a load issued after a
    // store or atomic would wait for it
    constexpr int kChunk = 12;
    const float4* l4 = (const float4*)(w.lacc + (size_t)s * Bp);
    for (int q0 = 0; q0 < Bp / 4; q0 += kChunk) {
      float4 l[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q)
        l[q] = q0 + q < Bp / 4 ? l4[q0 + q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      float cur[kUnique ? 4 * kChunk : 1];
      if constexpr (kUnique) {
#pragma unroll
        for (int e = 0; e < 4 * kChunk; ++e) {
          const int j = 4 * q0 + e;
          cur[e] = j < B ? img[(size_t)j * plane] : 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const float c4[4] = {l[q].x, l[q].y, l[q].z, l[q].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 4 * (q0 + q) + e;
          const float c = c4[e] * V.inv_spp;
          n_bad += (j < B && !isfinite(c)) ? 1u : 0u;
          if (j < B && c != 0.0f) {
            if constexpr (kUnique)
              img[(size_t)j * plane] = cur[4 * q + e] + c;
            else
              unsafeAtomicAdd(img + (size_t)j * plane, c);
          }
        }
      }
    }
  }
  // non-finite radiance (an overflow of huge but finite inputs, for example) is added to the
  // image as it is and counted; sdd_finish reports it. One atomic per wave that saw any.
  wave_add(&w.ctl->err_nonfinite, n_bad);
}

// ==========================================================================================
// persistent batched render: the whole batch of views in one kernel (plain mode)
// ==========================================================================================
// Work list: the path samples of every view as (view, tile, sample) items, a tile being 8 x 8
// pixels, one item per (tile, sample) pair and pixel of the tile (64 per tile and sample, those
// beyond a ragged view edge empty). View v owns items [item_base_v, item_base_v + T_v 64 spp_v),
// T_v tiles, in sample-major order (all tiles of sample 0, then sample 1, ...), so that the
// pixels of a tile at one sample are consecutive items and start together in one wave. The list
// is this index space, decoded on the device from the views' prefix offsets; waves take it in
// chunks of 64 items, each XCD from its own contiguous range first (an atomic on a per-XCD
// counter per chunk), then from the others'.
constexpr uint32_t kPersistTile = 8;
constexpr uint32_t kPersistChunk = 64;

// Item g of the work list: its view, pixel (row-major within the view) and sample; false for an
// empty item (a tile pixel outside the view).
__device__ __forceinline__ bool persist_item(const DevWS& w, uint64_t g, uint32_t& v, uint32_t& pix, uint32_t& smp) {
  int lo = 0, hi = w.n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (w.views[mid].item_base <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  v = (uint32_t)lo;
  const ViewDesc& V = w.views[lo];
  const uint32_t tx = ((uint32_t)V.width + kPersistTile - 1) / kPersistTile;
  const uint32_t ty = ((uint32_t)V.height + kPersistTile - 1) / kPersistTile;
  const uint64_t local = g - V.item_base;
  const uint32_t i = (uint32_t)(local % 64u);
  const uint64_t ts = local / 64u;
  const uint32_t nt = tx * ty;
  uint32_t t;
  if ((ts >> 32) == 0) {  // 32-bit division where it suffices
    t = (uint32_t)ts % nt;
    smp = (uint32_t)ts / nt + V.first_sample;
  } else {
    t = (uint32_t)(ts % nt);
    smp = (uint32_t)(ts / nt) + V.first_sample;
  }
  const uint32_t px = (t % tx) * kPersistTile + i % kPersistTile;
  const uint32_t py = (t / tx) * kPersistTile + i / kPersistTile;
  pix = py * (uint32_t)V.width + px;
  return px < (uint32_t)V.width && py < (uint32_t)V.height;
}

// The whole walk of each lane's ray through the cells, for the persistent kernel: a closest-hit
// ray until its first hit (st.best_id, st.tbest) or the grid's exit, a shadow ray until an opaque
// triangle blocks it (st.blocked) or it leaves the grid, its glass crossings recorded at slot
// `slot` (st.ncross). The lanes of a wave step together, one BVH node or triangle each per
// iteration, until every lane is done; lanes with go false only join the loop. Cells are entered
// in the half-open slab intervals of the traversal kernel, the first one from t > 0.
__device__ __forceinline__ void walk_ray(const DevScene& S, const DevWS& w, const float* s_planes, const int4* s_cells,
                                         bool cells_lds, bool go, const RayPre& R, bool shadow, uint32_t skip,
                                         uint32_t cell0, uint32_t slot, uint32_t* stack, uint32_t* spill,
                                         TraceState& st, uint32_t& n_visit, uint32_t& n_nodes, uint32_t& n_tris,
                                         uint32_t& n_cross) {
  int phase = go && cell0 != kInvalidCell ? kLaneEnter : kLaneDone;
  uint32_t cpos = 0;
  if (phase == kLaneEnter)
    cpos = (cell0 % (uint32_t)S.gx) | ((cell0 / (uint32_t)S.gx) % (uint32_t)S.gy) << 6 |
           (cell0 / (uint32_t)(S.gx * S.gy)) << 12;
  bool first = true;
  float t_lo = 0.0f, tf = 0.0f;
  int4 cinfo = make_int4(0, 0, 0, 0);
  uint32_t node = 0, pend = 0;
  int sp = 0;
  for (;;) {
    if (__ballot(phase != kLaneDone) == 0) break;
    int work = kStepNone;
    n_visit += (uint32_t)__popcll(__ballot(phase == kLaneEnter));
    if (phase == kLaneEnter) {
      float tn;
      const int ix = (int)(cpos & 63u), iy = (int)((cpos >> 6) & 63u), iz = (int)((cpos >> 12) & 63u);
      const int cell = (int)cpos_cell(S, cpos);
      int axis;
      cell_interval_pl(s_planes, S.gx, S.gy, ix, iy, iz, R.o, R.inv, tn, tf, axis);
      cpos = (cpos & ~(3u << 26)) | (uint32_t)axis << 26;
      t_lo = first ? -INFINITY : tn;
      if (cells_lds) {
        const __attribute__((address_space(3))) int* c = (const __attribute__((address_space(3))) int*)s_cells + 4 * cell;
        cinfo = make_int4(c[0], c[1], c[2], c[3]);
      } else {
        const __attribute__((address_space(1))) int* c = (const __attribute__((address_space(1))) int*)S.cells + 4 * cell;
        cinfo = make_int4(c[0], c[1], c[2], c[3]);
      }
      if (cinfo.y > 0 && t_lo < tf) {
        if (!shadow) st.tbest = tf;
        node = 0;
        sp = 0;
        pend = 0;
        phase = kLaneTrav;
      } else {
        phase = kLaneLeave;
      }
    }
    if (phase == kLaneTrav) {
      if (!trav_step(S, w, R, shadow, cinfo, stack, spill, w.trace_threads, skip, t_lo, tf, slot, st, node, sp, pend,
                     work))
        phase = (shadow && st.blocked) || (!shadow && st.best_id != 0xFFFFFFFFu) ? kLaneDone : kLaneLeave;
    }
    if (phase == kLaneLeave) {
      const int axis = (int)((cpos >> 26) & 3u);
      const float dc = comp(R.inv, axis);
      const int g = axis == 0 ? S.gx : (axis == 1 ? S.gy : S.gz);
      const int ni = (int)((cpos >> (6 * axis)) & 63u) + (dc > 0.0f ? 1 : -1);
      if (ni < 0 || ni >= g || !(tf < INFINITY)) {
        phase = kLaneDone;
      } else {
        cpos = (cpos & ~(63u << (6 * axis))) | ((uint32_t)ni << (6 * axis));
        first = false;
        phase = kLaneEnter;
      }
    }
    n_nodes += (uint32_t)__popcll(__ballot(work == kStepNode));
    n_tris += (uint32_t)__popcll(__ballot(work >= kStepTri));
    n_cross += (uint32_t)__popcll(__ballot(work == kStepCross));
  }
}

// One persistent kernel renders a batch of views. Each lane carries one path at a time through
// all its vertices with the arithmetic of the wavefront kernels (same random-number counters,
// lobe rules, Fresnel and slab factors, hit re-evaluation), its spectral rows in the workspace
// slot of its thread; a lane whose path ends adds the path's radiance / spp to its pixel
// (atomics: other samples of the pixel may be in flight) and takes the next item of the work
// list, so the wave's lanes stay busy until the list is exhausted. A loop iteration traces each
// lane's current ray (extension or shadow) through the cells, then shades: at an opaque vertex
// the direct-term weight and the continuation are computed, the shadow ray is traced in the next
// iteration and the continuation after it; at glass the continuation directly.
// Four waves per SIMD (128 registers, a little spilled): measured faster than three (161 registers,
// none spilled) and five on the church frame.
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) void k_persist(DevScene S, DevWS w, uint64_t total, uint32_t key0, uint32_t key1,
                                                 int max_depth) {
  __shared__ uint32_t s_stack[kShortStack * kWG];
  __shared__ float s_planes[3 * (kMaxGrid + 1)];
  __shared__ int4 s_cells[kLdsCells];
  __shared__ uint32_t s_st[10];
  const int n_planes = S.gx + S.gy + S.gz + 3;
  const bool cells_lds = S.n_cells <= kLdsCells;
  for (int q = threadIdx.x; q < n_planes; q += kWG) s_planes[q] = S.planes[q];
  if (cells_lds)
    for (int q = threadIdx.x; q < S.n_cells; q += kWG) s_cells[q] = S.cells[q];
  stats_init(s_st, 10);
  __syncthreads();
  const uint32_t slot = blockIdx.x * kWG + threadIdx.x;
  uint32_t* stack = s_stack + threadIdx.x;
  uint32_t* spill = w.spill + slot;
  const int B = S.n_bins, Bp = w.Bp, nq = Bp / 4;
  float4* b4 = (float4*)(w.beta + (size_t)slot * Bp);
  float4* e4 = (float4*)(w.nee + (size_t)slot * Bp);
  float4* l4 = (float4*)(w.lacc + (size_t)slot * Bp);
  const F3 ws = f3(S.sun[0], S.sun[1], S.sun[2]);
  const size_t W = w.W;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint64_t n_chunks = (total + kPersistChunk - 1) / kPersistChunk;
  uint32_t donor = 0;      // ranges of the work list this wave has exhausted (wave-uniform)
  uint64_t cb = 0, ce = 0; // items of the wave's current chunk not yet handed out (wave-uniform)
  bool active = false;     // the lane carries a path
  uint32_t view = 0, pix = 0, smp = 0;
  int depth = 0;           // surface vertices of the path so far
  bool shadow = false;     // the lane's current ray is a shadow ray
  bool cont = false;       // a continuation ray waits behind the shadow ray
  F3 ro = f3(0.0f, 0.0f, 0.0f), rd = ro, co = ro, cd = ro;
  uint32_t skip = 0, cskip = 0;
  uint32_t n_visit = 0, n_nodes = 0, n_tris = 0, n_cross = 0, n_bad = 0;
  for (;;) {
    // idle lanes take the next items of the work list, in lane order
    for (;;) {
      const uint64_t idle = __ballot(!active);
      if (idle == 0) break;
      if (cb == ce) {
        bool got = false;
        for (; donor < (uint32_t)kXcds; ++donor) {
          const uint32_t X = (xcd + donor) % kXcds;
          const uint64_t b = n_chunks * X / kXcds, e = n_chunks * (X + 1) / kXcds;
          uint32_t q = 0;
          if (lane_id() == 0) q = atomicAdd(&w.ctl->tile_next[X * kKeyStride], 1u);
          q = __builtin_amdgcn_readfirstlane(q);
          if (b + q < e) {
            cb = (b + q) * kPersistChunk;
            ce = min(total, cb + kPersistChunk);
            got = true;
            break;
          }
        }
        if (!got) break;
      }
      const uint32_t rank = count_below(idle);
      const uint64_t take = min((uint64_t)__popcll(idle), ce - cb);
      bool started = false;
      if (!active && rank < take) {
        uint32_t v, px, sm;
        if (persist_item(w, cb + rank, v, px, sm)) {
          // camera ray (vertex 0), as in ray generation
          view = v;
          pix = px;
          smp = sm;
          const ViewDesc& V = w.views[v];
          const uint32_t x = pix % (uint32_t)V.width, y = pix / (uint32_t)V.width;
          const uint4 rn = philox(make_uint4(pix, smp, 0u, V.view_id), key0, key1);
          const float sx = 2.0f * ((float)x + unif24(rn.x)) / (float)V.width - 1.0f;
          const float sy = 1.0f - 2.0f * ((float)y + unif24(rn.y)) / (float)V.height;
          const F3 fw = f3(V.fwd[0], V.fwd[1], V.fwd[2]);
          const F3 rt = f3(V.right[0], V.right[1], V.right[2]);
          const F3 up = f3(V.upv[0], V.upv[1], V.upv[2]);
          rd = norm3(fw + rt * sx + up * sy);
          ro = f3(V.eye[0], V.eye[1], V.eye[2]);
          skip = 0xFFFFFFFFu;
          shadow = false;
          cont = false;
          depth = 0;
          for (int q = 0; q < nq; ++q) {
            b4[q] = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
            l4[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          }
          active = true;
          started = true;
        }
      }
      stats_add_ballot(s_st, 0, started);
      cb += take;
    }
    if (__ballot(active) == 0) break;  // the list is exhausted and every path has ended
    // trace every lane's current ray through the cells
    const RayPre R = make_pre(ro, rd);
    const uint32_t cell0 = active ? start_cell_pl(S, s_planes, ro, rd) : kInvalidCell;
    TraceState st;
    st.tbest = INFINITY;
    st.best_id = 0xFFFFFFFFu;
    st.blocked = false;
    st.ncross = 0;
    walk_ray(S, w, s_planes, s_cells, cells_lds, active, R, shadow, skip, cell0, slot, stack, spill, st, n_visit,
             n_nodes, n_tris, n_cross);
    stats_add_ballot(s_st, 1, active && !shadow);
    stats_add_ballot(s_st, 2, active && shadow);
    bool done = false, escaped = false, shaded = false, overflow = false;
    if (active) {
      if (shadow) {
        // the direct term of the vertex, through the glass it crossed, unless an opaque triangle
        // blocked the way to the sun
        if (!st.blocked) {
          overflow = st.ncross > (uint32_t)kMaxCross;
          add_direct_seq(S, w, slot, min(st.ncross, (uint32_t)kMaxCross));
        }
        if (cont) {
          ro = co;
          rd = cd;
          skip = cskip;
          shadow = false;
          cont = false;
        } else {
          done = true;
        }
      } else if (st.best_id == 0xFFFFFFFFu) {
        // the path leaves the scene: environment radiance
        if (S.env_nonzero) {
          const float4* env = (const float4*)S.env;
          row_update<4>(l4, nq, [&](int q, float4 l) {
            const float4 a = b4[q], e = env[q];
            return make_float4(l.x + a.x * e.x, l.y + a.y * e.y, l.z + a.z * e.z, l.w + a.w * e.w);
          });
        }
        escaped = true;
        done = true;
      } else {
        ++depth;
        const Vertex V = make_vertex(S, ro, rd, st.best_id, st.tbest);
        const uint4 rn = philox(make_uint4(pix, smp, (uint32_t)depth, w.views[view].view_id), key0, key1);
        const float u0 = unif24(rn.x), u1 = unif24(rn.y), u2 = unif24(rn.z);
        const float4* nt = (const float4*)(S.ntab + V.m * Bp);
        const float4* kt = (const float4*)(S.ktab + V.m * Bp);
        shaded = S.mtype[V.m] == 0 || depth < max_depth;  // glass at the last vertex ends the path unshaded
        if (S.mtype[V.m] != 0) {
          // glass: thin slab, reflect or transmit straight through; no direct term
          if (depth < max_depth) {
            const float4* lam = (const float4*)S.lambda;
            const float th = S.thick[V.m];
            const int tx = S.n_tex > 0 ? S.mtex[V.m] : -1;
            TexTap tap;
            tap.base = nullptr;
            tap.r00 = tap.r10 = tap.r01 = tap.r11 = 0;
            tap.fx = tap.fy = 0.0f;
            if (tx >= 0) {
              float ss, tt;
              hit_st(S, V.id, V.bu, V.bv, ss, tt);
              tap = tex_tap(S, tx, ss, tt);
            }
            auto slab4 = [&](int q, float (&Rr)[4], float (&Tt)[4]) {
              const float4 nn = nt[q], kk = kt[q], la = lam[q];
              if (tx >= 0) {
                const float4 t4 = tex_quad(tap, q);
                slab_tau0(nn.x, kk.x, t4.x, V.cos_o, Rr[0], Tt[0]);
                slab_tau0(nn.y, kk.y, t4.y, V.cos_o, Rr[1], Tt[1]);
                slab_tau0(nn.z, kk.z, t4.z, V.cos_o, Rr[2], Tt[2]);
                slab_tau0(nn.w, kk.w, t4.w, V.cos_o, Rr[3], Tt[3]);
              } else {
                slab(nn.x, kk.x, la.x, th, V.cos_o, Rr[0], Tt[0]);
                slab(nn.y, kk.y, la.y, th, V.cos_o, Rr[1], Tt[1]);
                slab(nn.z, kk.z, la.z, th, V.cos_o, Rr[2], Tt[2]);
                slab(nn.w, kk.w, la.w, th, V.cos_o, Rr[3], Tt[3]);
              }
            };
            float mr = 0.0f, mt = 0.0f;
            for (int q = 0; q < nq; ++q) {
              float Rr[4], Tt[4];
              slab4(q, Rr, Tt);
#pragma unroll
              for (int c = 0; c < 4; ++c)
                if (4 * q + c < B) {
                  mr += Rr[c];
                  mt += Tt[c];
                }
            }
            const float Pr = mr / (mr + mt);
            const bool refl = u0 < Pr;
            const float inv_p = refl ? 1.0f / Pr : 1.0f / (1.0f - Pr);
            row_update<2>(b4, nq, [&](int q, float4 b) {
              float Rr[4], Tt[4];
              slab4(q, Rr, Tt);
              return make_float4(b.x * ((refl ? Rr[0] : Tt[0]) * inv_p), b.y * ((refl ? Rr[1] : Tt[1]) * inv_p),
                                 b.z * ((refl ? Rr[2] : Tt[2]) * inv_p), b.w * ((refl ? Rr[3] : Tt[3]) * inv_p));
            });
            rd = refl ? V.d - V.ng * (2.0f * V.dn) : V.d;
            ro = refl ? V.p + V.n * V.eps : V.p - V.n * V.eps;
            skip = V.id;
          } else {
            done = true;
          }
        } else {
          // opaque: direct term toward the sun (a shadow ray), Fresnel-split lobe choice
          const float4* rt = (const float4*)(S.rho + V.m * Bp);
          const float4* E4 = (const float4*)S.sunE;
          const float cs = dot_exact_sign(V.n, ws);
          const bool nee = cs > 0.0f;
          const float kn = cs * (1.0f / 3.14159265358979f);
          float a_sum = 0.0f, b_sum = 0.0f;
          row_write<2>(e4, nq, nee, [&](int q) {
            const float4 nn = nt[q], kk = kt[q], rr = rt[q];
            const float F[4] = {fresnel(nn.x, kk.x, V.cos_o), fresnel(nn.y, kk.y, V.cos_o),
                                fresnel(nn.z, kk.z, V.cos_o), fresnel(nn.w, kk.w, V.cos_o)};
            const float rho[4] = {rr.x, rr.y, rr.z, rr.w};
            float dif[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              dif[c] = (1.0f - F[c]) * rho[c];
              if (4 * q + c < B) {
                a_sum += F[c];
                b_sum += dif[c];
              }
            }
            float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (nee) {
              const float4 bb = b4[q], EE = E4[q];
              out = make_float4(bb.x * dif[0] * kn * EE.x, bb.y * dif[1] * kn * EE.y, bb.z * dif[2] * kn * EE.z,
                                bb.w * dif[3] * kn * EE.w);
            }
            return out;
          });
          const float am = a_sum / (float)B, bm = b_sum / (float)B;
          bool go_on = depth < max_depth && am + bm > 0.0f;
          bool mirror = false;
          float inv_p = 0.0f;
          if (go_on) {
            const float Ps = am / (am + bm);
            mirror = u0 < Ps;
            inv_p = mirror ? 1.0f / Ps : 1.0f / (1.0f - Ps);
            row_update<2>(b4, nq, [&](int q, float4 bb) {
              const float4 nn = nt[q], kk = kt[q], rr = rt[q];
              const float F0 = fresnel(nn.x, kk.x, V.cos_o), F1 = fresnel(nn.y, kk.y, V.cos_o),
                          F2 = fresnel(nn.z, kk.z, V.cos_o), F3v = fresnel(nn.w, kk.w, V.cos_o);
              bb.x *= (mirror ? F0 : (1.0f - F0) * rr.x) * inv_p;
              bb.y *= (mirror ? F1 : (1.0f - F1) * rr.y) * inv_p;
              bb.z *= (mirror ? F2 : (1.0f - F2) * rr.z) * inv_p;
              bb.w *= (mirror ? F3v : (1.0f - F3v) * rr.w) * inv_p;
              return bb;
            });
            F3 nd;
            if (mirror) {
              nd = V.d - V.ng * (2.0f * V.dn);
            } else {
              float sn, cn;
              sincosf(2.0f * 3.14159265358979f * u1, &sn, &cn);
              const float rr = sqrtf(u2);
              const float lx = rr * cn, ly = rr * sn, lz = sqrtf(fmaxf(0.0f, 1.0f - u2));
              const F3 nrm = V.n;
              const float sg = copysignf(1.0f, nrm.z);
              const float aa = -1.0f / (sg + nrm.z);
              const float bb = nrm.x * nrm.y * aa;
              const F3 t1 = f3(1.0f + sg * nrm.x * nrm.x * aa, sg * bb, -sg * nrm.x);
              const F3 t2 = f3(bb, sg + nrm.y * nrm.y * aa, -nrm.y);
              nd = t1 * lx + t2 * ly + nrm * lz;
            }
            co = V.p + V.n * V.eps;
            cd = nd;
            cskip = V.id;
          }
          if (nee) {
            // the shadow ray first (its record in the workspace serves the glass crossings), then
            // the continuation
            ro = V.p + V.n * V.eps;
            rd = ws;
            skip = V.id;
            shadow = true;
            cont = go_on;
            w.rays[2 * (W + slot)] = make_float4(ro.x, ro.y, ro.z, __uint_as_float(V.id));
            w.rays[2 * (W + slot) + 1] = make_float4(ws.x, ws.y, ws.z, __uint_as_float(slot | kShadowBit));
          } else if (go_on) {
            ro = co;
            rd = cd;
            skip = cskip;
          } else {
            done = true;
          }
        }
      }
    }
    stats_add_ballot(s_st, 3, escaped);
    stats_add_ballot(s_st, 4, shaded);
    stats_add_ballot(s_st, 8, overflow);
    if (done) {
      // the path's radiance / spp into its pixel
      const ViewDesc& V = w.views[view];
      const size_t plane = (size_t)V.width * V.height;
      float* img = V.image + pix;
      for (int q = 0; q < nq; ++q) {
        const float4 l = l4[q];
        const float c4[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 4 * q + e;
          const float c = c4[e] * V.inv_spp;
          n_bad += (j < B && !isfinite(c)) ? 1u : 0u;
          if (j < B && c != 0.0f) unsafeAtomicAdd(img + (size_t)j * plane, c);
        }
      }
      active = false;
    }
  }
  stats_add(s_st, 5, n_visit);
  stats_add(s_st, 6, n_nodes);
  stats_add(s_st, 7, n_tris);
  stats_add(s_st, 9, n_cross);
  wave_add(&w.ctl->err_nonfinite, n_bad);
  __syncthreads();
  stats_flush(s_st, 0, &w.ctl->st_paths);
  stats_flush(s_st, 1, &w.ctl->st_ext);
  stats_flush(s_st, 2, &w.ctl->st_shadow);
  stats_flush(s_st, 3, &w.ctl->st_escape);
  stats_flush(s_st, 4, &w.ctl->st_vertices);
  stats_flush(s_st, 5, &w.ctl->st_visits);
  stats_flush(s_st, 6, &w.ctl->st_nodes);
  stats_flush(s_st, 7, &w.ctl->st_tris);
  stats_flush(s_st, 8, &w.ctl->err_cross);
  stats_flush(s_st, 9, &w.ctl->st_glass);
}

// ==========================================================================================
// host-side launchers
// ==========================================================================================
// ==========================================================================================
// caustic photon map (section 4: photon maps filled from the light sources, one for caustics)
// ==========================================================================================
// Photon i of the map: random-number counter (i, i >> 32, vertex | 4 << 24, 0) -- purpose 4. The
// slot's pix / smp words hold the photon index, its view word the photon's flags (bit 0: it has
// been reflected, by a glass face or a mirror lobe).
constexpr uint32_t kPhotonPurpose = 4u << 24;
constexpr uint32_t kPhotonReflected = 1u;

// Emission: the window (glass triangle) whose integer threshold is the last not above the 24-bit
// random integer, a uniform point p on it, flux E_j A / N; the photon's first vertex is p (its
// ray from p + w_s toward -w_s, hit record at distance 1 on that triangle), and its incoming
// visibility is a shadow ray from p toward the sun, offset to the sun's side and skipping the
// window, queued like any shadow ray.
__global__ __launch_bounds__(kWG) void k_photon_gen(DevScene S, DevWS w, PhotonDev P, uint64_t k0, uint32_t n,
                                                    int gen) {
  __shared__ float s_planes[3 * (kMaxGrid + 1)];
  for (int q = threadIdx.x; q < S.gx + S.gy + S.gz + 3; q += kWG) s_planes[q] = S.planes[q];
  __syncthreads();
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  const bool valid = i < n;
  uint32_t cell = kInvalidCell, qdir = 0, xo = 0;
  if (valid) {
    const uint64_t id = k0 + i;
    const uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32);
    const uint4 rn = philox(make_uint4(c0, c1, kPhotonPurpose, 0u), P.seed_lo, P.seed_hi);
    const uint32_t x24 = rn.x >> 8;
    uint32_t lo = 0, hi = P.n_win;  // the last window whose threshold <= x24 (thr[0] = 0)
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (P.win_thr[mid] <= x24) lo = mid; else hi = mid;
    }
    const uint32_t tri = P.win_tri[lo];
    const float4* g = S.gtris + (size_t)tri * 3;
    const float4 A = g[0], B = g[1], C = g[2];
    const F3 v0 = f3(A.x, A.y, A.z), v1 = f3(B.x, B.y, B.z), v2 = f3(C.x, C.y, C.z);
    const float r = sqrtf(unif24(rn.y)), u2 = unif24(rn.z);
    const float bu = r * (1.0f - u2), bv = r * u2;
    const F3 p = v0 * (1.0f - bu - bv) + v1 * bu + v2 * bv;
    const F3 sun = f3(S.sun[0], S.sun[1], S.sun[2]);
    const F3 d = sun * -1.0f;
    const F3 o1 = p + sun;
    w.rays[2 * i] = make_float4(o1.x, o1.y, o1.z, __int_as_float(-1));
    w.rays[2 * i + 1] = make_float4(d.x, d.y, d.z, __uint_as_float(i));
    w.hit[i] = make_float4(1.0f, __uint_as_float(tri), 0.0f, 0.0f);
    const F3 ng = geo_normal(v0, v1, v2);
    const F3 nn = dot_exact_sign(d, ng) > 0.0f ? ng * -1.0f : ng;
    const F3 so = p + nn * (1e-5f * (1.0f + maxabs3(p)));
    w.rays[2 * ((size_t)w.W + i)] = make_float4(so.x, so.y, so.z, __uint_as_float(tri));
    w.rays[2 * ((size_t)w.W + i) + 1] = make_float4(sun.x, sun.y, sun.z, __uint_as_float(i | kShadowBit));
    w.shcnt[i] = 0;
    w.pix[i] = c0;
    w.smp[i] = c1;
    w.view[i] = 0;
    float4* b4 = (float4*)(w.beta + (size_t)i * w.Bp);
    const float4* e4 = (const float4*)S.sunE;
    for (int q = 0; q < w.Bp / 4; ++q) {
      const float4 e = e4[q];
      b4[q] = make_float4(e.x * P.flux_scale, e.y * P.flux_scale, e.z * P.flux_scale, e.w * P.flux_scale);
    }
    cell = start_cell_pl(S, s_planes, so, sun, &xo);
    qdir = dir_code(sun);
  }
  const int gp = gen & 1;
  const bool in_grid = valid && cell != kInvalidCell;
  const uint32_t key = in_grid ? qsub(w, cell, qdir, xo) : kNoKey;
  const uint32_t rank = wave_key_rank(in_grid, key, ccount_of(S, w, gp), w);
  if (valid) {
    w.lsrc[i] = (w.W + i) | kFirstVisit;
    w.ldst[i] = key;
    w.lrank[i] = rank;
    // a shadow ray that starts outside the grid reaches the sun at once
    if (!in_grid) w.catb[(size_t)w.W + i] = (uint8_t)(kCatShadowClear + 1);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctl->list_count[gp] = n;
}

// Incoming visibility of the photons: blocked ones are gone; through glass the flux takes the
// slabs' transmittance. The live photons become the glass vertices of the first bounce.
__global__ __launch_bounds__(kWG) void k_photon_vis(DevScene S, DevWS w, PhotonDev P, int par) {
  const uint32_t n_clear = w.ctl->cat_count[par][kCatShadowClear * kKeyStride];
  const uint32_t n_glass = w.ctl->cat_count[par][kCatShadowGlass * kKeyStride];
  const uint32_t n = n_clear + n_glass;
  const int Bp = w.Bp, nq = Bp / 4;
  if (blockIdx.x == 0 && threadIdx.x < kCats) w.ctl->cat_count[par ^ 1][threadIdx.x * kKeyStride] = 0;
  const uint32_t n_iter = (n + kWG - 1) / kWG * kWG;
  for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < n_iter; i += gridDim.x * kWG) {
    const bool valid = i < n;
    uint32_t s = 0;
    if (valid && i >= n_clear) {
      s = cat_list(w, par, kCatShadowGlass)[i - n_clear];
      const uint32_t nc = min(w.shcnt[s], (uint32_t)kMaxCross);
      int mq[kMaxCross], tx[kMaxCross];
      float cq[kMaxCross], sq[kMaxCross], tq[kMaxCross];
      crossings(S, w, s, nc, mq, cq, tx, sq, tq);
      const float4* lam = (const float4*)S.lambda;
      row_update<12>((float4*)(w.beta + (size_t)s * Bp), nq, [&](int q, float4 b) {
        const float4 la = lam[q];
        for (int c = 0; c < kMaxCross; ++c) {
          if ((uint32_t)c < nc) {
            const int m = mq[c];
            const float4 nn = ((const float4*)(S.ntab + m * Bp))[q], kk = ((const float4*)(S.ktab + m * Bp))[q];
            float R0, T0, R1, T1, R2, T2, R3, T3;
            if (tx[c] >= 0) {
              const float4 t4 = tex_quad(tex_tap(S, tx[c], sq[c], tq[c]), q);
              slab_tau0(nn.x, kk.x, t4.x, cq[c], R0, T0);
              slab_tau0(nn.y, kk.y, t4.y, cq[c], R1, T1);
              slab_tau0(nn.z, kk.z, t4.z, cq[c], R2, T2);
              slab_tau0(nn.w, kk.w, t4.w, cq[c], R3, T3);
            } else {
              slab(nn.x, kk.x, la.x, S.thick[m], cq[c], R0, T0);
              slab(nn.y, kk.y, la.y, S.thick[m], cq[c], R1, T1);
              slab(nn.z, kk.z, la.z, S.thick[m], cq[c], R2, T2);
              slab(nn.w, kk.w, la.w, S.thick[m], cq[c], R3, T3);
            }
            b = make_float4(b.x * T0, b.y * T1, b.z * T2, b.w * T3);
          }
        }
        return b;
      });
    } else if (valid) {
      s = cat_list(w, par, kCatShadowClear)[i];
    }
    wave_push(valid, s, &w.ctl->cat_count[par][kCatGlass * kKeyStride], cat_list(w, par, kCatGlass));
  }
}

// One photon vertex per thread, opaque vertices first (produced entries 0 .. n_opaque), then glass
// (n_opaque .. n_opaque + n_glass): the same lobe rules as camera paths, no direct term. An opaque
// vertex of a caustic map stores the photon when it has been reflected before, then takes the
// mirror lobe or ends (a diffuse bounce leaves the caustic paths); one of a global map stores every
// photon and continues it by either lobe. Vertex max_depth scatters nothing.
__global__ __launch_bounds__(kWG) void k_photon_shade(DevScene S, DevWS w, PhotonDev P, int depth, int gen) {
  __shared__ float s_planes[3 * (kMaxGrid + 1)];
  for (int q = threadIdx.x; q < S.gx + S.gy + S.gz + 3; q += kWG) s_planes[q] = S.planes[q];
  __syncthreads();
  const int p = depth & 1, gp = gen & 1;
  const uint32_t n_op = w.ctl->cat_count[p][kCatOpaque * kKeyStride];
  const uint32_t n_gl = w.ctl->cat_count[p][kCatGlass * kKeyStride];
  const uint32_t n = n_op + n_gl;
  const int B = S.n_bins, Bp = w.Bp, nq = Bp / 4;
  if (blockIdx.x == 0 && threadIdx.x == 0) w.ctl->list_count[gp] = n;
  if (blockIdx.x == 0 && threadIdx.x < kCats) w.ctl->cat_count[p ^ 1][threadIdx.x * kKeyStride] = 0;
  const bool last = depth >= P.max_depth;
  const uint32_t n_iter = (n + kWG - 1) / kWG * kWG;
  for (uint32_t a = blockIdx.x * kWG + threadIdx.x; a < n_iter; a += gridDim.x * kWG) {
    const bool valid = a < n;
    uint32_t s = 0, cell = kInvalidCell, qd = 0, xo = 0;
    if (valid) {
      const bool opaque = a < n_op;
      s = opaque ? cat_list(w, p, kCatOpaque)[a] : cat_list(w, p, kCatGlass)[a - n_op];
      const Vertex V = load_vertex(S, w, s);
      const uint32_t flags = w.view[s];
      const uint4 rn = philox(make_uint4(w.pix[s], w.smp[s], (uint32_t)depth | kPhotonPurpose, 0u), P.seed_lo,
                              P.seed_hi);
      const float u0 = unif24(rn.x);
      float4* brow = (float4*)(w.beta + (size_t)s * Bp);
      const float4* nt = (const float4*)(S.ntab + V.m * Bp);
      const float4* kt = (const float4*)(S.ktab + V.m * Bp);
      bool cont = false, refl = false, diffuse = false;
      F3 diff_dir = f3(0.0f, 0.0f, 1.0f);
      if (opaque) {
        // the photons stored by the wave's active lanes take consecutive records (one atomic per
        // wave); the flux is the throughput on arrival, before this vertex's lobe
        const bool store = P.global || (flags & kPhotonReflected) != 0;
        const uint64_t m = __ballot(store);
        if (m) {
          const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
          uint32_t base = 0;
          if (lane_id() == leader) base = atomicAdd(&P.ctl[0], (uint32_t)__popcll(m));
          base = __builtin_amdgcn_readlane(base, (int)leader);
          const uint32_t r = base + count_below(m);
          const uint64_t lost = __ballot(store && r >= P.cap);
          if (lost && lane_id() == leader) atomicAdd(&P.ctl[1], (uint32_t)__popcll(lost));
          if (store && r < P.cap) {
            float4* rec = P.rec + (size_t)r * P.rq;
            rec[0] = make_float4(V.p.x, V.p.y, V.p.z, __uint_as_float(w.pix[s]));
            rec[1] = make_float4(V.d.x, V.d.y, V.d.z, __uint_as_float((uint32_t)depth | (w.smp[s] << 8)));
            for (int q = 0; q < nq; ++q) rec[2 + q] = brow[q];
          }
        }
        if (!last) {
          const float4* rt = (const float4*)(S.rho + V.m * Bp);
          float a_ = 0.0f, b_ = 0.0f;
          for (int q = 0; q < nq; ++q) {
            const float4 nn = nt[q], kk = kt[q], rr = rt[q];
            const float F4[4] = {fresnel(nn.x, kk.x, V.cos_o), fresnel(nn.y, kk.y, V.cos_o),
                                 fresnel(nn.z, kk.z, V.cos_o), fresnel(nn.w, kk.w, V.cos_o)};
            const float R4[4] = {rr.x, rr.y, rr.z, rr.w};
            for (int c = 0; c < 4; ++c)
              if (4 * q + c < B) {
                a_ += F4[c];
                b_ += (1.0f - F4[c]) * R4[c];
              }
          }
          a_ /= (float)B;
          b_ /= (float)B;
          if (a_ + b_ > 0.0f) {
            const float Ps = a_ / (a_ + b_);
            if (u0 < Ps) {
              const float inv = 1.0f / Ps;
              row_update<8>(brow, nq, [&](int q, float4 b) {
                const float4 nn = nt[q], kk = kt[q];
                return make_float4(b.x * fresnel(nn.x, kk.x, V.cos_o) * inv, b.y * fresnel(nn.y, kk.y, V.cos_o) * inv,
                                   b.z * fresnel(nn.z, kk.z, V.cos_o) * inv, b.w * fresnel(nn.w, kk.w, V.cos_o) * inv);
              });
              cont = refl = true;
            } else if (P.global) {
              // diffuse lobe (cosine-weighted, as for camera paths); its Fresnel factor is that of
              // the direction the light leaves in, here the photon's new direction (cos = lz)
              const float u1 = unif24(rn.y), u2 = unif24(rn.z);
              float sn, cn;
              sincosf(2.0f * 3.14159265358979f * u1, &sn, &cn);
              const float rr_ = sqrtf(u2);
              const float lx = rr_ * cn, ly = rr_ * sn, lz = sqrtf(fmaxf(0.0f, 1.0f - u2));
              const F3 nrm = V.n;
              const float sg = copysignf(1.0f, nrm.z);
              const float aa = -1.0f / (sg + nrm.z);
              const float bb = nrm.x * nrm.y * aa;
              const F3 t1 = f3(1.0f + sg * nrm.x * nrm.x * aa, sg * bb, -sg * nrm.x);
              const F3 t2 = f3(bb, sg + nrm.y * nrm.y * aa, -nrm.y);
              diff_dir = t1 * lx + t2 * ly + nrm * lz;
              const float inv = 1.0f / (1.0f - Ps);
              const float4* rt = (const float4*)(S.rho + V.m * Bp);
              row_update<8>(brow, nq, [&](int q, float4 b) {
                const float4 nn = nt[q], kk = kt[q], rr = rt[q];
                return make_float4(b.x * ((1.0f - fresnel(nn.x, kk.x, lz)) * rr.x * inv),
                                   b.y * ((1.0f - fresnel(nn.y, kk.y, lz)) * rr.y * inv),
                                   b.z * ((1.0f - fresnel(nn.z, kk.z, lz)) * rr.z * inv),
                                   b.w * ((1.0f - fresnel(nn.w, kk.w, lz)) * rr.w * inv));
              });
              cont = diffuse = true;
            }
          }
        }
      } else if (!last) {
        const float4* lam = (const float4*)S.lambda;
        const float th = S.thick[V.m];
        const int tx = S.n_tex > 0 ? S.mtex[V.m] : -1;
        TexTap tap;
        tap.base = nullptr;
        tap.r00 = tap.r10 = tap.r01 = tap.r11 = 0;
        tap.fx = tap.fy = 0.0f;
        if (tx >= 0) {
          float ss, tt;
          hit_st(S, V.id, V.bu, V.bv, ss, tt);
          tap = tex_tap(S, tx, ss, tt);
        }
        auto slab4 = [&](int q, float (&R)[4], float (&T)[4]) {
          const float4 nn = nt[q], kk = kt[q], la = lam[q];
          if (tx >= 0) {
            const float4 t4 = tex_quad(tap, q);
            slab_tau0(nn.x, kk.x, t4.x, V.cos_o, R[0], T[0]);
            slab_tau0(nn.y, kk.y, t4.y, V.cos_o, R[1], T[1]);
            slab_tau0(nn.z, kk.z, t4.z, V.cos_o, R[2], T[2]);
            slab_tau0(nn.w, kk.w, t4.w, V.cos_o, R[3], T[3]);
          } else {
            slab(nn.x, kk.x, la.x, th, V.cos_o, R[0], T[0]);
            slab(nn.y, kk.y, la.y, th, V.cos_o, R[1], T[1]);
            slab(nn.z, kk.z, la.z, th, V.cos_o, R[2], T[2]);
            slab(nn.w, kk.w, la.w, th, V.cos_o, R[3], T[3]);
          }
        };
        float mr = 0.0f, mt = 0.0f;
        for (int q = 0; q < nq; ++q) {
          float R[4], T[4];
          slab4(q, R, T);
          for (int c = 0; c < 4; ++c)
            if (4 * q + c < B) {
              mr += R[c];
              mt += T[c];
            }
        }
        const float Pr = mr / (mr + mt);
        refl = u0 < Pr;
        const float inv = refl ? 1.0f / Pr : 1.0f / (1.0f - Pr);
        row_update<8>(brow, nq, [&](int q, float4 b) {
          float R[4], T[4];
          slab4(q, R, T);
          return make_float4(b.x * ((refl ? R[0] : T[0]) * inv), b.y * ((refl ? R[1] : T[1]) * inv),
                             b.z * ((refl ? R[2] : T[2]) * inv), b.w * ((refl ? R[3] : T[3]) * inv));
        });
        cont = true;
      }
      if (cont) {
        const F3 nd = diffuse ? diff_dir : (refl ? V.d - V.ng * (2.0f * V.dn) : V.d);
        const F3 no = (refl || diffuse) ? V.p + V.n * V.eps : V.p - V.n * V.eps;
        w.rays[2 * s] = make_float4(no.x, no.y, no.z, __uint_as_float(V.id));
        w.rays[2 * s + 1] = make_float4(nd.x, nd.y, nd.z, __uint_as_float(s));
        if (refl) w.view[s] = flags | kPhotonReflected;
        cell = start_cell_pl(S, s_planes, no, nd, &xo);
        qd = dir_code(nd);
      }
    }
    const bool ve = valid && cell != kInvalidCell;
    const uint32_t ke = ve ? qsub(w, cell, qd, xo) : kNoKey;
    const uint32_t re = wave_key_rank(ve, ke, ccount_of(S, w, gp), w);
    if (valid) {
      w.lsrc[a] = s | kFirstVisit;
      w.ldst[a] = ke;
      w.lrank[a] = re;
    }
  }
}

// Uniform grid over the stored photons with cells of the gather radius r: a gather ball meets
// the 3 x 3 x 3 block of cells around its centre's cell, of which only those whose box lies
// closer than r to the centre are read. Cell (i, j, k) goes to the bucket whose low 6 bits are
// (i mod 4, j mod 4, k mod 4), so the 27 cells of one block are 27 distinct buckets, and whose
// high bits are the spatial hash of Teschner et al. (2003) of the 4 x 4 x 4 super-cell
// (i >> 2, j >> 2, k >> 2), which spreads the occupied super-cells over the table; cells that
// share a bucket are still told apart by testing every entry read against the ball.
__device__ __forceinline__ uint32_t super_hash(int sx, int sy, int sz) {
  return (uint32_t)sx * 73856093u ^ (uint32_t)sy * 19349663u ^ (uint32_t)sz * 83492791u;
}
__device__ __forceinline__ uint32_t photon_bucket(const PhotonDev& P, int ix, int iy, int iz) {
  const uint32_t lo = ((uint32_t)ix & 3u) | (((uint32_t)iy & 3u) << 2) | (((uint32_t)iz & 3u) << 4);
  return lo | ((super_hash(ix >> 2, iy >> 2, iz >> 2) << 6) & (P.n_buckets - 1u));
}
// occupancy bit of the super-cell holding cell (i, j, k)
constexpr uint32_t kOccMask = kPhotonOccWords * 32u - 1u;
__device__ __forceinline__ uint32_t occ_bit(int sx, int sy, int sz) { return super_hash(sx, sy, sz) & kOccMask; }
__device__ __forceinline__ uint32_t photon_bucket_of(const PhotonDev& P, float4 q) {
  return photon_bucket(P, (int)floorf(q.x * P.inv_cell), (int)floorf(q.y * P.inv_cell), (int)floorf(q.z * P.inv_cell));
}

__global__ void k_photon_count(PhotonDev P) {
  const uint32_t n = min(P.ctl[0], P.cap);
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const float4 q = P.rec[(size_t)r * P.rq];
    const int ix = (int)floorf(q.x * P.inv_cell), iy = (int)floorf(q.y * P.inv_cell), iz = (int)floorf(q.z * P.inv_cell);
    atomicAdd(&P.bcount[photon_bucket(P, ix, iy, iz)], 1u);
    const uint32_t h = occ_bit(ix >> 2, iy >> 2, iz >> 2);
    atomicOr(&P.occ[h >> 5], 1u << (h & 31u));
  }
}

// Exclusive prefix sum of the bucket counts in three passes: the sum of each chunk of
// kPhotonScanChunk buckets, the scan of the chunk sums (one workgroup), then each chunk's own
// scan from its offset; the counts are cleared to serve as scatter cursors.
constexpr int kPhotonScanThreads = 256;
constexpr int kPhotonScanPer = kPhotonScanChunk / kPhotonScanThreads;
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_w, uint32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_w[wv] = incl;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
  for (int q = 0; q < kPhotonScanThreads / 64; ++q) {
    before += q < wv ? s_w[q] : 0u;
    total += s_w[q];
  }
  __syncthreads();
  return before + incl - x;
}
__global__ __launch_bounds__(kPhotonScanThreads) void k_photon_chunk_sums(PhotonDev P) {
  __shared__ uint32_t s_w[kPhotonScanThreads / 64];
  const uint32_t b0 = blockIdx.x * kPhotonScanChunk + threadIdx.x * kPhotonScanPer;
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < kPhotonScanPer; ++k) t += P.bcount[b0 + k];
  uint32_t total;
  block_excl_scan(t, s_w, total);
  if (threadIdx.x == 0) P.bsum[blockIdx.x] = total;
}
__global__ __launch_bounds__(kPhotonScanThreads) void k_photon_scan_sums(PhotonDev P, uint32_t n_chunks) {
  __shared__ uint32_t s_w[kPhotonScanThreads / 64];
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < n_chunks; c0 += kPhotonScanThreads) {
    const uint32_t c = c0 + threadIdx.x;
    const uint32_t x = c < n_chunks ? P.bsum[c] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan(x, s_w, total);
    if (c < n_chunks) P.bsum[c] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) P.bstart[P.n_buckets] = carry;
}
__global__ __launch_bounds__(kPhotonScanThreads) void k_photon_chunk_scan(PhotonDev P) {
  __shared__ uint32_t s_w[kPhotonScanThreads / 64];
  const uint32_t b0 = blockIdx.x * kPhotonScanChunk + threadIdx.x * kPhotonScanPer;
  uint32_t c[kPhotonScanPer], t = 0;
#pragma unroll
  for (int k = 0; k < kPhotonScanPer; ++k) {
    c[k] = P.bcount[b0 + k];
    t += c[k];
  }
  uint32_t total;
  uint32_t acc = P.bsum[blockIdx.x] + block_excl_scan(t, s_w, total);
#pragma unroll
  for (int k = 0; k < kPhotonScanPer; ++k) {
    P.bstart[b0 + k] = acc;
    P.bcount[b0 + k] = 0;
    acc += c[k];
  }
}

// Records into bucket order: each bucket's entries hold the position the gathering tests
// (contiguous per bucket) and the index of the record's copy in bucket order, through which the
// direction and flux of a record within the radius are read; the records a gather finds then
// lie next to each other in memory, bucket by bucket.
__global__ void k_photon_scatter(PhotonDev P) {
  const uint32_t n = min(P.ctl[0], P.cap);
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const float4* src = P.rec + (size_t)r * P.rq;
    const float4 q0 = src[0];
    const uint32_t b = photon_bucket_of(P, q0);
    const uint32_t e = P.bstart[b] + atomicAdd(&P.bcount[b], 1u);
    P.cand[e] = make_float4(q0.x, q0.y, q0.z, __uint_as_float(e));
    float4* dst = P.srec + (size_t)e * P.rq;
    for (uint32_t q = 0; q < P.rq; ++q) dst[q] = src[q];
  }
}

// The cells of the 3 x 3 x 3 block around a point that a ball of radius r (one cell) about it
// can reach: per axis the squared gap (in cells) to the lower neighbour, the own cell and the
// upper neighbour; a cell is read when the gaps of its three axes sum below one (with a margin
// of 1e-3 for the rounding of the point's cell coordinates).
struct CellBlock {
  int ix, iy, iz;
  float gx[3], gy[3], gz[3];
};
__device__ __forceinline__ CellBlock cell_block(const PhotonDev& P, F3 p) {
  CellBlock C;
  const float cx = p.x * P.inv_cell, cy = p.y * P.inv_cell, cz = p.z * P.inv_cell;
  const float fx = floorf(cx), fy = floorf(cy), fz = floorf(cz);
  C.ix = (int)fx;
  C.iy = (int)fy;
  C.iz = (int)fz;
  const float ux = cx - fx, uy = cy - fy, uz = cz - fz;  // exact, in [0, 1)
  C.gx[0] = ux * ux; C.gx[1] = 0.0f; C.gx[2] = (1.0f - ux) * (1.0f - ux);
  C.gy[0] = uy * uy; C.gy[1] = 0.0f; C.gy[2] = (1.0f - uy) * (1.0f - uy);
  C.gz[0] = uz * uz; C.gz[1] = 0.0f; C.gz[2] = (1.0f - uz) * (1.0f - uz);
  return C;
}
constexpr float kCellReach = 1.001f;

// Caustic radiance at the opaque vertices of a bounce, before their shading changes the
// throughput: (1 - F_j) rho_j / pi times the flux of the photons within the gather radius that
// arrived from the side the path sees, over pi r^2, added to the gathered radiance. A vertex
// whose block of cells touches no occupied super-cell (a bitmap in LDS) has nothing to gather; one
// whose own cell holds more than kGatherHeavy entries goes to the wave-wide pass. Otherwise the
// cells are read one 3 x 3 slab at a time (nine ranges loaded together), four entries at a time;
// an entry within the ball reads its record's direction, and its flux when it arrived from the
// side the path sees.
// NQ > 0: rows of NQ quads, the flux sums in registers; NQ = 0: any row length, the sums in
// dynamic LDS laid out lane-contiguous ([quad][lane], distinct banks across the wave).
constexpr int kGatherWG = 64;
constexpr uint32_t kGatherHeavy = 24;  // entries in the vertex's own cell above which it goes wave-wide

__device__ __forceinline__ float gap_of(const float (&g)[3], int o) { return o == 0 ? g[0] : (o == 1 ? 0.0f : g[2]); }

template <int NQ>
__global__ __launch_bounds__(kGatherWG) void k_photon_gather(DevScene S, DevWS w, PhotonDev P, int depth) {
  extern __shared__ float4 s_dyn[];
  __shared__ uint32_t s_occ[kPhotonOccWords];
  for (int q = threadIdx.x; q < kPhotonOccWords; q += kGatherWG) s_occ[q] = P.occ[q];
  __syncthreads();
  const int p = depth & 1;
  const uint32_t n = w.ctl->cat_count[p][kCatOpaque * kKeyStride];
  const uint32_t* list = cat_list(w, p, kCatOpaque);
  const int Bp = w.Bp, nq = NQ > 0 ? NQ : Bp / 4;
  const float r = P.radius, r2 = r * r;
  const float norm = 1.0f / (3.14159265358979f * 3.14159265358979f * r2);  // 1 / pi (BRDF) / (pi r^2)
  const int lane = threadIdx.x;
  if (blockIdx.x == 0 && lane == 0) w.ctl->ph_heavy[p ^ 1] = 0;  // the other parity's pass is done
  float4 acc_r[NQ > 0 ? NQ : 1];
  auto acc = [&](int q) -> float4& { return NQ > 0 ? acc_r[q] : s_dyn[q * kGatherWG + lane]; };
  uint32_t n_found = 0, n_vert = 0, n_lit = 0, n_cand = 0, m_cand = 0;
  for (uint32_t a = blockIdx.x * kGatherWG + threadIdx.x; a < n; a += gridDim.x * kGatherWG) {
    const uint32_t s = list[a];
    ++n_vert;
    const Vertex V = load_vertex(S, w, s);
    const CellBlock C = cell_block(P, V.p);
    // nothing to gather when no record lies in the super-cells that the block's cells touch
    bool occupied = false;
    {
      const int sx0 = (C.ix - 1) >> 2, sx1 = (C.ix + 1) >> 2, sy0 = (C.iy - 1) >> 2, sy1 = (C.iy + 1) >> 2;
      const int sz0 = (C.iz - 1) >> 2, sz1 = (C.iz + 1) >> 2;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const uint32_t h = occ_bit((c & 1) ? sx1 : sx0, (c & 2) ? sy1 : sy0, (c & 4) ? sz1 : sz0);
        occupied |= (s_occ[h >> 5] >> (h & 31u)) & 1u;
      }
    }
    if (!occupied) continue;
    // a vertex whose own cell holds many entries goes to the wave-wide pass (one wave per
    // vertex), which keeps a wave of this pass from waiting on its one lane in a dense caustic
    const uint32_t b_own = photon_bucket(P, C.ix, C.iy, C.iz);
    const bool heavy = P.bstart[b_own + 1] - P.bstart[b_own] > kGatherHeavy;
    const uint64_t hm = __ballot(heavy);
    if (hm) {
      const uint32_t leader = (uint32_t)__ffsll((unsigned long long)hm) - 1u;
      uint32_t base = 0;
      if ((uint32_t)lane == leader) base = atomicAdd(&w.ctl->ph_heavy[p], (uint32_t)__popcll(hm));
      base = __builtin_amdgcn_readlane(base, (int)leader);
      if (heavy) w.queue[base + count_below(hm)] = s;
    }
    if (heavy) continue;
    uint32_t v_cand = 0;
    for (int q = 0; q < nq; ++q) acc(q) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    bool any = false;
#pragma unroll 1
    for (int oz = 0; oz < 3; ++oz) {
      const float gz = gap_of(C.gz, oz);
      uint32_t e0[9], e1[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int ox = k % 3, oy = k / 3;
        const bool vis = C.gx[ox] + C.gy[oy] + gz < kCellReach;
        const uint32_t b = photon_bucket(P, C.ix + ox - 1, C.iy + oy - 1, C.iz + oz - 1);
        e0[k] = vis ? P.bstart[b] : 0u;
        e1[k] = vis ? P.bstart[b + 1] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) v_cand += e1[k] - e0[k];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const uint32_t end = e1[k];
        for (uint32_t e = e0[k]; e < end; e += 4) {
          float4 q0[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) q0[j] = P.cand[min(e + (uint32_t)j, end - 1u)];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float dx = q0[j].x - V.p.x, dy = q0[j].y - V.p.y, dz = q0[j].z - V.p.z;
            if (e + (uint32_t)j < end && dx * dx + dy * dy + dz * dz < r2) {
              // the direction and the flux row in one round trip (nearly every record within
              // the ball arrived from the side the path sees)
              const float4* R = P.srec + (size_t)__float_as_uint(q0[j].w) * P.rq;
              if constexpr (NQ > 0) {
                float4 x[NQ];
                const float4 q1 = R[1];
#pragma unroll
                for (int q = 0; q < NQ; ++q) x[q] = R[2 + q];
                if (q1.x * V.n.x + q1.y * V.n.y + q1.z * V.n.z < 0.0f) {
#pragma unroll
                  for (int q = 0; q < NQ; ++q)
                    acc_r[q] = make_float4(acc_r[q].x + x[q].x, acc_r[q].y + x[q].y, acc_r[q].z + x[q].z,
                                           acc_r[q].w + x[q].w);
                  any = true;
                  ++n_found;
                }
              } else {
                const float4 q1 = R[1];
                if (q1.x * V.n.x + q1.y * V.n.y + q1.z * V.n.z < 0.0f) {
                  for (int q = 0; q < nq; ++q) {
                    const float4 x = R[2 + q], t = acc(q);
                    acc(q) = make_float4(t.x + x.x, t.y + x.y, t.z + x.z, t.w + x.w);
                  }
                  any = true;
                  ++n_found;
                }
              }
            }
          }
        }
      }
    }
    n_cand += v_cand;
    m_cand = max(m_cand, v_cand);
    if (!any) continue;
    ++n_lit;
    const float4* nt = (const float4*)(S.ntab + V.m * Bp);
    const float4* kt = (const float4*)(S.ktab + V.m * Bp);
    const float4* rt = (const float4*)(S.rho + V.m * Bp);
    const float4* b4 = (const float4*)(w.beta + (size_t)s * Bp);
    row_update<2>((float4*)(w.lacc + (size_t)s * Bp), nq, [&](int q, float4 l) {
      const float4 nn = nt[q], kk = kt[q], rr = rt[q], b = b4[q], f = acc(q);
      const float F0 = fresnel(nn.x, kk.x, V.cos_o), F1 = fresnel(nn.y, kk.y, V.cos_o);
      const float F2 = fresnel(nn.z, kk.z, V.cos_o), F3v = fresnel(nn.w, kk.w, V.cos_o);
      return make_float4(l.x + b.x * (1.0f - F0) * rr.x * f.x * norm, l.y + b.y * (1.0f - F1) * rr.y * f.y * norm,
                         l.z + b.z * (1.0f - F2) * rr.z * f.z * norm, l.w + b.w * (1.0f - F3v) * rr.w * f.w * norm);
    });
  }
  // one atomic per wave and counter (the workgroup is one wave)
  for (int o = 32; o > 0; o >>= 1) {
    n_found += __shfl_xor(n_found, o);
    n_vert += __shfl_xor(n_vert, o);
    n_lit += __shfl_xor(n_lit, o);
    n_cand += __shfl_xor(n_cand, o);
    m_cand = max(m_cand, (uint32_t)__shfl_xor(m_cand, o));
  }
  if (lane == 0 && n_vert) {
    atomicAdd(&w.ctl->st_ph_vertices, (unsigned long long)n_vert);
    atomicAdd(&w.ctl->st_ph_found, (unsigned long long)n_found);
    if (n_lit) atomicAdd(&w.ctl->st_ph_lit, (unsigned long long)n_lit);
    atomicAdd(&w.ctl->st_ph_cand, (unsigned long long)n_cand);
    atomicMax(&w.ctl->st_ph_cand_max, (unsigned long long)m_cand);
  }
}

// The deferred vertices of a bounce (their slots in the queue buffer, which no kernel uses
// between two traversal phases), one wave each: for every reachable cell the lanes test its
// entries k = lane, lane + 64, ... (consecutive entries across the wave), each summing the flux of
// the ones it finds, then the wave adds its 64 partial sums per bin in a fixed butterfly order and
// lane q updates quad q of the gathered radiance.
template <int NQ>
__global__ __launch_bounds__(kGatherWG) void k_photon_gather_heavy(DevScene S, DevWS w, PhotonDev P, int depth) {
  const int p = depth & 1;
  const uint32_t n = w.ctl->ph_heavy[p];
  const int Bp = w.Bp, nq = Bp / 4;
  const float r = P.radius, r2 = r * r;
  const float norm = 1.0f / (3.14159265358979f * 3.14159265358979f * r2);
  const int lane = threadIdx.x;
  constexpr int kQ = NQ > 0 ? NQ : kMaxBins / 4;
  uint32_t n_found = 0, n_lit = 0;
  for (uint32_t h = blockIdx.x; h < n; h += gridDim.x) {
    const uint32_t s = w.queue[h];
    const Vertex V = load_vertex(S, w, s);
    const CellBlock C = cell_block(P, V.p);
    float4 acc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) acc[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t v_found = 0;
#pragma unroll 1
    for (int c = 0; c < 27; ++c) {
      const int ox = c % 3, oy = (c / 3) % 3, oz = c / 9;
      if (!(gap_of(C.gx, ox) + gap_of(C.gy, oy) + gap_of(C.gz, oz) < kCellReach)) continue;
      const uint32_t b = photon_bucket(P, C.ix + ox - 1, C.iy + oy - 1, C.iz + oz - 1);
      const uint32_t e0 = P.bstart[b], cnt = P.bstart[b + 1] - e0;
      for (uint32_t k = (uint32_t)lane; k < cnt; k += kGatherWG) {
        const float4 q0 = P.cand[(size_t)e0 + k];
        const float dx = q0.x - V.p.x, dy = q0.y - V.p.y, dz = q0.z - V.p.z;
        if (dx * dx + dy * dy + dz * dz < r2) {
          const float4* R = P.srec + (size_t)__float_as_uint(q0.w) * P.rq;
          const float4 q1 = R[1];
          if (q1.x * V.n.x + q1.y * V.n.y + q1.z * V.n.z < 0.0f) {
#pragma unroll
            for (int q = 0; q < kQ; ++q)
              if (q < nq) {
                const float4 x = R[2 + q];
                acc[q] = make_float4(acc[q].x + x.x, acc[q].y + x.y, acc[q].z + x.z, acc[q].w + x.w);
              }
            ++v_found;
          }
        }
      }
    }
    n_found += v_found;
    for (int o = 32; o > 0; o >>= 1) v_found += __shfl_xor(v_found, o);
    n_lit += v_found != 0;  // the same on every lane: added once, by lane 0 below
    // butterfly sums: every lane ends with the wave's totals, quad q kept by lane q
    float4 mine = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      if (q < nq) {
        float4 t = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
          t = make_float4(t.x + __shfl_xor(t.x, o), t.y + __shfl_xor(t.y, o), t.z + __shfl_xor(t.z, o),
                          t.w + __shfl_xor(t.w, o));
        if (lane == q) mine = t;
      }
    }
    if (lane < nq) {
      const int q = lane;
      const float4 nn = ((const float4*)(S.ntab + V.m * Bp))[q], kk = ((const float4*)(S.ktab + V.m * Bp))[q];
      const float4 rr = ((const float4*)(S.rho + V.m * Bp))[q];
      const float4 b = ((const float4*)(w.beta + (size_t)s * Bp))[q];
      float4* lp = (float4*)(w.lacc + (size_t)s * Bp) + q;
      const float4 l = *lp, f = mine;
      const float F0 = fresnel(nn.x, kk.x, V.cos_o), F1 = fresnel(nn.y, kk.y, V.cos_o);
      const float F2 = fresnel(nn.z, kk.z, V.cos_o), F3v = fresnel(nn.w, kk.w, V.cos_o);
      *lp = make_float4(l.x + b.x * (1.0f - F0) * rr.x * f.x * norm, l.y + b.y * (1.0f - F1) * rr.y * f.y * norm,
                        l.z + b.z * (1.0f - F2) * rr.z * f.z * norm, l.w + b.w * (1.0f - F3v) * rr.w * f.w * norm);
    }
  }
  for (int o = 32; o > 0; o >>= 1) n_found += __shfl_xor(n_found, o);
  if (lane == 0 && n_found) {
    atomicAdd(&w.ctl->st_ph_found, (unsigned long long)n_found);
    atomicAdd(&w.ctl->st_ph_lit, (unsigned long long)n_lit);
  }
}

static inline unsigned grid_for(size_t n, unsigned cap = 8192) {
  size_t g = (n + kWG - 1) / kWG;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

hipError_t launch_fill_f32(hipStream_t s, float* p, size_t n, float v) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(kWG), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t* p, size_t n, uint32_t v) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kWG), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_philox(hipStream_t s, const uint32_t ctr[4], const uint32_t key[2], uint64_t n, uint32_t* out) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3(grid_for(n)), dim3(kWG), 0, s, make_uint4(ctr[0], ctr[1], ctr[2], ctr[3]), key[0],
                     key[1], n, (uint4*)out);
  return hipGetLastError();
}

hipError_t launch_raygen(const Launch& L, const DevScene& S, const DevWS& w, uint64_t k0, uint32_t n, uint64_t seed,
                         int gen, const PathMode& pm) {
  if (pm.purpose)
    hipLaunchKernelGGL(k_raygen<true>, dim3((n + kWG - 1) / kWG), dim3(kWG), 0, L.stream, S, w, k0, n, (uint32_t)seed,
                       (uint32_t)(seed >> 32), gen, pm);
  else
    hipLaunchKernelGGL(k_raygen<false>, dim3((n + kWG - 1) / kWG), dim3(kWG), 0, L.stream, S, w, k0, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), gen, pm);
  return hipGetLastError();
}

hipError_t launch_scan(const Launch& L, const DevScene& S, const DevWS& w, int gen) {
  const size_t n_keys = (size_t)S.n_cells * kDirBins, nsub = (size_t)1 << w.sub_shift;
  const uint32_t g_sub = nsub <= 64 ? (uint32_t)((n_keys * nsub + kWG - 1) / kWG) : (uint32_t)n_keys;
  hipLaunchKernelGGL(k_subscan, dim3(g_sub), dim3(kWG), 0, L.stream, S, w, gen);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, L.stream, S, w, gen, L.cell_order);
  return hipGetLastError();
}

hipError_t launch_scatter(const Launch& L, const DevWS& w, int gen) {
  hipLaunchKernelGGL(k_scatter, dim3(grid_for((size_t)w.W / 2, 8192)), dim3(kWG), 0, L.stream, w, gen);
  return hipGetLastError();
}

hipError_t launch_trace(const Launch& L, const DevScene& S, const DevWS& w, int gen, int hops) {
  hipLaunchKernelGGL(k_trace, dim3(L.trace_blocks), dim3(kWG), 0, L.stream, S, w, gen, hops);
  return hipGetLastError();
}

hipError_t launch_gather_cats(const Launch& L, const DevWS& w, int par) {
  const size_t chunks = (2 * (size_t)w.W + (size_t)kWG * kGatherPer - 1) / ((size_t)kWG * kGatherPer);
  hipLaunchKernelGGL(k_gather_cats, dim3((unsigned)std::min<size_t>(chunks, 4096)), dim3(kWG), 0, L.stream, w, par);
  return hipGetLastError();
}

hipError_t launch_resolve(const Launch& L, const DevScene& S, const DevWS& w, int depth) {
  hipLaunchKernelGGL(k_resolve, dim3(grid_for(2 * (size_t)w.W, 4096)), dim3(kWG), 0, L.stream, S, w, depth);
  return hipGetLastError();
}

hipError_t launch_escape(const Launch& L, const DevScene& S, const DevWS& w, int depth) {
  hipLaunchKernelGGL(k_escape, dim3(grid_for(w.W, 2048)), dim3(kWG), 0, L.stream, S, w, depth);
  return hipGetLastError();
}

hipError_t launch_shade_opaque(const Launch& L, const DevScene& S, const DevWS& w, int depth, int max_depth,
                               uint64_t seed, int gen, const PathMode& pm) {
  const dim3 g(grid_for(w.W, 4096)), b(kWG);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const size_t tab = (size_t)3 * S.n_mat * w.Bp + w.Bp;  // LDS tables of the templated kernels
  const bool lds = tab <= (size_t)kShadeLdsFloats;
  const size_t bytes = lds ? tab * sizeof(float) : 0;
#define SDD_SHADE(nq, l) hipLaunchKernelGGL((k_shade_opaque<nq, l>), g, b, bytes, L.stream, S, w, depth, max_depth, k0, k1, gen, pm)
  switch (w.Bp / 4) {
    case 2:
      if (lds) SDD_SHADE(2, true); else SDD_SHADE(2, false);
      break;
    case 10:
      if (lds) SDD_SHADE(10, true); else SDD_SHADE(10, false);
      break;
    default: SDD_SHADE(0, false);
  }
#undef SDD_SHADE
  return hipGetLastError();
}

hipError_t launch_shade_glass(const Launch& L, const DevScene& S, const DevWS& w, int depth, uint64_t seed, int gen,
                              const PathMode& pm) {
  hipLaunchKernelGGL(k_shade_glass, dim3(grid_for(w.W, 1024)), dim3(kWG), 0, L.stream, S, w, depth, (uint32_t)seed,
                     (uint32_t)(seed >> 32), gen, pm);
  return hipGetLastError();
}

hipError_t launch_accumulate(const Launch& L, const DevScene& S, const DevWS& w, uint32_t s0, uint32_t n,
                             bool unique) {
  if (n == 0) return hipSuccess;
  if (unique)
    hipLaunchKernelGGL(k_accumulate<true>, dim3(grid_for(n, 8192)), dim3(kWG), 0, L.stream, S, w, s0, n);
  else
    hipLaunchKernelGGL(k_accumulate<false>, dim3(grid_for(n, 8192)), dim3(kWG), 0, L.stream, S, w, s0, n);
  return hipGetLastError();
}

// Workgroups of k_persist the device holds at once (its occupancy times the compute units), 0 if
// the runtime cannot tell.
uint32_t persist_resident_blocks(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_persist), kWG, 0) !=
          hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  return (uint32_t)(per_cu * cus);
}

hipError_t launch_persist(const Launch& L, const DevScene& S, const DevWS& w, uint64_t total, uint64_t seed,
                          int max_depth, uint32_t lanes) {
  hipLaunchKernelGGL(k_persist, dim3(lanes / kWG), dim3(kWG), 0, L.stream, S, w, total, (uint32_t)seed,
                     (uint32_t)(seed >> 32), max_depth);
  return hipGetLastError();
}

hipError_t launch_pack_rays(const Launch& L, const DevScene& S, const DevWS& w, const float* orig, const float* dir,
                            const int32_t* skip, uint32_t n, int shadow, int gen) {
  hipLaunchKernelGGL(k_pack_rays, dim3((n + kWG - 1) / kWG), dim3(kWG), 0, L.stream, S, w, orig, dir, skip, n, shadow,
                     gen);
  return hipGetLastError();
}

hipError_t launch_unpack_hits(const Launch& L, const DevScene& S, const DevWS& w, uint32_t n, float* t, int32_t* id,
                              float* u, float* v) {
  hipLaunchKernelGGL(k_unpack_hits, dim3(grid_for(n)), dim3(kWG), 0, L.stream, S, w, n, t, id, u, v);
  return hipGetLastError();
}

hipError_t launch_resolve_vis(const Launch& L, const DevScene& S, const DevWS& w, uint32_t n, float* vis) {
  hipLaunchKernelGGL(k_resolve_vis, dim3(grid_for(n)), dim3(kWG), 0, L.stream, S, w, n, vis);
  return hipGetLastError();
}

hipError_t launch_photon_gen(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, uint64_t k0,
                             uint32_t n, int gen) {
  hipLaunchKernelGGL(k_photon_gen, dim3((n + kWG - 1) / kWG), dim3(kWG), 0, L.stream, S, w, P, k0, n, gen);
  return hipGetLastError();
}
hipError_t launch_photon_vis(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, int par) {
  hipLaunchKernelGGL(k_photon_vis, dim3(grid_for(w.W, 4096)), dim3(kWG), 0, L.stream, S, w, P, par);
  return hipGetLastError();
}
hipError_t launch_photon_shade(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, int depth,
                               int gen) {
  hipLaunchKernelGGL(k_photon_shade, dim3(grid_for(w.W, 4096)), dim3(kWG), 0, L.stream, S, w, P, depth, gen);
  return hipGetLastError();
}
hipError_t launch_photon_build(hipStream_t s, const PhotonDev& P) {
  const uint32_t n_chunks = P.n_buckets / kPhotonScanChunk;  // n_buckets is a multiple of the chunk
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(P.n_buckets)), dim3(256), 0, s, P.bcount, (size_t)P.n_buckets, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(4), dim3(256), 0, s, P.occ, (size_t)kPhotonOccWords, 0u);
  hipLaunchKernelGGL(k_photon_count, dim3(grid_for(P.cap)), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_photon_chunk_sums, dim3(n_chunks), dim3(kPhotonScanThreads), 0, s, P);
  hipLaunchKernelGGL(k_photon_scan_sums, dim3(1), dim3(kPhotonScanThreads), 0, s, P, n_chunks);
  hipLaunchKernelGGL(k_photon_chunk_scan, dim3(n_chunks), dim3(kPhotonScanThreads), 0, s, P);
  hipLaunchKernelGGL(k_photon_scatter, dim3(grid_for(P.cap)), dim3(256), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_photon_gather(const Launch& L, const DevScene& S, const DevWS& w, const PhotonDev& P, int depth) {
  const size_t want = ((size_t)w.W + kGatherWG - 1) / kGatherWG;
  const dim3 g((unsigned)(want < 16384 ? want : 16384)), b(kGatherWG), gh(16384);
  switch (w.Bp / 4) {
    case 2:
      hipLaunchKernelGGL(k_photon_gather<2>, g, b, 0, L.stream, S, w, P, depth);
      hipLaunchKernelGGL(k_photon_gather_heavy<2>, gh, b, 0, L.stream, S, w, P, depth);
      break;
    case 10:
      hipLaunchKernelGGL(k_photon_gather<10>, g, b, 0, L.stream, S, w, P, depth);
      hipLaunchKernelGGL(k_photon_gather_heavy<10>, gh, b, 0, L.stream, S, w, P, depth);
      break;
    default:
      hipLaunchKernelGGL(k_photon_gather<0>, g, b, (size_t)(w.Bp / 4) * kGatherWG * sizeof(float4), L.stream, S, w,
                         P, depth);
      hipLaunchKernelGGL(k_photon_gather_heavy<0>, gh, b, 0, L.stream, S, w, P, depth);
  }
  return hipGetLastError();
}

}  // namespace sdd
