// Device helpers shared by the tracer and the radiance-cache kernels of libspecdd.
#pragma once

#include "internal.h"

namespace sdd {

struct F3 { float x, y, z; };
__device__ __forceinline__ F3 f3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ F3 operator+(F3 a, F3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ F3 operator-(F3 a, F3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ F3 operator*(F3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot3(F3 a, F3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ F3 cross3(F3 a, F3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ F3 norm3(F3 a) { return a * (1.0f / sqrtf(dot3(a, a))); }
__device__ __forceinline__ float maxabs3(F3 a) { return fmaxf(fabsf(a.x), fmaxf(fabsf(a.y), fabsf(a.z))); }
__device__ __forceinline__ float comp(F3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// Geometric normal and the dot products whose sign selects a branch (face side, sun side),
// evaluated without FMA contraction: an exactly cancelling sum (a vertical facet's z, for
// example) then stays exactly zero, as in exact arithmetic, instead of keeping the rounding
// error of one product, which would flip the sign-dependent choices downstream.
__device__ __forceinline__ F3 geo_normal(F3 v0, F3 v1, F3 v2) {
#pragma clang fp contract(off)
  const F3 e1 = v1 - v0, e2 = v2 - v0;
  const F3 c = {e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
  const float l2 = c.x * c.x + c.y * c.y + c.z * c.z;
  return c * (1.0f / sqrtf(l2));
}
__device__ __forceinline__ float dot_exact_sign(F3 a, F3 b) {
#pragma clang fp contract(off)
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}
__device__ __forceinline__ float unif24(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// Ray queues are keyed by (cell, direction bin): rays of one tile then share a cell, the signs of
// their direction components and their dominant axis, which keeps the lanes of a wave on similar
// BVH paths.
__device__ __forceinline__ uint32_t dir_bin(F3 d) {
  const uint32_t oct = (d.x < 0.0f ? 1u : 0u) | (d.y < 0.0f ? 2u : 0u) | (d.z < 0.0f ? 4u : 0u);
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  const uint32_t dom = (ax >= ay && ax >= az) ? 0u : (ay >= az ? 1u : 2u);
  return oct * 3u + dom;
}
__device__ __forceinline__ uint32_t qkey(uint32_t cell, uint32_t dbin) { return cell * (uint32_t)kDirBins + dbin; }
__device__ __forceinline__ uint32_t* ccount_of(const DevScene& S, const DevWS& w, int parity) {
  return w.ccount + (size_t)parity * S.n_cells * kDirBins * kKeyStride;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}


// Statistics counters of a workgroup in LDS: every wave adds its count with one LDS atomic, and
// at the end of the kernel one thread per counter adds the workgroup's totals to the global
// counters, a handful of global atomics per workgroup instead of one per wave and loop
// iteration on the same few addresses. stats_init is followed by a barrier before the first
// stats_add; stats_add is called by every lane of the wave; stats_flush by every thread.
__device__ __forceinline__ void stats_init(uint32_t* s, int n) {
  if ((int)threadIdx.x < n) s[threadIdx.x] = 0;
}
__device__ __forceinline__ void stats_add(uint32_t* s, int i, uint32_t wave_count) {
  if (lane_id() == 0 && wave_count) atomicAdd(&s[i], wave_count);
}
__device__ __forceinline__ void stats_add_ballot(uint32_t* s, int i, bool pred) {
  stats_add(s, i, (uint32_t)__popcll(__ballot(pred)));
}
__device__ __forceinline__ void stats_flush(const uint32_t* s, int i, unsigned long long* ctr) {
  if ((int)threadIdx.x == i && s[i]) atomicAdd(ctr, (unsigned long long)s[i]);
}

// Wave-level sum, then one 64-bit atomic per wave.
__device__ __forceinline__ void wave_add(unsigned long long* ctr, uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (lane_id() == 0 && x) atomicAdd(ctr, (unsigned long long)x);
}


// Geometry of the hit of slot s: vertex position, face-forward normal, geometric normal.
// Distance and barycentrics of the winning triangle re-evaluated in FP64 with the sheared
// formulation of the watertight test: the FP32 test of the traversal decides which triangle is
// hit, this pass (run by whoever reads the hit) removes the cancellation that makes FP32
// distances and barycentrics inaccurate for grazing rays. t, bu, bv are left as passed in when
// the FP64 determinant is zero.
__device__ __forceinline__ void refine_hit(F3 of, F3 df, F3 v0, F3 v1, F3 v2, float& t, float& bu, float& bv) {
  const double o[3] = {of.x, of.y, of.z}, d[3] = {df.x, df.y, df.z};
  const double ad[3] = {fabs(d[0]), fabs(d[1]), fabs(d[2])};
  const int kz = (ad[0] >= ad[1] && ad[0] >= ad[2]) ? 0 : (ad[1] >= ad[2] ? 1 : 2);
  const int kx = kz == 2 ? 0 : kz + 1, ky = kx == 2 ? 0 : kx + 1;
  const double Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0 / d[kz];
  const double A[3] = {v0.x - o[0], v0.y - o[1], v0.z - o[2]};
  const double B[3] = {v1.x - o[0], v1.y - o[1], v1.z - o[2]};
  const double C[3] = {v2.x - o[0], v2.y - o[1], v2.z - o[2]};
  const double Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
  const double Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
  const double Cx = C[kx] - Sx * C[kz], Cy = C[ky] - Sy * C[kz];
  const double U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
  const double det = U + V + W;
  if (det == 0.0) return;
  const double T = Sz * (U * A[kz] + V * B[kz] + W * C[kz]);
  const double inv_det = 1.0 / det;
  t = (float)(T * inv_det);
  bu = (float)(V * inv_det);
  bv = (float)(W * inv_det);
}

struct Vertex {
  F3 p, n, ng, d;
  float dn, cos_o, eps;
  uint32_t id;
  int m;
};

__device__ __forceinline__ Vertex load_vertex(const DevScene& S, const DevWS& w, uint32_t s) {
  Vertex V;
  const float4 h = w.hit[s];
  V.id = __float_as_uint(h.y);
  const float4 rdir = w.rays[2 * s + 1];
  V.d = f3(rdir.x, rdir.y, rdir.z);
  const float4 A = S.gtris[(size_t)V.id * 3 + 0], Bv = S.gtris[(size_t)V.id * 3 + 1], C = S.gtris[(size_t)V.id * 3 + 2];
  const F3 v0 = f3(A.x, A.y, A.z), v1 = f3(Bv.x, Bv.y, Bv.z), v2 = f3(C.x, C.y, C.z);
  V.m = (int)__float_as_uint(Bv.w);
  V.ng = geo_normal(v0, v1, v2);
  V.dn = dot_exact_sign(V.d, V.ng);
  V.n = V.dn > 0.0f ? V.ng * -1.0f : V.ng;
  V.cos_o = fabsf(V.dn);
  const float4 rorg = w.rays[2 * s];
  float t = h.x, bu = 1.0f / 3.0f, bv = 1.0f / 3.0f;
  refine_hit(f3(rorg.x, rorg.y, rorg.z), V.d, v0, v1, v2, t, bu, bv);
  V.p = v0 * (1.0f - bu - bv) + v1 * bu + v2 * bv;
  V.eps = 1e-5f * (1.0f + maxabs3(V.p));
  return V;
}

}  // namespace sdd
