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
// Sub-bin of a direction inside its class: whether each of the two components other than the
// dominant one exceeds half of the dominant one in magnitude (bit 0: the first, bit 1: the second).
__device__ __forceinline__ uint32_t dir_sub(F3 d) {
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  const bool xd = ax >= ay && ax >= az, yd = !xd && ay >= az;  // the dominant axis, as in dir_bin
  const float m = xd ? ax : (yd ? ay : az), u = xd ? ay : ax, v = (xd || yd) ? az : ay;
  return (u + u > m ? 1u : 0u) | (v + v > m ? 2u : 0u);
}
// direction class and sub-bin of a ray in one word: dir_bin | dir_sub << 8
__device__ __forceinline__ uint32_t dir_code(F3 d) { return dir_bin(d) | dir_sub(d) << 8; }
__device__ __forceinline__ uint32_t qkey(uint32_t cell, uint32_t dbin) { return cell * (uint32_t)kDirBins + dbin; }
// sub-range of a ray: its queue key (cell, direction class), its direction sub-bin (dc, from
// dir_code) and the block of its cell that holds its origin (blk, the Morton index at
// kMaxSubLevels levels, whose top 3 L bits are the index at L levels)
__device__ __forceinline__ uint32_t qsub(const DevWS& w, uint32_t cell, uint32_t dc, uint32_t blk) {
  const uint32_t bs = w.sub_shift - kDirSubBits;
  return (((qkey(cell, dc & 0xFFu) << kDirSubBits) | (dc >> 8)) << bs) | (blk >> (3u * kMaxSubLevels - bs));
}
// word of sub-range ks's counter in a counter array
__device__ __forceinline__ size_t ctr_word(const DevWS& w, uint32_t ks) {
  return (size_t)(ks >> w.sub_shift) * w.key_words + (ks & ((1u << w.sub_shift) - 1u));
}
__device__ __forceinline__ uint32_t* ccount_of(const DevScene& S, const DevWS& w, int parity) {
  return w.ccount + (size_t)parity * S.n_cells * kDirBins * w.key_words;
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


// Error-free transformations in FP32 (round to nearest): a + b = s + e exactly (Knuth's
// TwoSum) and a * b = p + e exactly (the FMA residual of the product).
__device__ __forceinline__ float two_sum(float a, float b, float& e) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
  return s;
}
__device__ __forceinline__ float two_prod(float a, float b, float& e) {
  const float p = a * b;
  e = __builtin_fmaf(a, b, -p);
  return p;
}
// Compensated dot product (Ogita, Rump, Oishi 2005, Dot2) of x = xh + xl and y = yh + yl: the
// high parts' products and sum are formed exactly, the terms with a low part added once, so the
// result hi + lo is as accurate as if computed in twice the working precision.
__device__ __forceinline__ float dot2(F3 xh, F3 xl, F3 yh, F3 yl, float& lo) {
#pragma clang fp contract(off)
  float r0, r1, r2, q1, q2;
  const float h0 = two_prod(xh.x, yh.x, r0), h1 = two_prod(xh.y, yh.y, r1), h2 = two_prod(xh.z, yh.z, r2);
  float p = two_sum(h0, h1, q1);
  p = two_sum(p, h2, q2);
  lo = (q1 + q2) + ((r0 + r1) + r2) + (dot3(xl, yh) + dot3(xh, yl));
  return p;
}

// a*b - c*d for a = ah + al, b = bh + bl, c = ch + cl, d = dh + dl (exact sums of two floats),
// returned as hi + lo: the products of the high parts and their difference are formed exactly,
// the terms with one low part added once, so the result is accurate to about twice the working
// precision even when the difference cancels.
__device__ __forceinline__ float cross_term(float ah, float al, float bh, float bl, float ch, float cl, float dh,
                                            float dl, float& lo) {
#pragma clang fp contract(off)
  float p1l, p2l, sl;
  const float p1 = two_prod(ah, bh, p1l), p2 = two_prod(ch, dh, p2l);
  const float sh = two_sum(p1, -p2, sl);
  const float c = (sl + (p1l - p2l)) + ((ah * bl + al * bh) - (ch * dl + cl * dh));
  const float hi = sh + c;      // |c| is below ulp(sh) unless sh == 0: fast two-sum
  lo = c - (hi - sh);
  return hi;
}

// Distance and barycentrics of the winning triangle, re-evaluated by whoever reads the hit.
// The traversal's FP32 watertight test decides WHICH triangle is hit; its sheared coordinates
// carry the rounding of v - o, which is of the size of the ray's origin and, for a hit at
// incidence cosine c, moves the distance by about eps |o| / c. Here the plane of the triangle
// is intersected in FP32 arithmetic made exact where it cancels: the edges v1 - v0, v2 - v0 and
// o - v0 are kept as exact sums of two floats, the normal is their compensated cross product
// (kept as a sum of two floats too), the two dot products are compensated, and the hit point relative to v0,
// q = (o - v0) + t d, is formed from the exact parts. On return t is the distance, q the hit
// point minus v0 and (bu, bv) the barycentrics of v1 and v2. t, q, bu, bv keep their incoming
// values when the ray is parallel to the triangle's plane.
__device__ __forceinline__ void refine_hit(F3 o, F3 d, F3 v0, F3 v1, F3 v2, float& t, F3& q, float& bu,
                                           float& bv) {
#pragma clang fp contract(off)
  F3 e1, e1l, e2, e2l, ah, al;
  e1.x = two_sum(v1.x, -v0.x, e1l.x);
  e1.y = two_sum(v1.y, -v0.y, e1l.y);
  e1.z = two_sum(v1.z, -v0.z, e1l.z);
  e2.x = two_sum(v2.x, -v0.x, e2l.x);
  e2.y = two_sum(v2.y, -v0.y, e2l.y);
  e2.z = two_sum(v2.z, -v0.z, e2l.z);
  F3 nl;
  const F3 n = f3(cross_term(e1.y, e1l.y, e2.z, e2l.z, e1.z, e1l.z, e2.y, e2l.y, nl.x),
                  cross_term(e1.z, e1l.z, e2.x, e2l.x, e1.x, e1l.x, e2.z, e2l.z, nl.y),
                  cross_term(e1.x, e1l.x, e2.y, e2l.y, e1.y, e1l.y, e2.x, e2l.x, nl.z));
  ah.x = two_sum(o.x, -v0.x, al.x);
  ah.y = two_sum(o.y, -v0.y, al.y);
  ah.z = two_sum(o.z, -v0.z, al.z);
  float num_lo, den_lo;
  const float num = dot2(ah, al, n, nl, num_lo);
  const float den = dot2(d, f3(0.0f, 0.0f, 0.0f), n, nl, den_lo);
  if (den == 0.0f) return;
  // (o - v0 + t d) . n = 0:  t = -(num + num_lo) / (den + den_lo), kept as th + tl
  const float th = -num / den;
  const float r = __builtin_fmaf(-th, den, -num) - num_lo - th * den_lo;
  const float tl = r / den;
  // q = (ah + al) + (th + tl) d: the large parts ah + th d cancel exactly in two_sum
  float px, py, pz, ex, ey, ez;
  const float mx = two_prod(th, d.x, px), my = two_prod(th, d.y, py), mz = two_prod(th, d.z, pz);
  const float sx = two_sum(ah.x, mx, ex), sy = two_sum(ah.y, my, ey), sz = two_sum(ah.z, mz, ez);
  q = f3(sx + (ex + px + al.x + tl * d.x), sy + (ey + py + al.y + tl * d.y), sz + (ez + pz + al.z + tl * d.z));
  t = th + tl;
  // q = bu e1 + bv e2:  bu = (q x e2) . n / |n|^2,  bv = (e1 x q) . n / |n|^2
  const float inv_nn = 1.0f / dot3(n, n);
  bu = dot3(cross3(q, e2), n) * inv_nn;
  bv = dot3(cross3(e1, q), n) * inv_nn;
}

struct Vertex {
  F3 p, n, ng, d;
  float dn, cos_o, eps;
  float bu, bv;  // barycentrics of v1 and v2
  uint32_t id;
  int m;
};

// The surface vertex where the ray (o, d) hits triangle id at the traversal's distance t: the
// hit re-evaluated by refine_hit, the face-forward normal and the spawn offset.
__device__ __forceinline__ Vertex make_vertex(const DevScene& S, F3 o, F3 d, uint32_t id, float t) {
  Vertex V;
  V.id = id;
  V.d = d;
  const float4 A = S.gtris[(size_t)V.id * 3 + 0], Bv = S.gtris[(size_t)V.id * 3 + 1], C = S.gtris[(size_t)V.id * 3 + 2];
  const F3 v0 = f3(A.x, A.y, A.z), v1 = f3(Bv.x, Bv.y, Bv.z), v2 = f3(C.x, C.y, C.z);
  V.m = (int)__float_as_uint(Bv.w);
  V.ng = geo_normal(v0, v1, v2);
  V.dn = dot_exact_sign(V.d, V.ng);
  V.n = V.dn > 0.0f ? V.ng * -1.0f : V.ng;
  V.cos_o = fabsf(V.dn);
  float bu = 1.0f / 3.0f, bv = 1.0f / 3.0f;
  F3 q = ((v1 - v0) + (v2 - v0)) * (1.0f / 3.0f);
  refine_hit(o, V.d, v0, v1, v2, t, q, bu, bv);
  V.p = v0 + q;
  V.bu = bu;
  V.bv = bv;
  V.eps = 1e-5f * (1.0f + maxabs3(V.p));
  return V;
}

// The vertex of path slot s: its extension ray and hit record from the workspace.
__device__ __forceinline__ Vertex load_vertex(const DevScene& S, const DevWS& w, uint32_t s) {
  const float4 h = w.hit[s];
  const float4 rorg = w.rays[2 * s], rdir = w.rays[2 * s + 1];
  return make_vertex(S, f3(rorg.x, rorg.y, rorg.z), f3(rdir.x, rdir.y, rdir.z), __float_as_uint(h.y), h.x);
}

}  // namespace sdd
