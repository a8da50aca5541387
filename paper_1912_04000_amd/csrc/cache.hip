// gfx950 kernels of the learned spectral radiance cache.
//
// The cache stands where the paper's photon maps supply indirect light (section 4): paths stop
// at their third surface vertex and add the network's estimate of the outgoing spectral
// radiance there. The network is the multiresolution hash encoding of Mueller et al. 2022
// (3D position grid + 2D octahedral direction grid), a material embedding and a one-blob
// wavelength encoding, followed by four 64-wide ReLU layers without biases and one output.
//
// Matrix-core layout (v_mfma_f32_32x32x16_bf16, FP32 accumulation). A layer is evaluated
// transposed, D[unit][vertex] = W[unit][k] . H^T[k][vertex], so that the 32 lanes of a half
// wave each own one query vertex (a row of the batch) and the weights are the A operand:
//   A (weights)      lane L holds A[L % 32][8 (L / 32) + i], i < 8
//   B (activations)  lane L holds B[8 (L / 32) + i][L % 32]
//   D                register r holds D[8 (r / 4) + 4 (L / 32) + r % 4][L % 32]
// A lane therefore ends a layer holding 32 of the 64 units of its own vertex. Those values are
// reused in place as the next layer's B operand: B block kb takes registers 8 (kb % 2) .. +7 of
// output tile kb / 2, which is unit U(k) = 32 (kb / 2) + 16 (kb % 2) + 8 (i / 4) + 4 h + i % 4
// for physical k = 16 kb + 8 h + i. The input columns of W1..W3 (and of the transposed weights
// of the backward pass) are stored in that order, so no data moves between lanes.
//
// The first layer is split: W0 [e_v ; blob_j] = W0_e e_v + W0_b blob_j. The per-vertex part z_v
// is one MFMA pass per 32 vertices; the per-bin part u_j is a small table; every bin of every
// vertex then costs h1 = relu(z_v + u_j) and three MFMA layers.
#include "device_common.h"

namespace sdd {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kCWG = kCacheWaves * 64;

__device__ __forceinline__ bf16x8 as_bf8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }
__device__ __forceinline__ uint4 as_u4(bf16x8 b) { return __builtin_bit_cast(uint4, b); }
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ float bf_f(__bf16 b) { return (float)b; }
__device__ __forceinline__ uint16_t bf_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ uint32_t bf_pair(float a, float b) {
  return (uint32_t)bf_bits(a) | ((uint32_t)bf_bits(b) << 16);
}

// ReLU of packed bf16 values: a negative bf16 is a negative int16, so max(x, 0) on the integer
// view zeroes exactly the negative values (and -0).
__device__ __forceinline__ bf16x8 relu8(bf16x8 b) {
  short8 s = __builtin_bit_cast(short8, b);
  const short8 z = {0, 0, 0, 0, 0, 0, 0, 0};
  s = __builtin_elementwise_max(s, z);
  return __builtin_bit_cast(bf16x8, s);
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.0f;
  return z;
}

// Two floats -> a packed bf16 pair (round to nearest even), one v_cvt_pk_bf16_f32: converting
// the two as a 2-vector keeps the compiler from converting them one by one and packing them
// with a permute.
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cvt_pk(float a, float b) {
  const f32x2v f = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2v));
}
// Eight floats (x[o .. o + 7] of a D tile) -> one B operand.
__device__ __forceinline__ bf16x8 pack8(const f32x16& x, int o) {
  return as_bf8(make_uint4(cvt_pk(x[o], x[o + 1]), cvt_pk(x[o + 2], x[o + 3]), cvt_pk(x[o + 4], x[o + 5]),
                           cvt_pk(x[o + 6], x[o + 7])));
}

// D tiles (two 32-unit output tiles) -> four B operands (bf16), optional ReLU.
__device__ __forceinline__ void pack_b(const f32x16& a0, const f32x16& a1, bf16x8 b[4]) {
  b[0] = pack8(a0, 0);
  b[1] = pack8(a0, 8);
  b[2] = pack8(a1, 0);
  b[3] = pack8(a1, 8);
}

// One 64x64 layer: (a0, a1) = W . B over the four K blocks.
__device__ __forceinline__ void layer64(const uint4* __restrict__ w, int lane, const bf16x8 b[4], f32x16& a0,
                                        f32x16& a1) {
  a0 = zero16();
  a1 = zero16();
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    a0 = mfma(as_bf8(w[(0 * 4 + kb) * 64 + lane]), b[kb], a0);
    a1 = mfma(as_bf8(w[(1 * 4 + kb) * 64 + lane]), b[kb], a1);
  }
}
__device__ __forceinline__ void layer64r(const bf16x8 w[2][4], const bf16x8 b[4], f32x16& a0, f32x16& a1) {
  a0 = zero16();
  a1 = zero16();
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    a0 = mfma(w[0][kb], b[kb], a0);
    a1 = mfma(w[1][kb], b[kb], a1);
  }
}

// Wave-scope ordering of LDS traffic between lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------------------------
// encoding
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t grid_index3(int x, int y, int z, int N, bool dense, uint32_t mask) {
  if (dense) {
    const uint32_t s = (uint32_t)N + 1u;
    return (uint32_t)x + s * ((uint32_t)y + s * (uint32_t)z);
  }
  return ((uint32_t)x ^ ((uint32_t)y * 2654435761u) ^ ((uint32_t)z * 805459861u)) & mask;
}
__device__ __forceinline__ uint32_t grid_index2(int x, int y, int N, bool dense, uint32_t mask) {
  if (dense) return (uint32_t)x + ((uint32_t)N + 1u) * (uint32_t)y;
  return ((uint32_t)x ^ ((uint32_t)y * 2654435761u)) & mask;
}

// Normalised position in [0, 1 - 2^-20]^3.
__device__ __forceinline__ F3 cache_pos(const CacheDev& C, F3 x) {
  const float hi = 1.0f - 0x1p-20f;
  return f3(fminf(fmaxf((x.x - C.lo[0]) / C.ext[0], 0.0f), hi), fminf(fmaxf((x.y - C.lo[1]) / C.ext[1], 0.0f), hi),
            fminf(fmaxf((x.z - C.lo[2]) / C.ext[2], 0.0f), hi));
}

// Octahedral map of a unit direction to [0,1]^2 (lower hemisphere folded outward).
__device__ __forceinline__ float2 octahedral(F3 w) {
  const float s = fabsf(w.x) + fabsf(w.y) + fabsf(w.z);
  float px = w.x / s, py = w.y / s;
  if (w.z < 0.0f) {
    const float fx = (1.0f - fabsf(py)) * copysignf(1.0f, px);
    const float fy = (1.0f - fabsf(px)) * copysignf(1.0f, py);
    px = fx;
    py = fy;
  }
  const float hi = 1.0f - 0x1p-20f;
  return make_float2(fminf(fmaxf((px + 1.0f) * 0.5f, 0.0f), hi), fminf(fmaxf((py + 1.0f) * 0.5f, 0.0f), hi));
}

// Trilinear interpolation of the two features of position level l.
__device__ __forceinline__ float2 enc_pos(const CacheDev& C, int l, F3 p) {
  const int N = C.Npos[l];
  const bool dense = (C.dense_pos >> l) & 1u;
  const uint32_t mask = (1u << C.Tp_log2) - 1u;
  const float xs = p.x * (float)N, ys = p.y * (float)N, zs = p.z * (float)N;
  const float x0 = floorf(xs), y0 = floorf(ys), z0 = floorf(zs);
  const float fx = xs - x0, fy = ys - y0, fz = zs - z0;
  const int ix = (int)x0, iy = (int)y0, iz = (int)z0;
  const uint32_t* tab = C.gpos + ((size_t)l << C.Tp_log2);
  float a = 0.0f, b = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
    const float w = (ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy) * (oz ? fz : 1.0f - fz);
    const uint32_t v = tab[grid_index3(ix + ox, iy + oy, iz + oz, N, dense, mask)];
    a += w * bf_lo(v);
    b += w * bf_hi(v);
  }
  return make_float2(a, b);
}

// Bilinear interpolation of the two features of direction level l.
__device__ __forceinline__ float2 enc_dir(const CacheDev& C, int l, float2 uv) {
  const int N = C.Ndir[l];
  const bool dense = (C.dense_dir >> l) & 1u;
  const uint32_t mask = (1u << C.Td_log2) - 1u;
  const float xs = uv.x * (float)N, ys = uv.y * (float)N;
  const float x0 = floorf(xs), y0 = floorf(ys);
  const float fx = xs - x0, fy = ys - y0;
  const int ix = (int)x0, iy = (int)y0;
  const uint32_t* tab = C.gdir + ((size_t)l << C.Td_log2);
  float a = 0.0f, b = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int ox = c & 1, oy = c >> 1;
    const float w = (ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy);
    const uint32_t v = tab[grid_index2(ix + ox, iy + oy, N, dense, mask)];
    a += w * bf_lo(v);
    b += w * bf_hi(v);
  }
  return make_float2(a, b);
}

// Encoding tile of one wave: row v = [pos features | dir features | material | 0 ...] (bf16),
// the wavelength columns left at zero (they enter through the u_j table). Lane (v, h) fills
// the levels l = h, h + 2, ... of vertex v.
__device__ __forceinline__ void encode_tile(const CacheDev& C, uint16_t* E, int v, int h, F3 x, F3 wo, int mat) {
  uint32_t* row = (uint32_t*)(E + v * kCacheERow);
  const F3 p = cache_pos(C, x);
  for (int l = h; l < C.Lp; l += 2) {
    const float2 f = enc_pos(C, l, p);
    row[l] = bf_pair(f.x, f.y);
  }
  const float2 uv = octahedral(wo);
  for (int l = h; l < C.Ld; l += 2) {
    const float2 f = enc_dir(C, l, uv);
    row[C.Lp + l] = bf_pair(f.x, f.y);
  }
  const int mc = C.Lp + C.Ld;  // word column of the material embedding
  const float* me = C.P + C.o_mat + (size_t)min(max(mat, 0), C.n_mat - 1) * kCacheMatDim;
  row[mc + 2 * h] = bf_pair(me[4 * h], me[4 * h + 1]);
  row[mc + 2 * h + 1] = bf_pair(me[4 * h + 2], me[4 * h + 3]);
  for (int c = mc + 4 + h; c < kCacheWidth / 2; c += 2) row[c] = 0u;
}

// z_v = W0 [e_v ; 0] for the 32 vertices of the tile (D layout).
__device__ __forceinline__ void first_layer(const CacheDev& C, const uint16_t* E, int lane, f32x16& z0, f32x16& z1) {
  const int v = lane & 31, h = lane >> 5;
  bf16x8 b[4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) b[kb] = as_bf8(*(const uint4*)(E + v * kCacheERow + 16 * kb + 8 * h));
  layer64(C.wf, lane, b, z0, z1);
}

// One-blob encoding of the wavelength parameter t (8 Gaussians of width 1/8), bf16-rounded.
__device__ __forceinline__ float blob(float t, int k) {
  const float c = ((float)k + 0.5f) * (1.0f / kCacheBlob);
  const float d = t - c;
  return bf_f((__bf16)expf(-0.5f * d * d * (float)(kCacheBlob * kCacheBlob)));
}

// u_j = W0_blob . blob_j for every bin (LDS table [B][64] FP32).
__device__ void build_u_table(const CacheDev& C, int B, float* u) {
  const int cb = 2 * (C.Lp + C.Ld) + kCacheMatDim;  // first wavelength column of W0
  const float* W0 = C.P + C.o_w[0];
  for (int i = threadIdx.x; i < B * kCacheWidth; i += blockDim.x) {
    const int j = i / kCacheWidth, unit = i % kCacheWidth;
    const float t = ((float)j + 0.5f) / (float)B;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kCacheBlob; ++k) s += bf_f((__bf16)W0[(size_t)unit * C.n_in + cb + k]) * blob(t, k);
    u[i] = s;
  }
}

// h1 = relu(z + u_j) as B operands.
__device__ __forceinline__ void hidden1(const f32x16& z0, const f32x16& z1, const float* uj, int h, bf16x8 b[4]) {
  uint32_t w[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 u0 = *(const float4*)(uj + 8 * q + 4 * h);
    const float4 u1 = *(const float4*)(uj + 32 + 8 * q + 4 * h);
    const int kb0 = q / 2, kb1 = 2 + q / 2, i0 = 2 * (q % 2);
    w[kb0][i0] = cvt_pk(z0[4 * q + 0] + u0.x, z0[4 * q + 1] + u0.y);
    w[kb0][i0 + 1] = cvt_pk(z0[4 * q + 2] + u0.z, z0[4 * q + 3] + u0.w);
    w[kb1][i0] = cvt_pk(z1[4 * q + 0] + u1.x, z1[4 * q + 1] + u1.y);
    w[kb1][i0 + 1] = cvt_pk(z1[4 * q + 2] + u1.z, z1[4 * q + 3] + u1.w);
  }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) b[kb] = relu8(as_bf8(make_uint4(w[kb][0], w[kb][1], w[kb][2], w[kb][3])));
}

// y = w4 . h4 over the lane's 32 units, then summed with the other half of the wave.
__device__ __forceinline__ float output_dot(const bf16x8 h4[4], const bf16x8 w4[4]) {
  float y = 0.0f;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
      const bf16x2v a = {h4[kb][i], h4[kb][i + 1]};
      const bf16x2v c = {w4[kb][i], w4[kb][i + 1]};
      y = __builtin_amdgcn_fdot2_f32_bf16(a, c, y, false);
    }
  }
  return y + __shfl_xor(y, 32);
}

// ------------------------------------------------------------------------------------------
// inference: render-time queries (lacc += beta max(y, 0)) and the evaluation entry point
// ------------------------------------------------------------------------------------------
struct QueryOut {
  // render mode: slot rows
  const float* beta;
  float* lacc;
  int Bp;
  // evaluation mode: out [n][B]
  float* out;
};

template <bool kRender>
__device__ __forceinline__ void query_wave(const CacheDev& C, int B, const float* u, uint16_t* E, float* Y, int lane,
                                           bool valid, uint32_t row_id, F3 x, F3 wo, int mat,
                                           const bf16x8 W[3][2][4], const bf16x8 w4[4], const QueryOut& o) {
  const int v = lane & 31, h = lane >> 5;
  encode_tile(C, E, v, h, x, wo, mat);
  wave_sync();
  f32x16 z0, z1;
  first_layer(C, E, lane, z0, z1);
  for (int j0 = 0; j0 < B; j0 += 8) {
    const int jn = min(8, B - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const int j = j0 + jj;
      bf16x8 b[4];
      hidden1(z0, z1, u + j * kCacheWidth, h, b);
      f32x16 a0, a1;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        layer64r(W[l], b, a0, a1);
        pack_b(a0, a1, b);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) b[kb] = relu8(b[kb]);
      }
      const float y = output_dot(b, w4);
      if (h == 0) Y[v * 8 + jj] = y;
    }
    wave_sync();
    // lane (v, h) owns bins j0 + 4h .. j0 + 4h + 3 of vertex v
    const int jb = j0 + 4 * h;
    if (valid && jb < B) {
      float y4[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) y4[c] = (jb + c < B) ? Y[v * 8 + 4 * h + c] : 0.0f;
      if (kRender) {
        const float4 be = *(const float4*)(o.beta + (size_t)row_id * o.Bp + jb);
        float4* lp = (float4*)(o.lacc + (size_t)row_id * o.Bp + jb);
        float4 l = *lp;
        l.x += be.x * fmaxf(y4[0], 0.0f);
        l.y += be.y * fmaxf(y4[1], 0.0f);
        l.z += be.z * fmaxf(y4[2], 0.0f);
        l.w += be.w * fmaxf(y4[3], 0.0f);
        *lp = l;
      } else {
        for (int c = 0; c < 4 && jb + c < B; ++c) o.out[(size_t)row_id * B + jb + c] = y4[c];
      }
    }
    wave_sync();
  }
}

__device__ __forceinline__ void load_weights(const CacheDev& C, int lane, bf16x8 W[3][2][4], bf16x8 w4[4]) {
  const int h = lane >> 5;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) W[l][mt][kb] = as_bf8(C.wf[(((l + 1) * 2 + mt) * 4 + kb) * 64 + lane]);
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) w4[kb] = as_bf8(C.w4b[kb * 2 + h]);
}

// Queries of the render: the hits of bounce-2 continuations (opaque and glass lists of the
// bounce parity p), 32 per wave.
__global__ __launch_bounds__(kCWG) __attribute__((amdgpu_waves_per_eu(2))) void k_cache_query(CacheDev C, DevScene S, DevWS w, int p) {
  __shared__ __attribute__((aligned(16))) float u[kMaxBins * kCacheWidth];
  __shared__ __attribute__((aligned(16))) uint16_t Es[kCacheWaves * kCacheVerts * kCacheERow];
  __shared__ float Ys[kCacheWaves * kCacheVerts * 8];
  __shared__ uint32_t s_st[1];
  const int B = S.n_bins;
  stats_init(s_st, 1);
  build_u_table(C, B, u);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, v = lane & 31;
  bf16x8 W[3][2][4], w4[4];
  load_weights(C, lane, W, w4);
  const uint32_t n_o = w.ctl->cat_count[p][kCatOpaque * kKeyStride], n_g = w.ctl->cat_count[p][kCatGlass * kKeyStride];
  const uint32_t n = n_o + n_g;
  const uint32_t* lo = w.cat + ((size_t)p * kCats + kCatOpaque) * w.W;
  const uint32_t* lg = w.cat + ((size_t)p * kCats + kCatGlass) * w.W;
  QueryOut o{w.beta, w.lacc, w.Bp, nullptr};
  for (uint32_t base = (blockIdx.x * kCacheWaves + wave) * kCacheVerts; base < n;
       base += gridDim.x * kCacheWaves * kCacheVerts) {
    const uint32_t i = base + v;
    const bool valid = i < n;
    F3 x = f3(0.0f, 0.0f, 0.0f), wo = f3(0.0f, 0.0f, 1.0f);
    int mat = 0;
    uint32_t s = 0;
    if (valid) {
      s = i < n_o ? lo[i] : lg[i - n_o];
      const Vertex V = load_vertex(S, w, s);
      x = V.p;
      wo = V.d * -1.0f;
      mat = V.m;
    }
    query_wave<true>(C, B, u, Es + wave * kCacheVerts * kCacheERow, Ys + wave * kCacheVerts * 8, lane, valid, s, x,
                     wo, mat, W, w4, o);
    stats_add_ballot(s_st, 0, valid && lane < 32);
  }
  __syncthreads();
  stats_flush(s_st, 0, &w.ctl->st_queries);
}

// Network output y (before the clamp at zero) for explicit vertices: out [n][B].
__global__ __launch_bounds__(kCWG) __attribute__((amdgpu_waves_per_eu(2))) void k_cache_eval(CacheDev C, const float* X, const float* WO, const int32_t* MAT,
                                                     uint32_t n, int B, float* out) {
  __shared__ __attribute__((aligned(16))) float u[kMaxBins * kCacheWidth];
  __shared__ __attribute__((aligned(16))) uint16_t Es[kCacheWaves * kCacheVerts * kCacheERow];
  __shared__ float Ys[kCacheWaves * kCacheVerts * 8];
  build_u_table(C, B, u);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, v = lane & 31;
  bf16x8 W[3][2][4], w4[4];
  load_weights(C, lane, W, w4);
  QueryOut o{nullptr, nullptr, 0, out};
  for (uint32_t base = (blockIdx.x * kCacheWaves + wave) * kCacheVerts; base < n;
       base += gridDim.x * kCacheWaves * kCacheVerts) {
    const uint32_t i = base + v;
    const bool valid = i < n;
    F3 x = f3(0.0f, 0.0f, 0.0f), wo = f3(0.0f, 0.0f, 1.0f);
    int mat = 0;
    if (valid) {
      x = f3(X[3 * i], X[3 * i + 1], X[3 * i + 2]);
      wo = f3(WO[3 * i], WO[3 * i + 1], WO[3 * i + 2]);
      mat = MAT[i];
    }
    query_wave<false>(C, B, u, Es + wave * kCacheVerts * kCacheERow, Ys + wave * kCacheVerts * 8, lane, valid, i, x,
                      wo, mat, W, w4, o);
  }
}

// ------------------------------------------------------------------------------------------
// training
// ------------------------------------------------------------------------------------------
// Tiles of stored activations / deltas: [layer][tile][unit 64][row 32] bf16, tile = block * B + j.
__device__ __forceinline__ uint16_t* tile_ptr(uint16_t* base, int layer, size_t n_tiles_max, size_t t) {
  return base + ((size_t)layer * n_tiles_max + t) * (kCacheWidth * 32);
}

// Store a B-operand set (lane holds units U(kb, h, i) of row v) into a tile. The bf16 bits are
// taken from the operand's 32-bit words with shifts (element i sits in word i / 2, high half for
// odd i): extracting single bf16 elements of the vector as 16-bit integers is miscompiled here
// (every element was stored from the first word).
__device__ __forceinline__ void store_tile_b(uint16_t* tile, int v, int h, const bf16x8 b[4]) {
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const uint4 u = as_u4(b[kb]);
    const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int U = 32 * (kb / 2) + 16 * (kb % 2) + 8 * (i / 4) + 4 * h + (i % 4);
      tile[U * 32 + v] = (uint16_t)(wd[i / 2] >> (16 * (i % 2)));
    }
  }
}

// delta = dh (D tiles) masked by h > 0, as B operands.
__device__ __forceinline__ void mask_delta(const f32x16& a0, const f32x16& a1, const bf16x8 hb[4], bf16x8 d[4]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    d[0][i] = (__bf16)(bf_f(hb[0][i]) > 0.0f ? a0[i] : 0.0f);
    d[1][i] = (__bf16)(bf_f(hb[1][i]) > 0.0f ? a0[8 + i] : 0.0f);
    d[2][i] = (__bf16)(bf_f(hb[2][i]) > 0.0f ? a1[i] : 0.0f);
    d[3][i] = (__bf16)(bf_f(hb[3][i]) > 0.0f ? a1[8 + i] : 0.0f);
  }
}

// Records of a training step: the compacted records [v0, v0 + nv) with nv = clamp(count - v0,
// 0, step_max). Returns nv.
__device__ __forceinline__ uint32_t step_range(const CacheDev& C, uint32_t v0, uint32_t step_max) {
  const uint32_t cnt = C.ridx[C.max_train];
  return cnt > v0 ? min(cnt - v0, step_max) : 0u;
}

// Forward and backward pass of 32 vertices x B bins per wave: stores the layer inputs and the
// deltas (for the weight gradients), the encoding gradient dE of every vertex, adds the output
// weights' gradient and the loss.
__global__ __launch_bounds__(kCWG) void k_cache_train(CacheDev C, int B, uint32_t v0, uint32_t step_max) {
  __shared__ __attribute__((aligned(16))) float u[kMaxBins * kCacheWidth];
  __shared__ __attribute__((aligned(16))) uint16_t Es[kCacheWaves * kCacheVerts * kCacheERow];
  __shared__ float gw4[kCacheWidth];
  __shared__ float lsum;
  const uint32_t nv = step_range(C, v0, step_max);
  const uint32_t blocks = (nv + kCacheVerts - 1) / kCacheVerts;
  if (blockIdx.x * kCacheWaves >= blocks) return;  // uniform over the workgroup
  build_u_table(C, B, u);
  if (threadIdx.x < kCacheWidth) gw4[threadIdx.x] = 0.0f;
  if (threadIdx.x == 0) lsum = 0.0f;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, v = lane & 31, h = lane >> 5;
  const uint32_t blk = blockIdx.x * kCacheWaves + wave;
  const size_t n_tiles_max = (size_t)((C.max_step + kCacheVerts - 1) / kCacheVerts) * C.max_bins;
  const float inv_rows = 1.0f / ((float)nv * (float)B);
  uint16_t* E = Es + wave * kCacheVerts * kCacheERow;
  if (blk < blocks) {
    const uint32_t k = blk * kCacheVerts + v;
    const bool valid = k < nv;
    uint32_t slot = 0;
    F3 x = f3(0.0f, 0.0f, 0.0f), wo = f3(0.0f, 0.0f, 1.0f);
    int mat = 0;
    if (valid) {
      slot = C.ridx[v0 + k];
      const float4 a = C.rx[slot], b = C.rw[slot];
      x = f3(a.x, a.y, a.z);
      mat = (int)__float_as_uint(a.w);
      wo = f3(b.x, b.y, b.z);
    }
    encode_tile(C, E, v, h, x, wo, mat);
    wave_sync();
    f32x16 z0, z1;
    first_layer(C, E, lane, z0, z1);
    bf16x8 w4[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) w4[kb] = as_bf8(C.w4b[kb * 2 + h]);
    // input row e_v (bf16, natural column order) for the stored layer-0 inputs
    const uint16_t* erow = E + v * kCacheERow;
    const int cb = 2 * (C.Lp + C.Ld) + kCacheMatDim;
    float dsum[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) dsum[r] = 0.0f;
    float gacc[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) gacc[r] = 0.0f;
    float lpart = 0.0f;
    for (int j = 0; j < B; ++j) {
      const size_t t = (size_t)blk * B + j;
      // layer-0 input tile: unit c of row v (columns 32 h .. 32 h + 31 by this lane)
      {
        uint16_t* tile = tile_ptr(C.hst, 0, n_tiles_max, t);
        const float tj = ((float)j + 0.5f) / (float)B;
        for (int c = 32 * h; c < 32 * h + 32; ++c) {
          uint16_t val = erow[c];
          if (c >= cb && c < cb + kCacheBlob) val = bf_bits(blob(tj, c - cb));
          tile[c * 32 + v] = valid ? val : (uint16_t)0;
        }
      }
      bf16x8 hb[4][4];  // h1..h4 as B operands
      hidden1(z0, z1, u + j * kCacheWidth, h, hb[0]);
      f32x16 a0, a1;
#pragma unroll
      for (int l = 1; l < 4; ++l) {
        layer64(C.wf + l * 512, lane, hb[l - 1], a0, a1);
        pack_b(a0, a1, hb[l]);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) hb[l][kb] = relu8(hb[l][kb]);
      }
      const float y = output_dot(hb[3], w4);
      const float tg = valid ? C.tgt[(size_t)slot * C.max_bins + j] : 0.0f;
      const float den = y * y + 0.01f;
      const float dy = valid ? 2.0f * (y - tg) / den * inv_rows : 0.0f;
      if (valid && h == 0) lpart += (y - tg) * (y - tg) / den;
      // output weights: dw4[U] += dy h4[U]
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 8; ++i) gacc[kb * 8 + i] += dy * bf_f(hb[3][kb][i]);
      // delta4 = dy w4 (h4 > 0)
      bf16x8 d[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 8; ++i) d[kb][i] = (__bf16)(bf_f(hb[3][kb][i]) > 0.0f ? dy * bf_f(w4[kb][i]) : 0.0f);
      for (int l = 3; l >= 1; --l) {
        store_tile_b(tile_ptr(C.hst, l, n_tiles_max, t), v, h, hb[l - 1]);
        store_tile_b(tile_ptr(C.dst, l, n_tiles_max, t), v, h, d);
        layer64(C.wb + l * 512, lane, d, a0, a1);  // dh_{l} = W_l^T delta_{l+1}
        mask_delta(a0, a1, hb[l - 1], d);
      }
      store_tile_b(tile_ptr(C.dst, 0, n_tiles_max, t), v, h, d);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 8; ++i) dsum[kb * 8 + i] += bf_f(d[kb][i]);
    }
    // dE = W0^T sum_j delta1 (hi/lo bf16 split of the FP32 sum)
    bf16x8 dh[4], dl[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const __bf16 hi = (__bf16)dsum[kb * 8 + i];
        dh[kb][i] = hi;
        dl[kb][i] = (__bf16)(dsum[kb * 8 + i] - bf_f(hi));
      }
    f32x16 e0, e1, f0, f1;
    layer64(C.wb, lane, dh, e0, e1);
    layer64(C.wb, lane, dl, f0, f1);
    if (valid) {
      float* de = C.dE + (size_t)k * kCacheWidth;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        *(float4*)(de + 8 * q + 4 * h) = make_float4(e0[4 * q] + f0[4 * q], e0[4 * q + 1] + f0[4 * q + 1],
                                                     e0[4 * q + 2] + f0[4 * q + 2], e0[4 * q + 3] + f0[4 * q + 3]);
        *(float4*)(de + 32 + 8 * q + 4 * h) = make_float4(e1[4 * q] + f1[4 * q], e1[4 * q + 1] + f1[4 * q + 1],
                                                          e1[4 * q + 2] + f1[4 * q + 2], e1[4 * q + 3] + f1[4 * q + 3]);
      }
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int U = 32 * (kb / 2) + 16 * (kb % 2) + 8 * (i / 4) + 4 * h + (i % 4);
        float g = gacc[kb * 8 + i];
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) g += __shfl_xor(g, o);
        if (v == 0) atomicAdd(&gw4[U], g);
      }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) lpart += __shfl_xor(lpart, o);
    if (lane == 0) atomicAdd(&lsum, lpart);
  }
  __syncthreads();
  if (threadIdx.x < kCacheWidth) atomicAdd(C.G + C.o_w4 + threadIdx.x, gw4[threadIdx.x]);
  if (threadIdx.x == 0) {
    atomicAdd(C.loss, lsum);
    if (blockIdx.x == 0) atomicAdd(C.loss + 1, (float)nv * (float)B);
  }
}

// Weight gradients dW_l = sum over rows of delta_{l+1} (x) h_l: MFMA with the rows as K.
// Workgroup = 4 waves, each wave a contiguous range of tiles of one layer.
__global__ __launch_bounds__(kCWG) void k_cache_wgrad(CacheDev C, int B, uint32_t v0, uint32_t step_max,
                                                      int tiles_per_wave) {
  const uint32_t nv = step_range(C, v0, step_max);
  const uint32_t n_tiles = (nv + kCacheVerts - 1) / kCacheVerts * (uint32_t)B;
  const int layer = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5, m = lane & 31;
  const uint32_t t0 = (blockIdx.x * kCacheWaves + wave) * (uint32_t)tiles_per_wave;
  if (t0 >= n_tiles) return;
  const uint32_t t1 = min(n_tiles, t0 + (uint32_t)tiles_per_wave);
  const size_t n_tiles_max = (size_t)((C.max_step + kCacheVerts - 1) / kCacheVerts) * C.max_bins;
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero16();
  for (uint32_t t = t0; t < t1; ++t) {
    const uint16_t* dt = tile_ptr(C.dst, layer, n_tiles_max, t);
    const uint16_t* ht = tile_ptr(C.hst, layer, n_tiles_max, t);
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      bf16x8 A[2], Bo[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        A[q] = as_bf8(*(const uint4*)(dt + (32 * q + m) * 32 + 16 * kb + 8 * h));
        Bo[q] = as_bf8(*(const uint4*)(ht + (32 * q + m) * 32 + 16 * kb + 8 * h));
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma(A[a], Bo[b], acc[a][b]);
    }
  }
  const int ncols = layer == 0 ? C.n_in : kCacheWidth;
  float* g = C.G + C.o_w[layer];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int out = 32 * a + 8 * (r / 4) + 4 * h + (r % 4);
        const int in = 32 * b + m;
        if (in < ncols) atomicAdd(g + (size_t)out * ncols + in, acc[a][b][r]);
      }
}

// Hash-grid and material-embedding gradients: scatter dE through the interpolation weights.
// One thread per (level, vertex) of position and direction plus one per vertex for the
// material; consecutive threads take consecutive vertices of one level, so the atomics of a
// wave on a coarse level fall on few table entries.
__global__ void k_cache_grid_bwd(CacheDev C, uint32_t v0, uint32_t step_max) {
  const uint32_t nv = step_range(C, v0, step_max);
  const int per = C.Lp + C.Ld + 1;
  const uint64_t total = (uint64_t)nv * per;
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)(q % nv);
    const int l = (int)(q / nv);
    const uint32_t slot = C.ridx[v0 + k];
    const float* de = C.dE + (size_t)k * kCacheWidth;
    if (l < C.Lp) {
      const float4 a = C.rx[slot];
      const F3 p = cache_pos(C, f3(a.x, a.y, a.z));
      const int N = C.Npos[l];
      const bool dense = (C.dense_pos >> l) & 1u;
      const uint32_t mask = (1u << C.Tp_log2) - 1u;
      const float xs = p.x * (float)N, ys = p.y * (float)N, zs = p.z * (float)N;
      const float x0 = floorf(xs), y0 = floorf(ys), z0 = floorf(zs);
      const float fx = xs - x0, fy = ys - y0, fz = zs - z0;
      const float g0 = de[2 * l], g1 = de[2 * l + 1];
      float* gt = C.G + C.o_pos + ((size_t)l << C.Tp_log2) * kCacheFeat;
      for (int c = 0; c < 8; ++c) {
        const int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
        const float w = (ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy) * (oz ? fz : 1.0f - fz);
        const uint32_t idx = grid_index3((int)x0 + ox, (int)y0 + oy, (int)z0 + oz, N, dense, mask);
        atomicAdd(gt + 2 * (size_t)idx, w * g0);
        atomicAdd(gt + 2 * (size_t)idx + 1, w * g1);
      }
    } else if (l < C.Lp + C.Ld) {
      const int ld = l - C.Lp;
      const float4 b = C.rw[slot];
      const float2 uv = octahedral(f3(b.x, b.y, b.z));
      const int N = C.Ndir[ld];
      const bool dense = (C.dense_dir >> ld) & 1u;
      const uint32_t mask = (1u << C.Td_log2) - 1u;
      const float xs = uv.x * (float)N, ys = uv.y * (float)N;
      const float x0 = floorf(xs), y0 = floorf(ys);
      const float fx = xs - x0, fy = ys - y0;
      const float g0 = de[2 * l], g1 = de[2 * l + 1];
      float* gt = C.G + C.o_dir + ((size_t)ld << C.Td_log2) * kCacheFeat;
      for (int c = 0; c < 4; ++c) {
        const int ox = c & 1, oy = c >> 1;
        const float w = (ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy);
        const uint32_t idx = grid_index2((int)x0 + ox, (int)y0 + oy, N, dense, mask);
        atomicAdd(gt + 2 * (size_t)idx, w * g0);
        atomicAdd(gt + 2 * (size_t)idx + 1, w * g1);
      }
    } else {
      const int mat = min(max((int)__float_as_uint(C.rx[slot].w), 0), C.n_mat - 1);
      const int mc = 2 * (C.Lp + C.Ld);
      for (int c = 0; c < kCacheMatDim; ++c) atomicAdd(C.G + C.o_mat + (size_t)mat * kCacheMatDim + c, de[mc + c]);
    }
  }
}

// Adam bookkeeping of one step: skipped (flag 0) when the step has no records; else the step
// count advances and the bias corrections 1/(1 - b^t) are formed as -1/expm1(t log1p(b - 1)),
// which keeps FP32 accuracy when b^t is close to 1 (b - 1 is exact for b in [1/2, 1]).
__global__ void k_cache_adam_prep(CacheDev C, uint32_t v0, uint32_t step_max, float* opt, float b1, float b2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t nv = step_range(C, v0, step_max);
  if (nv == 0) {
    opt[3] = 0.0f;
    return;
  }
  const uint32_t t = __float_as_uint(opt[0]) + 1u;
  opt[0] = __uint_as_float(t);
  opt[1] = -1.0f / expm1f((float)t * log1pf(b1 - 1.0f));
  opt[2] = -1.0f / expm1f((float)t * log1pf(b2 - 1.0f));
  opt[3] = 1.0f;
}

// Adam (Kingma & Ba 2015) over every parameter pair, the bf16 grid copies refreshed and the
// gradients cleared for the next step.
__global__ void k_cache_adam(CacheDev C, const float* opt, float lr, float b1, float b2, float eps) {
  if (opt[3] == 0.0f) return;
  const float c1 = opt[1], c2 = opt[2];
  const int64_t n = C.n_param;
  const int64_t pairs = (n + 1) / 2;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < pairs; q += (int64_t)gridDim.x * blockDim.x) {
    float pv[2];
    for (int e = 0; e < 2; ++e) {
      const int64_t i = 2 * q + e;
      if (i >= n) {
        pv[e] = 0.0f;
        continue;
      }
      const float g = C.G[i];
      const float m = b1 * C.M[i] + (1.0f - b1) * g;
      const float vv = b2 * C.V[i] + (1.0f - b2) * g * g;
      C.M[i] = m;
      C.V[i] = vv;
      const float p = C.P[i] - lr * (m * c1) / (sqrtf(vv * c2) + eps);
      C.P[i] = p;
      C.G[i] = 0.0f;
      pv[e] = p;
    }
    const int64_t i = 2 * q;
    if (i < C.o_dir)
      C.gpos[q] = bf_pair(pv[0], pv[1]);
    else if (i < C.o_mat)
      C.gdir[q - C.o_dir / 2] = bf_pair(pv[0], pv[1]);
  }
}

// bf16 copies of the grids from the masters.
__global__ void k_cache_refresh_grids(CacheDev C) {
  const int64_t pairs = C.o_mat / 2;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < pairs; q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t w = bf_pair(C.P[2 * q], C.P[2 * q + 1]);
    if (2 * q < C.o_dir)
      C.gpos[q] = w;
    else
      C.gdir[q - C.o_dir / 2] = w;
  }
}

// Matrix-core operands of the four layers (forward, transposed for the backward pass) and the
// output weights, from the masters. Thread = (layer, mt, kb, lane).
__global__ void k_cache_pack(CacheDev C) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id < 4 * 2 * 4 * 64) {
    const int lane = id & 63, kb = (id >> 6) & 3, mt = (id >> 8) & 1, l = id >> 9;
    const int h = lane >> 5;
    const int M = 32 * mt + (lane & 31);
    const int ncols = l == 0 ? C.n_in : kCacheWidth;
    const float* W = C.P + C.o_w[l];
    bf16x8 f, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 16 * kb + 8 * h + i;
      const int U = 32 * (kb / 2) + 16 * (kb % 2) + 8 * (i / 4) + 4 * h + (i % 4);
      // forward: layer 0 reads its input in natural column order, layers 1..3 in U order
      const int col = l == 0 ? k : U;
      f[i] = (__bf16)(col < ncols ? W[(size_t)M * ncols + col] : 0.0f);
      // backward: A[M = input unit][k] = W[U(k)][M]
      b[i] = (__bf16)(M < ncols ? W[(size_t)U * ncols + M] : 0.0f);
    }
    C.wf[id] = as_u4(f);
    C.wb[id] = as_u4(b);
  } else if (id < 4 * 2 * 4 * 64 + 8) {
    const int e = id - 4 * 2 * 4 * 64;
    const int kb = e >> 1, h = e & 1;
    bf16x8 w;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int U = 32 * (kb / 2) + 16 * (kb % 2) + 8 * (i / 4) + 4 * h + (i % 4);
      w[i] = (__bf16)C.P[C.o_w4 + U];
    }
    C.w4b[e] = as_u4(w);
  }
}

// Deterministic initialisation from Philox (counter = parameter index, purpose 3):
// grids U(-1e-4, 1e-4), material embedding U(-1, 1), weights Glorot-uniform.
__global__ void k_cache_init(CacheDev C, uint32_t k0, uint32_t k1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < C.n_param;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint4 r = philox(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 3u << 24, 0u), k0, k1);
    const float u = unif24(r.x) * 2.0f - 1.0f;
    float lim;
    if (i < C.o_mat)
      lim = 1e-4f;
    else if (i < C.o_w[0])
      lim = 1.0f;
    else if (i < C.o_w[1])
      lim = sqrtf(6.0f / (float)(C.n_in + kCacheWidth));
    else if (i < C.o_w4)
      lim = sqrtf(6.0f / (float)(2 * kCacheWidth));
    else
      lim = sqrtf(6.0f / (float)(kCacheWidth + 1));
    C.P[i] = u * lim;
    C.M[i] = 0.0f;
    C.V[i] = 0.0f;
    C.G[i] = 0.0f;
  }
}

// Explicit records (entry points that train on caller data): slot k = record k.
__global__ void k_cache_load_records(CacheDev C, const float* X, const float* WO, const int32_t* MAT,
                                     const float* T, uint32_t n, int B) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    C.rx[k] = make_float4(X[3 * k], X[3 * k + 1], X[3 * k + 2], __uint_as_float((uint32_t)MAT[k]));
    C.rw[k] = make_float4(WO[3 * k], WO[3 * k + 1], WO[3 * k + 2], 1.0f);
    for (int j = 0; j < B; ++j) C.tgt[(size_t)k * C.max_bins + j] = T[(size_t)k * B + j];
    C.ridx[k] = k;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) C.ridx[C.max_train] = n;
}

// Training paths: each path slot that reached its third vertex holds a record; its suffix
// radiance (gathered after the throughput reset there) becomes the target.
__global__ void k_cache_gather(CacheDev C, DevWS w, uint32_t n, int B) {
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    if (C.rw[s].w == 0.0f) continue;
    const float* l = w.lacc + (size_t)s * w.Bp;
    for (int j = 0; j < B; ++j) C.tgt[(size_t)s * C.max_bins + j] = l[j];
  }
}

// Records in slot order (one workgroup): ridx[0 .. count) and ridx[max_train] = count, count
// capped at cap.
__global__ __launch_bounds__(1024) void k_cache_compact(CacheDev C, uint32_t n, uint32_t cap) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t c0 = 0; c0 < n; c0 += 1024) {
    const uint32_t s = c0 + threadIdx.x;
    const bool ok = s < n && C.rw[s].w != 0.0f;
    const uint64_t m = __ballot(ok);
    if (lane == 0) wsum[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t off = base;
    for (int q = 0; q < wv; ++q) off += wsum[q];
    const uint32_t pos = off + count_below(m);
    if (ok && pos < cap) C.ridx[pos] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int q = 0; q < 16; ++q) t += wsum[q];
      base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) C.ridx[C.max_train] = min(base, cap);
}

// ------------------------------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------------------------------
static inline unsigned cgrid(uint64_t n, unsigned per, unsigned cap) {
  uint64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

hipError_t launch_cache_init(hipStream_t s, const CacheDev& C, uint64_t seed) {
  hipLaunchKernelGGL(k_cache_init, dim3(cgrid(C.n_param, 256, 8192)), dim3(256), 0, s, C, (uint32_t)seed,
                     (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_cache_sync(hipStream_t s, const CacheDev& C) {
  hipLaunchKernelGGL(k_cache_refresh_grids, dim3(cgrid(C.o_mat / 2, 256, 8192)), dim3(256), 0, s, C);
  hipLaunchKernelGGL(k_cache_pack, dim3((4 * 2 * 4 * 64 + 8 + 255) / 256), dim3(256), 0, s, C);
  return hipGetLastError();
}

hipError_t launch_cache_eval(hipStream_t s, const CacheDev& C, const float* x, const float* wo, const int32_t* mat,
                             uint32_t n, int B, float* out) {
  hipLaunchKernelGGL(k_cache_eval, dim3(cgrid(n, kCacheWaves * kCacheVerts, 2048)), dim3(kCWG), 0, s, C, x, wo, mat, n,
                     B, out);
  return hipGetLastError();
}

hipError_t launch_cache_query(hipStream_t s, const CacheDev& C, const DevScene& S, const DevWS& w, int p) {
  hipLaunchKernelGGL(k_cache_query, dim3(cgrid(w.W, kCacheWaves * kCacheVerts, 2048)), dim3(kCWG), 0, s, C, S, w, p);
  return hipGetLastError();
}

hipError_t launch_cache_load_records(hipStream_t s, const CacheDev& C, const float* x, const float* wo,
                                     const int32_t* mat, const float* t, uint32_t n, int B) {
  hipLaunchKernelGGL(k_cache_load_records, dim3(cgrid(n, 256, 4096)), dim3(256), 0, s, C, x, wo, mat, t, n, B);
  return hipGetLastError();
}

hipError_t launch_cache_gather(hipStream_t s, const CacheDev& C, const DevWS& w, uint32_t n, int B) {
  hipLaunchKernelGGL(k_cache_gather, dim3(cgrid(n, 256, 4096)), dim3(256), 0, s, C, w, n, B);
  return hipGetLastError();
}

hipError_t launch_cache_compact(hipStream_t s, const CacheDev& C, uint32_t n, uint32_t cap) {
  hipLaunchKernelGGL(k_cache_compact, dim3(1), dim3(1024), 0, s, C, n, cap);
  return hipGetLastError();
}

// Gradients of one step over records [v0, v0 + step_max) (clamped on the device to the
// record count): loss and gradients accumulate into C.loss and C.G.
hipError_t launch_cache_backward(hipStream_t s, const CacheDev& C, int B, uint32_t v0, uint32_t step_max) {
  const uint32_t blocks = (step_max + kCacheVerts - 1) / kCacheVerts;
  hipLaunchKernelGGL(k_cache_train, dim3((blocks + kCacheWaves - 1) / kCacheWaves), dim3(kCWG), 0, s, C, B, v0,
                     step_max);
  const uint32_t tiles = blocks * (uint32_t)B;
  const int tpw = 16;
  const uint32_t waves = (tiles + tpw - 1) / tpw;
  hipLaunchKernelGGL(k_cache_wgrad, dim3((waves + kCacheWaves - 1) / kCacheWaves, 4), dim3(kCWG), 0, s, C, B, v0,
                     step_max, tpw);
  const uint64_t per = (uint64_t)step_max * (C.Lp + C.Ld + 1);
  hipLaunchKernelGGL(k_cache_grid_bwd, dim3(cgrid(per, 256, 8192)), dim3(256), 0, s, C, v0, step_max);
  return hipGetLastError();
}

hipError_t launch_cache_adam(hipStream_t s, const CacheDev& C, uint32_t v0, uint32_t step_max, float* opt, float lr,
                             float b1, float b2, float eps) {
  hipLaunchKernelGGL(k_cache_adam_prep, dim3(1), dim3(64), 0, s, C, v0, step_max, opt, b1, b2);
  hipLaunchKernelGGL(k_cache_adam, dim3(cgrid((C.n_param + 1) / 2, 256, 8192)), dim3(256), 0, s, C, (const float*)opt,
                     lr, b1, b2, eps);
  hipLaunchKernelGGL(k_cache_pack, dim3((4 * 2 * 4 * 64 + 8 + 255) / 256), dim3(256), 0, s, C);
  return hipGetLastError();
}

}  // namespace sdd
