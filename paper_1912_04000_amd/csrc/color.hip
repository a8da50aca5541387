// Colorimetry of the spectral image on gfx950: [B][n] radiance -> CIE 1931 XYZ -> sRGB.
//
// The paper maps its spectral renderings to RGB by colorimetry for display (section 6), the
// observer's visual adaptation being a colorimetric matter (section 1). The colour-matching
// functions of the CIE 1931 2-degree observer are evaluated from the multi-lobe analytic fit of
// Wyman, Sloan and Shirley (JCGT 2013): sums of piecewise Gaussians exp(-((l - mu) / s)^2 / 2),
// s = s1 below mu and s2 above. Per pixel:
//   XYZ = exposure * sum_j I_j cmf(l_j) / sum_j ybar(l_j)     (bin centres l_j, point samples)
//   linear sRGB = M XYZ (IEC 61966-2-1, D65), clamped to [0, 1], then the sRGB transfer function.
// One pass over the image: the kernel is bound by reading the B planes (HBM).
#include <stdint.h>
#include "internal.h"

namespace sdd {

constexpr int kColorWG = 256;

__device__ __forceinline__ float cie_lobe(float l, float a, float mu, float s1, float s2) {
  const float x = (l - mu) / (l < mu ? s1 : s2);
  return a * expf(-0.5f * x * x);
}

__device__ __forceinline__ float srgb_encode(float c) {
  c = fminf(1.0f, fmaxf(0.0f, c));
  return c <= 0.0031308f ? 12.92f * c : 1.055f * powf(c, 1.0f / 2.4f) - 0.055f;
}

__global__ __launch_bounds__(kColorWG) void k_spectral_to_srgb(const float* __restrict__ img, int B, float lmin,
                                                                float lmax, uint64_t n, float exposure,
                                                                float* __restrict__ xyz, float* __restrict__ srgb,
                                                                bool vec) {
  // per-bin weights cmf(l_j) exposure / sum_k ybar(l_k), staged in LDS by every workgroup
  __shared__ float s_w[3][kMaxBins];
  __shared__ float s_ysum;
  for (int j = threadIdx.x; j < B; j += kColorWG) {
    const float l = lmin + ((float)j + 0.5f) * (lmax - lmin) / (float)B;
    s_w[0][j] = cie_lobe(l, 1.056f, 599.8f, 37.9f, 31.0f) + cie_lobe(l, 0.362f, 442.0f, 16.0f, 26.7f) +
                cie_lobe(l, -0.065f, 501.1f, 20.4f, 26.2f);
    s_w[1][j] = cie_lobe(l, 0.821f, 568.8f, 46.9f, 40.5f) + cie_lobe(l, 0.286f, 530.9f, 16.3f, 31.1f);
    s_w[2][j] = cie_lobe(l, 1.217f, 437.0f, 11.8f, 36.0f) + cie_lobe(l, 0.681f, 459.0f, 26.0f, 13.8f);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float y = 0.0f;
    for (int j = 0; j < B; ++j) y += s_w[1][j];
    s_ysum = exposure / y;
  }
  __syncthreads();
  const float k = s_ysum;
  for (int j = threadIdx.x; j < B; j += kColorWG) {
    s_w[0][j] *= k;
    s_w[1][j] *= k;
    s_w[2][j] *= k;
  }
  __syncthreads();
  // Four consecutive pixels per thread when every plane starts 16-byte aligned: one float4 load
  // per plane, the XYZ planes and the interleaved sRGB triples stored as whole float4 (full
  // 64-byte segments per wave); the remaining pixels one per thread.
  const uint64_t n4 = vec ? n / 4 : 0;
  for (uint64_t q = (uint64_t)blockIdx.x * kColorWG + threadIdx.x; q < n4; q += (uint64_t)gridDim.x * kColorWG) {
    float4 X = make_float4(0.0f, 0.0f, 0.0f, 0.0f), Y = X, Z = X;
    const float4* src = (const float4*)img + q;
    const uint64_t n_4 = n / 4;
    int j = 0;
    for (; j + 2 <= B; j += 2) {
      const float4 v0 = src[(uint64_t)j * n_4], v1 = src[(uint64_t)(j + 1) * n_4];
      const float a0 = s_w[0][j], a1 = s_w[0][j + 1], b0 = s_w[1][j], b1 = s_w[1][j + 1];
      const float c0 = s_w[2][j], c1 = s_w[2][j + 1];
      X.x += a0 * v0.x + a1 * v1.x; X.y += a0 * v0.y + a1 * v1.y; X.z += a0 * v0.z + a1 * v1.z; X.w += a0 * v0.w + a1 * v1.w;
      Y.x += b0 * v0.x + b1 * v1.x; Y.y += b0 * v0.y + b1 * v1.y; Y.z += b0 * v0.z + b1 * v1.z; Y.w += b0 * v0.w + b1 * v1.w;
      Z.x += c0 * v0.x + c1 * v1.x; Z.y += c0 * v0.y + c1 * v1.y; Z.z += c0 * v0.z + c1 * v1.z; Z.w += c0 * v0.w + c1 * v1.w;
    }
    if (j < B) {
      const float4 v = src[(uint64_t)j * n_4];
      const float a = s_w[0][j], b = s_w[1][j], c = s_w[2][j];
      X.x += a * v.x; X.y += a * v.y; X.z += a * v.z; X.w += a * v.w;
      Y.x += b * v.x; Y.y += b * v.y; Y.z += b * v.z; Y.w += b * v.w;
      Z.x += c * v.x; Z.y += c * v.y; Z.z += c * v.z; Z.w += c * v.w;
    }
    if (xyz) {
      ((float4*)xyz)[q] = X;
      ((float4*)xyz)[n_4 + q] = Y;
      ((float4*)xyz)[2 * n_4 + q] = Z;
    }
    if (srgb) {
      const float x4[4] = {X.x, X.y, X.z, X.w}, y4[4] = {Y.x, Y.y, Y.z, Y.w}, z4[4] = {Z.x, Z.y, Z.z, Z.w};
      float o[12];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[3 * e] = srgb_encode(3.2406f * x4[e] - 1.5372f * y4[e] - 0.4986f * z4[e]);
        o[3 * e + 1] = srgb_encode(-0.9689f * x4[e] + 1.8758f * y4[e] + 0.0415f * z4[e]);
        o[3 * e + 2] = srgb_encode(0.0557f * x4[e] - 0.2040f * y4[e] + 1.0570f * z4[e]);
      }
      float4* d = (float4*)srgb + 3 * q;
      d[0] = make_float4(o[0], o[1], o[2], o[3]);
      d[1] = make_float4(o[4], o[5], o[6], o[7]);
      d[2] = make_float4(o[8], o[9], o[10], o[11]);
    }
  }
  for (uint64_t p = 4 * n4 + (uint64_t)blockIdx.x * kColorWG + threadIdx.x; p < n; p += (uint64_t)gridDim.x * kColorWG) {
    float X = 0.0f, Y = 0.0f, Z = 0.0f;
    const float* src = img + p;
    for (int j = 0; j < B; ++j) {
      const float v = src[(uint64_t)j * n];
      X += s_w[0][j] * v;
      Y += s_w[1][j] * v;
      Z += s_w[2][j] * v;
    }
    if (xyz) {
      xyz[p] = X;
      xyz[n + p] = Y;
      xyz[2 * n + p] = Z;
    }
    if (srgb) {
      srgb[3 * p] = srgb_encode(3.2406f * X - 1.5372f * Y - 0.4986f * Z);
      srgb[3 * p + 1] = srgb_encode(-0.9689f * X + 1.8758f * Y + 0.0415f * Z);
      srgb[3 * p + 2] = srgb_encode(0.0557f * X - 0.2040f * Y + 1.0570f * Z);
    }
  }
}

hipError_t launch_spectral_to_srgb(hipStream_t s, const float* img, int B, float lmin, float lmax, uint64_t n,
                                   float exposure, float* xyz, float* srgb) {
  // the vector path needs every plane (and output) 16-byte aligned: n a multiple of 4 and aligned bases
  const bool vec = n % 4 == 0 && ((uintptr_t)img & 15) == 0 && ((uintptr_t)xyz & 15) == 0 && ((uintptr_t)srgb & 15) == 0;
  const uint64_t items = vec ? n / 4 : n;
  const uint64_t want = (items + kColorWG - 1) / kColorWG;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(k_spectral_to_srgb, dim3(blocks), dim3(kColorWG), 0, s, img, B, lmin, lmax, n, exposure, xyz,
                     srgb, vec);
  return hipGetLastError();
}

}  // namespace sdd
