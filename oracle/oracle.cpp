// Plain CPU oracle of the spectral path tracer -- TEST INFRASTRUCTURE ONLY.
//
// Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load this
// library. It shares no code with the HIP renderer: it is a separate, deliberately simple
// FP64 implementation of what the renderer computes, built with g++.
//
//   * wavelength bins, complex refractive index n + ik           (section 3, eq. 1)
//   * directional (plane-wave) sun, spectrum given per bin        (section 3)
//   * direct term of N directional sources (next-event estimation) (section 4, eq. 3)
//   * path estimate of the rendering equation                     (section 4, eq. 2)
//   * spatial decomposition does not change the image: the oracle has no cells at all,
//     the global closest hit is the definition                    (section 5)
//
// Intersection uses the Moeller-Trumbore test in FP64 (a different algorithm from the
// renderer's watertight test) over all triangles (brute force) or a median-split BVH
// whose only role is to skip triangles that cannot matter.
//
// Paths whose outcome could flip under FP32 rounding (hits near an edge, nearly equal
// distances, near misses, lobe choices with u ~ P) are flagged as "tied" so that the
// comparison can exclude and count them.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of a multiply-xor bijection
// on four 32-bit words, with a Weyl-sequence key schedule.
// ------------------------------------------------------------------------------------------
struct U4 { uint32_t x[4]; };

U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = M0 * (uint64_t)c.x[0];
    uint64_t p1 = M1 * (uint64_t)c.x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    U4 n;
    n.x[0] = hi1 ^ c.x[1] ^ k0;
    n.x[1] = lo1;
    n.x[2] = hi0 ^ c.x[3] ^ k1;
    n.x[3] = lo0;
    c = n;
  }
  return c;
}

// Uniform in [0,1) from the top 24 bits: exact in both FP32 and FP64.
inline double unif(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline V3 normalize(V3 a) { return a * (1.0 / std::sqrt(dot(a, a))); }
inline double maxabs(V3 a) { return std::max(std::fabs(a.x), std::max(std::fabs(a.y), std::fabs(a.z))); }

// ------------------------------------------------------------------------------------------
// Unpolarised Fresnel reflectance at the interface air -> (n + ik)   (eq. 1 gives n + ik)
//   eta^2 = (n + ik)^2,  w = sqrt(eta^2 - sin^2 theta)  (principal branch)
//   r_s = (cos - w)/(cos + w),  r_p = (eta^2 cos - w)/(eta^2 cos + w),  F = (|r_s|^2+|r_p|^2)/2
// Written with explicit real/imaginary parts so nothing depends on std::complex.
// ------------------------------------------------------------------------------------------
struct Cx { double re, im; };
inline double cabs2(Cx a) { return a.re * a.re + a.im * a.im; }
inline Cx csqrt_principal(Cx z) {
  double r = std::hypot(z.re, z.im);
  if (r == 0.0) return {0.0, 0.0};
  if (z.re >= 0.0) {
    double s = std::sqrt(0.5 * (r + z.re));
    return {s, z.im / (2.0 * s)};
  }
  double s = std::sqrt(0.5 * (r - z.re));
  double im = std::copysign(s, z.im);
  return {z.im / (2.0 * im), im};
}

double fresnel(double n, double k, double cos_t) {
  cos_t = std::min(1.0, std::max(0.0, cos_t));
  double sin2 = 1.0 - cos_t * cos_t;
  Cx eta2 = {n * n - k * k, 2.0 * n * k};
  Cx w = csqrt_principal({eta2.re - sin2, eta2.im});
  Cx rs_num = {cos_t - w.re, -w.im}, rs_den = {cos_t + w.re, w.im};
  Cx e2c = {eta2.re * cos_t, eta2.im * cos_t};
  Cx rp_num = {e2c.re - w.re, e2c.im - w.im}, rp_den = {e2c.re + w.re, e2c.im + w.im};
  double Rs = cabs2(rs_num) / cabs2(rs_den);
  double Rp = cabs2(rp_num) / cabs2(rp_den);
  return 0.5 * (Rs + Rp);
}

// Thin absorbing slab of thickness d on a zero-thickness quad, incoherent multiple
// reflections between its two faces; Beer-Lambert absorption alpha = 4 pi k / lambda over
// the internal path d / cos(theta_t), refraction angle from the real index.
void slab(double n, double k, double lambda_nm, double d_m, double cos_t, double* R, double* T) {
  cos_t = std::min(1.0, std::max(0.0, cos_t));
  double sin_t = std::sqrt(std::max(0.0, 1.0 - cos_t * cos_t));
  double sin_i = sin_t / n;
  double cos_i = std::sqrt(std::max(0.0, 1.0 - sin_i * sin_i));
  double alpha = 4.0 * M_PI * k / (lambda_nm * 1e-9);
  double tau = std::exp(-alpha * d_m / cos_i);
  double R1 = fresnel(n, k, cos_t);
  double den = 1.0 - R1 * R1 * tau * tau;
  *R = R1 + (1.0 - R1) * (1.0 - R1) * tau * tau * R1 / den;
  *T = (1.0 - R1) * (1.0 - R1) * tau / den;
}

// The same slab when its internal transmittance at normal incidence tau0 is given directly (a
// measured spectral transmittance map of the glass, section 3) instead of by k: Beer-Lambert
// over the internal path d / cos(theta_t) makes it tau0^(1 / cos(theta_t)); the faces still
// reflect by the Fresnel factor of n + ik.
void slab_tau0(double n, double k, double tau0, double cos_t, double* R, double* T) {
  cos_t = std::min(1.0, std::max(0.0, cos_t));
  double sin_t = std::sqrt(std::max(0.0, 1.0 - cos_t * cos_t));
  double sin_i = sin_t / n;
  double cos_i = std::sqrt(std::max(0.0, 1.0 - sin_i * sin_i));
  double tau = std::pow(tau0, 1.0 / cos_i);
  double R1 = fresnel(n, k, cos_t);
  double den = 1.0 - R1 * R1 * tau * tau;
  *R = R1 + (1.0 - R1) * (1.0 - R1) * tau * tau * R1 / den;
  *T = (1.0 - R1) * (1.0 - R1) * tau / den;
}

// ------------------------------------------------------------------------------------------
// Scene in FP64
// ------------------------------------------------------------------------------------------
struct Tri { V3 v0, v1, v2; int mat; bool degenerate; double area2; double elen[3]; };

struct Box { V3 lo, hi; };
struct BNode { Box b; int left, right, first, count; };  // leaf if count > 0

struct Tie {
  double t_rel;      // nearly-equal distances: t2 <= t1 * (1 + t_rel)
  double edge_abs;   // edge margin: m = edge_abs * (1 + max|o|) + edge_rel_t * t
  double edge_rel_t;
  double lobe;       // |u0 - P| <= lobe
  double cos_sun;    // 0 < |n . w_s| <= cos_sun
};

struct Scene {
  std::vector<Tri> tris;
  std::vector<BNode> nodes;
  std::vector<int> order;
  bool use_bvh = false;
};

void build_bvh(Scene& S) {
  int n = (int)S.tris.size();
  S.order.resize(n);
  for (int i = 0; i < n; ++i) S.order[i] = i;
  std::vector<V3> cen(n);
  for (int i = 0; i < n; ++i) cen[i] = (S.tris[i].v0 + S.tris[i].v1 + S.tris[i].v2) * (1.0 / 3.0);
  struct Item { int node, first, count; };
  S.nodes.clear();
  S.nodes.push_back({});
  std::vector<Item> work{{0, 0, n}};
  while (!work.empty()) {
    Item it = work.back();
    work.pop_back();
    Box b{{1e300, 1e300, 1e300}, {-1e300, -1e300, -1e300}};
    Box cb = b;
    for (int i = it.first; i < it.first + it.count; ++i) {
      const Tri& t = S.tris[S.order[i]];
      for (const V3& v : {t.v0, t.v1, t.v2}) {
        b.lo = {std::min(b.lo.x, v.x), std::min(b.lo.y, v.y), std::min(b.lo.z, v.z)};
        b.hi = {std::max(b.hi.x, v.x), std::max(b.hi.y, v.y), std::max(b.hi.z, v.z)};
      }
      V3 c = cen[S.order[i]];
      cb.lo = {std::min(cb.lo.x, c.x), std::min(cb.lo.y, c.y), std::min(cb.lo.z, c.z)};
      cb.hi = {std::max(cb.hi.x, c.x), std::max(cb.hi.y, c.y), std::max(cb.hi.z, c.z)};
    }
    S.nodes[it.node].b = b;
    if (it.count <= 4) {
      S.nodes[it.node].left = S.nodes[it.node].right = -1;
      S.nodes[it.node].first = it.first;
      S.nodes[it.node].count = it.count;
      continue;
    }
    V3 ext = cb.hi - cb.lo;
    int axis = (ext.x >= ext.y && ext.x >= ext.z) ? 0 : (ext.y >= ext.z ? 1 : 2);
    auto key = [&](int i) { const V3& c = cen[i]; return axis == 0 ? c.x : axis == 1 ? c.y : c.z; };
    int mid = it.first + it.count / 2;
    std::nth_element(S.order.begin() + it.first, S.order.begin() + mid, S.order.begin() + it.first + it.count,
                     [&](int a, int b2) { return key(a) < key(b2) || (key(a) == key(b2) && a < b2); });
    int l = (int)S.nodes.size();
    S.nodes.push_back({});
    S.nodes.push_back({});
    S.nodes[it.node].left = l;
    S.nodes[it.node].right = l + 1;
    S.nodes[it.node].count = 0;
    work.push_back({l, it.first, mid - it.first});
    work.push_back({l + 1, mid, it.first + it.count - mid});
  }
}

// Ray-box overlap for the interval [t0, t1], box grown by `pad` on every side.
bool box_hit(const Box& b, V3 o, V3 d, double t0, double t1, double pad) {
  const double lo[3] = {b.lo.x - pad, b.lo.y - pad, b.lo.z - pad};
  const double hi[3] = {b.hi.x + pad, b.hi.y + pad, b.hi.z + pad};
  const double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
  for (int a = 0; a < 3; ++a) {
    if (dd[a] == 0.0) {
      if (oo[a] < lo[a] || oo[a] > hi[a]) return false;
      continue;
    }
    double ta = (lo[a] - oo[a]) / dd[a], tb = (hi[a] - oo[a]) / dd[a];
    if (ta > tb) std::swap(ta, tb);
    t0 = std::max(t0, ta);
    t1 = std::min(t1, tb * (1.0 + 1e-12) + 1e-12);
    if (t0 > t1) return false;
  }
  return true;
}

// Moeller-Trumbore in FP64. Returns false for parallel rays / degenerate triangles.
// Also returns the signed distance of the hit point (on the triangle's plane) to the
// nearest edge line: >= 0 inside, < 0 outside.
bool mt(const Tri& T, V3 o, V3 d, double* t, double* u, double* v, double* edge_dist) {
  if (T.degenerate) return false;
  V3 e1 = T.v1 - T.v0, e2 = T.v2 - T.v0;
  V3 pv = cross(d, e2);
  double det = dot(e1, pv);
  if (det == 0.0) return false;
  double inv = 1.0 / det;
  V3 tv = o - T.v0;
  *u = dot(tv, pv) * inv;
  V3 qv = cross(tv, e1);
  *v = dot(d, qv) * inv;
  *t = dot(e2, qv) * inv;
  double w0 = 1.0 - *u - *v;
  // distance to the edge opposite vertex i = w_i * 2A / |edge_i|
  double d0 = w0 * T.area2 / T.elen[0];   // edge v1-v2
  double d1 = *u * T.area2 / T.elen[1];   // edge v2-v0
  double d2 = *v * T.area2 / T.elen[2];   // edge v0-v1
  *edge_dist = std::min(d0, std::min(d1, d2));
  return true;
}

struct Hit { bool hit = false; double t = 0, u = 0, v = 0; int id = -1; double edge = 0; };

// Closest hit with tie analysis (definition: minimum t > 0 over all non-degenerate triangles
// other than `skip`, inclusive barycentric test, equal t -> smaller id).
struct Cand { double t, edge; int id; };

template <class L, class F>
void for_candidates(const Scene& S, V3 o, V3 d, double pad, L&& tmax_hint, F&& f) {
  if (!S.use_bvh) {
    for (int i = 0; i < (int)S.tris.size(); ++i) f(i);
    return;
  }
  int stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    int ni = stack[--sp];
    const BNode& N = S.nodes[ni];
    if (!box_hit(N.b, o, d, -pad, tmax_hint(), pad)) continue;
    if (N.count > 0) {
      for (int i = N.first; i < N.first + N.count; ++i) f(S.order[i]);
    } else {
      stack[sp++] = N.left;
      stack[sp++] = N.right;
    }
  }
}

Hit closest_hit(const Scene& S, V3 o, V3 d, int skip, const Tie& tie, bool* tied) {
  Hit best;
  double pad = tie.edge_abs * (1.0 + maxabs(o)) * 4.0 + 1e-9;
  std::vector<Cand> cands;
  double t_best = INFINITY;
  auto limit = [&]() { return std::isinf(t_best) ? 1e300 : t_best * (1.0 + tie.t_rel) * 1.001 + pad; };
  for_candidates(S, o, d, pad + tie.edge_rel_t * 1e3, limit, [&](int i) {
    if (i == skip) return;
    double t, u, v, ed;
    if (!mt(S.tris[i], o, d, &t, &u, &v, &ed)) return;
    double m = tie.edge_abs * (1.0 + maxabs(o)) + tie.edge_rel_t * std::fabs(t);
    if (ed >= -m) cands.push_back({t, ed, i});
    bool inside = (u >= 0.0 && v >= 0.0 && u + v <= 1.0);
    if (inside && t > 0.0) {
      if (!best.hit || t < best.t || (t == best.t && i < best.id)) {
        best.hit = true; best.t = t; best.u = u; best.v = v; best.id = i; best.edge = ed;
        t_best = t;
      }
    }
  });
  // tie analysis
  bool tie_flag = false;
  double t_lim = best.hit ? best.t * (1.0 + tie.t_rel) : INFINITY;
  double tiny = 1e-9 * (1.0 + maxabs(o));
  for (const Cand& c : cands) {
    if (c.id == best.id) continue;
    if (c.t <= t_lim && c.t > -tiny) { tie_flag = true; break; }
  }
  if (best.hit) {
    double m = tie.edge_abs * (1.0 + maxabs(o)) + tie.edge_rel_t * best.t;
    if (best.edge <= m) tie_flag = true;
    if (best.t <= tiny) tie_flag = true;
  }
  if (tie_flag) *tied = true;
  return best;
}

// Shadow ray toward the sun: any opaque hit (t > 0) blocks; every glass triangle crossed
// multiplies the visibility by its slab transmittance at that crossing.
struct GlassCross { int mat; double cos_t; int tri; double u, v; };

bool shadow_visibility(const Scene& S, const std::vector<int>& mat_type, V3 o, V3 d, int skip, const Tie& tie,
                       std::vector<GlassCross>* crossings, bool* tied) {
  double pad = tie.edge_abs * (1.0 + maxabs(o)) * 4.0 + 1e-9;
  bool robust_block = false, any_block = false, near_edge = false;
  crossings->clear();
  for_candidates(S, o, d, pad + tie.edge_rel_t * 1e3, [&]() { return 1e300; }, [&](int i) {
    if (i == skip) return;
    const Tri& T = S.tris[i];
    double t, u, v, ed;
    if (!mt(T, o, d, &t, &u, &v, &ed)) return;
    double m = tie.edge_abs * (1.0 + maxabs(o)) + tie.edge_rel_t * std::fabs(t);
    bool inside = (u >= 0.0 && v >= 0.0 && u + v <= 1.0);
    double tiny = 1e-9 * (1.0 + maxabs(o));
    if (ed >= -m && (std::fabs(ed) <= m || std::fabs(t) <= tiny) && t > -tiny) near_edge = true;
    if (!(inside && t > 0.0)) return;
    if (mat_type[T.mat] == 0) {
      any_block = true;
      if (ed > m && t > tiny) robust_block = true;
    } else {
      V3 ng = normalize(cross(T.v1 - T.v0, T.v2 - T.v0));
      crossings->push_back({T.mat, std::fabs(dot(d, ng)), i, u, v});
    }
  });
  if (robust_block) return false;
  if (near_edge) *tied = true;
  return !any_block;
}

}  // namespace

// ==========================================================================================
// C ABI (ctypes)
// ==========================================================================================
extern "C" {

typedef struct {
  const float* verts;        // [N][3][3]
  int64_t n_tri;
  const uint16_t* mat;       // [N]
  int32_t n_mat;
  const int32_t* mat_type;   // [n_mat] 0 opaque, 1 glass slab
  const float* thickness_m;  // [n_mat]
  const float* n_tab;        // [n_mat][B]
  const float* k_tab;        // [n_mat][B]
  const float* rho_tab;      // [n_mat][B]
  int32_t n_bins;
  double lambda_min_nm, lambda_max_nm;
  const float* sun_dir;      // [3] toward the sun
  const float* sun_E;        // [B]
  const float* env;          // [B]
  // spectral transmittance maps of glass (n_tex = 0: none)
  const float* uv;           // [N][3][2] texture coordinates of the triangle's vertices
  int32_t n_tex;
  const int32_t* tex_dims;   // [n_tex][2] width, height
  const int64_t* tex_offset; // [n_tex] float offset of the map in texels
  const float* texels;       // maps [h][w][B]: internal transmittance at normal incidence
  const int32_t* mat_tex;    // [n_mat] map of the material, -1 none
} orc_scene;

// Internal transmittance at normal incidence of map t, bin j, at texture coordinates (s, t):
// bilinear interpolation between texel centres ((i + 1/2) / w, (k + 1/2) / h), the map repeated
// periodically in both directions.
static double tex_tau0(const orc_scene* sc, int t, double s, double tt, int j) {
  const int w = sc->tex_dims[2 * t], h = sc->tex_dims[2 * t + 1], B = sc->n_bins;
  const float* T = sc->texels + sc->tex_offset[t];
  double x = s * w - 0.5, y = tt * h - 0.5;
  double fx0 = std::floor(x), fy0 = std::floor(y);
  double fx = x - fx0, fy = y - fy0;
  auto wrap = [](long long i, int n) { long long r = i % n; return (int)(r < 0 ? r + n : r); };
  int i0 = wrap((long long)fx0, w), i1 = wrap((long long)fx0 + 1, w);
  int k0 = wrap((long long)fy0, h), k1 = wrap((long long)fy0 + 1, h);
  auto at = [&](int k, int i) { return (double)T[((int64_t)k * w + i) * B + j]; };
  return (1 - fx) * (1 - fy) * at(k0, i0) + fx * (1 - fy) * at(k0, i1) + (1 - fx) * fy * at(k1, i0) +
         fx * fy * at(k1, i1);
}

// Slab response of glass material m at bin j for a hit on triangle tri with barycentrics
// (u, v): the material's map at the interpolated texture coordinates when it has one, else
// Beer-Lambert with its k.
static void glass_slab(const orc_scene* sc, int m, int j, double lambda_nm, double cos_t, int tri, double u, double v,
                       double* R, double* T) {
  const int B = sc->n_bins;
  const int t = (sc->n_tex > 0 && sc->mat_tex) ? sc->mat_tex[m] : -1;
  if (t < 0) {
    slab(sc->n_tab[m * B + j], sc->k_tab[m * B + j], lambda_nm, sc->thickness_m[m], cos_t, R, T);
    return;
  }
  const float* q = sc->uv + 6 * (int64_t)tri;
  const double w0 = 1.0 - u - v;
  const double s = w0 * q[0] + u * q[2] + v * q[4], tt = w0 * q[1] + u * q[3] + v * q[5];
  slab_tau0(sc->n_tab[m * B + j], sc->k_tab[m * B + j], tex_tau0(sc, t, s, tt, j), cos_t, R, T);
}

typedef struct {
  double eye[3], target[3], up[3];
  double vfov_deg;
  int32_t width, height;
} orc_camera;

typedef struct {
  int32_t spp, max_depth;
  uint64_t seed;
  uint32_t view;
  int32_t threads;
  int32_t force_bvh;         // -1 auto (BVH above 1e4 triangles), 0 brute force, 1 BVH
  double tie_t_rel, tie_edge_abs, tie_edge_rel_t, tie_lobe, tie_cos_sun;
  int32_t cached;            // 1: stop at vertex 3 and record the cache query instead
  int32_t first_sample;      // sample indices first_sample .. first_sample + spp - 1
  uint32_t purpose;          // random-number purpose: added to the depth word (0 or 1 << 24)
  int32_t record_depth;      // > 0: training paths; record that vertex and restart beta and L there
  int32_t sample_per_entry;  // 1: entry i of the pixel list is one path with sample first_sample + i
  // caustic photon map (n_photons = 0: none): density estimate added at every opaque vertex
  const double* ph_pos;      // [n][3] where a photon was stored
  const double* ph_dir;      // [n][3] its direction of travel on arrival
  const double* ph_flux;     // [n][B] its flux
  int64_t n_photons;
  double ph_radius;
  double tie_radius;         // relative margin of the gather radius: photons within it are uncertain
  double* ph_unc;            // [B][n_pix] or null: the radiance those photons could change
  // global photon map (gl_depth = 0: none): at every opaque vertex from vertex gl_depth on, the
  // diffuse radiance leaving it is the map's density estimate (no direct term, no caustic map),
  // and the path goes on only by the mirror lobe
  const double* gl_pos;
  const double* gl_dir;
  const double* gl_flux;
  int64_t n_global;
  double gl_radius;
  int32_t gl_depth;
  int32_t pad_gl;
} orc_params;

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  U4 c{{ctr[0], ctr[1], ctr[2], ctr[3]}};
  U4 r = philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = r.x[i];
}

void orc_philox_stream(const uint32_t* ctr_base, const uint32_t* key, int64_t n, uint32_t* out) {
  // counters (base0 + i, base1, base2, base3), i < n  -> out[i][4]
  for (int64_t i = 0; i < n; ++i) {
    U4 c{{ctr_base[0] + (uint32_t)i, ctr_base[1], ctr_base[2], ctr_base[3]}};
    U4 r = philox4x32_10(c, key[0], key[1]);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = r.x[j];
  }
}

double orc_fresnel(double n, double k, double cos_t) { return fresnel(n, k, cos_t); }

void orc_slab(double n, double k, double lambda_nm, double d_m, double cos_t, double* R, double* T) {
  slab(n, k, lambda_nm, d_m, cos_t, R, T);
}

static void load_scene(const orc_scene* sc, int force_bvh, Scene* S) {
  S->tris.resize(sc->n_tri);
  for (int64_t i = 0; i < sc->n_tri; ++i) {
    const float* p = sc->verts + 9 * i;
    Tri& T = S->tris[i];
    T.v0 = {p[0], p[1], p[2]};
    T.v1 = {p[3], p[4], p[5]};
    T.v2 = {p[6], p[7], p[8]};
    T.mat = sc->mat ? sc->mat[i] : 0;
    V3 c = cross(T.v1 - T.v0, T.v2 - T.v0);
    T.area2 = std::sqrt(dot(c, c));
    T.degenerate = (T.area2 == 0.0);
    V3 e0 = T.v2 - T.v1, e1 = T.v0 - T.v2, e2 = T.v1 - T.v0;
    T.elen[0] = std::sqrt(dot(e0, e0));
    T.elen[1] = std::sqrt(dot(e1, e1));
    T.elen[2] = std::sqrt(dot(e2, e2));
  }
  S->use_bvh = force_bvh == 1 || (force_bvh < 0 && sc->n_tri > 10000);
  if (S->use_bvh) build_bvh(*S);
}

// Closest hit for a batch of rays (FP32 inputs, converted exactly).
// out_t (inf on miss), out_id (-1 on miss), out_u, out_v, out_tie.
int orc_intersect(const orc_scene* sc, const float* orig, const float* dir, const int32_t* skip, int64_t n_rays,
                  int32_t force_bvh, double tie_t_rel, double tie_edge_abs, double tie_edge_rel_t, int32_t threads,
                  double* out_t, int64_t* out_id, double* out_u, double* out_v, uint8_t* out_tie) {
  Scene S;
  load_scene(sc, force_bvh, &S);
  Tie tie{tie_t_rel, tie_edge_abs, tie_edge_rel_t, 0.0, 0.0};
  auto work = [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      V3 o{orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]};
      V3 d{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
      bool tied = false;
      Hit h = closest_hit(S, o, d, skip ? skip[i] : -1, tie, &tied);
      out_t[i] = h.hit ? h.t : INFINITY;
      out_id[i] = h.hit ? h.id : -1;
      out_u[i] = h.u;
      out_v[i] = h.v;
      out_tie[i] = tied ? 1 : 0;
    }
  };
  int nt = std::max(1, threads);
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k) th.emplace_back(work, n_rays * k / nt, n_rays * (k + 1) / nt);
  for (auto& t : th) t.join();
  return 0;
}

// Shadow query for a batch of rays: visibility per bin (0 if blocked) and tie flag.
int orc_shadow(const orc_scene* sc, const float* orig, const float* dir, const int32_t* skip, int64_t n_rays,
               double tie_edge_abs, double tie_edge_rel_t, double* out_vis /*[n][B]*/, uint8_t* out_tie) {
  Scene S;
  load_scene(sc, -1, &S);
  Tie tie{1e-5, tie_edge_abs, tie_edge_rel_t, 0.0, 0.0};
  std::vector<int> mat_type(sc->mat_type, sc->mat_type + sc->n_mat);
  int B = sc->n_bins;
  std::vector<double> lam(B);
  for (int j = 0; j < B; ++j) lam[j] = sc->lambda_min_nm + (j + 0.5) * (sc->lambda_max_nm - sc->lambda_min_nm) / B;
  std::vector<GlassCross> cr;
  for (int64_t i = 0; i < n_rays; ++i) {
    V3 o{orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]};
    V3 d{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
    bool tied = false;
    bool vis = shadow_visibility(S, mat_type, o, d, skip ? skip[i] : -1, tie, &cr, &tied);
    for (int j = 0; j < B; ++j) {
      double V = vis ? 1.0 : 0.0;
      if (vis)
        for (const GlassCross& g : cr) {
          double R, T;
          glass_slab(sc, g.mat, j, lam[j], g.cos_t, g.tri, g.u, g.v, &R, &T);
          V *= T;
        }
      out_vis[i * B + j] = V;
    }
    out_tie[i] = tied ? 1 : 0;
  }
  return 0;
}

// Cache queries recorded in cached mode (the vertex after bounce 2): position, direction
// toward the previous vertex, material and the path throughput, per (pixel subset index,
// sample). valid = 0 when the path never reached that vertex.
typedef struct {
  double* x;       // [n_pix*spp][3]
  double* wo;      // [n_pix*spp][3]
  int32_t* mat;    // [n_pix*spp]
  double* beta;    // [n_pix*spp][B]
  uint8_t* valid;  // [n_pix*spp]
} orc_cache_queries;

// Render the spectral image (or a pixel subset). image: [B][n_pix] FP64, the mean over
// spp samples; tied: number of tied samples per pixel; stats[0..3]: paths, vertices,
// shadow rays, tied paths.
int orc_render(const orc_scene* sc, const orc_camera* cam, const orc_params* prm, const int64_t* pixels,
               int64_t n_pix, double* image, int32_t* tied_out, int64_t* stats, orc_cache_queries* cq) {
  Scene S;
  load_scene(sc, prm->force_bvh, &S);
  const int B = sc->n_bins;
  const int W = cam->width, H = cam->height;
  const int spp = prm->spp, D = prm->max_depth;
  const Tie tie{prm->tie_t_rel, prm->tie_edge_abs, prm->tie_edge_rel_t, prm->tie_lobe, prm->tie_cos_sun};
  std::vector<int> mat_type(sc->mat_type, sc->mat_type + sc->n_mat);
  std::vector<double> lam(B), E(B), env(B);
  for (int j = 0; j < B; ++j) {
    lam[j] = sc->lambda_min_nm + (j + 0.5) * (sc->lambda_max_nm - sc->lambda_min_nm) / B;
    E[j] = sc->sun_E[j];
    env[j] = sc->env[j];
  }
  V3 ws = normalize({sc->sun_dir[0], sc->sun_dir[1], sc->sun_dir[2]});
  // camera basis
  V3 eye{cam->eye[0], cam->eye[1], cam->eye[2]};
  V3 f = normalize(V3{cam->target[0], cam->target[1], cam->target[2]} - eye);
  V3 r = normalize(cross(f, {cam->up[0], cam->up[1], cam->up[2]}));
  V3 up = cross(r, f);
  double tf = std::tan(cam->vfov_deg * M_PI / 360.0);
  const uint32_t k0 = (uint32_t)prm->seed, k1 = (uint32_t)(prm->seed >> 32);
  const int64_t npx = pixels ? n_pix : (int64_t)W * H;

  std::atomic<int64_t> st_paths{0}, st_vert{0}, st_shadow{0}, st_tied{0};

  auto render_pixel = [&](int64_t i, std::vector<double>& acc, std::vector<double>& L, std::vector<double>& beta,
                          std::vector<double>& F, std::vector<GlassCross>& cr, int64_t* nv, int64_t* ns, int32_t* ntie) {
    thread_local std::vector<double> acc_ph, acc_unc, Lu, acc_u;
    acc_ph.assign(B, 0.0);
    acc_unc.assign(B, 0.0);
    acc_u.assign(B, 0.0);
    int64_t pix = pixels ? pixels[i] : i;
    int px = (int)(pix % W), py = (int)(pix / W);
    std::fill(acc.begin(), acc.end(), 0.0);
    for (int si = 0; si < spp; ++si) {
      const int s = prm->sample_per_entry ? prm->first_sample + (int)i : prm->first_sample + si;
      bool tied = false;
      std::fill(L.begin(), L.end(), 0.0);
      Lu.assign(B, 0.0);
      std::fill(beta.begin(), beta.end(), 1.0);
      U4 rn = philox4x32_10({{(uint32_t)pix, (uint32_t)s, prm->purpose, prm->view}}, k0, k1);
      double sx = (2.0 * (px + unif(rn.x[0])) / W - 1.0) * tf * W / H;
      double sy = (1.0 - 2.0 * (py + unif(rn.x[1])) / H) * tf;
      V3 o = eye, d = normalize(f + r * sx + up * sy);
      int skip = -1;
      for (int dep = 1; dep <= D; ++dep) {
        Hit h = closest_hit(S, o, d, skip, tie, &tied);
        if (!h.hit) {
          for (int j = 0; j < B; ++j) L[j] += beta[j] * env[j];
          break;
        }
        ++*nv;
        const Tri& T = S.tris[h.id];
        V3 ng = normalize(cross(T.v1 - T.v0, T.v2 - T.v0));
        double dn = dot(d, ng);
        V3 n = dn > 0 ? ng * -1.0 : ng;  // face forward: -sign(d . n_g) n_g
        double cos_o = std::fabs(dn);
        // grazing hit: the side the surface is seen from (and so the spawn side) is uncertain
        if (cos_o <= tie.cos_sun) tied = true;
        V3 p = T.v0 * (1.0 - h.u - h.v) + T.v1 * h.u + T.v2 * h.v;
        double eps = 1e-5 * (1.0 + maxabs(p));
        int m = T.mat;
        if (prm->record_depth == dep) {
          // training path: this vertex is the record; what the path gathers from here on is the
          // radiance leaving it toward the previous vertex
          int64_t q = i * spp + si;
          cq->x[3 * q] = p.x; cq->x[3 * q + 1] = p.y; cq->x[3 * q + 2] = p.z;
          cq->wo[3 * q] = -d.x; cq->wo[3 * q + 1] = -d.y; cq->wo[3 * q + 2] = -d.z;
          cq->mat[q] = m;
          cq->valid[q] = 1;
          std::fill(L.begin(), L.end(), 0.0);
          std::fill(beta.begin(), beta.end(), 1.0);
        }
        if (prm->cached && dep == 3) {
          int64_t q = i * spp + si;
          cq->x[3 * q] = p.x; cq->x[3 * q + 1] = p.y; cq->x[3 * q + 2] = p.z;
          cq->wo[3 * q] = -d.x; cq->wo[3 * q + 1] = -d.y; cq->wo[3 * q + 2] = -d.z;
          cq->mat[q] = m;
          for (int j = 0; j < B; ++j) cq->beta[q * B + j] = beta[j];
          cq->valid[q] = 1;
          break;
        }
        U4 rv = philox4x32_10({{(uint32_t)pix, (uint32_t)s, (uint32_t)dep | prm->purpose, prm->view}}, k0, k1);
        double u0 = unif(rv.x[0]), u1 = unif(rv.x[1]), u2 = unif(rv.x[2]);
        const float* nt = sc->n_tab + m * B;
        const float* kt = sc->k_tab + m * B;
        const float* rt = sc->rho_tab + m * B;
        if (mat_type[m] == 0) {
          for (int j = 0; j < B; ++j) F[j] = fresnel(nt[j], kt[j], cos_o);
          // density estimate of a photon map: (1 - F) rho / pi times the flux of the photons
          // within the gather radius that arrived from the side the path sees, over the disc
          // area pi r^2; photons within r (1 +- tie_radius) could fall on either side of r in
          // FP32: their flux bounds how far another rounding of the same estimate can go
          auto density = [&](const double* mp, const double* md, const double* mf, int64_t nm, double r) {
            const double r2 = r * r;
            const double lo2 = r2 * (1.0 - prm->tie_radius) * (1.0 - prm->tie_radius);
            const double hi2 = r2 * (1.0 + prm->tie_radius) * (1.0 + prm->tie_radius);
            std::fill(acc_ph.begin(), acc_ph.end(), 0.0);
            std::fill(acc_unc.begin(), acc_unc.end(), 0.0);
            for (int64_t q = 0; q < nm; ++q) {
              const double* pp = mp + 3 * q;
              const double dx = pp[0] - p.x, dy = pp[1] - p.y, dz = pp[2] - p.z;
              const double d2 = dx * dx + dy * dy + dz * dz;
              if (d2 > hi2) continue;
              const double* pd = md + 3 * q;
              const double side = pd[0] * n.x + pd[1] * n.y + pd[2] * n.z;
              if (std::fabs(side) <= tie.cos_sun) tied = true;
              if (d2 < r2 && side < 0.0)
                for (int j = 0; j < B; ++j) acc_ph[j] += mf[q * B + j];
              if (d2 >= lo2 && side < 0.0)
                for (int j = 0; j < B; ++j) acc_unc[j] += mf[q * B + j];
            }
            for (int j = 0; j < B; ++j) Lu[j] += beta[j] * (1.0 - F[j]) * rt[j] / M_PI * acc_unc[j] / (M_PI * r2);
            for (int j = 0; j < B; ++j) L[j] += beta[j] * (1.0 - F[j]) * rt[j] / M_PI * acc_ph[j] / (M_PI * r2);
          };
          const bool gm = prm->gl_depth > 0 && dep >= prm->gl_depth;
          if (gm) {
            // the global map holds the light arriving here by every route (the sun's direct
            // light, caustics, interreflections): its estimate is the whole diffuse part
            if (prm->n_global > 0) density(prm->gl_pos, prm->gl_dir, prm->gl_flux, prm->n_global, prm->gl_radius);
          } else if (prm->n_photons > 0) {
            density(prm->ph_pos, prm->ph_dir, prm->ph_flux, prm->n_photons, prm->ph_radius);
          }
          // next-event estimation toward the sun (eq. 3)
          double cs = dot(n, ws);
          if (!gm && cs != 0.0 && std::fabs(cs) <= tie.cos_sun) tied = true;
          if (!gm && cs > 0.0) {
            ++*ns;
            bool vis = shadow_visibility(S, mat_type, p + n * eps, ws, h.id, tie, &cr, &tied);
            if (vis) {
              for (int j = 0; j < B; ++j) {
                double V = 1.0;
                for (const GlassCross& g : cr) {
                  double R, Tt;
                  glass_slab(sc, g.mat, j, lam[j], g.cos_t, g.tri, g.u, g.v, &R, &Tt);
                  V *= Tt;
                }
                L[j] += beta[j] * (1.0 - F[j]) * rt[j] / M_PI * E[j] * cs * V;
              }
            }
          }
          if (dep == D) break;
          double a = 0, b = 0;
          for (int j = 0; j < B; ++j) { a += F[j]; b += (1.0 - F[j]) * rt[j]; }
          a /= B;
          b /= B;
          if (a + b == 0.0) break;
          double Ps = a / (a + b);
          if (std::fabs(u0 - Ps) <= tie.lobe) tied = true;
          if (u0 < Ps) {
            for (int j = 0; j < B; ++j) beta[j] *= F[j] / Ps;
            d = d - ng * (2.0 * dn);
          } else if (gm) {
            break;   // the diffuse lobe's light came from the global map
          } else {
            for (int j = 0; j < B; ++j) beta[j] *= (1.0 - F[j]) * rt[j] / (1.0 - Ps);
            double phi = 2.0 * M_PI * u1, rr = std::sqrt(u2);
            double lx = rr * std::cos(phi), ly = rr * std::sin(phi), lz = std::sqrt(std::max(0.0, 1.0 - u2));
            // orthonormal basis around n (Duff et al. 2017); the frame switches with the sign
            // of n_z, so a normal with a tiny non-zero z could land on either side in FP32
            if (n.z != 0.0 && std::fabs(n.z) <= tie.cos_sun) tied = true;
            double sgn = std::copysign(1.0, n.z);
            double aa = -1.0 / (sgn + n.z);
            double bb = n.x * n.y * aa;
            V3 t1{1.0 + sgn * n.x * n.x * aa, sgn * bb, -sgn * n.x};
            V3 t2{bb, sgn + n.y * n.y * aa, -n.y};
            d = t1 * lx + t2 * ly + n * lz;
          }
          o = p + n * eps;
        } else {
          if (dep == D) break;
          double mr = 0, mt_ = 0;
          for (int j = 0; j < B; ++j) {
            double R, Tt;
            glass_slab(sc, m, j, lam[j], cos_o, h.id, h.u, h.v, &R, &Tt);
            F[j] = R;       // slab reflectance per bin
            F[B + j] = Tt;  // slab transmittance per bin
            mr += R;
            mt_ += Tt;
          }
          double Pr = mr / (mr + mt_);
          if (std::fabs(u0 - Pr) <= tie.lobe) tied = true;
          if (u0 < Pr) {
            for (int j = 0; j < B; ++j) beta[j] *= F[j] / Pr;
            d = d - ng * (2.0 * dn);
            o = p + n * eps;
          } else {
            for (int j = 0; j < B; ++j) beta[j] *= F[B + j] / (1.0 - Pr);
            o = p - n * eps;
          }
        }
        skip = h.id;
      }
      for (int j = 0; j < B; ++j) acc[j] += L[j];
      for (int j = 0; j < B; ++j) acc_u[j] += Lu[j];
      if (tied) ++*ntie;
    }
    for (int j = 0; j < B; ++j) image[(int64_t)j * npx + i] = acc[j] / spp;
    if (prm->ph_unc)
      for (int j = 0; j < B; ++j) prm->ph_unc[(int64_t)j * npx + i] = acc_u[j] / spp;
  };

  int nt = std::max(1, prm->threads);
  // static image-space partition over rows of the pixel list (the paper's classical scheme)
  auto worker = [&](int64_t a, int64_t b) {
    std::vector<double> acc(B), L(B), beta(B), F(2 * B);
    std::vector<GlassCross> cr;
    int64_t nv = 0, ns = 0, ntied = 0;
    for (int64_t i = a; i < b; ++i) {
      int32_t nti = 0;
      render_pixel(i, acc, L, beta, F, cr, &nv, &ns, &nti);
      if (tied_out) tied_out[i] = nti;
      ntied += nti;
    }
    st_paths += (b - a) * spp;
    st_vert += nv;
    st_shadow += ns;
    st_tied += ntied;
  };
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k) th.emplace_back(worker, npx * k / nt, npx * (k + 1) / nt);
  for (auto& t : th) t.join();
  if (stats) {
    stats[0] = st_paths;
    stats[1] = st_vert;
    stats[2] = st_shadow;
    stats[3] = st_tied;
  }
  return 0;
}

// ------------------------------------------------------------------------------------------
// Caustic photon map (section 4: photon maps filled from the light sources, one of them for
// caustics). Photons leave the sun (a plane wave, section 3) through the windows: photon i picks
// a glass triangle with probability proportional to its area projected on the sun's direction (the
// window whose threshold floor(cdf_w / A 2^24) is the last not above the 24-bit random integer
// x >> 8, cdf_w the projected area of the windows before it) and a uniform point p on it
// (random-number counter (i, i >> 32, 0 | 4 << 24, 0)); it carries the
// flux E_j A / N of the sun's beam through the windows' total projected area A, times the
// transmittance of whatever lies between p and the sun (a shadow ray from p, as for the direct
// term). Its first vertex is p on that window. At vertex d (counter (i, i >> 32, d | 4 << 24, 0)):
//   glass:  reflect with probability P_r = mean R / (mean R + mean T) (weight R / P_r), else
//           transmit straight (weight T / (1 - P_r)), as for camera paths;
//   opaque: if the photon has been reflected at least once (by a glass face or a mirror lobe) it
//           is stored with its flux and direction (light reaching a diffuse surface only by
//           transmission through thin glass is the direct term, which the paths' eq. 3 already
//           counts); then the mirror lobe is taken with P_s = mean F / (mean F + mean (1-F) rho)
//           (weight F / P_s), else the photon ends (a diffuse bounce leaves the caustic paths).
// Vertex max_depth stores but does not scatter. Records come out ordered by (photon, vertex).
// Global map (global = 1): an opaque vertex stores every photon, and a photon that does not take
// the mirror lobe takes the cosine-weighted diffuse lobe (direction from the vertex's second and
// third uniforms, as for camera paths; weight (1 - F(cos of the new direction)) rho / (1 - P_s),
// the adjoint of the camera paths' diffuse weight) instead of ending.
// With stride k > 1 only the photons i = 0, k, 2k, ... are traced (a sample of the same map:
// every photon still carries E_j A / N).
// ------------------------------------------------------------------------------------------
typedef struct {
  int64_t n_photons;
  int32_t max_depth;
  uint64_t seed;
  int32_t threads;
  double tie_t_rel, tie_edge_abs, tie_edge_rel_t, tie_lobe, tie_cos_sun;
  int64_t stride;
  int32_t global;            // 1: global map (stored at every opaque vertex, diffuse lobe too)
  int32_t pad;
} orc_photon_params;

int64_t orc_photons(const orc_scene* sc, const orc_photon_params* pp, int64_t cap, double* pos, double* dir,
                    double* flux, int64_t* pid, int32_t* pdepth, int32_t* ptri, uint8_t* tied_out, double* area_out) {
  Scene S;
  load_scene(sc, -1, &S);
  const int B = sc->n_bins;
  const Tie tie{pp->tie_t_rel, pp->tie_edge_abs, pp->tie_edge_rel_t, pp->tie_lobe, pp->tie_cos_sun};
  std::vector<int> mat_type(sc->mat_type, sc->mat_type + sc->n_mat);
  std::vector<double> lam(B), E(B);
  for (int j = 0; j < B; ++j) {
    lam[j] = sc->lambda_min_nm + (j + 0.5) * (sc->lambda_max_nm - sc->lambda_min_nm) / B;
    E[j] = sc->sun_E[j];
  }
  const V3 ws = normalize({sc->sun_dir[0], sc->sun_dir[1], sc->sun_dir[2]});
  // windows: glass triangles and the prefix sums of their projected areas, taken on the sun's
  // unit direction rounded to FP32 (the form a scene stores it in)
  const double sl = std::sqrt((double)sc->sun_dir[0] * sc->sun_dir[0] + (double)sc->sun_dir[1] * sc->sun_dir[1] +
                              (double)sc->sun_dir[2] * sc->sun_dir[2]);
  const V3 ws32{(double)(float)(sc->sun_dir[0] / sl), (double)(float)(sc->sun_dir[1] / sl),
                (double)(float)(sc->sun_dir[2] / sl)};
  std::vector<int> wtri;
  std::vector<double> cdf{0.0};
  for (int64_t t = 0; t < sc->n_tri; ++t) {
    const Tri& T = S.tris[t];
    if (mat_type[T.mat] != 1 || T.degenerate) continue;
    const V3 c = cross(T.v1 - T.v0, T.v2 - T.v0);
    const double a = 0.5 * std::fabs(dot(c, ws32));
    if (!(a > 0.0)) continue;
    wtri.push_back((int)t);
    cdf.push_back(cdf.back() + a);
  }
  const double A = cdf.back();
  if (area_out) *area_out = A;
  if (wtri.empty() || !(A > 0.0) || pp->n_photons <= 0) return 0;
  std::vector<uint32_t> thr(wtri.size());
  for (size_t w = 0; w < wtri.size(); ++w) thr[w] = (uint32_t)std::floor(cdf[w] / A * 16777216.0);
  const uint32_t k0 = (uint32_t)pp->seed, k1 = (uint32_t)(pp->seed >> 32);
  const uint32_t kPurpose = 4u << 24;
  struct Rec { V3 p, d; int64_t id; int depth; int tri; std::vector<double> f; };
  const int nt = std::max(1, pp->threads);
  std::vector<std::vector<Rec>> out(nt);
  auto work = [&](int th, int64_t a, int64_t b) {
    std::vector<double> beta(B), F(B), R(B), Tt(B);
    std::vector<GlassCross> cr;
    const int64_t k = std::max<int64_t>(1, pp->stride);
    for (int64_t i = (a + k - 1) / k * k; i < b; i += k) {
      bool tied = false;
      const uint32_t c0 = (uint32_t)i, c1 = (uint32_t)((uint64_t)i >> 32);
      U4 rn = philox4x32_10({{c0, c1, 0u | kPurpose, 0u}}, k0, k1);
      // window w when its integer threshold floor(cdf_w / A 2^24) <= (x >> 8) < the next one
      const uint32_t x24 = rn.x[0] >> 8;
      int w = (int)(std::upper_bound(thr.begin(), thr.end(), x24) - thr.begin()) - 1;
      w = std::min(std::max(w, 0), (int)wtri.size() - 1);
      int tri = wtri[w];
      const Tri& T0 = S.tris[tri];
      const double r = std::sqrt(unif(rn.x[1])), u2 = unif(rn.x[2]);
      double bu = r * (1.0 - u2), bv = r * u2;
      V3 p = T0.v0 * (1.0 - bu - bv) + T0.v1 * bu + T0.v2 * bv;
      V3 d = ws * -1.0;
      // incoming visibility: from p toward the sun, stopped by opaque, attenuated by other glass
      {
        const V3 ng = normalize(cross(T0.v1 - T0.v0, T0.v2 - T0.v0));
        const double dn = dot(d, ng);
        const V3 n = dn > 0 ? ng * -1.0 : ng;
        const double eps = 1e-5 * (1.0 + maxabs(p));
        if (!shadow_visibility(S, mat_type, p + n * eps, ws, tri, tie, &cr, &tied)) {
          if (tied_out) tied_out[i] = tied;
          continue;
        }
        for (int j = 0; j < B; ++j) {
          double V = 1.0;
          for (const GlassCross& g : cr) {
            double Rr, Tr;
            glass_slab(sc, g.mat, j, lam[j], g.cos_t, g.tri, g.u, g.v, &Rr, &Tr);
            V *= Tr;
          }
          beta[j] = E[j] * A / (double)pp->n_photons * V;
        }
      }
      bool reflected = false;
      for (int dep = 1; dep <= pp->max_depth; ++dep) {
        const Tri& T = S.tris[tri];
        const V3 ng = normalize(cross(T.v1 - T.v0, T.v2 - T.v0));
        const double dn = dot(d, ng);
        const V3 n = dn > 0 ? ng * -1.0 : ng;
        const double cos_o = std::fabs(dn);
        if (cos_o <= tie.cos_sun) tied = true;
        const double eps = 1e-5 * (1.0 + maxabs(p));
        const int m = T.mat;
        U4 rv = philox4x32_10({{c0, c1, (uint32_t)dep | kPurpose, 0u}}, k0, k1);
        const double u0 = unif(rv.x[0]);
        V3 o;
        if (mat_type[m] == 0) {
          if (reflected || pp->global) out[th].push_back({p, d, i, dep, tri, beta});
          if (dep == pp->max_depth) break;
          double a = 0, b = 0;
          for (int j = 0; j < B; ++j) {
            F[j] = fresnel(sc->n_tab[m * B + j], sc->k_tab[m * B + j], cos_o);
            a += F[j];
            b += (1.0 - F[j]) * sc->rho_tab[m * B + j];
          }
          a /= B;
          b /= B;
          if (a + b == 0.0) break;
          const double Ps = a / (a + b);
          if (std::fabs(u0 - Ps) <= tie.lobe) tied = true;
          if (u0 < Ps) {
            for (int j = 0; j < B; ++j) beta[j] *= F[j] / Ps;
            d = d - ng * (2.0 * dn);
            reflected = true;
          } else if (!pp->global) {
            break;   // the diffuse lobe ends the photon's caustic path
          } else {
            const double u1 = unif(rv.x[1]), u2 = unif(rv.x[2]);
            const double phi = 2.0 * M_PI * u1, rr = std::sqrt(u2);
            const double lx = rr * std::cos(phi), ly = rr * std::sin(phi), lz = std::sqrt(std::max(0.0, 1.0 - u2));
            // The diffuse lobe's Fresnel factor belongs to the direction the light leaves in (for
            // camera paths the direction toward the viewer): a photon carries power the other
            // way, so its weight takes F at its new direction, cos = lz (the adjoint of the
            // camera paths' (1 - F(view)) rho)
            for (int j = 0; j < B; ++j)
              beta[j] *= (1.0 - fresnel(sc->n_tab[m * B + j], sc->k_tab[m * B + j], lz)) * sc->rho_tab[m * B + j] /
                         (1.0 - Ps);
            if (n.z != 0.0 && std::fabs(n.z) <= tie.cos_sun) tied = true;
            const double sgn = std::copysign(1.0, n.z);
            const double aa = -1.0 / (sgn + n.z);
            const double bb = n.x * n.y * aa;
            const V3 t1{1.0 + sgn * n.x * n.x * aa, sgn * bb, -sgn * n.x};
            const V3 t2{bb, sgn + n.y * n.y * aa, -n.y};
            d = t1 * lx + t2 * ly + n * lz;
          }
          o = p + n * eps;
        } else {
          if (dep == pp->max_depth) break;
          double mr = 0, mt = 0;
          for (int j = 0; j < B; ++j) {
            glass_slab(sc, m, j, lam[j], cos_o, tri, bu, bv, &R[j], &Tt[j]);
            mr += R[j];
            mt += Tt[j];
          }
          const double Pr = mr / (mr + mt);
          if (std::fabs(u0 - Pr) <= tie.lobe) tied = true;
          if (u0 < Pr) {
            for (int j = 0; j < B; ++j) beta[j] *= R[j] / Pr;
            d = d - ng * (2.0 * dn);
            o = p + n * eps;
            reflected = true;
          } else {
            for (int j = 0; j < B; ++j) beta[j] *= Tt[j] / (1.0 - Pr);
            o = p - n * eps;
          }
        }
        Hit h = closest_hit(S, o, d, tri, tie, &tied);
        if (!h.hit) break;
        tri = h.id;
        bu = h.u;
        bv = h.v;
        const Tri& Tn = S.tris[tri];
        p = Tn.v0 * (1.0 - bu - bv) + Tn.v1 * bu + Tn.v2 * bv;
      }
      if (tied_out) tied_out[i] = tied;
    }
  };
  std::vector<std::thread> ths;
  for (int k = 0; k < nt; ++k) ths.emplace_back(work, k, pp->n_photons * k / nt, pp->n_photons * (k + 1) / nt);
  for (auto& t : ths) t.join();
  int64_t n = 0;
  for (auto& v : out)
    for (const Rec& r : v) {
      if (n < cap) {
        pos[3 * n] = r.p.x; pos[3 * n + 1] = r.p.y; pos[3 * n + 2] = r.p.z;
        dir[3 * n] = r.d.x; dir[3 * n + 1] = r.d.y; dir[3 * n + 2] = r.d.z;
        for (int j = 0; j < B; ++j) flux[n * B + j] = r.f[j];
        pid[n] = r.id;
        pdepth[n] = r.depth;
        if (ptri) ptri[n] = r.tri;
      }
      ++n;
    }
  return n;
}

}  // extern "C"
