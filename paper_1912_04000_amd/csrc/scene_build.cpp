// Host scene build: spatial cells (the paper's sub-models, section 5) and one BVH per cell.
//
// The padded scene box is split into a regular grid of cells. A triangle is referenced by
// every cell whose (slightly grown) box its surface overlaps, tested with the separating-axis
// theorem (Akenine-Moeller 2001), so no geometry is ever moved between cells while rendering:
// rays move instead. Each cell gets a binned-SAH BVH (Wald 2007) over its references, with
// reference boxes clipped to the cell; nodes are stored in breadth-first order so the top
// levels of every cell are a contiguous prefix that kernels can stage in LDS.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "host.h"

namespace sdd {

namespace {

struct D3 { double x, y, z; };
inline D3 sub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline D3 crs(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double dt(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double comp(D3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Separating-axis test of a triangle against an axis-aligned box (centre c, half extents h).
bool tri_box_overlap(D3 c, D3 h, D3 a, D3 b, D3 e) {
  D3 v[3] = {sub(a, c), sub(b, c), sub(e, c)};
  auto separated = [&](D3 ax) {
    double p0 = dt(v[0], ax), p1 = dt(v[1], ax), p2 = dt(v[2], ax);
    double mn = std::min(p0, std::min(p1, p2)), mx = std::max(p0, std::max(p1, p2));
    double r = h.x * std::fabs(ax.x) + h.y * std::fabs(ax.y) + h.z * std::fabs(ax.z);
    return mn > r || mx < -r;
  };
  const D3 ex[3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int i = 0; i < 3; ++i)
    if (separated(ex[i])) return false;
  D3 f[3] = {sub(v[1], v[0]), sub(v[2], v[1]), sub(v[0], v[2])};
  if (separated(crs(f[0], f[1]))) return false;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      D3 ax = crs(ex[i], f[j]);
      if (ax.x == 0 && ax.y == 0 && ax.z == 0) continue;
      if (separated(ax)) return false;
    }
  return true;
}

struct Box3 {
  float lo[3], hi[3];
  void empty() { for (int i = 0; i < 3; ++i) { lo[i] = INFINITY; hi[i] = -INFINITY; } }
  void grow(const Box3& b) {
    for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], b.lo[i]); hi[i] = std::max(hi[i], b.hi[i]); }
  }
  void grow_pt(const float* p) {
    for (int i = 0; i < 3; ++i) { lo[i] = std::min(lo[i], p[i]); hi[i] = std::max(hi[i], p[i]); }
  }
  double area() const {
    double dx = std::max(0.0f, hi[0] - lo[0]), dy = std::max(0.0f, hi[1] - lo[1]), dz = std::max(0.0f, hi[2] - lo[2]);
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct Ref { int32_t tri; Box3 box; float cen[3]; };

struct Child { Box3 box; uint32_t idx; uint32_t cnt; };  // cnt > 0 leaf, 0 inner, idx==kEmptyChild none

struct BNode { Child c[2]; };
struct WNode { Child c[kWide]; };  // node of the 4-wide tree the traversal reads

struct CellBVH {
  std::vector<WNode> nodes;      // 4-wide, breadth-first order
  std::vector<int32_t> tris;     // reference order (leaves are contiguous ranges)
  int depth = 0;                 // binary build depth
  int wdepth = 0;                // 4-wide depth
  int max_leaf = 0;
};

constexpr int kBins = 64;
constexpr int kLeafMax = 4;        // largest leaf the cost rule may keep
constexpr double kCostNode = 1.0;      // a node visit against one triangle test
constexpr int kDepthCap = 46;  // binary depth cap: 4-wide depth <= 23, stack <= 3 * 23 + 1 < kMaxStack

// Recursive binned-SAH build. Returns the child descriptor for refs[first, first+count).
Child build_rec(std::vector<Ref>& refs, int first, int count, int depth, std::vector<BNode>& nodes, CellBVH& out) {
  Box3 bb, cb;
  bb.empty();
  cb.empty();
  for (int i = first; i < first + count; ++i) {
    bb.grow(refs[i].box);
    cb.grow_pt(refs[i].cen);
  }
  out.depth = std::max(out.depth, depth);
  auto make_leaf = [&]() {
    Child ch;
    ch.box = bb;
    ch.idx = (uint32_t)first;
    ch.cnt = (uint32_t)count;
    out.max_leaf = std::max(out.max_leaf, count);
    return ch;
  };
  if (count <= 1 || depth >= kDepthCap) return make_leaf();

  int best_axis = -1, best_split = -1;
  double best_cost = INFINITY;
  for (int ax = 0; ax < 3; ++ax) {
    double ext = (double)cb.hi[ax] - cb.lo[ax];
    if (!(ext > 0)) continue;
    Box3 bbox[kBins];
    int bcnt[kBins] = {0};
    for (int b = 0; b < kBins; ++b) bbox[b].empty();
    for (int i = first; i < first + count; ++i) {
      int b = (int)((refs[i].cen[ax] - cb.lo[ax]) / ext * kBins);
      b = std::min(kBins - 1, std::max(0, b));
      bcnt[b]++;
      bbox[b].grow(refs[i].box);
    }
    double la[kBins], ra[kBins];
    int lc[kBins], rc[kBins];
    Box3 acc;
    acc.empty();
    int c = 0;
    for (int b = 0; b < kBins - 1; ++b) {
      acc.grow(bbox[b]);
      c += bcnt[b];
      la[b] = acc.area();
      lc[b] = c;
    }
    acc.empty();
    c = 0;
    for (int b = kBins - 1; b > 0; --b) {
      acc.grow(bbox[b]);
      c += bcnt[b];
      ra[b - 1] = acc.area();
      rc[b - 1] = c;
    }
    for (int s = 0; s < kBins - 1; ++s) {
      if (lc[s] == 0 || rc[s] == 0) continue;
      double cost = la[s] * lc[s] + ra[s] * rc[s];
      if (cost < best_cost) { best_cost = cost; best_axis = ax; best_split = s; }
    }
  }
  // a leaf costs one test per triangle; a split one node visit plus the children's triangles
  // weighted by the chance that a ray through this box enters each child (area ratio)
  if (count <= kLeafMax && best_axis >= 0 && count <= kCostNode + best_cost / bb.area()) return make_leaf();
  if (count <= kLeafMax && best_axis < 0) return make_leaf();
  int mid;
  if (best_axis < 0) {
    // all centroids coincide: split the list in halves (boxes overlap, still correct)
    mid = first + count / 2;
  } else {
    double ext = (double)cb.hi[best_axis] - cb.lo[best_axis];
    auto it = std::partition(refs.begin() + first, refs.begin() + first + count, [&](const Ref& r) {
      int b = (int)((r.cen[best_axis] - cb.lo[best_axis]) / ext * kBins);
      b = std::min(kBins - 1, std::max(0, b));
      return b <= best_split;
    });
    mid = (int)(it - refs.begin());
    if (mid == first || mid == first + count) mid = first + count / 2;
  }
  uint32_t me = (uint32_t)nodes.size();
  nodes.push_back(BNode{});
  Child l = build_rec(refs, first, mid - first, depth + 1, nodes, out);
  Child r = build_rec(refs, mid, first + count - mid, depth + 1, nodes, out);
  nodes[me].c[0] = l;
  nodes[me].c[1] = r;
  Child ch;
  ch.box = bb;
  ch.idx = me;
  ch.cnt = 0;
  return ch;
}

// Wide node for binary node i2 (children gathered as described in build_cell); returns its
// index in `wide`.
uint32_t collapse(const std::vector<BNode>& bin, uint32_t i2, int depth, std::vector<WNode>& wide, CellBVH& out) {
  out.wdepth = std::max(out.wdepth, depth);
  Child ch[kWide];
  int n = 0;
  for (int c = 0; c < 2; ++c)
    if (bin[i2].c[c].idx != kEmptyChild) ch[n++] = bin[i2].c[c];
  while (n < kWide) {
    int best = -1;
    double ba = -1.0;
    for (int k = 0; k < n; ++k)
      if (ch[k].cnt == 0 && ch[k].box.area() > ba) {
        ba = ch[k].box.area();
        best = k;
      }
    if (best < 0) break;
    const BNode& o = bin[ch[best].idx];
    ch[best] = ch[--n];
    for (int c = 0; c < 2; ++c)
      if (o.c[c].idx != kEmptyChild) ch[n++] = o.c[c];
  }
  const uint32_t me = (uint32_t)wide.size();
  wide.push_back(WNode{});
  WNode w;
  for (int k = 0; k < kWide; ++k) {
    if (k < n) {
      w.c[k] = ch[k];
      if (ch[k].cnt == 0) w.c[k].idx = collapse(bin, ch[k].idx, depth + 1, wide, out);
    } else {
      w.c[k].box.empty();
      w.c[k].idx = kEmptyChild;
      w.c[k].cnt = 0;
    }
  }
  wide[me] = w;
  return me;
}

void build_cell(std::vector<Ref>& refs, CellBVH& out) {
  out.nodes.clear();
  out.tris.clear();
  if (refs.empty()) return;
  std::vector<BNode> nodes;
  nodes.reserve(refs.size());
  nodes.push_back(BNode{});  // root
  Child top = build_rec(refs, 0, (int)refs.size(), 1, nodes, out);
  if (top.cnt > 0) {
    nodes[0].c[0] = top;
    nodes[0].c[1].box.empty();
    nodes[0].c[1].idx = kEmptyChild;
    nodes[0].c[1].cnt = 0;
  } else {
    // the recursion allocated a fresh node for the top split; make it the root
    nodes[0] = nodes[top.idx];
    nodes[top.idx].c[0].idx = kEmptyChild;  // orphan, dropped by the BFS pass
  }
  // 4-wide tree: every wide node takes a binary node's children and opens its largest inner
  // child (by box area) until it holds four, so a traversal step tests four boxes
  std::vector<WNode> wide;
  wide.reserve(nodes.size() / 2 + 1);
  collapse(nodes, 0, 1, wide, out);
  // breadth-first renumbering (the top levels of a cell form a contiguous prefix)
  std::vector<uint32_t> order{0}, remap(wide.size(), kEmptyChild);
  remap[0] = 0;
  for (size_t q = 0; q < order.size(); ++q) {
    const WNode& n = wide[order[q]];
    for (int c = 0; c < kWide; ++c)
      if (n.c[c].cnt == 0 && n.c[c].idx != kEmptyChild) {
        remap[n.c[c].idx] = (uint32_t)order.size();
        order.push_back(n.c[c].idx);
      }
  }
  out.nodes.resize(order.size());
  for (size_t q = 0; q < order.size(); ++q) {
    WNode n = wide[order[q]];
    for (int c = 0; c < kWide; ++c)
      if (n.c[c].cnt == 0 && n.c[c].idx != kEmptyChild) n.c[c].idx = remap[n.c[c].idx];
    out.nodes[q] = n;
  }
  out.tris.resize(refs.size());
  for (size_t i = 0; i < refs.size(); ++i) out.tris[i] = refs[i].tri;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// A 4-wide node in 64 bytes (four 16-byte words): the child boxes quantised to 8 bits per bound
// on a grid of the node's own box (after Ylitie, Karras and Laine, "Efficient incoherent ray
// traversal on GPUs through compressed wide BVHs", HPG 2017):
//   word 0: origin x, y, z (the node box's low corner, FP32) | exponents e_x, e_y, e_z (bytes 0..2)
//   word 1: the four child words (inner node index, count << 27 | first triangle, or empty)
//   word 2: lo.x, hi.x, lo.y, hi.y of the four children, one byte per child (child c in byte c)
//   word 3: lo.z, hi.z of the four children | 0 | 0
// A child's bound is origin + q 2^(e - 127); e is the smallest power of two with 255 steps
// covering the node box, lo rounded down and hi rounded up, so the stored box always contains
// the child's box. Empty children have zero bytes and the empty word. Returns false if the
// containment check (exact, in double) fails.
bool quantize_node(const WNode& n, uint32_t* o) {
  double L[3], Hh[3];
  for (int a = 0; a < 3; ++a) {
    L[a] = INFINITY;
    Hh[a] = -INFINITY;
  }
  for (int k = 0; k < kWide; ++k) {
    if (n.c[k].idx == kEmptyChild) continue;
    for (int a = 0; a < 3; ++a) {
      L[a] = std::min(L[a], (double)n.c[k].box.lo[a]);
      Hh[a] = std::max(Hh[a], (double)n.c[k].box.hi[a]);
    }
  }
  uint32_t ebytes = 0;
  double scale[3];
  float origin[3];
  for (int a = 0; a < 3; ++a) {
    if (!(L[a] <= Hh[a])) L[a] = Hh[a] = 0.0;   // a node without children (not produced)
    origin[a] = (float)L[a];                   // the children's bounds are floats: exact
    const double ext = Hh[a] - L[a];
    int e = -126;
    while (e < 127 && std::ldexp(255.0, e) < ext) ++e;
    scale[a] = std::ldexp(1.0, e);
    ebytes |= (uint32_t)(e + 127) << (8 * a);
  }
  uint32_t q[6] = {0, 0, 0, 0, 0, 0};   // lo.x hi.x lo.y hi.y lo.z hi.z
  uint32_t words[kWide];
  for (int k = 0; k < kWide; ++k) {
    const Child& c = n.c[k];
    words[k] = c.idx == kEmptyChild ? kEmptyChild : (c.cnt > 0 ? (c.cnt << 27) | c.idx : c.idx);
    if (c.idx == kEmptyChild) continue;
    for (int a = 0; a < 3; ++a) {
      const double ql = std::floor((c.box.lo[a] - L[a]) / scale[a]);
      const double qh = std::ceil((c.box.hi[a] - L[a]) / scale[a]);
      const uint32_t bl = (uint32_t)std::min(255.0, std::max(0.0, ql));
      const uint32_t bh = (uint32_t)std::min(255.0, std::max(0.0, qh));
      if (!(L[a] + bl * scale[a] <= (double)c.box.lo[a]) || !(L[a] + bh * scale[a] >= (double)c.box.hi[a]))
        return false;
      q[2 * a] |= bl << (8 * k);
      q[2 * a + 1] |= bh << (8 * k);
    }
  }
  std::memcpy(o, origin, 12);
  o[3] = ebytes;
  std::memcpy(o + 4, words, 16);
  for (int j = 0; j < 6; ++j) o[8 + j] = q[j];
  o[14] = o[15] = 0;
  return true;
}

}  // namespace

std::string build_scene(const sdd_scene_desc& d, sdd_scene* out) {
  // ---------------- validation ----------------
  if (!d.verts || !d.mat || !d.materials || !d.n_tab || !d.k_tab || !d.rho_tab || !d.sun_irradiance)
    return "null pointer in scene description";
  if (d.n_tri < 1 || d.n_tri > (int64_t)INT32_MAX / 4) return "n_tri out of range";
  if (d.n_mat < 1 || d.n_mat > 65535) return "n_mat out of range";
  if (d.n_bins < 1 || d.n_bins > kMaxBins) return "n_bins out of range (1..128)";
  if (!(d.lambda_min_nm > 0) || !(d.lambda_max_nm > d.lambda_min_nm) || !std::isfinite(d.lambda_max_nm))
    return "wavelength range invalid";
  for (int i = 0; i < 3; ++i)
    if (d.grid[i] < 1 || d.grid[i] > kMaxGrid) return "grid out of range (1..64 per axis)";
  const int B = d.n_bins, M = d.n_mat;
  const int64_t N = d.n_tri;
  for (int m = 0; m < M; ++m) {
    if (d.materials[m].type != SDD_MAT_OPAQUE && d.materials[m].type != SDD_MAT_GLASS) return "bad material type";
    if (d.materials[m].type == SDD_MAT_GLASS && !(d.materials[m].thickness_m >= 0 && std::isfinite(d.materials[m].thickness_m)))
      return "bad glass thickness";
    for (int j = 0; j < B; ++j) {
      float n = d.n_tab[m * B + j], k = d.k_tab[m * B + j], r = d.rho_tab[m * B + j];
      if (!(n > 0) || !std::isfinite(n)) return "n must be finite and > 0";
      if (!(k >= 0) || !std::isfinite(k)) return "k must be finite and >= 0";
      if (!(r >= 0 && r <= 1)) return "rho must lie in [0,1]";
    }
  }
  for (int j = 0; j < B; ++j) {
    if (!(d.sun_irradiance[j] >= 0) || !std::isfinite(d.sun_irradiance[j])) return "sun irradiance must be finite >= 0";
    if (d.env_radiance && (!(d.env_radiance[j] >= 0) || !std::isfinite(d.env_radiance[j])))
      return "env radiance must be finite >= 0";
  }
  double sl = std::sqrt((double)d.sun_dir[0] * d.sun_dir[0] + (double)d.sun_dir[1] * d.sun_dir[1] +
                        (double)d.sun_dir[2] * d.sun_dir[2]);
  if (!(sl > 1e-12) || !std::isfinite(sl)) return "sun direction must be non-zero and finite";
  // spectral transmittance maps of glass
  const int NT = d.n_tex;
  uint64_t texel_floats = 0;
  if (NT < 0 || NT > 65535) return "n_tex out of range (0..65535)";
  if (NT > 0) {
    if (!d.uv || !d.textures || !d.mat_texture) return "maps need uv, textures and mat_texture";
    for (int t = 0; t < NT; ++t) {
      const sdd_texture& T = d.textures[t];
      if (!T.tau0 || T.width < 1 || T.height < 1 || (int64_t)T.width * T.height > (1 << 24))
        return "map " + std::to_string(t) + ": bad size or null data";
      const int64_t nv = (int64_t)T.width * T.height * B;
      for (int64_t i = 0; i < nv; ++i)
        if (!(T.tau0[i] >= 0.0f && T.tau0[i] <= 1.0f)) return "map " + std::to_string(t) + ": values must lie in [0,1]";
      texel_floats += (uint64_t)T.width * T.height * ((B + 3) & ~3);
    }
    if (texel_floats > (uint64_t)INT32_MAX) return "maps too large (more than 2^31 texel values)";
    for (int m = 0; m < M; ++m) {
      const int t = d.mat_texture[m];
      if (t < -1 || t >= NT) return "mat_texture out of range";
      if (t >= 0 && d.materials[m].type != SDD_MAT_GLASS) return "only glass materials take a transmittance map";
    }
    for (int64_t i = 0; i < 6 * N; ++i)
      if (!(std::fabs(d.uv[i]) <= 1e6f)) return "texture coordinates must be finite, |uv| <= 1e6";
  }
  double maxabs = 0;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < N; ++i) {
    if (d.mat[i] >= M) return "material id >= n_mat at triangle " + std::to_string(i);
    for (int k = 0; k < 9; ++k) {
      float v = d.verts[9 * i + k];
      if (!std::isfinite(v)) return "non-finite vertex at triangle " + std::to_string(i);
      lo[k % 3] = std::min(lo[k % 3], v);
      hi[k % 3] = std::max(hi[k % 3], v);
      maxabs = std::max(maxabs, (double)std::fabs(v));
    }
  }

  // ---------------- grid ----------------
  double ext = std::max({(double)hi[0] - lo[0], (double)hi[1] - lo[1], (double)hi[2] - lo[2], 1e-6});
  double pad = 1e-4 * ext + 1e-6 * (1.0 + maxabs);
  const int g[3] = {d.grid[0], d.grid[1], d.grid[2]};
  std::vector<float> planes;
  float glo[3], ghi[3];
  double cs_max = 0;
  for (int a = 0; a < 3; ++a) {
    double l = (double)lo[a] - pad, h = (double)hi[a] + pad;
    glo[a] = (float)l;
    ghi[a] = (float)h;
    for (int i = 0; i <= g[a]; ++i) {
      float p = (i == g[a]) ? ghi[a] : (float)(l + (h - l) * i / g[a]);
      if (i > 0 && !(p > planes.back())) return "degenerate cell grid (cells too thin for FP32)";
      planes.push_back(p);
    }
    cs_max = std::max(cs_max, (h - l) / g[a]);
  }
  const float* px = planes.data();
  const float* py = px + g[0] + 1;
  const float* pz = py + g[1] + 1;
  const float* pl[3] = {px, py, pz};
  const int n_cells = g[0] * g[1] * g[2];
  // binning slack: covers FP32 error of hit distances and cell intervals near cell faces
  const double bpad = 1e-4 * cs_max + 4e-6 * (1.0 + maxabs);

  // ---------------- cell binning ----------------
  int nth = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  std::vector<std::vector<std::vector<int32_t>>> per_thread(nth, std::vector<std::vector<int32_t>>(n_cells));
  std::atomic<int64_t> next{0};
  auto bin_worker = [&](int tid) {
    auto& lists = per_thread[tid];
    const int64_t chunk = 4096;
    for (;;) {
      int64_t a = next.fetch_add(chunk);
      if (a >= N) break;
      int64_t b = std::min(N, a + chunk);
      for (int64_t i = a; i < b; ++i) {
        const float* v = d.verts + 9 * i;
        D3 A{v[0], v[1], v[2]}, Bv{v[3], v[4], v[5]}, Cv{v[6], v[7], v[8]};
        D3 nn = crs(sub(Bv, A), sub(Cv, A));
        if (nn.x == 0 && nn.y == 0 && nn.z == 0) continue;  // zero area: never hit
        int r0[3], r1[3];
        for (int ax = 0; ax < 3; ++ax) {
          double mn = std::min({comp(A, ax), comp(Bv, ax), comp(Cv, ax)}) - bpad;
          double mx = std::max({comp(A, ax), comp(Bv, ax), comp(Cv, ax)}) + bpad;
          int i0 = 0, i1 = g[ax] - 1;
          while (i0 < g[ax] - 1 && pl[ax][i0 + 1] < mn) ++i0;
          while (i1 > 0 && pl[ax][i1] > mx) --i1;
          r0[ax] = i0;
          r1[ax] = i1;
        }
        for (int iz = r0[2]; iz <= r1[2]; ++iz)
          for (int iy = r0[1]; iy <= r1[1]; ++iy)
            for (int ix = r0[0]; ix <= r1[0]; ++ix) {
              D3 c{0.5 * ((double)px[ix] + px[ix + 1]), 0.5 * ((double)py[iy] + py[iy + 1]),
                   0.5 * ((double)pz[iz] + pz[iz + 1])};
              D3 h{0.5 * ((double)px[ix + 1] - px[ix]) + bpad, 0.5 * ((double)py[iy + 1] - py[iy]) + bpad,
                   0.5 * ((double)pz[iz + 1] - pz[iz]) + bpad};
              bool single = (r0[0] == r1[0] && r0[1] == r1[1] && r0[2] == r1[2]);
              if (single || tri_box_overlap(c, h, A, Bv, Cv)) lists[(iz * g[1] + iy) * g[0] + ix].push_back((int32_t)i);
            }
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(bin_worker, t);
    for (auto& t : th) t.join();
  }

  // ---------------- per-cell BVH ----------------
  std::vector<CellBVH> cells(n_cells);
  std::atomic<int> next_cell{0};
  std::vector<int> corder(n_cells);
  std::vector<size_t> csize(n_cells, 0);
  for (int c = 0; c < n_cells; ++c) {
    corder[c] = c;
    for (int t = 0; t < nth; ++t) csize[c] += per_thread[t][c].size();
  }
  std::sort(corder.begin(), corder.end(), [&](int a, int b) { return csize[a] > csize[b]; });
  auto bvh_worker = [&]() {
    std::vector<Ref> refs;
    for (;;) {
      int k = next_cell.fetch_add(1);
      if (k >= n_cells) break;
      int c = corder[k];
      int ix = c % g[0], iy = (c / g[0]) % g[1], iz = c / (g[0] * g[1]);
      float clo[3] = {(float)(px[ix] - bpad), (float)(py[iy] - bpad), (float)(pz[iz] - bpad)};
      float chi[3] = {(float)(px[ix + 1] + bpad), (float)(py[iy + 1] + bpad), (float)(pz[iz + 1] + bpad)};
      refs.clear();
      for (int t = 0; t < nth; ++t) {
        std::vector<int32_t>& L = per_thread[t][c];
        std::sort(L.begin(), L.end());
        for (int32_t tri : L) {
          Ref r;
          r.tri = tri;
          r.box.empty();
          const float* v = d.verts + 9 * (int64_t)tri;
          for (int k2 = 0; k2 < 3; ++k2) r.box.grow_pt(v + 3 * k2);
          for (int a = 0; a < 3; ++a) {  // clip to the grown cell box: hits outside it are rejected anyway
            r.box.lo[a] = std::max(r.box.lo[a], clo[a]);
            r.box.hi[a] = std::min(r.box.hi[a], chi[a]);
            if (r.box.lo[a] > r.box.hi[a]) r.box.lo[a] = r.box.hi[a] = 0.5f * (clo[a] + chi[a]);
            r.cen[a] = 0.5f * (r.box.lo[a] + r.box.hi[a]);
          }
          refs.push_back(r);
        }
        std::vector<int32_t>().swap(L);
      }
      build_cell(refs, cells[c]);
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(bvh_worker);
    for (auto& t : th) t.join();
  }

  // ---------------- serialise ----------------
  uint64_t n_nodes = 0, n_refs = 0;
  int max_depth = 0, max_leaf = 0;
  int64_t empty = 0;
  for (auto& c : cells) {
    n_nodes += c.nodes.size();
    n_refs += c.tris.size();
    max_depth = std::max(max_depth, c.wdepth);
    max_leaf = std::max(max_leaf, c.max_leaf);
    if (c.tris.empty()) ++empty;
  }
  // a wide node visit pushes at most three entries
  if (3 * max_depth + 1 > kMaxStack) return "internal: BVH depth exceeds the traversal stack";
  // the traversal stack encodes a leaf as (first triangle, count) in one word
  if (max_leaf > (int)kStackLeafMaxCount) return "scene too degenerate: a BVH leaf holds more than 15 triangles";
  for (auto& c : cells)
    if (c.tris.size() > (size_t)kStackLeafMaxIndex) return "scene too large: a cell holds more than 2^27 triangles";
  if (n_refs > (uint64_t)INT32_MAX || n_nodes > (uint64_t)INT32_MAX) return "scene too large for 32-bit indices";

  SceneHeader H;
  std::memset(&H, 0, sizeof(H));
  H.magic = 0x53444431u;  // "SDD1"
  H.version = 1;
  H.n_tri = (int32_t)N;
  H.n_mat = M;
  H.n_bins = B;
  H.n_cells = n_cells;
  for (int a = 0; a < 3; ++a) {
    H.grid[a] = g[a];
    H.lo[a] = glo[a];
    H.hi[a] = ghi[a];
    H.sun[a] = (float)(d.sun_dir[a] / sl);
  }
  H.max_depth = max_depth;
  H.max_leaf = max_leaf;
  H.lambda_min_nm = d.lambda_min_nm;
  H.lambda_max_nm = d.lambda_max_nm;
  int env_nz = 0;
  if (d.env_radiance)
    for (int j = 0; j < B; ++j) env_nz |= d.env_radiance[j] != 0.0f;
  H.env_nonzero = env_nz;
  size_t off = kHeaderBytes;
  H.off_planes = off; off = align256(off + planes.size() * 4);
  H.off_cells = off;  off = align256(off + (size_t)n_cells * 16);
  H.off_nodes = off;  off = align256(off + n_nodes * 64);
  H.off_ctris = off;  off = align256(off + n_refs * 48);
  H.off_gtris = off;  off = align256(off + (size_t)N * 48);
  H.off_mtype = off;  off = align256(off + (size_t)M * 4);
  H.off_thick = off;  off = align256(off + (size_t)M * 4);
  // spectral tables use a row stride of Bp = B rounded up to 4 so kernels read them as float4;
  // the padding bins hold harmless values (n = 1.5, k = 0, rho = 0, E = 0, lambda = 500 nm)
  const int Bp = (B + 3) & ~3;
  H.off_n = off;      off = align256(off + (size_t)M * Bp * 4);
  H.off_k = off;      off = align256(off + (size_t)M * Bp * 4);
  H.off_rho = off;    off = align256(off + (size_t)M * Bp * 4);
  H.off_lambda = off; off = align256(off + (size_t)Bp * 4);
  H.off_sunE = off;   off = align256(off + (size_t)Bp * 4);
  H.off_env = off;    off = align256(off + (size_t)Bp * 4);
  H.n_tex = NT;
  H.off_uv = off;      off = align256(off + (NT > 0 ? (size_t)N * 32 : 0));
  H.off_texinfo = off; off = align256(off + (size_t)NT * 16);
  H.off_texel = off;   off = align256(off + texel_floats * 4);
  H.off_mtex = off;    off = align256(off + (size_t)M * 4);
  H.bins_pad = Bp;
  H.n_nodes = n_nodes;
  H.n_refs = n_refs;
  out->image.assign(off, 0);
  uint8_t* img = out->image.data();
  std::memcpy(img, &H, sizeof(H));
  std::memcpy(img + H.off_planes, planes.data(), planes.size() * 4);
  int4* ctab = (int4*)(img + H.off_cells);
  float* nodes = (float*)(img + H.off_nodes);
  float* ctris = (float*)(img + H.off_ctris);
  uint64_t nb = 0, tb = 0;
  for (int c = 0; c < n_cells; ++c) {
    CellBVH& cb = cells[c];
    ctab[c] = make_int4((int)nb, (int)cb.nodes.size(), (int)tb, (int)cb.tris.size());
    for (size_t i = 0; i < cb.nodes.size(); ++i) {
      const WNode& n = cb.nodes[i];
      uint32_t* o = (uint32_t*)(nodes + (nb + i) * 16);
      if (!quantize_node(n, o)) return "internal: a quantised child box does not contain its child";
    }
    for (size_t i = 0; i < cb.tris.size(); ++i) {
      int32_t t = cb.tris[i];
      const float* v = d.verts + 9 * (int64_t)t;
      float* o = ctris + (tb + i) * 12;
      uint32_t id = (uint32_t)t, m = d.mat[t];
      o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; std::memcpy(o + 3, &id, 4);
      o[4] = v[3]; o[5] = v[4]; o[6] = v[5]; std::memcpy(o + 7, &m, 4);
      o[8] = v[6]; o[9] = v[7]; o[10] = v[8]; o[11] = 0.0f;
    }
    nb += cb.nodes.size();
    tb += cb.tris.size();
  }
  float* gt = (float*)(img + H.off_gtris);
  for (int64_t t = 0; t < N; ++t) {
    const float* v = d.verts + 9 * t;
    float* o = gt + t * 12;
    uint32_t id = (uint32_t)t, m = d.mat[t];
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; std::memcpy(o + 3, &id, 4);
    o[4] = v[3]; o[5] = v[4]; o[6] = v[5]; std::memcpy(o + 7, &m, 4);
    o[8] = v[6]; o[9] = v[7]; o[10] = v[8]; o[11] = 0.0f;
  }
  int32_t* mt = (int32_t*)(img + H.off_mtype);
  float* th = (float*)(img + H.off_thick);
  for (int m = 0; m < M; ++m) {
    mt[m] = d.materials[m].type;
    th[m] = d.materials[m].thickness_m;
  }
  float* tn = (float*)(img + H.off_n);
  float* tk = (float*)(img + H.off_k);
  float* tr = (float*)(img + H.off_rho);
  for (int m = 0; m < M; ++m)
    for (int j = 0; j < Bp; ++j) {
      tn[m * Bp + j] = j < B ? d.n_tab[m * B + j] : 1.5f;
      tk[m * Bp + j] = j < B ? d.k_tab[m * B + j] : 0.0f;
      tr[m * Bp + j] = j < B ? d.rho_tab[m * B + j] : 0.0f;
    }
  float* lam = (float*)(img + H.off_lambda);
  float* sE = (float*)(img + H.off_sunE);
  float* sL = (float*)(img + H.off_env);
  for (int j = 0; j < Bp; ++j) {
    lam[j] = j < B ? (float)((double)d.lambda_min_nm + (j + 0.5) * ((double)d.lambda_max_nm - d.lambda_min_nm) / B)
                   : 500.0f;
    sE[j] = j < B ? d.sun_irradiance[j] : 0.0f;
    sL[j] = (j < B && d.env_radiance) ? d.env_radiance[j] : 0.0f;
  }

  int32_t* mtex = (int32_t*)(img + H.off_mtex);
  for (int m = 0; m < M; ++m) mtex[m] = NT > 0 ? d.mat_texture[m] : -1;
  if (NT > 0) {
    float* uv = (float*)(img + H.off_uv);
    for (int64_t t = 0; t < N; ++t) {
      const float* q = d.uv + 6 * t;
      float* o = uv + 8 * t;
      for (int k = 0; k < 6; ++k) o[k] = q[k];
      o[6] = o[7] = 0.0f;
    }
    int4* ti = (int4*)(img + H.off_texinfo);
    float* tx = (float*)(img + H.off_texel);
    uint64_t at = 0;
    for (int t = 0; t < NT; ++t) {
      const sdd_texture& T = d.textures[t];
      ti[t] = make_int4((int)at, T.width, T.height, 0);
      for (int64_t p = 0; p < (int64_t)T.width * T.height; ++p)
        for (int j = 0; j < Bp; ++j) tx[at + p * Bp + j] = j < B ? T.tau0[p * B + j] : 1.0f;
      at += (uint64_t)T.width * T.height * Bp;
    }
  }

  out->hdr = H;
  sdd_scene_info& I = out->info;
  std::memset(&I, 0, sizeof(I));
  I.n_tri = N;
  I.n_refs = (int64_t)n_refs;
  I.n_nodes = (int64_t)n_nodes;
  I.n_cells = n_cells;
  I.n_empty_cells = empty;
  I.max_depth = max_depth;
  I.max_leaf = max_leaf;
  I.device_bytes = off;
  for (int a = 0; a < 3; ++a) {
    I.grid_lo[a] = glo[a];
    I.grid_hi[a] = ghi[a];
  }
  return "";
}

DevScene device_view(const sdd_scene* s) {
  const SceneHeader& H = s->hdr;
  const uint8_t* b = (const uint8_t*)s->dev;
  DevScene S;
  std::memset(&S, 0, sizeof(S));
  S.nodes = (const float4*)(b + H.off_nodes);
  S.ctris = (const float4*)(b + H.off_ctris);
  S.gtris = (const float4*)(b + H.off_gtris);
  S.cells = (const int4*)(b + H.off_cells);
  S.planes = (const float*)(b + H.off_planes);
  S.mtype = (const int32_t*)(b + H.off_mtype);
  S.thick = (const float*)(b + H.off_thick);
  S.ntab = (const float*)(b + H.off_n);
  S.ktab = (const float*)(b + H.off_k);
  S.rho = (const float*)(b + H.off_rho);
  S.lambda = (const float*)(b + H.off_lambda);
  S.sunE = (const float*)(b + H.off_sunE);
  S.env = (const float*)(b + H.off_env);
  S.guv = (const float4*)(b + H.off_uv);
  S.texinfo = (const int4*)(b + H.off_texinfo);
  S.texel = (const float*)(b + H.off_texel);
  S.mtex = (const int32_t*)(b + H.off_mtex);
  S.n_tex = H.n_tex;
  S.gx = H.grid[0];
  S.gy = H.grid[1];
  S.gz = H.grid[2];
  S.n_cells = H.n_cells;
  for (int a = 0; a < 3; ++a) {
    S.lo[a] = H.lo[a];
    S.hi[a] = H.hi[a];
    S.inv_cs[a] = (float)(H.grid[a] / ((double)H.hi[a] - H.lo[a]));
    S.sun[a] = H.sun[a];
  }
  S.n_bins = H.n_bins;
  S.bins_pad = H.bins_pad;
  S.n_mat = H.n_mat;
  S.env_nonzero = H.env_nonzero;
  return S;
}

}  // namespace sdd
