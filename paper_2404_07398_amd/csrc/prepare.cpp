// Mesh-only preparation of the implicit filter (Sect. 2.2.1): active cells,
// dofs, flat-facet geometry, lumped mass, stiffness, order-n operator and a
// locality ordering. Host C++, run once per mesh; the result is reused for
// every field and every scale.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace ifl {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }

// Corner positions of triangle t; periodic edges are unwrapped by the
// minimum image relative to corner 0. Planar points get z = 0.
void corners(const ifl_mesh& m, const int32_t* t, V3 p[3]) {
  if (m.geometry == IFL_GEOM_SPHERE) {
    for (int i = 0; i < 3; ++i) {
      const double* c = m.coords + 3 * (int64_t)t[i];
      p[i] = {c[0], c[1], c[2]};
    }
    return;
  }
  const double* c0 = m.coords + 2 * (int64_t)t[0];
  p[0] = {c0[0], c0[1], 0.0};
  for (int i = 1; i < 3; ++i) {
    const double* c = m.coords + 2 * (int64_t)t[i];
    double dx = c[0] - c0[0], dy = c[1] - c0[1];
    if (m.geometry == IFL_GEOM_PERIODIC) {
      dx -= m.period[0] * std::nearbyint(dx / m.period[0]);
      dy -= m.period[1] * std::nearbyint(dy / m.period[1]);
    }
    p[i] = {c0[0] + dx, c0[1] + dy, 0.0};
  }
}

// COO triplets -> CSR with sorted columns; duplicates are summed in the
// order they were added, so two rows that receive the same contributions in
// the same order get bitwise equal entries.
struct Triplets {
  std::vector<int64_t> r;
  std::vector<int32_t> c;
  std::vector<double> v;
  void add(int64_t i, int64_t j, double x) {
    r.push_back(i);
    c.push_back((int32_t)j);
    v.push_back(x);
  }
};

void to_csr(int64_t n, const Triplets& t, std::vector<int64_t>& row_ptr, std::vector<int32_t>& col,
            std::vector<double>& val) {
  const int64_t m = (int64_t)t.r.size();
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t e = 0; e < m; ++e) cnt[t.r[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  std::vector<int32_t> bc(m);
  std::vector<double> bv(m);
  for (int64_t e = 0; e < m; ++e) {
    int64_t p = pos[t.r[e]]++;
    bc[p] = t.c[e];
    bv[p] = t.v[e];
  }
  row_ptr.assign(n + 1, 0);
  col.clear();
  val.clear();
  col.reserve(m);
  val.reserve(m);
  std::vector<int64_t> idx;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t b = cnt[i], e = cnt[i + 1];
    idx.resize(e - b);
    std::iota(idx.begin(), idx.end(), b);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t q) { return bc[a] < bc[q]; });
    for (size_t k = 0; k < idx.size();) {
      const int32_t cc = bc[idx[k]];
      double s = 0.0;
      while (k < idx.size() && bc[idx[k]] == cc) s += bv[idx[k++]];
      col.push_back(cc);
      val.push_back(s);
    }
    row_ptr[i + 1] = (int64_t)col.size();
  }
}

// C = A diag(1/m) B for CSR A, B with sorted columns. Entry (i, j) sums
// (A_ik B_kj) / m_k over k ascending; with A = B symmetric this makes C
// bitwise symmetric.
void spgemm_scaled(int64_t n, const std::vector<int64_t>& ap, const std::vector<int32_t>& ac,
                   const std::vector<double>& av, const std::vector<int64_t>& bp,
                   const std::vector<int32_t>& bc, const std::vector<double>& bv,
                   const std::vector<double>& m, std::vector<int64_t>& cp, std::vector<int32_t>& cc,
                   std::vector<double>& cv) {
  std::vector<double> acc(n, 0.0);
  std::vector<int64_t> mark(n, -1);
  std::vector<int32_t> touched;
  cp.assign(n + 1, 0);
  cc.clear();
  cv.clear();
  for (int64_t i = 0; i < n; ++i) {
    touched.clear();
    for (int64_t a = ap[i]; a < ap[i + 1]; ++a) {
      const int32_t k = ac[a];
      const double aik = av[a];
      for (int64_t b = bp[k]; b < bp[k + 1]; ++b) {
        const int32_t j = bc[b];
        const double t = (aik * bv[b]) / m[k];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = t;
          touched.push_back(j);
        } else {
          acc[j] += t;
        }
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int32_t j : touched) {
      cc.push_back(j);
      cv.push_back(acc[j]);
    }
    cp[i + 1] = (int64_t)cc.size();
  }
}

// C = (A + A^T) / 2 for a CSR matrix with a symmetric pattern and sorted
// columns; the result is bitwise symmetric (each pair is one sum).
void symmetrize_csr(int64_t n, const std::vector<int64_t>& p, const std::vector<int32_t>& c, std::vector<double>& v) {
  std::vector<double> out(v.size());
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = p[i]; e < p[i + 1]; ++e) {
      const int32_t j = c[e];
      const auto b = c.begin() + p[j], en = c.begin() + p[j + 1];
      const auto t = std::lower_bound(b, en, (int32_t)i);
      const double vji = (t != en && *t == i) ? v[t - c.begin()] : 0.0;
      out[e] = 0.5 * (v[e] + vji);
    }
  }
  v.swap(out);
}

// Order-n operator K_n = K (M^-1 K)^(n-1), n = 1..4 (Sect. 2.1.1; n = 2 is
// the biharmonic form of Eq. 5, n = 4 the highest order of Fig. 8). Even
// orders are squares, K_4 = K_2 M^-1 K_2: a product X M^-1 X of a bitwise
// symmetric X is bitwise symmetric (entry (i,j) and (j,i) sum the same
// products in the same order), and n = 3 is symmetrised explicitly.
void order_n_csr(int64_t n, int32_t order, const std::vector<int64_t>& kp, const std::vector<int32_t>& kc,
                 const std::vector<double>& kv, const std::vector<double>& m, std::vector<int64_t>& np,
                 std::vector<int32_t>& nc, std::vector<double>& nv) {
  np = kp;
  nc = kc;
  nv = kv;
  if (order == 1) return;
  std::vector<int64_t> p2;
  std::vector<int32_t> c2;
  std::vector<double> v2;
  spgemm_scaled(n, kp, kc, kv, kp, kc, kv, m, p2, c2, v2);
  if (order == 2) {
    np.swap(p2);
    nc.swap(c2);
    nv.swap(v2);
  } else if (order == 3) {
    spgemm_scaled(n, p2, c2, v2, kp, kc, kv, m, np, nc, nv);
    symmetrize_csr(n, np, nc, nv);
  } else {
    spgemm_scaled(n, p2, c2, v2, p2, c2, v2, m, np, nc, nv);
  }
}

// Reverse Cuthill-McKee ordering of a graph given by CSR adjacency (self
// loops ignored). Each connected component starts from a pseudo-peripheral
// node; neighbours are visited by increasing degree. Returns order[new] = old.
std::vector<int64_t> rcm(int64_t n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj) {
  std::vector<int32_t> deg(n);
  for (int64_t i = 0; i < n; ++i) {
    int32_t d = 0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) d += (adj[e] != i);
    deg[i] = d;
  }
  std::vector<int64_t> order;
  order.reserve(n);
  std::vector<char> seen(n, 0);
  std::vector<int64_t> level(n, -1);
  std::vector<int64_t> queue;
  std::vector<int64_t> nb;
  auto bfs_last = [&](int64_t s, int64_t* depth) {
    // returns a minimum-degree node of the last BFS level from s
    queue.clear();
    queue.push_back(s);
    level[s] = 0;
    std::vector<int64_t> touched{s};
    size_t h = 0;
    int64_t maxl = 0;
    while (h < queue.size()) {
      int64_t u = queue[h++];
      for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
        int64_t w = adj[e];
        if (w == u || level[w] >= 0) continue;
        level[w] = level[u] + 1;
        maxl = std::max(maxl, level[w]);
        queue.push_back(w);
        touched.push_back(w);
      }
    }
    int64_t best = s;
    for (int64_t u : touched)
      if (level[u] == maxl && (best == s || deg[u] < deg[best])) best = u;
    for (int64_t u : touched) level[u] = -1;
    *depth = maxl;
    return best;
  };
  for (int64_t s0 = 0; s0 < n; ++s0) {
    if (seen[s0]) continue;
    int64_t start = s0, depth = 0, d2 = 0;
    int64_t cand = bfs_last(start, &depth);
    for (int it = 0; it < 4; ++it) {
      int64_t c2 = bfs_last(cand, &d2);
      if (d2 <= depth) break;
      start = cand;
      depth = d2;
      cand = c2;
    }
    // Cuthill-McKee BFS from start
    size_t head = order.size();
    order.push_back(start);
    seen[start] = 1;
    while (head < order.size()) {
      int64_t u = order[head++];
      nb.clear();
      for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
        int64_t w = adj[e];
        if (w != u && !seen[w]) {
          seen[w] = 1;
          nb.push_back(w);
        }
      }
      std::stable_sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) { return deg[a] < deg[b]; });
      for (int64_t w : nb) order.push_back(w);
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Morton (Z-order) key of a point quantised to 21 bits per axis.
uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Locality ordering for the GPU kernels. Small graphs: reverse Cuthill-McKee.
// Larger ones: the nodes are cut into kParts parts of equal size along the
// Morton curve of their positions (one part per XCD of the device: a
// kernel's blocks on one XCD walk one contiguous eighth of the rows), and
// each part is ordered by RCM on its induced subgraph. A part is compact,
// so its RCM levels are short and a row's neighbours are a few hundred rows
// away instead of a great circle's worth; the few edges between parts are
// far apart in the numbering.
constexpr int kParts = 8;
constexpr int64_t kPartMin = 32768;  // below this, plain RCM

std::vector<int64_t> locality_order(int64_t n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj,
                                    const std::vector<V3>& pts) {
  if (n < kPartMin) return rcm(n, ptr, adj);
  V3 lo = pts[0], hi = pts[0];
  for (const V3& q : pts) {
    lo = V3{std::min(lo.x, q.x), std::min(lo.y, q.y), std::min(lo.z, q.z)};
    hi = V3{std::max(hi.x, q.x), std::max(hi.y, q.y), std::max(hi.z, q.z)};
  }
  const double ext = std::max({hi.x - lo.x, hi.y - lo.y, hi.z - lo.z, 1e-300});
  const double qs = 2097151.0 / ext;
  std::vector<std::pair<uint64_t, int64_t>> key(n);
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t ix = (uint64_t)((pts[i].x - lo.x) * qs), iy = (uint64_t)((pts[i].y - lo.y) * qs),
                   iz = (uint64_t)((pts[i].z - lo.z) * qs);
    key[i] = {spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2), i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int64_t> order;
  order.reserve(n);
  std::vector<int64_t> loc(n, -1);
  for (int p = 0; p < kParts; ++p) {
    const int64_t b = n * p / kParts, e = n * (p + 1) / kParts;
    const int64_t m = e - b;
    for (int64_t i = 0; i < m; ++i) loc[key[b + i].second] = i;
    std::vector<int64_t> sp(m + 1, 0);
    std::vector<int32_t> sa;
    for (int64_t i = 0; i < m; ++i) {
      const int64_t u = key[b + i].second;
      for (int64_t k = ptr[u]; k < ptr[u + 1]; ++k)
        if (loc[adj[k]] >= 0) sa.push_back((int32_t)loc[adj[k]]);
      sp[i + 1] = (int64_t)sa.size();
    }
    const std::vector<int64_t> r = rcm(m, sp, sa);
    for (int64_t i = 0; i < m; ++i) order.push_back(key[b + r[i]].second);
    for (int64_t i = 0; i < m; ++i) loc[key[b + i].second] = -1;
  }
  return order;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

ifl_status validate(const ifl_mesh& m) {
  if (m.n_vertices < 3 || m.n_triangles < 1) return fail(IFL_EINVAL, "mesh needs >= 3 vertices and >= 1 triangle");
  if (m.n_vertices > INT32_MAX || m.n_triangles > INT32_MAX / 2)
    return fail(IFL_EINVAL, "mesh too large for 32-bit indices");
  if (!m.coords || !m.triangles) return fail(IFL_EINVAL, "mesh coords / triangles are NULL");
  if (m.geometry < IFL_GEOM_PLANAR || m.geometry > IFL_GEOM_SPHERE) return fail(IFL_EINVAL, "unknown geometry");
  const int dim = m.geometry == IFL_GEOM_SPHERE ? 3 : 2;
  for (int64_t i = 0; i < m.n_vertices * dim; ++i)
    if (!std::isfinite(m.coords[i])) return fail(IFL_EINVAL, "non-finite vertex coordinate");
  if (m.geometry == IFL_GEOM_PERIODIC &&
      !(m.period[0] > 0 && m.period[1] > 0 && std::isfinite(m.period[0]) && std::isfinite(m.period[1])))
    return fail(IFL_EINVAL, "periodic mesh needs positive finite periods");
  for (int64_t i = 0; i < 3 * m.n_triangles; ++i)
    if (m.triangles[i] < 0 || m.triangles[i] >= m.n_vertices) return fail(IFL_EINVAL, "triangle vertex id out of range");
  return IFL_OK;
}

std::vector<char> active_triangles(const ifl_mesh& m) {
  std::vector<char> act(m.n_triangles, 1);
  if (m.wet) {
    for (int64_t t = 0; t < m.n_triangles; ++t) {
      const int32_t* v = m.triangles + 3 * t;
      act[t] = (m.wet[v[0]] != 0) && (m.wet[v[1]] != 0) && (m.wet[v[2]] != 0);
    }
  }
  return act;
}

// Renumber rows/cols of a CSR by order[new] = old; columns re-sorted.
void permute_csr(int64_t n, const std::vector<int64_t>& order, const std::vector<int64_t>& p,
                 const std::vector<int32_t>& c, const std::vector<double>& v, std::vector<int64_t>& np,
                 std::vector<int32_t>& nc, std::vector<double>& nv) {
  std::vector<int64_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[order[i]] = i;
  np.assign(n + 1, 0);
  nc.resize(c.size());
  nv.resize(v.size());
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t r = 0; r < n; ++r) {
    const int64_t o = order[r];
    row.clear();
    for (int64_t e = p[o]; e < p[o + 1]; ++e) row.push_back({(int32_t)inv[c[e]], v[e]});
    std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    int64_t base = np[r];
    for (size_t k = 0; k < row.size(); ++k) {
      nc[base + k] = row[k].first;
      nv[base + k] = row[k].second;
    }
    np[r + 1] = base + (int64_t)row.size();
  }
}

// Scalars on vertices. Median-dual control volumes and P1 elements (Sect.
// 2.1.1), or (voronoi) the quasi-hexagonal control volumes of Eq. 3-5: the
// flux weight of Eq. 3, l/d (circumcentre distance across the edge over the
// edge length), is the cotangent weight of the P1 stiffness, triangle by
// triangle (a triangle's circumcentre lies (d/2) cot(theta) from the edge
// midpoint, theta the angle opposite the edge), so the two share K and
// differ in the mass: the circumcentric (Voronoi) cell area. A corner i of a
// triangle (i, j, k) contributes (|ij|^2 cot(theta_k) + |ik|^2 cot(theta_j)) / 8.
ifl_status build_vertex_scalar(const ifl_mesh& m, int32_t order, int32_t reorder, bool voronoi, HostOperator* out) {
  const std::vector<char> act = active_triangles(m);
  std::vector<int64_t> dof_of(m.n_vertices, -1);
  for (int64_t t = 0; t < m.n_triangles; ++t)
    if (act[t])
      for (int k = 0; k < 3; ++k) dof_of[m.triangles[3 * t + k]] = 0;
  std::vector<int64_t> vert_of;
  for (int64_t v = 0; v < m.n_vertices; ++v)
    if (dof_of[v] == 0) {
      dof_of[v] = (int64_t)vert_of.size();
      vert_of.push_back(v);
    }
  const int64_t n = (int64_t)vert_of.size();
  if (n == 0) return fail(IFL_EDEGENERATE, "no active triangle (all triangles touch a dry vertex)");

  Triplets tr;
  tr.r.reserve(9 * (size_t)m.n_triangles);
  tr.c.reserve(9 * (size_t)m.n_triangles);
  tr.v.reserve(9 * (size_t)m.n_triangles);
  std::vector<double> mass(n, 0.0);
  for (int64_t t = 0; t < m.n_triangles; ++t) {
    if (!act[t]) continue;
    const int32_t* tv = m.triangles + 3 * t;
    V3 p[3];
    corners(m, tv, p);
    // e[i] is the edge opposite corner i; grad N_i = (normal x e_i) / (2 area),
    // so A_T grad N_i . grad N_j = e_i . e_j / (4 A_T).
    const V3 e[3] = {sub(p[2], p[1]), sub(p[0], p[2]), sub(p[1], p[0])};
    const double twoA = norm(cross(e[2], scale(e[1], -1.0)));
    const double ee = dot(e[0], e[0]) + dot(e[1], e[1]) + dot(e[2], e[2]);
    if (!(twoA > 1e-14 * ee)) return fail(IFL_EDEGENERATE, "zero-area active triangle " + std::to_string(t));
    const double inv = 1.0 / (2.0 * twoA);
    int64_t d[3] = {dof_of[tv[0]], dof_of[tv[1]], dof_of[tv[2]]};
    for (int i = 0; i < 3; ++i) {
      tr.add(d[i], d[i], dot(e[i], e[i]) * inv);
      for (int j = i + 1; j < 3; ++j) {
        const double kij = dot(e[i], e[j]) * inv;
        tr.add(d[i], d[j], kij);
        tr.add(d[j], d[i], kij);
      }
      if (voronoi) {
        // corners j, k of i; cot of the angle at corner c is -e_a.e_b / 2A
        // with a, b the other two corners
        const int j = (i + 1) % 3, k = (i + 2) % 3;
        const double cot_k = -dot(e[i], e[j]) / twoA, cot_j = -dot(e[i], e[k]) / twoA;
        mass[d[i]] += (dot(e[k], e[k]) * cot_k + dot(e[j], e[j]) * cot_j) / 8.0;
      } else {
        mass[d[i]] += twoA / 6.0;
      }
    }
  }
  if (voronoi)
    for (int64_t v = 0; v < n; ++v)
      if (!(mass[v] > 0.0))
        return fail(IFL_EDEGENERATE, "non-positive Voronoi cell area at vertex " + std::to_string(vert_of[v]) +
                                         " (the triangulation is not well centred there)");
  std::vector<int64_t> kp;
  std::vector<int32_t> kc;
  std::vector<double> kv;
  to_csr(n, tr, kp, kc, kv);
  tr = Triplets();

  std::vector<int64_t> np;
  std::vector<int32_t> nc;
  std::vector<double> nv;
  order_n_csr(n, order, kp, kc, kv, mass, np, nc, nv);
  std::vector<int64_t> ord(n);
  if (reorder) {
    const int dim = m.geometry == IFL_GEOM_SPHERE ? 3 : 2;
    std::vector<V3> pts(n);
    for (int64_t i = 0; i < n; ++i) {
      const double* c = m.coords + dim * vert_of[i];
      pts[i] = V3{c[0], c[1], dim == 3 ? c[2] : 0.0};
    }
    ord = locality_order(n, kp, kc, pts);
  } else {
    std::iota(ord.begin(), ord.end(), 0);
  }

  out->placement = voronoi ? IFL_VORONOI_SCALAR : IFL_VERTEX_SCALAR;
  out->order = order;
  out->n = n;
  out->n_components = 1;
  out->field_len = m.n_vertices;
  permute_csr(n, ord, np, nc, nv, out->row_ptr, out->col, out->val);
  if (order >= 2) permute_csr(n, ord, kp, kc, kv, out->k1_row_ptr, out->k1_col, out->k1_val);
  out->mass.resize(n);
  out->entity.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    out->mass[i] = mass[ord[i]];
    out->entity[i] = vert_of[ord[i]];
  }
  return IFL_OK;
}

// Velocities on vertices (Sect. 2.1.2): the FE vector Laplacian
// D_2 = [[D~, T], [-T, D~]] in (east, north) components, unknowns of dof d
// at rows 2d (east) and 2d+1 (north). Over each active triangle, with P1
// basis N, flat-facet gradients and m = tan(latitude of the centroid) / R_e
// (R_e the mean corner radius; planar meshes: m = 0, 1/R_e^2 = 0):
//   D~_ij += A grad N_i . grad N_j + (1/R_e^2 + m^2) A (1 + [i = j]) / 12,
//   T_ij  += m A / 3 (d_x N_j - d_x N_i),
// d_x the derivative along the zonal unit vector at the centroid (constant
// on the triangle). T is antisymmetric entry by entry, so D_2 is bitwise
// symmetric. Mass: the median-dual area per component. The right-hand side
// R_vc u_c (R_vc = A_c / 3 for each corner of an active cell) is kept as a
// projection onto the rows divided by the mass, so that M times the
// projected field is R_vc u_c.
ifl_status build_vertex_vector(const ifl_mesh& m, int32_t order, int32_t reorder, HostOperator* out) {
  const std::vector<char> act = active_triangles(m);
  std::vector<int64_t> dof_of(m.n_vertices, -1);
  for (int64_t t = 0; t < m.n_triangles; ++t)
    if (act[t])
      for (int k = 0; k < 3; ++k) dof_of[m.triangles[3 * t + k]] = 0;
  std::vector<int64_t> vert_of;
  for (int64_t v = 0; v < m.n_vertices; ++v)
    if (dof_of[v] == 0) {
      dof_of[v] = (int64_t)vert_of.size();
      vert_of.push_back(v);
    }
  const int64_t nd = (int64_t)vert_of.size();
  if (nd == 0) return fail(IFL_EDEGENERATE, "no active triangle (all triangles touch a dry vertex)");
  const int64_t n = 2 * nd;
  const bool sphere = m.geometry == IFL_GEOM_SPHERE;

  Triplets tr, pat;
  std::vector<double> mass(nd, 0.0);
  std::vector<double> tri_w(m.n_triangles, 0.0);
  for (int64_t t = 0; t < m.n_triangles; ++t) {
    if (!act[t]) continue;
    const int32_t* tv = m.triangles + 3 * t;
    V3 p[3];
    corners(m, tv, p);
    const V3 e[3] = {sub(p[2], p[1]), sub(p[0], p[2]), sub(p[1], p[0])};
    const V3 nrm_raw = cross(e[2], scale(e[1], -1.0));
    const double twoA = norm(nrm_raw);
    const double ee = dot(e[0], e[0]) + dot(e[1], e[1]) + dot(e[2], e[2]);
    if (!(twoA > 1e-14 * ee)) return fail(IFL_EDEGENERATE, "zero-area active triangle " + std::to_string(t));
    const double area = 0.5 * twoA;
    const V3 nrm = scale(nrm_raw, 1.0 / twoA);
    double mf = 0.0, inv_r2 = 0.0;
    V3 east{1.0, 0.0, 0.0};
    if (sphere) {
      V3 cd = add(add(p[0], p[1]), p[2]);
      cd = scale(cd, 1.0 / norm(cd));
      const double re = (norm(p[0]) + norm(p[1]) + norm(p[2])) / 3.0;
      const double coslat = std::hypot(cd.x, cd.y);
      if (!(coslat > 1e-12))
        return fail(IFL_EDEGENERATE, "active triangle " + std::to_string(t) +
                                         " has its centroid on the polar axis (the metric factor is infinite)");
      mf = cd.z / (coslat * re);
      inv_r2 = 1.0 / (re * re);
      east = V3{-cd.y / coslat, cd.x / coslat, 0.0};
    }
    double dx[3];
    for (int i = 0; i < 3; ++i) dx[i] = dot(cross(nrm, e[i]), east) / twoA;
    const double inv = 1.0 / (2.0 * twoA);
    const double w0 = (inv_r2 + mf * mf) * area / 12.0;
    const double mt = mf * area / 3.0;
    const int64_t d[3] = {dof_of[tv[0]], dof_of[tv[1]], dof_of[tv[2]]};
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) {
        const double dij = dot(e[i], e[j]) * inv + w0 * (i == j ? 2.0 : 1.0);
        tr.add(2 * d[i], 2 * d[j], dij);
        tr.add(2 * d[i] + 1, 2 * d[j] + 1, dij);
        if (i != j) {  // T_vv = 0: no east-north entry of a dof with itself
          const double tij = mt * (dx[j] - dx[i]);
          tr.add(2 * d[i], 2 * d[j] + 1, tij);
          tr.add(2 * d[i] + 1, 2 * d[j], -tij);
        }
        pat.add(d[i], d[j], 1.0);
      }
      mass[d[i]] += twoA / 6.0;
    }
    tri_w[t] = area / 3.0;
  }
  std::vector<double> mass2(n);
  for (int64_t i = 0; i < nd; ++i) mass2[2 * i] = mass2[2 * i + 1] = mass[i];
  std::vector<int64_t> kp;
  std::vector<int32_t> kc;
  std::vector<double> kv;
  to_csr(n, tr, kp, kc, kv);
  tr = Triplets();
  std::vector<int64_t> np;
  std::vector<int32_t> ncol;
  std::vector<double> nv;
  order_n_csr(n, order, kp, kc, kv, mass2, np, ncol, nv);

  // locality ordering of the vertices; both components of a dof stay adjacent
  std::vector<int64_t> vord(nd);
  if (reorder) {
    std::vector<int64_t> gp;
    std::vector<int32_t> gc;
    std::vector<double> gv;
    to_csr(nd, pat, gp, gc, gv);
    const int dim = sphere ? 3 : 2;
    std::vector<V3> pts(nd);
    for (int64_t i = 0; i < nd; ++i) {
      const double* c = m.coords + dim * vert_of[i];
      pts[i] = V3{c[0], c[1], dim == 3 ? c[2] : 0.0};
    }
    vord = locality_order(nd, gp, gc, pts);
  } else {
    std::iota(vord.begin(), vord.end(), 0);
  }
  pat = Triplets();
  std::vector<int64_t> ord(n);
  for (int64_t i = 0; i < nd; ++i) {
    ord[2 * i] = 2 * vord[i];
    ord[2 * i + 1] = 2 * vord[i] + 1;
  }
  out->placement = IFL_VERTEX_VECTOR;
  out->order = order;
  out->n = n;
  out->n_components = 2;
  out->field_len = 2 * m.n_vertices;
  permute_csr(n, ord, np, ncol, nv, out->row_ptr, out->col, out->val);
  if (order >= 2) permute_csr(n, ord, kp, kc, kv, out->k1_row_ptr, out->k1_col, out->k1_val);
  out->mass.resize(n);
  out->entity.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    out->mass[i] = mass2[ord[i]];
    out->entity[i] = 2 * vert_of[ord[i] / 2] + ord[i] % 2;
  }
  // projection, dofs in row order
  std::vector<int64_t> cnt(nd + 1, 0);
  for (int64_t t = 0; t < m.n_triangles; ++t)
    if (act[t])
      for (int k = 0; k < 3; ++k) cnt[dof_of[m.triangles[3 * t + k]] + 1]++;
  for (int64_t i = 0; i < nd; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> inc(cnt[nd]);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < m.n_triangles; ++t)
      if (act[t])
        for (int k = 0; k < 3; ++k) inc[fill[dof_of[m.triangles[3 * t + k]]]++] = (int32_t)t;
  }
  out->n_cells = m.n_triangles;
  out->proj_ptr.assign(nd + 1, 0);
  out->proj_tri.clear();
  out->proj_w.clear();
  for (int64_t i = 0; i < nd; ++i) {
    const int64_t d = vord[i];
    for (int64_t e = cnt[d]; e < cnt[d + 1]; ++e) {
      out->proj_tri.push_back(inc[e]);
      out->proj_w.push_back(tri_w[inc[e]] / mass[d]);
    }
    out->proj_ptr[i + 1] = (int64_t)out->proj_tri.size();
  }
  return IFL_OK;
}

// Scalars at triangle circumcentres (Eq. 6): dofs are the active triangles,
// mass their (flat-facet) areas, and a pair of active triangles sharing an
// edge of length l is coupled with weight l / d, d the distance between
// their circumcentres measured through the edge midpoint: each circumcentre
// lies (l/2) cot(theta) from it, theta the triangle's angle opposite the
// edge, so l / d = 2 / (cot(theta_1) + cot(theta_2)). The triangulation must
// be well centred (d > 0); two right triangles sharing their hypotenuse, for
// instance, have coincident circumcentres.
ifl_status build_circumcenter_scalar(const ifl_mesh& m, int32_t order, int32_t reorder, HostOperator* out) {
  const std::vector<char> act = active_triangles(m);
  std::vector<int64_t> tri_of;
  for (int64_t t = 0; t < m.n_triangles; ++t)
    if (act[t]) tri_of.push_back(t);
  const int64_t n = (int64_t)tri_of.size();
  if (n == 0) return fail(IFL_EDEGENERATE, "no active triangle (all triangles touch a dry vertex)");
  std::vector<double> area(n);
  // cot of the angle at each corner (the angle opposite edge (k+1, k+2))
  std::vector<double> cot(3 * n);
  for (int64_t c = 0; c < n; ++c) {
    V3 p[3];
    corners(m, m.triangles + 3 * tri_of[c], p);
    const V3 e[3] = {sub(p[2], p[1]), sub(p[0], p[2]), sub(p[1], p[0])};
    const double twoA = norm(cross(e[2], scale(e[1], -1.0)));
    const double ee = dot(e[0], e[0]) + dot(e[1], e[1]) + dot(e[2], e[2]);
    if (!(twoA > 1e-14 * ee)) return fail(IFL_EDEGENERATE, "zero-area active triangle " + std::to_string(tri_of[c]));
    area[c] = 0.5 * twoA;
    for (int k = 0; k < 3; ++k) cot[3 * c + k] = -dot(e[(k + 1) % 3], e[(k + 2) % 3]) / twoA;
  }
  struct EC {
    int64_t key;
    int64_t cell;
    int corner;  // the corner opposite the edge
  };
  std::vector<EC> ec;
  ec.reserve(3 * n);
  for (int64_t c = 0; c < n; ++c) {
    const int32_t* tv = m.triangles + 3 * tri_of[c];
    for (int k = 0; k < 3; ++k) {
      const int64_t a = tv[(k + 1) % 3], b = tv[(k + 2) % 3];
      ec.push_back({std::min(a, b) * m.n_vertices + std::max(a, b), c, k});
    }
  }
  std::stable_sort(ec.begin(), ec.end(), [](const EC& x, const EC& y) { return x.key < y.key; });
  Triplets tr;
  std::vector<double> diag(n, 0.0);
  std::vector<int64_t> gp(n + 1, 0);
  std::vector<std::pair<int64_t, int64_t>> pairs;
  std::vector<double> wts;
  for (size_t i = 0; i < ec.size();) {
    size_t j = i;
    while (j < ec.size() && ec[j].key == ec[i].key) ++j;
    if (j - i > 2) return fail(IFL_EINVAL, "edge shared by more than two active triangles");
    if (j - i == 2) {
      const int64_t c1 = ec[i].cell, c2 = ec[i + 1].cell;
      const double cs = cot[3 * c1 + ec[i].corner] + cot[3 * c2 + ec[i + 1].corner];
      if (!(cs > 1e-12))
        return fail(IFL_EDEGENERATE, "circumcentres of triangles " + std::to_string(tri_of[c1]) + " and " +
                                         std::to_string(tri_of[c2]) + " coincide or cross (not well centred)");
      pairs.push_back({c1, c2});
      wts.push_back(2.0 / cs);
    }
    i = j;
  }
  for (size_t q = 0; q < pairs.size(); ++q) {
    const int64_t c1 = pairs[q].first, c2 = pairs[q].second;
    tr.add(c1, c2, -wts[q]);
    tr.add(c2, c1, -wts[q]);
    diag[c1] += wts[q];
    diag[c2] += wts[q];
    gp[c1 + 1]++;
    gp[c2 + 1]++;
  }
  for (int64_t c = 0; c < n; ++c) tr.add(c, c, diag[c]);
  std::vector<int64_t> kp;
  std::vector<int32_t> kc;
  std::vector<double> kv;
  to_csr(n, tr, kp, kc, kv);
  tr = Triplets();
  std::vector<int64_t> np;
  std::vector<int32_t> ncol;
  std::vector<double> nv;
  order_n_csr(n, order, kp, kc, kv, area, np, ncol, nv);
  std::vector<int64_t> ord(n);
  if (reorder) {
    for (int64_t c = 0; c < n; ++c) gp[c + 1] += gp[c];
    std::vector<int32_t> adj(gp[n]);
    std::vector<int64_t> fill(gp.begin(), gp.end() - 1);
    for (const auto& pr : pairs) {
      adj[fill[pr.first]++] = (int32_t)pr.second;
      adj[fill[pr.second]++] = (int32_t)pr.first;
    }
    std::vector<V3> pts(n);
    for (int64_t c = 0; c < n; ++c) {
      V3 p[3];
      corners(m, m.triangles + 3 * tri_of[c], p);
      pts[c] = scale(add(add(p[0], p[1]), p[2]), 1.0 / 3.0);
    }
    ord = locality_order(n, gp, adj, pts);
  } else {
    std::iota(ord.begin(), ord.end(), 0);
  }
  out->placement = IFL_CIRCUMCENTER_SCALAR;
  out->order = order;
  out->n = n;
  out->n_components = 1;
  out->field_len = m.n_triangles;
  permute_csr(n, ord, np, ncol, nv, out->row_ptr, out->col, out->val);
  if (order >= 2) permute_csr(n, ord, kp, kc, kv, out->k1_row_ptr, out->k1_col, out->k1_val);
  out->mass.resize(n);
  out->entity.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    out->mass[i] = area[ord[i]];
    out->entity[i] = tri_of[ord[i]];
  }
  return IFL_OK;
}

ifl_status build_cell_vector(const ifl_mesh& m, int32_t order, double A, int32_t reorder, HostOperator* out) {
  const std::vector<char> act = active_triangles(m);
  std::vector<int64_t> cell_of(m.n_triangles, -1), tri_of;
  for (int64_t t = 0; t < m.n_triangles; ++t)
    if (act[t]) {
      cell_of[t] = (int64_t)tri_of.size();
      tri_of.push_back(t);
    }
  const int64_t nc = (int64_t)tri_of.size();
  if (nc == 0) return fail(IFL_EDEGENERATE, "no active triangle (all triangles touch a dry vertex)");
  std::vector<double> area(nc);
  std::vector<V3> eE(nc), eN(nc);
  for (int64_t c = 0; c < nc; ++c) {
    const int32_t* tv = m.triangles + 3 * tri_of[c];
    V3 p[3];
    corners(m, tv, p);
    const V3 a = sub(p[1], p[0]), b = sub(p[2], p[0]);
    const double twoA = norm(cross(a, b));
    const double ee = dot(a, a) + dot(b, b) + dot(sub(p[2], p[1]), sub(p[2], p[1]));
    if (!(twoA > 1e-14 * ee)) return fail(IFL_EDEGENERATE, "zero-area active triangle " + std::to_string(tri_of[c]));
    area[c] = 0.5 * twoA;
    if (m.geometry == IFL_GEOM_SPHERE) {
      V3 cd = add(add(p[0], p[1]), p[2]);
      cd = scale(cd, 1.0 / norm(cd));
      V3 e = cross(V3{0.0, 0.0, 1.0}, cd);
      const double ne = norm(e);
      e = ne > 1e-300 ? scale(e, 1.0 / ne) : V3{1.0, 0.0, 0.0};
      eE[c] = e;
      eN[c] = cross(cd, e);
    } else {
      eE[c] = {1.0, 0.0, 0.0};
      eN[c] = {0.0, 1.0, 0.0};
    }
  }
  // edges of active cells, grouped by vertex pair
  struct EC {
    int64_t key;
    int64_t cell;
  };
  std::vector<EC> ec;
  ec.reserve(3 * nc);
  for (int64_t c = 0; c < nc; ++c) {
    const int32_t* tv = m.triangles + 3 * tri_of[c];
    for (int k = 0; k < 3; ++k) {
      int64_t a = tv[k], b = tv[(k + 1) % 3];
      ec.push_back({std::min(a, b) * m.n_vertices + std::max(a, b), c});
    }
  }
  std::stable_sort(ec.begin(), ec.end(), [](const EC& x, const EC& y) { return x.key < y.key; });
  Triplets tr;
  std::vector<double> deg(nc, 0.0);
  std::vector<int64_t> gp(nc + 1, 0);  // cell graph for the ordering
  std::vector<std::pair<int64_t, int64_t>> pairs;
  for (size_t i = 0; i < ec.size();) {
    size_t j = i;
    while (j < ec.size() && ec[j].key == ec[i].key) ++j;
    if (j - i > 2) return fail(IFL_EINVAL, "edge shared by more than two active triangles");
    if (j - i == 2) pairs.push_back({ec[i].cell, ec[i + 1].cell});
    i = j;
  }
  for (const auto& pr : pairs) {
    const int64_t c1 = pr.first, c2 = pr.second;
    // P maps components at c2 into the (east, north) frame at c1
    const V3 f1[2] = {eE[c1], eN[c1]}, f2[2] = {eE[c2], eN[c2]};
    for (int r = 0; r < 2; ++r)
      for (int s = 0; s < 2; ++s) {
        const double w = -A * dot(f1[r], f2[s]);
        tr.add(2 * c1 + r, 2 * c2 + s, w);
        tr.add(2 * c2 + s, 2 * c1 + r, w);
      }
    deg[c1] += 1.0;
    deg[c2] += 1.0;
    gp[c1 + 1]++;
    gp[c2 + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c)
    for (int r = 0; r < 2; ++r) tr.add(2 * c + r, 2 * c + r, A * deg[c]);
  const int64_t n = 2 * nc;
  std::vector<double> mass(n);
  for (int64_t c = 0; c < nc; ++c) mass[2 * c] = mass[2 * c + 1] = area[c];
  std::vector<int64_t> kp;
  std::vector<int32_t> kc;
  std::vector<double> kv;
  to_csr(n, tr, kp, kc, kv);
  tr = Triplets();
  std::vector<int64_t> np;
  std::vector<int32_t> ncol;
  std::vector<double> nv;
  order_n_csr(n, order, kp, kc, kv, mass, np, ncol, nv);
  // locality ordering of cells; both components of a cell stay adjacent
  std::vector<int64_t> cord(nc);
  if (reorder) {
    for (int64_t c = 0; c < nc; ++c) gp[c + 1] += gp[c];
    std::vector<int32_t> adj(gp[nc]);
    std::vector<int64_t> fill(gp.begin(), gp.end() - 1);
    for (const auto& pr : pairs) {
      adj[fill[pr.first]++] = (int32_t)pr.second;
      adj[fill[pr.second]++] = (int32_t)pr.first;
    }
    std::vector<V3> pts(nc);
    for (int64_t c = 0; c < nc; ++c) {
      V3 p[3];
      corners(m, m.triangles + 3 * tri_of[c], p);
      pts[c] = scale(add(add(p[0], p[1]), p[2]), 1.0 / 3.0);
    }
    cord = locality_order(nc, gp, adj, pts);
  } else {
    std::iota(cord.begin(), cord.end(), 0);
  }
  std::vector<int64_t> ord(n);
  for (int64_t c = 0; c < nc; ++c) {
    ord[2 * c] = 2 * cord[c];
    ord[2 * c + 1] = 2 * cord[c] + 1;
  }
  out->placement = IFL_CELL_VECTOR;
  out->order = order;
  out->n = n;
  out->n_components = 2;
  out->field_len = 2 * m.n_triangles;
  permute_csr(n, ord, np, ncol, nv, out->row_ptr, out->col, out->val);
  if (order >= 2) permute_csr(n, ord, kp, kc, kv, out->k1_row_ptr, out->k1_col, out->k1_val);
  out->mass.resize(n);
  out->entity.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    out->mass[i] = mass[ord[i]];
    const int64_t c = ord[i] / 2, comp = ord[i] % 2;
    out->entity[i] = 2 * tri_of[c] + comp;
  }
  return IFL_OK;
}

}  // namespace

ifl_status build_operator(const ifl_mesh& mesh, int32_t placement, int32_t order, double cell_A,
                          int32_t reorder, HostOperator* out) {
  ifl_status st = validate(mesh);
  if (st != IFL_OK) return st;
  if (order < 1 || order > 4) return fail(IFL_EUNSUPPORTED, "filter order n must be 1 to 4");
  if (placement == IFL_VERTEX_SCALAR || placement == IFL_VORONOI_SCALAR) {
    st = build_vertex_scalar(mesh, order, reorder, placement == IFL_VORONOI_SCALAR, out);
  } else if (placement == IFL_CELL_VECTOR) {
    if (!(cell_A > 0) || !std::isfinite(cell_A)) return fail(IFL_EINVAL, "cell_A must be positive and finite");
    st = build_cell_vector(mesh, order, cell_A, reorder, out);
  } else if (placement == IFL_CIRCUMCENTER_SCALAR) {
    st = build_circumcenter_scalar(mesh, order, reorder, out);
  } else if (placement == IFL_VERTEX_VECTOR) {
    st = build_vertex_vector(mesh, order, reorder, out);
  } else {
    return fail(IFL_EINVAL, "unknown placement");
  }
  if (st != IFL_OK) return st;
  uint64_t h = 1469598103934665603ull;
  const int dim = mesh.geometry == IFL_GEOM_SPHERE ? 3 : 2;
  h = fnv1a(h, mesh.coords, sizeof(double) * dim * mesh.n_vertices);
  h = fnv1a(h, mesh.triangles, sizeof(int32_t) * 3 * mesh.n_triangles);
  if (mesh.wet) h = fnv1a(h, mesh.wet, (size_t)mesh.n_vertices);
  h = fnv1a(h, &placement, sizeof placement);
  h = fnv1a(h, &order, sizeof order);
  out->mesh_hash = h;
  return IFL_OK;
}

void pack_sell_csr(int64_t n, const std::vector<int64_t>& row_ptr, const std::vector<int32_t>& col,
                   const std::vector<double>& val, const std::vector<double>& mass, SellPack* out) {
  const int64_t ns = (n + 63) / 64;
  out->n = n;
  out->n_slices = ns;
  out->slice_ptr.assign(ns + 1, 0);
  out->diag.assign(ns * 64, 0.0);
  out->mass.assign(ns * 64, 0.0);
  out->max_width = 0;
  out->stored_offdiag = 0;
  std::vector<int32_t> width(ns, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int64_t r = s * 64; r < std::min(n, s * 64 + 64); ++r) {
      int32_t len = 0;
      for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) len += (col[e] != r);
      w = std::max(w, len);
      out->stored_offdiag += len;
    }
    width[s] = w;
    out->max_width = std::max(out->max_width, w);
    out->slice_ptr[s + 1] = out->slice_ptr[s] + 64 * (int64_t)w;
  }
  // kSellTail zero entries (column 0, value 0) follow the last slice, so that
  // kernels may load a fixed number of entries per row without bounds checks
  out->col.assign(out->slice_ptr[ns] + kSellTail, 0);
  out->val.assign(out->slice_ptr[ns] + kSellTail, 0.0);
  for (int64_t s = 0; s < ns; ++s) {
    for (int64_t l = 0; l < 64; ++l) {
      const int64_t r = s * 64 + l;
      const int32_t self = (int32_t)std::min(r, n - 1);
      int32_t k = 0;
      if (r < n) {
        out->mass[r] = mass[r];
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
          if (col[e] == r) {
            out->diag[r] = val[e];
          } else {
            out->col[out->slice_ptr[s] + 64 * k + l] = col[e];
            out->val[out->slice_ptr[s] + 64 * k + l] = val[e];
            ++k;
          }
        }
      }
      for (; k < width[s]; ++k) {
        out->col[out->slice_ptr[s] + 64 * k + l] = self;
        out->val[out->slice_ptr[s] + 64 * k + l] = 0.0;
      }
    }
  }
}

void pack_sell(const HostOperator& op, SellPack* out) { pack_sell_csr(op.n, op.row_ptr, op.col, op.val, op.mass, out); }

bool pack_pairs(const HostOperator& op, PairPack* out) {
  if (op.n_components != 2 || op.n % 2 != 0) return false;
  const int64_t nb = op.n / 2, ns = (nb + 63) / 64;
  // the blocks of block row b in increasing block column: the CSR rows 2b
  // and 2b + 1 (sorted columns) merged; emit(j, v) for every block with at
  // least one off-diagonal entry
  auto blocks = [&](int64_t b, auto&& emit) {
    int64_t e0 = op.row_ptr[2 * b], e0e = op.row_ptr[2 * b + 1];
    int64_t e1 = op.row_ptr[2 * b + 1], e1e = op.row_ptr[2 * b + 2];
    while (e0 < e0e || e1 < e1e) {
      const int64_t j0 = e0 < e0e ? op.col[e0] / 2 : INT64_MAX, j1 = e1 < e1e ? op.col[e1] / 2 : INT64_MAX;
      const int64_t j = std::min(j0, j1);
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      bool any = false;
      for (; e0 < e0e && op.col[e0] / 2 == j; ++e0)
        if (op.col[e0] != 2 * b) {
          v[op.col[e0] % 2] = op.val[e0];
          any = true;
        }
      for (; e1 < e1e && op.col[e1] / 2 == j; ++e1)
        if (op.col[e1] != 2 * b + 1) {
          v[2 + op.col[e1] % 2] = op.val[e1];
          any = true;
        }
      if (any) emit((int32_t)j, v);
    }
  };
  out->nb = nb;
  out->n_slices = ns;
  out->slice_ptr.assign(ns + 1, 0);
  out->stored_blocks = 0;
  std::vector<int32_t> width(ns, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int64_t b = s * 64; b < std::min(nb, s * 64 + 64); ++b) {
      int32_t len = 0;
      blocks(b, [&](int32_t, const double*) { ++len; });
      w = std::max(w, len);
      out->stored_blocks += len;
    }
    width[s] = w;
    out->slice_ptr[s + 1] = out->slice_ptr[s] + 64 * (int64_t)w;
  }
  out->col.assign(out->slice_ptr[ns] + kSellTail, 0);
  out->val.assign(4 * (out->slice_ptr[ns] + kSellTail), 0.0);
  for (int64_t s = 0; s < ns; ++s) {
    for (int64_t l = 0; l < 64; ++l) {
      const int64_t b = s * 64 + l;
      const int32_t self = (int32_t)std::min(b, nb - 1);
      int32_t k = 0;
      if (b < nb)
        blocks(b, [&](int32_t j, const double* v) {
          const int64_t e = out->slice_ptr[s] + 64 * (int64_t)k + l;
          out->col[e] = j;
          for (int q = 0; q < 4; ++q) out->val[4 * e + q] = v[q];
          ++k;
        });
      for (; k < width[s]; ++k) out->col[out->slice_ptr[s] + 64 * (int64_t)k + l] = self;
    }
  }
  return true;
}

}  // namespace ifl
