// mesh_build.cpp -- host problem setup: a reduced Gaussian grid, its
// triangulation, the edge and node->edge tables, and the median-dual
// geometry.
//
// Grid: Section 4.2.3.5 (Gaussian latitudes = roots of the Legendre
// polynomial of degree 2N; first point of every parallel at lon 0) and
// Section 4.2.3.7 (any number of points per parallel); O<N> is Listing 6
// (nx = 20 + 4j to the equator, mirrored), F<N> is Section 4.2.3.6
// (nx = 4N on every parallel).
// Mesh: Section 4.3 (the structured mesh generator triangulates between
// parallels; edges are mesh lines between nodes).  Geometry: the
// ingredients of the edge-based finite-volume method of Section 4.7
// (dual volumes and dual-face normals per edge), built as the median dual
// in the (lon, lat) plane with the polar cells closed up to the pole line.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace atlasx {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Root finding in extended precision: Newton on P_n with the three-term
// recurrence, from the Tricomi initial guess.  The roots come out sorted
// north to south (mu decreasing).
void gaussian_mu(int N, std::vector<double> &mu) {
  const int n = 2 * N;
  mu.assign(n, 0.0);
  for (int j = 0; j < N; ++j) {
    long double theta = (long double)kPi * (4.0L * j + 3.0L) / (4.0L * n + 2.0L);
    long double x = std::cos(theta) *
                    (1.0L - (n - 1.0L) / (8.0L * n * n * n));  // Tricomi
    for (int it = 0; it < 60; ++it) {
      long double pm = 1.0L, p = x;
      for (int k = 2; k <= n; ++k) {
        long double pk = ((2 * k - 1) * x * p - (k - 1) * pm) / k;
        pm = p;
        p = pk;
      }
      long double dp = n * (pm - x * p) / (1.0L - x * x);
      long double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    mu[j] = (double)x;
    mu[n - 1 - j] = -(double)x;
  }
}

}  // namespace

// Builds every array of an atlas_mesh_desc for O<N>.
int build_octahedral(int N, double R, HostMesh &h) {
  std::vector<int32_t> nx(2 * N);
  for (int j = 0; j < N; ++j) nx[j] = nx[2 * N - 1 - j] = 20 + 4 * j;
  return build_reduced_gaussian(nx, R, h);
}

// Builds every array of an atlas_mesh_desc for the reduced Gaussian grid
// with nx[j] points on parallel j (nx.size() = 2N parallels; every nx >= 4,
// the two polar parallels even).
int build_reduced_gaussian(const std::vector<int32_t> &nx_in, double R, HostMesh &h) {
  return build_grid(nx_in, nullptr, false, false, R, h);
}

// Any grid of parallels: nx[j] points on parallel j at latitude lat[j]
// (strictly decreasing inside (-pi/2, pi/2); NULL: the Gaussian latitudes of
// degree nx.size()).  shifted: every point half a spacing east of the
// unshifted position (equal counts on all parallels).  quads: a strip
// between parallels of equal counts becomes a row of quadrilaterals
// (U_a, L_a, L_a+1, U_a+1) -- the blocked quadrilaterals of Section 4.3 --
// and the other strips stay triangulated.
int build_grid(const std::vector<int32_t> &nx_in, const std::vector<double> *lat_in,
               bool shifted, bool quads, double R, HostMesh &h) {
  const int nr = (int)nx_in.size();
  const int N = nr / 2;
  h.N = N;
  h.radius = R;
  h.nx = nx_in;
  h.ring_off.resize(nr + 1);
  h.ring_off[0] = 0;
  for (int j = 0; j < nr; ++j) h.ring_off[j + 1] = h.ring_off[j] + h.nx[j];
  const int64_t V = h.ring_off[nr];

  std::vector<double> mu;
  if (!lat_in) gaussian_mu(N, mu);
  h.lon.resize(V);
  h.lat.resize(V);
  h.cos_lat.resize(V);
  for (int j = 0; j < nr; ++j) {
    const double th = lat_in ? (*lat_in)[j] : std::asin(mu[j]);
    const double c = std::cos(th);
    const int64_t o = h.ring_off[j];
    for (int i = 0; i < h.nx[j]; ++i) {
      h.lon[o + i] = shifted ? 2.0 * kPi * ((double)i + 0.5) / (double)h.nx[j]
                             : 2.0 * kPi * (double)i / (double)h.nx[j];
      h.lat[o + i] = th;
      h.cos_lat[o + i] = c;
    }
  }

  // --- triangles: walk each strip, consuming whichever of the two next
  // points lies further west (exact integer comparison of i/n); ties
  // advance the ring with more points, the lower ring if counts are equal.
  std::vector<int32_t> &tri = h.tri;
  std::vector<int32_t> &quad = h.quad;
  tri.clear();
  quad.clear();
  tri.reserve((size_t)3 * (2 * V));
  for (int j = 0; j + 1 < nr; ++j) {
    const int64_t nu = h.nx[j], nl = h.nx[j + 1];
    const int64_t ou = h.ring_off[j], ol = h.ring_off[j + 1];
    if (quads && nu == nl) {
      for (int64_t a = 0; a < nu; ++a) {
        const int32_t q4[4] = {(int32_t)(ou + a), (int32_t)(ol + a),
                               (int32_t)(ol + (a + 1) % nl), (int32_t)(ou + (a + 1) % nu)};
        quad.insert(quad.end(), q4, q4 + 4);
      }
      continue;
    }
    int64_t iu = 0, il = 0;
    for (int64_t step = 0; step < nu + nl; ++step) {
      bool take_upper;
      if (iu == nu) take_upper = false;
      else if (il == nl) take_upper = true;
      else {
        const int64_t lhs = (iu + 1) * nl, rhs = (il + 1) * nu;
        take_upper = lhs < rhs || (lhs == rhs && nu > nl);
      }
      const int32_t u0 = (int32_t)(ou + iu % nu), l0 = (int32_t)(ol + il % nl);
      tri.push_back(u0);
      tri.push_back(l0);
      if (take_upper) { tri.push_back((int32_t)(ou + (iu + 1) % nu)); ++iu; }
      else            { tri.push_back((int32_t)(ol + (il + 1) % nl)); ++il; }
    }
  }
  const int64_t F = (int64_t)tri.size() / 3;
  const int64_t Q = (int64_t)quad.size() / 4;

  // --- edges: per node, its higher-numbered neighbours, sorted; reading
  // the nodes in order enumerates the pairs (a < b) lexicographically.
  // (element sides: every triangle side, then every quadrilateral side)
  auto for_each_side = [&](auto &&fn) {
    for (int64_t t = 0; t < F; ++t)
      for (int k = 0; k < 3; ++k) fn(tri[3 * t + k], tri[3 * t + (k + 1) % 3]);
    for (int64_t t = 0; t < Q; ++t)
      for (int k = 0; k < 4; ++k) fn(quad[4 * t + k], quad[4 * t + (k + 1) % 4]);
  };
  std::vector<int64_t> up_ptr(V + 1, 0);
  for_each_side([&](int32_t p, int32_t q) { up_ptr[std::min(p, q) + 1]++; });
  for (int64_t i = 0; i < V; ++i) up_ptr[i + 1] += up_ptr[i];
  std::vector<int32_t> up(up_ptr[V]);
  {
    std::vector<int64_t> fill(up_ptr.begin(), up_ptr.end() - 1);
    for_each_side([&](int32_t p, int32_t q) { up[fill[std::min(p, q)]++] = std::max(p, q); });
  }
  h.edge2node.clear();
  h.edge2node.reserve((size_t)2 * 3 * V);
  std::vector<int64_t> first(V + 1, 0);  // first edge of each smaller node
  for (int64_t a = 0; a < V; ++a) {
    first[a] = (int64_t)h.edge2node.size() / 2;
    int32_t *b0 = up.data() + up_ptr[a], *b1 = up.data() + up_ptr[a + 1];
    std::sort(b0, b1);
    int32_t *bend = std::unique(b0, b1);
    for (int32_t *b = b0; b != bend; ++b) {
      h.edge2node.push_back((int32_t)a);
      h.edge2node.push_back(*b);
    }
  }
  const int64_t E = (int64_t)h.edge2node.size() / 2;
  first[V] = E;
  auto edge_id = [&](int32_t p, int32_t q) -> int64_t {
    const int32_t a = std::min(p, q), b = std::max(p, q);
    const int32_t *lo = h.edge2node.data() + 2 * first[a];
    int64_t n = first[a + 1] - first[a];
    for (int64_t k = 0; k < n; ++k)
      if (lo[2 * k + 1] == b) return first[a] + k;
    return -1;
  };

  // --- median-dual geometry ----------------------------------------------
  // Each triangle corner owns the quadrilateral (vertex, midpoint,
  // centroid, midpoint): one third of the triangle.  The face between the
  // corner's two quadrilaterals on edge (a, b) is the segment midpoint ->
  // centroid; its normal (dy, -dx) is turned to point from a to b.
  h.dual_normals.assign((size_t)2 * E, 0.0);
  std::vector<double> area(V, 0.0);
  for (int64_t t = 0; t < F; ++t) {
    const int32_t v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
    double x[3], y[3];
    for (int k = 0; k < 3; ++k) {
      x[k] = h.lon[v[k]];
      y[k] = h.lat[v[k]];
      if (k) {  // bring the corner within half a turn of the first one
        if (x[k] - x[0] > kPi) x[k] -= 2.0 * kPi;
        else if (x[k] - x[0] < -kPi) x[k] += 2.0 * kPi;
      }
    }
    const double gx = (x[0] + x[1] + x[2]) / 3.0, gy = (y[0] + y[1] + y[2]) / 3.0;
    const double twice = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
    for (int k = 0; k < 3; ++k) area[v[k]] += 0.5 * twice / 3.0;
    for (int k = 0; k < 3; ++k) {
      const int p = k, q = (k + 1) % 3;
      const int64_t e = edge_id(v[p], v[q]);
      const double sx = gy - 0.5 * (y[p] + y[q]);   // normal of (g - m)
      const double sy = -(gx - 0.5 * (x[p] + x[q]));
      const int from = v[p] < v[q] ? p : q, to = from == p ? q : p;
      const double dot = sx * (x[to] - x[from]) + sy * (y[to] - y[from]);
      const double sgn = dot < 0.0 ? -1.0 : 1.0;
      h.dual_normals[2 * e] += sgn * sx;
      h.dual_normals[2 * e + 1] += sgn * sy;
    }
  }
  // Quadrilaterals: the same construction about the element centre g (mean
  // of the four corners): corner k owns the polygon (corner, midpoint
  // towards k+1, g, midpoint towards k-1), its area by the shoelace
  // formula; the face on side (k, k+1) is the segment midpoint -> g.
  for (int64_t t = 0; t < Q; ++t) {
    const int32_t v[4] = {quad[4 * t], quad[4 * t + 1], quad[4 * t + 2], quad[4 * t + 3]};
    double x[4], y[4];
    for (int k = 0; k < 4; ++k) {
      x[k] = h.lon[v[k]];
      y[k] = h.lat[v[k]];
      if (k) {
        if (x[k] - x[0] > kPi) x[k] -= 2.0 * kPi;
        else if (x[k] - x[0] < -kPi) x[k] += 2.0 * kPi;
      }
    }
    const double gx = 0.25 * (x[0] + x[1] + x[2] + x[3]);
    const double gy = 0.25 * (y[0] + y[1] + y[2] + y[3]);
    for (int k = 0; k < 4; ++k) {
      const int q = (k + 1) % 4, r = (k + 3) % 4;
      const double ax = 0.5 * (x[k] + x[q]), ay = 0.5 * (y[k] + y[q]);  // towards k+1
      const double bx = 0.5 * (x[k] + x[r]), by = 0.5 * (y[k] + y[r]);  // towards k-1
      const double cxs[4] = {x[k], ax, gx, bx}, cys[4] = {y[k], ay, gy, by};
      double twice = 0.0;
      for (int c = 0; c < 4; ++c)
        twice += cxs[c] * cys[(c + 1) % 4] - cxs[(c + 1) % 4] * cys[c];
      area[v[k]] += 0.5 * twice;
      const int64_t e = edge_id(v[k], v[q]);
      const double sx = gy - ay, sy = -(gx - ax);
      const int from = v[k] < v[q] ? k : q, to = from == k ? q : k;
      const double dot = sx * (x[to] - x[from]) + sy * (y[to] - y[from]);
      const double sgn = dot < 0.0 ? -1.0 : 1.0;
      h.dual_normals[2 * e] += sgn * sx;
      h.dual_normals[2 * e + 1] += sgn * sy;
    }
  }
  // polar closure: cells of the first / last parallel reach the pole line;
  // each polar node's face there is one spacing of its parallel wide
  h.pole_edges.clear();
  h.pole_normals.clear();
  for (int side = 0; side < 2; ++side) {
    const int j = side ? nr - 1 : 0;
    const double sigma = side ? -1.0 : 1.0;
    const int64_t o = h.ring_off[j];
    const int n = h.nx[j];
    const double dlon0 = 2.0 * kPi / (double)n;
    const double height = 0.5 * kPi - std::fabs(h.lat[o]);
    for (int i = 0; i < n; ++i) {
      const int32_t p = (int32_t)(o + i), q = (int32_t)(o + (i + 1) % n);
      const int64_t e = edge_id(p, q);
      // vertical face at the midpoint between p and its eastern neighbour
      // q; its normal points east, i.e. from a to b iff a == p.
      const double sx = (h.edge2node[2 * e] == p) ? height : -height;
      h.dual_normals[2 * e] += sx;
      area[p] += dlon0 * height;
    }
    for (int i = 0; i < n / 2; ++i) {
      h.pole_edges.push_back((int32_t)(o + i));
      h.pole_edges.push_back((int32_t)(o + i + n / 2));
      h.pole_normals.push_back(sigma * dlon0);
    }
  }
  h.dual_volumes.resize(V);
  for (int64_t i = 0; i < V; ++i) h.dual_volumes[i] = R * R * h.cos_lat[i] * area[i];

  // --- CSR node -> edge, ascending edge id, signed ----------------------
  h.node2edge_ptr.assign(V + 1, 0);
  for (int64_t e = 0; e < E; ++e) {
    h.node2edge_ptr[h.edge2node[2 * e] + 1]++;
    h.node2edge_ptr[h.edge2node[2 * e + 1] + 1]++;
  }
  for (int64_t i = 0; i < V; ++i) h.node2edge_ptr[i + 1] += h.node2edge_ptr[i];
  h.node2edge.resize(2 * E);
  h.node2edge_sign.resize(2 * E);
  {
    std::vector<int64_t> fill(h.node2edge_ptr.begin(), h.node2edge_ptr.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      const int32_t a = h.edge2node[2 * e], b = h.edge2node[2 * e + 1];
      h.node2edge[fill[a]] = (int32_t)e;
      h.node2edge_sign[fill[a]++] = 1;
      h.node2edge[fill[b]] = (int32_t)e;
      h.node2edge_sign[fill[b]++] = -1;
    }
  }
  h.fill_desc();
  return 0;
}

void HostMesh::fill_desc() {
  std::memset(&desc, 0, sizeof(desc));
  desc.nnodes = (int64_t)lon.size();
  desc.lon = lon.data();
  desc.lat = lat.data();
  desc.cos_lat = cos_lat.data();
  desc.nrings = (int32_t)nx.size();
  desc.ring_off = ring_off.data();
  desc.nedges = (int64_t)edge2node.size() / 2;
  desc.edge2node = edge2node.data();
  desc.node2edge_ptr = node2edge_ptr.data();
  desc.node2edge = node2edge.data();
  desc.node2edge_sign = node2edge_sign.data();
  desc.dual_volumes = dual_volumes.data();
  desc.dual_normals = dual_normals.data();
  desc.npole_edges = (int64_t)pole_normals.size();
  desc.pole_edges = pole_edges.data();
  desc.pole_normals = pole_normals.data();
  desc.radius = radius;
  desc.ntriangles = (int64_t)tri.size() / 3;
  desc.triangles = tri.empty() ? nullptr : tri.data();
  desc.nquads = (int64_t)quad.size() / 4;
  desc.quads = quad.empty() ? nullptr : quad.data();
}

}  // namespace atlasx
