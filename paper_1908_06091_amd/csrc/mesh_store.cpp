// mesh_store.cpp -- device mesh store: validation of a host mesh
// description, the processing order (tiles), the signed node->edge table in
// that order, and the one-time copy to the device.
//
// Section 4.3 (Block/Irregular connectivity: the node->edge table is an
// irregular table, edge2node a block table) and Section 5 (mesh data is
// made available on the device once, then stays resident).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace atlasx {

MeshStore::~MeshStore() {
  for (void *p : allocations) (void)hipFree(p);
  if (ws) (void)hipFree(ws);
}

namespace {

atlas_status validate(const atlas_mesh_desc *d) {
  if (!d) return fail(ATLAS_EINVAL, "mesh description is NULL");
  const int64_t V = d->nnodes, E = d->nedges;
  if (V < 1 || V >= (int64_t)1 << 31)
    return fail(ATLAS_EINVAL, "nnodes must be in [1, 2^31)");
  if (E < 1 || 2 * E >= (int64_t)1 << 31)
    return fail(ATLAS_EINVAL, "nedges must be in [1, 2^30)");
  if (!d->lon || !d->lat || !d->cos_lat || !d->edge2node || !d->node2edge_ptr ||
      !d->node2edge || !d->node2edge_sign || !d->dual_volumes || !d->dual_normals)
    return fail(ATLAS_EINVAL, "a required mesh array is NULL");
  if (d->npole_edges < 0 || (d->npole_edges > 0 && (!d->pole_edges || !d->pole_normals)))
    return fail(ATLAS_EINVAL, "pole edge arrays missing");
  if (!(d->radius > 0.0) || !std::isfinite(d->radius))
    return fail(ATLAS_EINVAL, "radius must be positive and finite");
  for (int64_t e = 0; e < E; ++e) {
    const int32_t a = d->edge2node[2 * e], b = d->edge2node[2 * e + 1];
    if (a < 0 || b >= V || !(a < b))
      return fail(ATLAS_EINVAL, "edge2node[" + std::to_string(e) + "] must satisfy 0 <= a < b < nnodes");
    if (!std::isfinite(d->dual_normals[2 * e]) || !std::isfinite(d->dual_normals[2 * e + 1]))
      return fail(ATLAS_EINVAL, "non-finite dual normal at edge " + std::to_string(e));
  }
  if (d->node2edge_ptr[0] != 0 || d->node2edge_ptr[V] != 2 * E)
    return fail(ATLAS_EINVAL, "node2edge_ptr must run from 0 to 2*nedges");
  std::vector<uint8_t> seen(E, 0);
  for (int64_t i = 0; i < V; ++i) {
    const int64_t r0 = d->node2edge_ptr[i], r1 = d->node2edge_ptr[i + 1];
    if (r1 < r0) return fail(ATLAS_EINVAL, "node2edge_ptr is not monotone");
    for (int64_t r = r0; r < r1; ++r) {
      const int32_t e = d->node2edge[r];
      if (e < 0 || e >= E) return fail(ATLAS_EINVAL, "node2edge entry out of range");
      if (r > r0 && !(d->node2edge[r - 1] < e))
        return fail(ATLAS_EINVAL, "node2edge rows must list edges in ascending id");
      const int8_t s = d->node2edge_sign[r];
      const int32_t a = d->edge2node[2 * e], b = d->edge2node[2 * e + 1];
      if (!((s == 1 && a == i) || (s == -1 && b == i)))
        return fail(ATLAS_EINVAL, "node2edge_sign / endpoint mismatch at node " + std::to_string(i));
      seen[e] |= (s == 1) ? 1 : 2;
    }
    if (!(d->dual_volumes[i] > 0.0) || !std::isfinite(d->dual_volumes[i]))
      return fail(ATLAS_EINVAL, "dual volume must be positive at node " + std::to_string(i));
    if (!(d->cos_lat[i] > 0.0) || d->cos_lat[i] > 1.0 || !std::isfinite(d->lat[i]) ||
        !std::isfinite(d->lon[i]))
      return fail(ATLAS_EINVAL, "bad coordinates at node " + std::to_string(i));
  }
  for (int64_t e = 0; e < E; ++e)
    if (seen[e] != 3) return fail(ATLAS_EINVAL, "edge " + std::to_string(e) + " missing from node2edge");
  std::vector<uint8_t> polar(V, 0);
  for (int64_t k = 0; k < d->npole_edges; ++k) {
    const int32_t a = d->pole_edges[2 * k], b = d->pole_edges[2 * k + 1];
    if (a < 0 || b < 0 || a >= V || b >= V || a == b)
      return fail(ATLAS_EINVAL, "pole edge endpoints out of range");
    if (polar[a]++ || polar[b]++)
      return fail(ATLAS_EINVAL, "a node belongs to more than one pole edge");
    if (!std::isfinite(d->pole_normals[k])) return fail(ATLAS_EINVAL, "non-finite pole normal");
  }
  return ATLAS_OK;
}

// Parallels: explicit ring_off, or runs of equal latitude in node order.
std::vector<int64_t> rings_of(const atlas_mesh_desc *d) {
  std::vector<int64_t> off;
  if (d->nrings > 0 && d->ring_off) {
    off.assign(d->ring_off, d->ring_off + d->nrings + 1);
    bool ok = off.front() == 0 && off.back() == d->nnodes;
    for (size_t j = 0; ok && j + 1 < off.size(); ++j) ok = off[j] < off[j + 1];
    if (ok) return off;
    off.clear();
  }
  off.push_back(0);
  for (int64_t i = 1; i < d->nnodes; ++i)
    if (d->lat[i] != d->lat[i - 1]) off.push_back(i);
  off.push_back(d->nnodes);
  return off;
}

}  // namespace

bool zipper_conforming(const atlas_mesh_desc *d, const std::vector<int64_t> &off) {
  const int64_t nr = (int64_t)off.size() - 1;
  if (nr < 2) return false;
  const double twopi = 6.283185307179586476925;
  for (int64_t j = 0; j < nr; ++j) {
    const int64_t o = off[j], n = off[j + 1] - o;
    if (n < 3 || d->lon[o] != 0.0) return false;
    if (j > 0 && !(d->lat[o] < d->lat[off[j - 1]])) return false;
    for (int64_t i = 0; i < n; ++i) {
      if (d->lat[o + i] != d->lat[o]) return false;
      if (!(d->lon[o + i] < twopi) || (i > 0 && !(d->lon[o + i] > d->lon[o + i - 1])))
        return false;
    }
  }
  // is {p, q} an edge?  (scan the smaller node's CSR row)
  auto has_edge = [&](int64_t p, int64_t q) {
    const int64_t a = std::min(p, q), b = std::max(p, q);
    for (int64_t r = d->node2edge_ptr[a]; r < d->node2edge_ptr[a + 1]; ++r) {
      const int32_t e = d->node2edge[r];
      if (d->edge2node[2 * e] == a && d->edge2node[2 * e + 1] == b) return true;
    }
    return false;
  };
  int64_t count = 0;
  for (int64_t j = 0; j < nr; ++j) {  // edges along each parallel
    const int64_t o = off[j], n = off[j + 1] - o;
    for (int64_t i = 0; i < n; ++i)
      if (!has_edge(o + i, o + (i + 1) % n)) return false;
    count += n;
  }
  for (int64_t j = 0; j + 1 < nr; ++j) {  // edges across each strip, walked
    const int64_t ou = off[j], nu = off[j + 1] - ou;
    const int64_t ol = off[j + 1], nl = off[j + 2] - ol;
    int64_t a = 0, b = 0;
    while (a + b < nu + nl) {
      if (!has_edge(ou + a % nu, ol + b % nl)) return false;
      const bool up = a < nu && (b == nl || (a + 1) * nl < (b + 1) * nu ||
                                 ((a + 1) * nl == (b + 1) * nu && nu > nl));
      if (up) ++a; else ++b;
    }
    count += nu + nl;
  }
  return count == d->nedges;
}

// Processing order: bands of `band` parallels; each band is cut into
// longitude sectors holding about `width` nodes of its widest parallel;
// a tile is one sector of one band, listed parallel by parallel.  Meshes
// without a parallel structure fall back to blocks of consecutive nodes.
static void processing_order(const atlas_mesh_desc *d, int band, int width,
                             std::vector<int32_t> &perm, std::vector<int32_t> &tile_ptr,
                             int32_t &nrings) {
  const int64_t V = d->nnodes;
  std::vector<int64_t> off = rings_of(d);
  const int64_t nr = (int64_t)off.size() - 1;
  nrings = (int32_t)nr;
  perm.clear();
  perm.reserve(V);
  tile_ptr.assign(1, 0);
  if (nr > V / 4) {
    for (int64_t i = 0; i < V; ++i) {
      perm.push_back((int32_t)i);
      if ((i + 1) % (band * width) == 0 || i + 1 == V) tile_ptr.push_back((int32_t)(i + 1));
    }
    return;
  }
  const double twopi = 6.283185307179586476925;
  for (int64_t j0 = 0; j0 < nr; j0 += band) {
    const int64_t j1 = std::min(nr, j0 + band);
    int64_t widest = 0;
    for (int64_t j = j0; j < j1; ++j) widest = std::max(widest, off[j + 1] - off[j]);
    const int64_t nsec = std::max<int64_t>(1, (widest + width / 2) / width);
    std::vector<std::vector<int32_t>> bucket(nsec);
    for (int64_t j = j0; j < j1; ++j) {
      for (int64_t i = off[j]; i < off[j + 1]; ++i) {
        double x = std::fmod(d->lon[i], twopi);
        if (x < 0) x += twopi;
        int64_t sec = (int64_t)(x / twopi * (double)nsec);
        if (sec >= nsec) sec = nsec - 1;
        bucket[sec].push_back((int32_t)i);
      }
    }
    for (int64_t s = 0; s < nsec; ++s) {
      perm.insert(perm.end(), bucket[s].begin(), bucket[s].end());
      if ((int64_t)perm.size() > tile_ptr.back()) tile_ptr.push_back((int32_t)perm.size());
    }
  }
}

// Parallel-sweep plan.  For every tile: the parallels it owns plus one
// above and one below, each reduced to the shortest cyclic run of nodes that
// holds the tile's own nodes and all their neighbours; the slot of every
// position in its run and of every neighbour in its run.  A kernel keeps
// the runs of three consecutive parallels in LDS and reads every neighbour
// from there.  Returns false if a neighbour lies more than one parallel away
// (then the plan is not used).
struct SweepPlan {
  std::vector<int32_t> tile_seg, selfslot, lref;
  std::vector<int4> seg;
  std::vector<int2> seg_pos;
  int32_t segmax = 0;
};

static bool sweep_plan(const std::vector<int64_t> &off, const std::vector<int32_t> &perm,
                       const std::vector<int32_t> &tile_ptr, const std::vector<int32_t> &rowp,
                       const std::vector<int32_t> &nbr, SweepPlan &sp) {
  const int64_t V = (int64_t)perm.size();
  const int64_t nr = (int64_t)off.size() - 1;
  std::vector<int32_t> ring_of(V);
  for (int64_t j = 0; j < nr; ++j)
    for (int64_t i = off[j]; i < off[j + 1]; ++i) ring_of[i] = (int32_t)j;
  const int64_t T = (int64_t)tile_ptr.size() - 1;
  sp.tile_seg.assign(1, 0);
  sp.selfslot.assign(V, 0);
  sp.lref.assign(nbr.size(), -1);
  std::vector<std::vector<int32_t>> need;
  for (int64_t t = 0; t < T; ++t) {
    const int32_t p0 = tile_ptr[t], p1 = tile_ptr[t + 1];
    int32_t jmin = INT32_MAX, jmax = -1;
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t j = ring_of[perm[p]];
      if (p > p0 && j < ring_of[perm[p - 1]]) return false;  // parallels in order
      jmin = std::min(jmin, j);
      jmax = std::max(jmax, j);
    }
    const int32_t rlo = std::max<int32_t>(0, jmin - 1);
    const int32_t rhi = std::min<int32_t>((int32_t)nr - 1, jmax + 1);
    need.assign(rhi - rlo + 1, {});
    std::vector<int2> pos(rhi - rlo + 1, make_int2(0, 0));
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = perm[p], j = ring_of[i];
      need[j - rlo].push_back((int32_t)(i - off[j]));
      if (pos[j - rlo].y == 0) pos[j - rlo] = make_int2(p, p + 1);
      else pos[j - rlo].y = p + 1;
      for (int32_t r = rowp[p]; r < rowp[p + 1]; ++r) {
        const int32_t n = (int32_t)((uint32_t)nbr[r] & ~kPoleBit), jn = ring_of[n];
        if (jn < j - 1 || jn > j + 1) return false;
        need[jn - rlo].push_back((int32_t)(n - off[jn]));
      }
    }
    std::vector<int32_t> lo(rhi - rlo + 1), len(rhi - rlo + 1);
    for (int32_t q = 0; q <= rhi - rlo; ++q) {
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      auto &a = need[q];
      std::sort(a.begin(), a.end());
      a.erase(std::unique(a.begin(), a.end()), a.end());
      if (a.empty()) { lo[q] = 0; len[q] = 0; }
      else if ((int32_t)a.size() == nx) { lo[q] = 0; len[q] = nx; }
      else {
        // the run is the complement of the widest cyclic gap
        int32_t best = -1, at = 0;
        for (size_t k = 0; k < a.size(); ++k) {
          const int32_t g = (k + 1 < a.size()) ? a[k + 1] - a[k] : a[0] + nx - a[k];
          if (g > best) { best = g; at = (int32_t)k; }
        }
        lo[q] = a[(at + 1) % a.size()];
        len[q] = nx - best + 1;
      }
      if (len[q] >= 65536) return false;
      sp.segmax = std::max(sp.segmax, len[q]);
      sp.seg.push_back(make_int4((int32_t)off[rlo + q], nx, lo[q], len[q]));
      sp.seg_pos.push_back(pos[q]);
    }
    sp.tile_seg.push_back((int32_t)sp.seg.size());
    auto slot = [&](int32_t node, int32_t q) {
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      int32_t s = (int32_t)(node - off[rlo + q]) - lo[q];
      if (s < 0) s += nx;
      return s;
    };
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = perm[p], q = ring_of[i] - rlo;
      sp.selfslot[p] = slot(i, q);
      for (int32_t r = rowp[p]; r < rowp[p + 1]; ++r) {
        const bool pole = ((uint32_t)nbr[r] & kPoleBit) != 0;
        const int32_t n = (int32_t)((uint32_t)nbr[r] & ~kPoleBit);
        const int32_t qn = ring_of[n] - rlo;
        const int32_t s = slot(n, qn);
        if (s >= len[qn]) return false;
        sp.lref[r] = (pole ? kLrefPole : 0) | ((qn - q + 1) << 16) | s;
      }
    }
  }
  return true;
}

// Two-ring plan of the fused Laplacian.  For every tile: its own
// parallels [ja, jb]; the gradient is needed at the tile's nodes and their
// neighbours (parallels ja-1 .. jb+1), and those gradients need the field at
// their own neighbours (parallels ja-2 .. jb+2).  Per parallel of that
// window: the f-run (shortest cyclic run holding every node whose field is
// read), the g-run (the same for the nodes whose gradient is formed; every
// node of the g-run gets one, so all of them are covered by the f-runs), and
// the tile's own positions.  Per g-run node: its incidence row start, count,
// its slot in its f-run and its neighbours' f-run slots; per own position:
// its slot in its g-run and its neighbours' g-run slots.  References are
// ((dq + 1) << 16) | slot (dq = neighbour parallel - own parallel) plus
// kLrefPole for a pole edge.  Returns false if a neighbour lies more than
// one parallel away.
struct LaplPlan {
  std::vector<int32_t> tile_seg;  // [T+1] window range of a tile in fseg/gseg
  std::vector<int4> fseg;         // {ring offset, ring size, f-run first, f-run length}
  std::vector<int4> gseg;         // {g-run first, g-run length, first g record, 0}
  std::vector<int2> seg_pos;      // own positions on the parallel [lo, hi)
  std::vector<int4> gnode;        // per g record {row start, row length, f self slot, position}
  std::vector<int32_t> glref;     // per g record: kGRefs references into the f-runs
  std::vector<int32_t> lref;      // per incidence (own positions): into the g-runs
  std::vector<int32_t> lself;     // per position: slot in its g-run
  int32_t fmax = 0, gmax = 0, pmax = 0;
};

static bool cyclic_run(std::vector<int32_t> &a, int32_t nx, int32_t &lo, int32_t &len) {
  std::sort(a.begin(), a.end());
  a.erase(std::unique(a.begin(), a.end()), a.end());
  if (a.empty()) {
    lo = 0;
    len = 0;
  } else if ((int32_t)a.size() == nx) {
    lo = 0;
    len = nx;
  } else {
    int32_t best = -1, at = 0;  // the run is the complement of the widest gap
    for (size_t k = 0; k < a.size(); ++k) {
      const int32_t g = (k + 1 < a.size()) ? a[k + 1] - a[k] : a[0] + nx - a[k];
      if (g > best) {
        best = g;
        at = (int32_t)k;
      }
    }
    lo = a[(at + 1) % a.size()];
    len = nx - best + 1;
  }
  return len < 65536;
}

static bool lapl_plan(const std::vector<int64_t> &off, const std::vector<int32_t> &perm,
                      const std::vector<int32_t> &tile_ptr, const std::vector<int32_t> &rowp,
                      const std::vector<int32_t> &nbr, LaplPlan &lp) {
  const int64_t V = (int64_t)perm.size();
  const int32_t nr = (int32_t)off.size() - 1;
  std::vector<int32_t> ring_of(V), inv(V);
  for (int32_t j = 0; j < nr; ++j)
    for (int64_t i = off[j]; i < off[j + 1]; ++i) ring_of[i] = j;
  for (int64_t p = 0; p < V; ++p) inv[perm[p]] = (int32_t)p;
  const int64_t T = (int64_t)tile_ptr.size() - 1;
  lp.tile_seg.assign(1, 0);
  lp.lref.assign(nbr.size(), 1 << 16);
  lp.lself.assign(V, 0);
  auto nb = [&](int32_t r) { return (int32_t)((uint32_t)nbr[r] & ~kPoleBit); };
  for (int64_t t = 0; t < T; ++t) {
    const int32_t p0 = tile_ptr[t], p1 = tile_ptr[t + 1];
    int32_t ja = INT32_MAX, jb = -1;
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t j = ring_of[perm[p]];
      if (p > p0 && j < ring_of[perm[p - 1]]) return false;  // parallels in order
      ja = std::min(ja, j);
      jb = std::max(jb, j);
    }
    const int32_t rlo = std::max(0, ja - 2), rhi = std::min(nr - 1, jb + 2);
    const int32_t W = rhi - rlo + 1;
    std::vector<std::vector<int32_t>> gneed(W), fneed(W);
    std::vector<int2> pos(W, make_int2(0, 0));
    auto local = [&](int32_t node) { return (int32_t)(node - off[ring_of[node]]); };
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = perm[p], j = ring_of[i];
      gneed[j - rlo].push_back(local(i));
      if (pos[j - rlo].y == 0) pos[j - rlo] = make_int2(p, p + 1);
      else pos[j - rlo].y = p + 1;
      for (int32_t r = rowp[p]; r < rowp[p + 1]; ++r) {
        const int32_t n = nb(r), jn = ring_of[n];
        if (jn < j - 1 || jn > j + 1) return false;
        gneed[jn - rlo].push_back(local(n));
      }
    }
    std::vector<int32_t> glo(W), glen(W), flo(W), flen(W);
    for (int32_t q = 0; q < W; ++q) {
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      if (!cyclic_run(gneed[q], nx, glo[q], glen[q])) return false;
      // every node of the g-run gets a gradient: its field and its
      // neighbours' fields are read
      for (int32_t s = 0; s < glen[q]; ++s) {
        const int32_t i = (int32_t)off[rlo + q] + (glo[q] + s) % nx;
        const int32_t p = inv[i], j = rlo + q;
        fneed[q].push_back(local(i));
        for (int32_t r = rowp[p]; r < rowp[p + 1]; ++r) {
          const int32_t n = nb(r), jn = ring_of[n];
          if (jn < j - 1 || jn > j + 1 || jn < rlo || jn > rhi) return false;
          fneed[jn - rlo].push_back(local(n));
        }
      }
    }
    for (int32_t q = 0; q < W; ++q) {
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      if (!cyclic_run(fneed[q], nx, flo[q], flen[q])) return false;
    }
    auto fslot = [&](int32_t node) {
      const int32_t q = ring_of[node] - rlo;
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      int32_t s = local(node) - flo[q];
      if (s < 0) s += nx;
      return s;
    };
    auto gslot = [&](int32_t node) {
      const int32_t q = ring_of[node] - rlo;
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      int32_t s = local(node) - glo[q];
      if (s < 0) s += nx;
      return s;
    };
    for (int32_t q = 0; q < W; ++q) {
      const int32_t nx = (int32_t)(off[rlo + q + 1] - off[rlo + q]);
      lp.fmax = std::max(lp.fmax, flen[q]);
      lp.gmax = std::max(lp.gmax, glen[q]);
      lp.pmax = std::max(lp.pmax, pos[q].y - pos[q].x);
      lp.fseg.push_back(make_int4((int32_t)off[rlo + q], nx, flo[q], flen[q]));
      lp.gseg.push_back(make_int4(glo[q], glen[q], (int32_t)lp.gnode.size(), 0));
      lp.seg_pos.push_back(pos[q]);
      const int32_t j = rlo + q;
      for (int32_t s = 0; s < glen[q]; ++s) {
        const int32_t i = (int32_t)off[j] + (glo[q] + s) % nx;
        const int32_t p = inv[i], n0 = rowp[p], n1 = rowp[p + 1];
        if (n1 - n0 > kGRefs) return false;
        const int32_t self = fslot(i);
        if (self >= flen[q]) return false;
        lp.gnode.push_back(make_int4(n0, n1 - n0, self, p));
        for (int32_t k = 0; k < kGRefs; ++k) {
          int32_t ref = 1 << 16;  // padding: the own parallel, slot 0
          if (k < n1 - n0) {
            const int32_t r = n0 + k, n = nb(r), qn = ring_of[n] - rlo;
            const int32_t sl = fslot(n);
            if (sl >= flen[qn]) return false;
            ref = ((((uint32_t)nbr[r] & kPoleBit) != 0) ? kLrefPole : 0) |
                  ((ring_of[n] - j + 1) << 16) | sl;
          }
          lp.glref.push_back(ref);
        }
      }
    }
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = perm[p], j = ring_of[i];
      lp.lself[p] = gslot(i);
      if (lp.lself[p] >= glen[j - rlo]) return false;
      for (int32_t r = rowp[p]; r < rowp[p + 1]; ++r) {
        const int32_t n = nb(r), qn = ring_of[n] - rlo;
        const int32_t sl = gslot(n);
        if (sl >= glen[qn]) return false;
        lp.lref[r] = ((((uint32_t)nbr[r] & kPoleBit) != 0) ? kLrefPole : 0) |
                     ((ring_of[n] - j + 1) << 16) | sl;
      }
    }
    lp.tile_seg.push_back((int32_t)lp.fseg.size());
  }
  return true;
}

template <class T>
static atlas_status upload_array(MeshStore &m, const std::vector<T> &h, const T **dptr) {
  void *p = nullptr;
  const size_t bytes = std::max<size_t>(1, h.size() * sizeof(T));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(ATLAS_ENOMEM, "hipMalloc of mesh store failed");
  m.allocations.push_back(p);
  m.bytes += bytes;
  if (!h.empty()) ATLASX_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *dptr = static_cast<const T *>(p);
  return ATLAS_OK;
}

atlas_status upload_mesh(const atlas_mesh_desc *d, int band, int width, MeshStore **out) {
  atlas_status st = validate(d);
  if (st != ATLAS_OK) return st;
  const int64_t V = d->nnodes, E = d->nedges, NP = d->npole_edges;

  std::vector<int32_t> perm, tile_ptr;
  int32_t nrings = 0;
  processing_order(d, band, width, perm, tile_ptr, nrings);
  if ((int64_t)perm.size() != V) return fail(ATLAS_EINVAL, "processing order lost nodes");

  std::vector<int32_t> pole_of(V, -1);
  for (int64_t k = 0; k < NP; ++k) {
    pole_of[d->pole_edges[2 * k]] = (int32_t)k;
    pole_of[d->pole_edges[2 * k + 1]] = (int32_t)k;
  }
  // incidences in processing order: mesh edges in ascending id, pole last
  std::vector<int32_t> rowp(V + 1, 0), nbr, inc_edge;
  std::vector<double2> S;
  std::vector<double> vol_p(V), cos_p(V);
  nbr.reserve(2 * E + 2 * NP);
  inc_edge.reserve(2 * E + 2 * NP);
  S.reserve(2 * E + 2 * NP);
  int32_t maxdeg = 0, mindeg = INT32_MAX;
  for (int64_t p = 0; p < V; ++p) {
    const int32_t i = perm[p];
    mindeg = std::min<int32_t>(mindeg, (int32_t)(d->node2edge_ptr[i + 1] - d->node2edge_ptr[i]));
    for (int64_t r = d->node2edge_ptr[i]; r < d->node2edge_ptr[i + 1]; ++r) {
      const int32_t e = d->node2edge[r];
      const int8_t s = d->node2edge_sign[r];
      const int32_t other = s > 0 ? d->edge2node[2 * e + 1] : d->edge2node[2 * e];
      nbr.push_back(other);
      inc_edge.push_back(s > 0 ? e : (int32_t)(e | (int32_t)kPoleBit));
      S.push_back(make_double2(s * d->dual_normals[2 * e], s * d->dual_normals[2 * e + 1]));
    }
    if (pole_of[i] >= 0) {
      const int32_t k = pole_of[i];
      const int32_t a = d->pole_edges[2 * k], b = d->pole_edges[2 * k + 1];
      nbr.push_back((int32_t)((uint32_t)(a == i ? b : a) | kPoleBit));
      inc_edge.push_back((int32_t)(E + k));
      S.push_back(make_double2(0.0, d->pole_normals[k]));
    }
    rowp[p + 1] = (int32_t)nbr.size();
    maxdeg = std::max(maxdeg, rowp[p + 1] - rowp[p]);
    vol_p[p] = d->dual_volumes[i];
    cos_p[p] = d->cos_lat[i];
  }
  if (maxdeg > 64) return fail(ATLAS_EINVAL, "node degree above 64");
  std::vector<int32_t> e2n(2 * (E + NP));
  std::vector<double2> eS(E + NP);
  for (int64_t e = 0; e < E; ++e) {
    e2n[2 * e] = d->edge2node[2 * e];
    e2n[2 * e + 1] = d->edge2node[2 * e + 1];
    eS[e] = make_double2(d->dual_normals[2 * e], d->dual_normals[2 * e + 1]);
  }
  for (int64_t k = 0; k < NP; ++k) {
    e2n[2 * (E + k)] = d->pole_edges[2 * k];
    e2n[2 * (E + k) + 1] = d->pole_edges[2 * k + 1];
    eS[E + k] = make_double2(0.0, d->pole_normals[k]);
  }
  std::vector<double> cos_n(d->cos_lat, d->cos_lat + V);
  SweepPlan sp;
  const bool sweep_ok = nrings <= V / 4 && sweep_plan(rings_of(d), perm, tile_ptr, rowp, nbr, sp);
  if (!sweep_ok) sp = SweepPlan();
  LaplPlan lp;
  const bool l2_ok = sweep_ok && lapl_plan(rings_of(d), perm, tile_ptr, rowp, nbr, lp);
  if (!l2_ok) lp = LaplPlan();
  // cos(lat) of every incidence's neighbour, so a node's row is read with
  // contiguous loads
  std::vector<double> ncos(nbr.size());
  for (size_t r = 0; r < nbr.size(); ++r) ncos[r] = d->cos_lat[(uint32_t)nbr[r] & ~kPoleBit];
  // kernels read the incidences of a node in groups of kIncPad without
  // clamping: pad every incidence array by one group
  nbr.resize(nbr.size() + kIncPad, 0);
  S.resize(S.size() + kIncPad, make_double2(0.0, 0.0));
  inc_edge.resize(inc_edge.size() + kIncPad, 0);
  ncos.resize(ncos.size() + kIncPad, 1.0);
  sp.lref.resize(sp.lref.size() + kIncPad, 1 << 16);
  if (l2_ok) lp.lref.resize(lp.lref.size() + kIncPad, 1 << 16);

  MeshStore *m = new (std::nothrow) MeshStore();
  if (!m) return fail(ATLAS_ENOMEM, "out of host memory");
  (void)hipGetDevice(&m->device);
  m->d.V = (int32_t)V;
  m->d.E = (int32_t)E;
  m->d.npole = (int32_t)NP;
  m->d.ntiles = (int32_t)tile_ptr.size() - 1;
  m->nincid = (int64_t)nbr.size() - kIncPad;
  m->radius = d->radius;
  m->nrings = nrings;
  m->max_degree = maxdeg;
  for (size_t t = 0; t + 1 < tile_ptr.size(); ++t)
    m->max_tile = std::max<int64_t>(m->max_tile, tile_ptr[t + 1] - tile_ptr[t]);
  if (sweep_ok) {
    const std::vector<int64_t> off = rings_of(d);
    for (size_t j = 0; j + 1 < off.size(); ++j) m->max_run = std::max(m->max_run, off[j + 1] - off[j]);
  }
  m->d.maxdeg = maxdeg;
  m->d.mindeg = V > 0 ? mindeg : 0;
  m->d.sweep_ok = sweep_ok ? 1 : 0;
  m->d.segmax = sp.segmax;
  m->d.l2_ok = l2_ok ? 1 : 0;
  m->d.l2_fmax = lp.fmax;
  m->d.l2_gmax = lp.gmax;
  m->d.l2_pmax = lp.pmax;
  const double *vol_d = nullptr, *cos_pd = nullptr;
  std::vector<double> zeros(V, 0.0);
  if ((st = upload_array(*m, perm, &m->d.perm)) != ATLAS_OK ||
      (st = upload_array(*m, rowp, &m->d.rowp)) != ATLAS_OK ||
      (st = upload_array(*m, nbr, &m->d.nbr)) != ATLAS_OK ||
      (st = upload_array(*m, S, &m->d.S)) != ATLAS_OK ||
      (st = upload_array(*m, inc_edge, &m->d.inc_edge)) != ATLAS_OK ||
      (st = upload_array(*m, zeros, &m->d.alpha)) != ATLAS_OK ||
      (st = upload_array(*m, zeros, &m->d.beta)) != ATLAS_OK ||
      (st = upload_array(*m, cos_n, &m->d.coslat)) != ATLAS_OK ||
      (st = upload_array(*m, tile_ptr, &m->d.tile_ptr)) != ATLAS_OK ||
      (st = upload_array(*m, e2n, &m->d.e2n)) != ATLAS_OK ||
      (st = upload_array(*m, eS, &m->d.eS)) != ATLAS_OK ||
      (st = upload_array(*m, vol_p, &vol_d)) != ATLAS_OK ||
      (st = upload_array(*m, cos_p, &cos_pd)) != ATLAS_OK ||
      (st = upload_array(*m, sp.tile_seg, &m->d.tile_seg)) != ATLAS_OK ||
      (st = upload_array(*m, sp.seg, &m->d.seg)) != ATLAS_OK ||
      (st = upload_array(*m, sp.seg_pos, &m->d.seg_pos)) != ATLAS_OK ||
      (st = upload_array(*m, sp.selfslot, &m->d.selfslot)) != ATLAS_OK ||
      (st = upload_array(*m, sp.lref, &m->d.lref)) != ATLAS_OK ||
      (st = upload_array(*m, ncos, &m->d.ncos)) != ATLAS_OK ||
      (st = upload_array(*m, lp.tile_seg, &m->d.l2_tile_seg)) != ATLAS_OK ||
      (st = upload_array(*m, lp.fseg, &m->d.l2_fseg)) != ATLAS_OK ||
      (st = upload_array(*m, lp.gseg, &m->d.l2_gseg)) != ATLAS_OK ||
      (st = upload_array(*m, lp.seg_pos, &m->d.l2_seg_pos)) != ATLAS_OK ||
      (st = upload_array(*m, lp.gnode, &m->d.l2_gnode)) != ATLAS_OK ||
      (st = upload_array(*m, lp.glref, &m->d.l2_glref)) != ATLAS_OK ||
      (st = upload_array(*m, lp.lref, &m->d.l2_lref)) != ATLAS_OK ||
      (st = upload_array(*m, lp.lself, &m->d.l2_lself)) != ATLAS_OK) {
    delete m;
    return st;
  }
  std::vector<PosRec> pos(V);
  for (int64_t p = 0; p < V; ++p) {
    pos[p].node = perm[p];
    pos[p].r0 = rowp[p];
    pos[p].r1 = rowp[p + 1];
    pos[p].selfslot = sweep_ok ? sp.selfslot[p] : 0;
    pos[p].alpha = 0.0;  // derived on the device below
    pos[p].beta = 0.0;
  }
  if ((st = upload_array(*m, pos, &m->d.pos)) != ATLAS_OK) {
    delete m;
    return st;
  }
  if ((st = derive_scales(*m, vol_d, cos_pd, d->radius)) != ATLAS_OK) {
    delete m;
    return st;
  }
  if (l2_ok && (st = pack_lapl_geometry(*m, (int64_t)lp.gnode.size())) != ATLAS_OK) {
    delete m;
    return st;
  }
  if (sweep_ok && (st = pack_sweep_geometry(*m)) != ATLAS_OK) {
    delete m;
    return st;
  }
  // node coordinates by node id (remap targets and sources), and the
  // parallels of a mesh a remap can start from
  {
    std::vector<double> lon_n(d->lon, d->lon + V), lat_n(d->lat, d->lat + V);
    if ((st = upload_array(*m, lon_n, &m->node_lon)) != ATLAS_OK ||
        (st = upload_array(*m, lat_n, &m->node_lat)) != ATLAS_OK) {
      delete m;
      return st;
    }
    const std::vector<int64_t> off = rings_of(d);
    if (zipper_conforming(d, off)) {
      std::vector<double> rlat(off.size() - 1);
      for (size_t j = 0; j + 1 < off.size(); ++j) rlat[j] = d->lat[off[j]];
      if ((st = upload_array(*m, off, &m->rs.ring_off)) != ATLAS_OK ||
          (st = upload_array(*m, rlat, &m->rs.ring_lat)) != ATLAS_OK) {
        delete m;
        return st;
      }
      m->rs.nrings = (int32_t)rlat.size();
      m->rs.ok = 1;
    }
  }
  // the volumes stay (diagnostics); cos by position was only for the scales
  m->d.vol = vol_d;
  (void)hipDeviceSynchronize();
  // bytes one operator pass reads from the mesh store (column/flat forms):
  // per position perm + rowp + alpha/beta; per incidence nbr + S;
  // per node cos(lat) (div/curl)
  m->geometry_bytes = (double)V * (4 + 4 + 16) + (double)m->nincid * (4 + 16);
  *out = m;
  return ATLAS_OK;
}

}  // namespace atlasx
