// capi.cpp -- the extern "C" entry points of atlas_nabla.h.
//
// The C layer follows the pattern of Section 4.1 / Figure 3: an opaque
// handle to a native object, driven through plain C functions that return a
// status instead of throwing (the grid classes' valid() in Section 4.2.3).
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "internal.h"

namespace atlasx {

static thread_local std::string g_last_error;

// host mesh descriptions handed out by atlas_mesh_desc_octahedral and
// atlas_mesh_desc_reduced_gaussian
static std::mutex g_desc_mu;
static std::unordered_map<const atlas_mesh_desc *, HostMesh *> g_descs;

atlas_status fail(atlas_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

atlas_status hip_fail(hipError_t err, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(err);
  return err == hipErrorOutOfMemory ? ATLAS_ENOMEM : ATLAS_EDEVICE;
}

atlas_status upload_mesh(const atlas_mesh_desc *d, int band, int width, MeshStore **out);

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

static size_t in_bytes(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt) {
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  const bool vec_in = op == ATLAS_OP_DIVERGENCE || op == ATLAS_OP_CURL;
  return (size_t)m.d.V * nlev * w * (vec_in ? 2 : 1);
}
static size_t out_bytes(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt) {
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  return (size_t)m.d.V * nlev * w * (op == ATLAS_OP_GRADIENT ? 2 : 1);
}
static size_t lapl_ws_bytes(const MeshStore &m, int nlev, atlas_dtype dt) {
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  return (size_t)m.d.V * nlev * 2 * w;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

// Whether fields of `nlev` levels fit the library's offsets: all values of
// a field below 2^40; the byte offsets inside one buffer resource (a
// parallel of columns, 16 bytes per level at most) and the element
// counters of one tile below 2^31.
bool levels_fit(const MeshStore &m, int64_t nlev, std::string *why) {
  const int64_t lim = (int64_t)1 << 31;
  if ((int64_t)m.d.V * nlev * 2 >= ((int64_t)1 << 40)) {
    if (why) *why = "nnodes * nlev too large";
    return false;
  }
  if (m.max_run * nlev * 16 >= lim || m.max_tile * nlev * 2 >= lim) {
    if (why)
      *why = "nlev too large for this mesh: at most " +
             std::to_string(max_levels(m)) + " levels (longest parallel " +
             std::to_string(m.max_run) + " nodes, largest tile " + std::to_string(m.max_tile) + ")";
    return false;
  }
  return true;
}

int64_t max_levels(const MeshStore &m) {
  const int64_t lim = ((int64_t)1 << 31) - 1;
  int64_t n = std::min(lim / (16 * m.max_run), lim / (2 * m.max_tile));
  return std::min<int64_t>(n, (((int64_t)1 << 40) - 1) / (2 * (int64_t)m.d.V));
}

// Validates every argument of an operator call before anything is enqueued.
atlas_status check_call(atlas_mesh_t mesh, atlas_op op, const void *in, int nlev,
                        atlas_dtype dt, void *out) {
  if (!mesh || !mesh->store) return fail(ATLAS_EINVAL, "mesh handle is NULL");
  if (op < ATLAS_OP_GRADIENT || op > ATLAS_OP_LAPLACIAN) return fail(ATLAS_EINVAL, "unknown operator");
  if (dt != ATLAS_F32 && dt != ATLAS_F64) return fail(ATLAS_EINVAL, "unknown dtype");
  if (nlev < 1) return fail(ATLAS_EINVAL, "nlev must be >= 1");
  if (std::string why; !levels_fit(*mesh->store, nlev, &why)) return fail(ATLAS_EINVAL, why);
  if (!in || !out) return fail(ATLAS_EINVAL, "field pointer is NULL");
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  const size_t vw = (op == ATLAS_OP_GRADIENT) ? 2 * w : w;
  const size_t iw = (op == ATLAS_OP_DIVERGENCE || op == ATLAS_OP_CURL) ? 2 * w : w;
  if (!aligned(in, iw) || !aligned(out, vw))
    return fail(ATLAS_EINVAL, "field pointer not aligned to its element size");
  const MeshStore &m = *mesh->store;
  if (overlap(in, in_bytes(m, op, nlev, dt), out, out_bytes(m, op, nlev, dt)))
    return fail(ATLAS_EINVAL, "input and output overlap");
  return ATLAS_OK;
}

static atlas_status internal_ws(MeshStore &m, size_t bytes, void **ws) {
  std::lock_guard<std::mutex> g(m.ws_mu);
  if (m.ws_bytes < bytes) {
    if (m.ws) ATLASX_HIP(hipFree(m.ws));
    m.ws = nullptr;
    m.ws_bytes = 0;
    hipError_t e = hipMalloc(&m.ws, bytes);
    if (e != hipSuccess) {
      m.ws = nullptr;
      return fail(ATLAS_ENOMEM, "cannot allocate the operator workspace");
    }
    m.ws_bytes = bytes;
  }
  *ws = m.ws;
  return ATLAS_OK;
}

LaunchShape shape_from(const atlas_launch *l, const MeshStore &m, atlas_op op, int nlev,
                       atlas_dtype dt);

atlas_status apply(atlas_mesh_t mesh, atlas_op op, const void *in, int32_t nlev,
                   atlas_dtype dt, void *out, void *workspace, const atlas_launch *shape,
                   hipStream_t stream) {
  atlas_status st = check_call(mesh, op, in, nlev, dt, out);
  if (st != ATLAS_OK) return st;
  MeshStore &m = *mesh->store;
  LaunchShape sh = shape_from(shape, m, op, nlev, dt);
  if (sh.block < 64 || sh.block > 1024 || (sh.block & 63) != 0)
    return fail(ATLAS_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
  if (sh.nodes_per_block < 0) return fail(ATLAS_EINVAL, "nodes_per_block must be >= 0");
  if (sh.level_chunk < 0 || sh.level_chunk > 64)
    return fail(ATLAS_EINVAL, "level_chunk must be in [0, 64]");
  if (sh.blocks_per_cu < 0 || sh.blocks_per_cu > 32)
    return fail(ATLAS_EINVAL, "blocks_per_cu must be in [0, 32]");
  if (sh.level_vec < 0 || sh.level_vec > 4)
    return fail(ATLAS_EINVAL, "level_vec must be in [0, 4]");
  size_t need = 0;
  if (op == ATLAS_OP_LAPLACIAN && !lapl_fused_runs(m, nlev, dt, sh))
    need += lapl_ws_bytes(m, nlev, dt);  // the fused form needs none
  if (sh.variant == ATLAS_VARIANT_FLUX) need += flux_ws_bytes(m, op, nlev, dt);
  void *ws = workspace;
  if (need && !ws) {
    st = internal_ws(m, need, &ws);
    if (st != ATLAS_OK) return st;
  }
  if (ws && !aligned(ws, 16)) return fail(ATLAS_EINVAL, "workspace must be 16-byte aligned");
  if (ws && (overlap(ws, need, in, in_bytes(m, op, nlev, dt)) ||
             overlap(ws, need, out, out_bytes(m, op, nlev, dt))))
    return fail(ATLAS_EINVAL, "workspace overlaps a field");
  return launch_op(m, op, dt, in, nlev, out, ws, sh, stream);
}

}  // namespace atlasx

using namespace atlasx;

extern "C" {

const char *atlas_last_error(void) { return g_last_error.c_str(); }

const char *atlas_version(void) { return "atlas-nabla-mi355x 0.1 (gfx950)"; }

atlas_status atlas_mesh_desc_octahedral(int32_t N, double radius, atlas_mesh_desc **out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 1 || N > 8192) return fail(ATLAS_EINVAL, "N must be in [1, 8192]");
  if (!(radius > 0.0)) return fail(ATLAS_EINVAL, "radius must be positive");
  HostMesh *h = new (std::nothrow) HostMesh();
  if (!h) return fail(ATLAS_ENOMEM, "out of host memory");
  try {
    build_octahedral(N, radius, *h);
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(ATLAS_ENOMEM, "out of host memory building the mesh");
  }
  {
    std::lock_guard<std::mutex> g(g_desc_mu);
    g_descs[&h->desc] = h;
  }
  *out = &h->desc;
  return ATLAS_OK;
}

atlas_status atlas_mesh_desc_reduced_gaussian(int32_t nrings, const int32_t *nx, double radius,
                                              atlas_mesh_desc **out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!nx) return fail(ATLAS_EINVAL, "nx is NULL");
  if (nrings < 2 || nrings > 16384 || (nrings & 1))
    return fail(ATLAS_EINVAL, "nrings must be even and in [2, 16384]");
  int64_t total = 0;
  for (int j = 0; j < nrings; ++j) {
    if (nx[j] < 4 || nx[j] > (1 << 20)) return fail(ATLAS_EINVAL, "every nx must be in [4, 2^20]");
    total += nx[j];
  }
  if ((nx[0] & 1) || (nx[nrings - 1] & 1))
    return fail(ATLAS_EINVAL, "the polar parallels need an even number of points");
  if (total * 3 >= ((int64_t)1 << 31)) return fail(ATLAS_EINVAL, "grid too large");
  if (!(radius > 0.0)) return fail(ATLAS_EINVAL, "radius must be positive");
  HostMesh *h = new (std::nothrow) HostMesh();
  if (!h) return fail(ATLAS_ENOMEM, "out of host memory");
  try {
    build_reduced_gaussian(std::vector<int32_t>(nx, nx + nrings), radius, *h);
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(ATLAS_ENOMEM, "out of host memory building the mesh");
  }
  {
    std::lock_guard<std::mutex> g(g_desc_mu);
    g_descs[&h->desc] = h;
  }
  *out = &h->desc;
  return ATLAS_OK;
}

atlas_status atlas_mesh_desc_grid(int32_t nrings, const int32_t *nx, const double *lat,
                                  int32_t flags, double radius, atlas_mesh_desc **out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!nx) return fail(ATLAS_EINVAL, "nx is NULL");
  if (flags & ~(ATLAS_MESH_SHIFTED | ATLAS_MESH_QUADS)) return fail(ATLAS_EINVAL, "unknown flags");
  if (nrings < 2 || nrings > 16384) return fail(ATLAS_EINVAL, "nrings must be in [2, 16384]");
  if (!lat && (nrings & 1)) return fail(ATLAS_EINVAL, "Gaussian latitudes need an even nrings");
  int64_t total = 0;
  for (int j = 0; j < nrings; ++j) {
    if (nx[j] < 4 || nx[j] > (1 << 20)) return fail(ATLAS_EINVAL, "every nx must be in [4, 2^20]");
    if ((flags & ATLAS_MESH_SHIFTED) && nx[j] != nx[0])
      return fail(ATLAS_EINVAL, "a shifted grid needs equal counts on all parallels");
    total += nx[j];
  }
  if ((nx[0] & 1) || (nx[nrings - 1] & 1))
    return fail(ATLAS_EINVAL, "the polar parallels need an even number of points");
  if (total * 3 >= ((int64_t)1 << 31)) return fail(ATLAS_EINVAL, "grid too large");
  if (!(radius > 0.0)) return fail(ATLAS_EINVAL, "radius must be positive");
  std::vector<double> lv;
  if (lat) {
    lv.assign(lat, lat + nrings);
    for (int j = 0; j < nrings; ++j) {
      if (!std::isfinite(lv[j]) || !(std::fabs(lv[j]) < 0.5 * 3.14159265358979323846))
        return fail(ATLAS_EINVAL, "latitudes must lie inside (-pi/2, pi/2)");
      if (j > 0 && !(lv[j] < lv[j - 1]))
        return fail(ATLAS_EINVAL, "latitudes must decrease strictly");
    }
  }
  HostMesh *h = new (std::nothrow) HostMesh();
  if (!h) return fail(ATLAS_ENOMEM, "out of host memory");
  try {
    build_grid(std::vector<int32_t>(nx, nx + nrings), lat ? &lv : nullptr,
               (flags & ATLAS_MESH_SHIFTED) != 0, (flags & ATLAS_MESH_QUADS) != 0, radius, *h);
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(ATLAS_ENOMEM, "out of host memory building the mesh");
  }
  {
    std::lock_guard<std::mutex> g(g_desc_mu);
    g_descs[&h->desc] = h;
  }
  *out = &h->desc;
  return ATLAS_OK;
}

atlas_status atlas_mesh_desc_free(atlas_mesh_desc *desc) {
  if (!desc) return ATLAS_OK;
  HostMesh *h = nullptr;
  {
    std::lock_guard<std::mutex> g(g_desc_mu);
    auto it = g_descs.find(desc);
    if (it == g_descs.end())
      return fail(ATLAS_EINVAL, "description was not created by atlas_mesh_desc_*");
    h = it->second;
    g_descs.erase(it);
  }
  delete h;
  return ATLAS_OK;
}

atlas_status atlas_mesh_upload(const atlas_mesh_desc *desc, atlas_mesh_t *out) {
  return atlas_mesh_upload_ex(desc, nullptr, out);
}

atlas_status atlas_mesh_upload_ex(const atlas_mesh_desc *desc, const atlas_mesh_layout *layout,
                                  atlas_mesh_t *out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  int band = kDefaultBand, width = kDefaultWidth;
  if (layout) {
    if (layout->band_rings < 0 || layout->sector_nodes < 0)
      return fail(ATLAS_EINVAL, "layout fields must be >= 0");
    if (layout->band_rings) band = layout->band_rings;
    if (layout->sector_nodes) width = layout->sector_nodes;
  }
  MeshStore *m = nullptr;
  atlas_status st;
  try {
    st = upload_mesh(desc, band, width, &m);
  } catch (const std::bad_alloc &) {
    return fail(ATLAS_ENOMEM, "out of host memory during upload");
  }
  if (st != ATLAS_OK) return st;
  atlas_mesh_t h = new (std::nothrow) atlas_mesh_s{m};
  if (!h) {
    delete m;
    return fail(ATLAS_ENOMEM, "out of host memory");
  }
  *out = h;
  return ATLAS_OK;
}

atlas_status atlas_mesh_create_octahedral(int32_t N, double radius, atlas_mesh_t *out) {
  atlas_mesh_desc *d = nullptr;
  atlas_status st = atlas_mesh_desc_octahedral(N, radius, &d);
  if (st != ATLAS_OK) return st;
  st = atlas_mesh_upload(d, out);
  atlas_mesh_desc_free(d);
  return st;
}

atlas_status atlas_mesh_free(atlas_mesh_t mesh) {
  if (!mesh) return ATLAS_OK;
  if (mesh->store && mesh->store->serve_refs > 0)
    return fail(ATLAS_EBUSY, "mesh is registered with a server");
  delete mesh->store;
  delete mesh;
  return ATLAS_OK;
}

atlas_status atlas_mesh_get_info(atlas_mesh_t mesh, atlas_mesh_info *info) {
  if (!mesh || !mesh->store || !info) return fail(ATLAS_EINVAL, "NULL argument");
  const MeshStore &m = *mesh->store;
  info->nnodes = m.d.V;
  info->nedges = m.d.E;
  info->nincidences = m.nincid;
  info->npole_edges = m.d.npole;
  info->ntiles = m.d.ntiles;
  info->nrings = m.nrings;
  info->max_degree = m.max_degree;
  info->device_bytes = m.bytes;
  info->geometry_bytes_per_call = m.geometry_bytes;
  info->max_levels = max_levels(m);
  return ATLAS_OK;
}

atlas_status atlas_nabla_apply(atlas_mesh_t mesh, atlas_op op, const void *in, int32_t nlev,
                               atlas_dtype dtype, void *out, void *workspace,
                               const atlas_launch *shape, hipStream_t stream) {
  return apply(mesh, op, in, nlev, dtype, out, workspace, shape, stream);
}

atlas_status atlas_nabla_gradient(atlas_mesh_t mesh, const void *f, int32_t nlev,
                                  atlas_dtype dtype, void *out, hipStream_t stream) {
  return apply(mesh, ATLAS_OP_GRADIENT, f, nlev, dtype, out, nullptr, nullptr, stream);
}

atlas_status atlas_nabla_divergence(atlas_mesh_t mesh, const void *uv, int32_t nlev,
                                    atlas_dtype dtype, void *out, hipStream_t stream) {
  return apply(mesh, ATLAS_OP_DIVERGENCE, uv, nlev, dtype, out, nullptr, nullptr, stream);
}

atlas_status atlas_nabla_curl(atlas_mesh_t mesh, const void *uv, int32_t nlev,
                              atlas_dtype dtype, void *out, hipStream_t stream) {
  return apply(mesh, ATLAS_OP_CURL, uv, nlev, dtype, out, nullptr, nullptr, stream);
}

atlas_status atlas_nabla_div_curl(atlas_mesh_t mesh, const void *uv, int32_t nlev,
                                  atlas_dtype dtype, void *out_div, void *out_curl,
                                  hipStream_t stream) {
  atlas_status st = check_call(mesh, ATLAS_OP_DIVERGENCE, uv, nlev, dtype, out_div);
  if (st != ATLAS_OK) return st;
  st = check_call(mesh, ATLAS_OP_CURL, uv, nlev, dtype, out_curl);
  if (st != ATLAS_OK) return st;
  const MeshStore &m = *mesh->store;
  const size_t ob = out_bytes(m, ATLAS_OP_DIVERGENCE, nlev, dtype);
  if (overlap(out_div, ob, out_curl, ob)) return fail(ATLAS_EINVAL, "the two outputs overlap");
  return launch_div_curl(m, dtype, uv, nlev, out_div, out_curl, stream);
}

atlas_status atlas_nabla_gradient_lonlat(atlas_mesh_t mesh, const void *f, int32_t nlev,
                                         atlas_dtype dtype, void *out, hipStream_t stream) {
  const atlas_status st = check_call(mesh, ATLAS_OP_GRADIENT, f, nlev, dtype, out);
  if (st != ATLAS_OK) return st;
  return gradient_lonlat(*mesh->store, dtype, f, nlev, out, stream);
}

atlas_status atlas_nabla_laplacian(atlas_mesh_t mesh, const void *f, int32_t nlev,
                                   atlas_dtype dtype, void *out, void *workspace,
                                   hipStream_t stream) {
  return apply(mesh, ATLAS_OP_LAPLACIAN, f, nlev, dtype, out, workspace, nullptr, stream);
}

atlas_status atlas_nabla_get_shape(atlas_mesh_t mesh, atlas_op op, int32_t nlev,
                                   atlas_dtype dtype, atlas_launch *out) {
  if (!mesh || !mesh->store || !out) return fail(ATLAS_EINVAL, "NULL argument");
  if (op < ATLAS_OP_GRADIENT || op > ATLAS_OP_LAPLACIAN) return fail(ATLAS_EINVAL, "unknown operator");
  if (dtype != ATLAS_F32 && dtype != ATLAS_F64) return fail(ATLAS_EINVAL, "unknown dtype");
  if (nlev < 1) return fail(ATLAS_EINVAL, "nlev must be >= 1");
  const MeshStore &m = *mesh->store;
  LaunchShape s = shape_from(nullptr, m, op, nlev, dtype);
  if (op == ATLAS_OP_LAPLACIAN) {
    if (lapl_fused_runs(m, nlev, dtype, s)) {
      s.variant = ATLAS_VARIANT_FUSED;
    } else {
      // two passes: report the gradient pass (the divergence pass is what
      // ATLAS_OP_DIVERGENCE reports)
      if (s.variant == ATLAS_VARIANT_FUSED || s.per_pass)
        s = shape_from(nullptr, m, ATLAS_OP_GRADIENT, nlev, dtype);
    }
  }
  out->variant = s.variant;
  out->block_threads = s.block;
  out->nodes_per_block = s.nodes_per_block;
  out->level_chunk = s.level_chunk;
  out->blocks_per_cu = s.blocks_per_cu;
  out->level_vec = s.level_vec;
  return ATLAS_OK;
}

size_t atlas_laplacian_workspace_bytes(atlas_mesh_t mesh, int32_t nlev, atlas_dtype dtype) {
  if (!mesh || !mesh->store || nlev < 1) return 0;
  return lapl_ws_bytes(*mesh->store, nlev, dtype);
}

atlas_status atlas_bandwidth_probe(const void *in, void *out, int64_t n, int32_t elem_bytes,
                                   hipStream_t stream) {
  if (!in || !out) return fail(ATLAS_EINVAL, "NULL pointer");
  if (n < 2 || (n & 1)) return fail(ATLAS_EINVAL, "n must be even and >= 2");
  if (elem_bytes != 4 && elem_bytes != 8) return fail(ATLAS_EINVAL, "elem_bytes must be 4 or 8");
  if (!aligned(in, 16) || !aligned(out, 16)) return fail(ATLAS_EINVAL, "pointers must be 16-byte aligned");
  if (overlap(in, (size_t)n * elem_bytes, out, (size_t)2 * n * elem_bytes))
    return fail(ATLAS_EINVAL, "input and output overlap");
  return bandwidth_probe(in, out, n, elem_bytes, stream);
}

size_t atlas_flux_workspace_bytes(atlas_mesh_t mesh, atlas_op op, int32_t nlev,
                                  atlas_dtype dtype) {
  if (!mesh || !mesh->store || nlev < 1) return 0;
  return flux_ws_bytes(*mesh->store, op, nlev, dtype);
}

}  // extern "C"

namespace atlasx {
LaunchShape shape_from(const atlas_launch *l, const MeshStore &m, atlas_op op, int nlev,
                       atlas_dtype dt) {
  LaunchShape s = default_shape(m, op, nlev, dt);
  if (!l || l->variant == ATLAS_VARIANT_AUTO) {
    // an autotuned shape for this (op, dtype, nlev), if any (for the
    // Laplacian: the fused form, or the two passes each with its own shape)
    MeshStore &ms = const_cast<MeshStore &>(m);
    std::lock_guard<std::mutex> g(ms.tune_mu);
    auto it = ms.tuned.find(TuneKey{(int)op, (int)dt, nlev});
    if (it != ms.tuned.end()) s = it->second;
  }
  if (l && l->variant != ATLAS_VARIANT_AUTO) {
    s.per_pass = 0;  // an explicit shape serves both Laplacian passes
    s.variant = l->variant;
    s.block = l->block_threads;
    s.nodes_per_block = l->nodes_per_block;
    s.level_chunk = l->level_chunk;
    s.blocks_per_cu = l->blocks_per_cu;
    s.level_vec = l->level_vec;
  }
  return s;
}
}  // namespace atlasx
