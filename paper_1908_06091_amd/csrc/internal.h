// internal.h -- shared declarations of the MI355X nabla library (not part of
// the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "atlas_nabla.h"

namespace atlasx {

// ---------------------------------------------------------------- errors
atlas_status fail(atlas_status code, const std::string &msg);
atlas_status hip_fail(hipError_t err, const char *what);
#define ATLASX_HIP(call)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::atlasx::hip_fail(e_, #call); \
  } while (0)

// ------------------------------------------------------- host-side mesh
struct HostMesh {
  int N = 0;
  double radius = 1.0;
  std::vector<int32_t> nx;
  std::vector<int64_t> ring_off;
  std::vector<double> lon, lat, cos_lat;
  std::vector<int32_t> edge2node;
  std::vector<int64_t> node2edge_ptr;
  std::vector<int32_t> node2edge;
  std::vector<int8_t> node2edge_sign;
  std::vector<double> dual_volumes, dual_normals;
  std::vector<int32_t> pole_edges;
  std::vector<double> pole_normals;
  std::vector<int32_t> tri, quad;  // element blocks
  atlas_mesh_desc desc{};
  void fill_desc();
};

int build_octahedral(int N, double R, HostMesh &h);
int build_reduced_gaussian(const std::vector<int32_t> &nx, double R, HostMesh &h);
int build_grid(const std::vector<int32_t> &nx, const std::vector<double> *lat, bool shifted,
               bool quads, double R, HostMesh &h);

// ------------------------------------------------------ device mesh store
// All "position" arrays follow the processing order: the nodes re-ordered
// into tiles (bands of parallels x longitude sectors) so that a tile's
// neighbours were touched by the tiles just before it.
constexpr uint32_t kPoleBit = 0x80000000u;
constexpr int kIncPad = 8;               // incidence arrays carry one extra group
constexpr int32_t kLrefPole = 1 << 30;  // sweep reference of a pole edge
constexpr int kGRefs = 8;               // references per gradient node (two-ring plan)
constexpr int kDefaultBand = 32;   // parallels per band of the processing order
constexpr int kDefaultWidth = 32;  // nodes per sector of a band's widest parallel

// One processing position, packed for a single scalar load.
struct __align__(32) PosRec {
  int32_t node, r0, r1, selfslot;
  double alpha, beta;
};

struct DevMesh {
  int32_t V = 0;          // nodes
  int32_t E = 0;          // mesh edges
  int32_t npole = 0;      // pole edges
  int32_t ntiles = 0;     // tiles in the processing order
  const int32_t *perm = nullptr;     // [V]   node at position p
  const int32_t *rowp = nullptr;     // [V+1] incidence range of position p
  const int32_t *nbr = nullptr;      // [I]   neighbour node | kPoleBit
  const double2 *S = nullptr;        // [I]   signed dual normal (s S_lon, s S_lat)
  const int32_t *inc_edge = nullptr; // [I]   flux slot (E + k for pole edge k)
  const double *alpha = nullptr;     // [V]   R / V_i          (by position)
  const double *beta = nullptr;      // [V]   R cos(lat_i)/V_i (by position)
  const double *coslat = nullptr;    // [V]   cos(lat)         (by node id)
  const int32_t *tile_ptr = nullptr; // [ntiles+1] position range of a tile
  const PosRec *pos = nullptr;       // [V]   packed position records
  const int32_t *e2n = nullptr;      // [E+npole][2] endpoints (flux kernel)
  const double2 *eS = nullptr;       // [E+npole] unsigned normals; pole: (0, sigma dlon0)
  // parallel-sweep plan: per tile, the parallels it touches (its own and
  // one above / below), each as a segment of consecutive nodes
  int32_t maxdeg = 0;                // longest incidence row
  int32_t mindeg = 0;                // fewest mesh (non-pole) incidences of a row
  int32_t sweep_ok = 0;              // plan valid for this mesh
  int32_t segmax = 0;                // longest segment (nodes)
  const int32_t *tile_seg = nullptr; // [ntiles+1] segment range of a tile
  const int4 *seg = nullptr;         // {ring offset, ring size, first index, length}
  const int2 *seg_pos = nullptr;     // owned positions of the segment [lo, hi)
  const int32_t *selfslot = nullptr; // [V]  slot of position p in its segment
  const int32_t *lref = nullptr;     // [I]  ((dq + 1) << 16) | slot, plus
                                     //      kLrefPole for a pole edge
  const double *ncos = nullptr;      // [I]  cos(lat) of the incidence's neighbour
  const double *vol = nullptr;       // [V]  dual volume V_i (by position; diagnostics)
  // two-ring plan of the fused Laplacian: per tile a window of parallels,
  // each with an f-run (field), a g-run (gradients formed) and own positions
  int32_t l2_ok = 0;                 // plan valid for this mesh
  int32_t l2_fmax = 0, l2_gmax = 0;  // longest f-run / g-run
  const int32_t *l2_tile_seg = nullptr; // [ntiles+1] window range of a tile
  const int4 *l2_fseg = nullptr;     // {ring offset, ring size, f first, f length}
  const int4 *l2_gseg = nullptr;     // {g first, g length, first g record, 0}
  const int2 *l2_seg_pos = nullptr;  // own positions on the parallel [lo, hi)
  const int4 *l2_gnode = nullptr;    // per g record {row start, row length, f self slot, position}
  const int32_t *l2_glref = nullptr; // [kGRefs] per g record: references into f-runs
  const int32_t *l2_lref = nullptr;  // [I] references of own positions into g-runs
  const int32_t *l2_lself = nullptr; // [V] slot of position p in its g-run
  int32_t l2_pmax = 0;               // most own positions of a tile on one parallel
  const int4 *l2_ggeo = nullptr;     // packed gradient-node records (device-built)
  const int4 *l2_lgeo = nullptr;     // packed own-position records (device-built)
  const int4 *sgeo = nullptr;        // packed per-position sweep geometry (device-built)
};

// ------------------------------------------------------------- kernels
struct MeshStore;

struct LaunchShape {
  int variant = ATLAS_VARIANT_COLUMN;
  int block = 256;
  int nodes_per_block = 0;  // 0 = the mesh's tiles
  int level_chunk = 0;      // column form: levels per unit, 0 = all
  int blocks_per_cu = 0;    // > 0: persistent wave-cyclic grid
  int level_vec = 0;        // column form: levels per lane, 0 = auto
  int per_pass = 0;         // Laplacian: each pass takes its built-in shape
};

// ------------------------------------------------------------- batches
enum { FORM_COLUMN = 0, FORM_FLAT = 1 };

struct BatchItem {       // device table entry of a batch
  DevMesh m;
  int32_t op;            // OP code of a single pass (Laplacian: see lapl)
  int32_t lapl;          // 1: gradient into ws (phase 0), divergence (phase 1)
  int32_t nlev;
  int32_t form;          // FORM_COLUMN / FORM_FLAT
  int32_t level_vec;     // column form, phase 0: as atlas_launch::level_vec
  int32_t level_vec1;    // column form, phase 1 (divergence of a Laplacian)
  int32_t pad[2];
  const void *in;
  void *out;
  void *ws;
};

struct BatchUnit {
  int32_t item, p0, p1, phase;
};

atlas_status launch_batch(atlas_dtype dt, const BatchItem *items, const BatchUnit *units,
                          const int *qbeg0, const int *qbeg1, bool two_pass, int *heads,
                          int grid, int block, hipStream_t st);
int batch_blocks_per_cu(atlas_dtype dt, int block);
atlas_status launch_fill(int *p, int n, int value, hipStream_t st);

// Tile shape of an item inside a batch: the form and positions per unit.
struct ItemShape {
  int form, npb, level_vec;
};
ItemShape heuristic_shape(int op, atlas_dtype dt, int nlev);
void plan_units(const std::vector<BatchItem> &items, const std::vector<ItemShape> &shapes,
                std::vector<BatchUnit> &units, std::vector<int> &qbeg);

struct TuneKey {
  int op, dtype, nlev;
  bool operator<(const TuneKey &o) const {
    return op != o.op ? op < o.op : dtype != o.dtype ? dtype < o.dtype : nlev < o.nlev;
  }
};

// Source side of a remap (atlas_remap.h): the parallels of a mesh
// triangulated strip by strip by the library's rule, first point of every
// parallel at lon 0.  ok == 0 for any other mesh.
struct RemapSource {
  int ok = 0;
  int32_t nrings = 0;
  const int64_t *ring_off = nullptr;  // device [nrings+1]
  const double *ring_lat = nullptr;   // device [nrings]
};

// True if the description's edges are exactly those of the strip-by-strip
// triangulation of its parallels `off` (see atlas_remap.h), its parallels
// have constant, strictly decreasing latitudes and their longitudes start
// at 0 and increase below 2 pi.
bool zipper_conforming(const atlas_mesh_desc *d, const std::vector<int64_t> &off);

struct MeshStore {
  DevMesh d;
  int device = 0;
  RemapSource rs;
  const double *node_lon = nullptr;  // device [V], by node id
  const double *node_lat = nullptr;  // device [V], by node id
  int64_t nincid = 0;
  int32_t nrings = 0, max_degree = 0;
  // most nodes a sweep kernel addresses through one buffer resource (the
  // longest parallel of a mesh with a sweep plan, else one column): the
  // byte offsets inside it are 32-bit
  int64_t max_run = 1;
  // most nodes one workgroup's unit of work holds (the largest tile, and
  // at least the 1024 nodes of a batch unit): its element counters are
  // 32-bit
  int64_t max_tile = 1024;
  size_t bytes = 0;
  std::vector<void *> allocations;
  // internal Laplacian / flux workspace, grown on demand
  std::mutex ws_mu;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int serve_refs = 0;
  double geometry_bytes = 0.0;
  // scales of the derivatives in the computational plane (built on the
  // first call that needs them)
  double radius = 1.0;
  std::mutex comp_mu;
  bool comp_ready = false;
  DevMesh dcomp;
  // autotuned launch shapes, keyed by (op, dtype, nlev)
  std::mutex tune_mu;
  std::map<TuneKey, LaunchShape> tuned;
  ~MeshStore();
};

int device_cu_count();

// Whether fields of `nlev` levels fit the mesh's 32-bit offsets (else the
// reason in *why), and the most levels that do.
bool levels_fit(const MeshStore &m, int64_t nlev, std::string *why);
int64_t max_levels(const MeshStore &m);

atlas_status launch_op(const MeshStore &m, atlas_op op, atlas_dtype dt,
                       const void *in, int nlev, void *out, void *ws,
                       const LaunchShape &shape, hipStream_t s);
size_t flux_ws_bytes(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt);
atlas_status derive_scales(MeshStore &m, const double *vol_by_pos,
                           const double *cos_by_pos, double radius);
atlas_status bandwidth_probe(const void *in, void *out, int64_t n, int elem, hipStream_t st);
LaunchShape default_shape(const MeshStore &m, atlas_op op, int nlev, atlas_dtype dt);
// True if a Laplacian launched with `sh` runs the fused one-pass form
// (which needs no workspace) rather than falling back to the two passes.
bool lapl_fused_runs(const MeshStore &ms, int nlev, atlas_dtype dt, const LaunchShape &sh);
// (d phi / d lon, d phi / d lat) of a scalar field, [V][nlev][2].
atlas_status gradient_lonlat(MeshStore &ms, atlas_dtype dt, const void *in, int nlev, void *out,
                             hipStream_t st);
// Divergence and curl of one vector field (one read of the field).
atlas_status launch_div_curl(const MeshStore &ms, atlas_dtype dt, const void *in, int nlev,
                             void *out_div, void *out_curl, hipStream_t st);
// Packs the fused Laplacian's geometry records of a mesh with a two-ring
// plan of `ngrec` gradient records (after derive_scales).
atlas_status pack_lapl_geometry(MeshStore &m, int64_t ngrec);
// Packs the wave-specialised sweep's per-position geometry (after
// derive_scales; a mesh with a sweep plan).
atlas_status pack_sweep_geometry(MeshStore &m);
// The shape a call with launch `l` (NULL: tuned, else built-in) runs with.
LaunchShape shape_from(const atlas_launch *l, const MeshStore &m, atlas_op op, int nlev,
                       atlas_dtype dt);

// ------------------------------------------------------------- remaps
// One target of a remap: its three source nodes and weights (the fourth
// slot pads the record to 48 bytes; its weight is 0 and its node valid).
struct __align__(16) RemapRec {
  int32_t i[4];
  double w[4];
};

struct RemapPlan {
  int device = 0;
  int64_t nsrc = 0, nt = 0, touched = 0, npolar = 0;
  RemapRec *rec = nullptr;  // device [nt]
  size_t bytes = 0;
  int serve_refs = 0;       // servers holding the remap
  ~RemapPlan() {
    if (rec) (void)hipFree(rec);
  }
};

// Enqueues out[t][c] = sum_k w_k in[i_k][c] for every target t and column c
// (arguments already validated).
atlas_status remap_launch(const RemapPlan &p, const void *in, int32_t ncol, atlas_dtype dt,
                          void *out, hipStream_t st);

}  // namespace atlasx

// the opaque mesh handle of the C ABI
struct atlas_mesh_s {
  atlasx::MeshStore *store;
};

// the opaque remap handle of the C ABI
struct atlas_remap_s {
  atlasx::RemapPlan *plan;
};
