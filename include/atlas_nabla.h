/*
 * atlas_nabla.h -- C ABI of the MI355X (gfx950) library for the edge-based
 * median-dual finite-volume nabla operators on the octahedral reduced
 * Gaussian grid.
 *
 * Paper anchors (Atlas, ESCAPE D1.3, arXiv:1908.06091):
 *   grid       Section 4.2.3.5, Section 4.2.3.7 and Listing 6
 *   mesh       Section 4.3 (nodes, cells, edges; Eq. 1; block and
 *              irregular connectivity tables; vertical levels extruded)
 *   fields     Section 4.5 and Figure 31 (NodeColumns: a node's vertical
 *              column is contiguous, layout [node][level]); Listing 12
 *              (gradient output has two variables)
 *   operators  Section 4.7, Figure 33 and Listing 12 (fvm::Method and
 *              Nabla: gradient, divergence, curl, Laplacian)
 *   device     Section 5 (connectivity and fields resident on the device,
 *              copied to it once)
 *   C layer    Section 4.1 and Figure 3 (an opaque handle to a native object
 *              driven through plain C functions)
 *
 * Conventions shared by every entry point:
 *   - Every function returns an atlas_status; ATLAS_OK (0) is success.  On
 *     failure nothing has been enqueued and atlas_last_error() returns a
 *     thread-local message describing the first problem found.
 *   - Field pointers are DEVICE pointers owned by the caller.  Scalar
 *     fields are [nnodes][nlev]; vector fields are [nnodes][nlev][2] with
 *     the two components interleaved (zonal, meridional).  Pointers must be
 *     aligned to the element size and input and output must not overlap.
 *   - Operator calls only enqueue work on `stream` (0 = the null stream);
 *     they never synchronise the host.  Buffers must stay valid until the
 *     stream has passed the call.  An asynchronous device fault surfaces at
 *     the caller's next synchronisation.
 *   - Every operator is deterministic: each node sums its own edges in a
 *     fixed order without atomics, so repeated calls give identical bits,
 *     whatever the launch shape.
 */
#ifndef ATLAS_NABLA_H
#define ATLAS_NABLA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ATLAS_OK = 0,
  ATLAS_EINVAL = -1,   /* invalid argument or malformed mesh description  */
  ATLAS_ENOMEM = -2,   /* host or device allocation failed / over budget  */
  ATLAS_EDEVICE = -3,  /* a HIP runtime call failed                        */
  ATLAS_EBUSY = -4,    /* resource in use (e.g. freeing a registered mesh) */
  ATLAS_ESTATE = -5,   /* call not valid in the object's current state    */
  ATLAS_ETIMEOUT = -6, /* a bounded wait expired                           */
  ATLAS_ECANCELLED = -7 /* the request was cancelled before it ran         */
} atlas_status;

typedef enum { ATLAS_F32 = 0, ATLAS_F64 = 1 } atlas_dtype;

typedef enum {
  ATLAS_OP_GRADIENT = 0,
  ATLAS_OP_DIVERGENCE = 1,
  ATLAS_OP_CURL = 2,
  ATLAS_OP_LAPLACIAN = 3
} atlas_op;

typedef struct atlas_mesh_s *atlas_mesh_t;

/*
 * Host description of a median-dual mesh (all pointers are HOST pointers,
 * read only; FP64 geometry in the (lon, lat) plane, radians).
 *
 *   nnodes, lon, lat, cos_lat   node coordinates and cos(lat), [nnodes]
 *   nrings, ring_off            optional: nodes grouped by parallel,
 *                               ring_off[nrings+1]; 0 / NULL = derive the
 *                               parallels from runs of equal latitude
 *   nedges, edge2node           [nedges][2], edge2node[e][0] < [e][1]
 *   node2edge_ptr, node2edge    CSR node -> edge, [nnodes+1] and [2*nedges],
 *                               each row in ascending edge id (this is the
 *                               summation order of every node)
 *   node2edge_sign              [2*nedges], +1 if the node is edge2node[e][0],
 *                               -1 if it is edge2node[e][1]
 *   dual_volumes                [nnodes] physical dual volumes
 *                               V_i = R^2 cos(lat_i) A_i
 *   dual_normals                [nedges][2] dual-face normal (S_lon, S_lat),
 *                               oriented from edge2node[e][0] to [e][1]
 *   npole_edges, pole_edges     [npole_edges][2] pole edges: pairs of nodes
 *                               on the first or last parallel half-way round
 *   pole_normals                [npole_edges] lat component of the pole-face
 *                               normal carried by each pole edge (+-2pi/nx)
 *   radius                      sphere radius R
 *   ntriangles, triangles       optional element blocks (Section 4.3,
 *   nquads, quads               Figure 27: one block per element type):
 *                               [ntriangles][3] and [nquads][4] node ids,
 *                               counter-clockwise in (lon, lat).  Filled by
 *                               the library's generators; not read by
 *                               atlas_mesh_upload (0 / NULL allowed)
 */
typedef struct {
  int64_t nnodes;
  const double *lon, *lat, *cos_lat;
  int32_t nrings;
  const int64_t *ring_off;
  int64_t nedges;
  const int32_t *edge2node;
  const int64_t *node2edge_ptr;
  const int32_t *node2edge;
  const int8_t *node2edge_sign;
  const double *dual_volumes;
  const double *dual_normals;
  int64_t npole_edges;
  const int32_t *pole_edges;
  const double *pole_normals;
  double radius;
  int64_t ntriangles;
  const int32_t *triangles;
  int64_t nquads;
  const int32_t *quads;
} atlas_mesh_desc;

/* Sizes of an uploaded mesh. */
typedef struct {
  int64_t nnodes, nedges, nincidences, npole_edges, ntiles;
  int32_t nrings, max_degree;
  size_t device_bytes;      /* device memory held by the mesh store        */
  double geometry_bytes_per_call; /* mesh bytes one operator pass reads   */
  int64_t max_levels;       /* most levels a field on this mesh may have:  */
                            /* byte offsets inside one parallel of columns */
                            /* and element counters of one tile are 32-bit */
} atlas_mesh_info;

/* ---------------------------------------------------------------------- */
/* Host problem setup (Section 4.2.3.7 grid, Section 4.3 mesh generator,   */
/* Section 4.7 fvm::Method geometry).                                      */
/* ---------------------------------------------------------------------- */

/* Build the description of grid O<N> (2N Gaussian parallels with
 * 20 + 4j points, mirrored) triangulated between consecutive parallels,
 * with its median-dual geometry on a sphere of radius `radius`.  The arrays
 * are owned by the library; release them with atlas_mesh_desc_free.
 * Errors: ATLAS_EINVAL for N < 1, N > 8192 or radius <= 0; ATLAS_ENOMEM. */
atlas_status atlas_mesh_desc_octahedral(int32_t N, double radius,
                                        atlas_mesh_desc **out);
/* The same for any reduced Gaussian grid (Section 4.2.3.7): nrings = 2N
 * parallels at the Gaussian latitudes of degree 2N, nx[j] points on
 * parallel j (first at lon 0, equispaced), triangulated between consecutive
 * parallels; the regular Gaussian grid F<N> of Section 4.2.3.6 has
 * nx[j] = 4N.  The polar parallels' nodes pair up across the pole, so those
 * two parallels need an even count.  nx: host array, read during the call.
 * Errors: ATLAS_EINVAL (nrings odd or outside [2, 16384], an nx outside
 * [4, 2^20], an odd polar parallel, radius <= 0, grid too large),
 * ATLAS_ENOMEM. */
atlas_status atlas_mesh_desc_reduced_gaussian(int32_t nrings, const int32_t *nx, double radius,
                                              atlas_mesh_desc **out);
/* Flags of atlas_mesh_desc_grid. */
#define ATLAS_MESH_SHIFTED 1 /* every point half a spacing east of lon 0 + i dlon */
#define ATLAS_MESH_QUADS 2   /* strips between parallels of equal counts become
                                quadrilaterals; the others stay triangles */

/* Any grid of parallels: nx[j] points on parallel j (first point at lon 0,
 * or half a spacing east of it with ATLAS_MESH_SHIFTED, which needs equal
 * counts on all parallels), at latitude lat[j] in radians (strictly
 * decreasing, inside (-pi/2, pi/2): no point on a pole), or at the Gaussian
 * latitudes of degree nrings when lat is NULL (nrings even).  With
 * ATLAS_MESH_QUADS a strip between two parallels of equal counts is meshed
 * with quadrilaterals (U_a, L_a, L_a+1, U_a+1), the blocked quadrilaterals
 * of Section 4.3, and the others with triangles as above: the description's
 * element blocks then hold both types (Figure 27), and the median-dual
 * cells of the quadrilaterals are built about their centres (the mean of
 * the four corners).  The regular longitude-latitude grids of Section
 * 4.2.3.8 without points on the poles: SLAT<nlon>x<nlat> is nx[j] = nlon,
 * lat[j] = pi/2 - (j + 1/2) pi / nlat; S<nlon>x<nlat> adds
 * ATLAS_MESH_SHIFTED.  Errors: as atlas_mesh_desc_reduced_gaussian, plus
 * ATLAS_EINVAL for latitudes out of order or range, unknown flags, or
 * ATLAS_MESH_SHIFTED with unequal counts. */
atlas_status atlas_mesh_desc_grid(int32_t nrings, const int32_t *nx, const double *lat,
                                  int32_t flags, double radius, atlas_mesh_desc **out);
atlas_status atlas_mesh_desc_free(atlas_mesh_desc *desc);

/* ---------------------------------------------------------------------- */
/* Device mesh store (Section 5: connectivity and geometry resident on     */
/* the device, copied once).                                               */
/* ---------------------------------------------------------------------- */

/* Validate `desc`, copy it to the current device (synchronous) and derive
 * the per-node scales.  The host arrays may be freed on return.  The mesh
 * belongs to the library until atlas_mesh_free.
 * Errors: ATLAS_EINVAL (malformed description: counts, index ranges, CSR
 * order, signs, non-positive volumes, non-finite geometry), ATLAS_ENOMEM,
 * ATLAS_EDEVICE. */
atlas_status atlas_mesh_upload(const atlas_mesh_desc *desc, atlas_mesh_t *out);

/* Processing layout of the device store: the nodes are visited in tiles,
 * each tile one longitude sector (about `sector_nodes` nodes of its widest
 * parallel) of a band of `band_rings` consecutive parallels, so that a
 * tile's neighbours were touched just before it.  Zero fields take the
 * library defaults.  Results do not depend on the layout. */
typedef struct {
  int32_t band_rings;
  int32_t sector_nodes;
} atlas_mesh_layout;

/* atlas_mesh_upload with an explicit layout (NULL = defaults).
 * Errors: as atlas_mesh_upload; ATLAS_EINVAL for a negative field. */
atlas_status atlas_mesh_upload_ex(const atlas_mesh_desc *desc,
                                  const atlas_mesh_layout *layout,
                                  atlas_mesh_t *out);

/* Convenience: atlas_mesh_desc_octahedral + atlas_mesh_upload. */
atlas_status atlas_mesh_create_octahedral(int32_t N, double radius,
                                          atlas_mesh_t *out);

/* Release the device store.  ATLAS_EBUSY if a server still holds it. */
atlas_status atlas_mesh_free(atlas_mesh_t mesh);
atlas_status atlas_mesh_get_info(atlas_mesh_t mesh, atlas_mesh_info *info);

/* ---------------------------------------------------------------------- */
/* Operators (Section 4.7, Figure 33, Listing 12).                          */
/*   gradient   f [V][nlev]       -> out [V][nlev][2] (zonal, meridional)   */
/*   divergence (u,v) [V][nlev][2] -> out [V][nlev]                          */
/*   curl       (u,v) [V][nlev][2] -> out [V][nlev] (radial component)       */
/*   laplacian  f [V][nlev]       -> out [V][nlev], = divergence(gradient)  */
/* dtype ATLAS_F64: FP64 fields and arithmetic.  dtype ATLAS_F32: FP32      */
/* fields, FP64 geometry, FP32 edge terms with a compensated (Kahan) node   */
/* sum, final scaling in FP64.                                              */
/* Errors (nothing enqueued): ATLAS_EINVAL for a NULL or misaligned pointer,*/
/* nlev < 1 or above the mesh's max_levels (atlas_mesh_info), overlapping   */
/* input/output, unknown dtype; ATLAS_EDEVICE if the launch fails.          */
/* ---------------------------------------------------------------------- */
atlas_status atlas_nabla_gradient(atlas_mesh_t mesh, const void *f, int32_t nlev,
                                  atlas_dtype dtype, void *out, hipStream_t stream);
atlas_status atlas_nabla_divergence(atlas_mesh_t mesh, const void *uv,
                                    int32_t nlev, atlas_dtype dtype, void *out,
                                    hipStream_t stream);
atlas_status atlas_nabla_curl(atlas_mesh_t mesh, const void *uv, int32_t nlev,
                              atlas_dtype dtype, void *out, hipStream_t stream);
/* The derivatives in the computational (lon, lat) plane instead of the
 * physical components: out[i][k] = (d f/d lon, d f/d lat) =
 * (R cos(lat_i) grad_lon, R grad_lat), both the node's edge sums divided by
 * its dual area in the (lon, lat) plane.  Same layout, arguments and errors
 * as atlas_nabla_gradient (plus ATLAS_ENOMEM: the first call on a mesh
 * allocates 48 bytes per node of scales). */
atlas_status atlas_nabla_gradient_lonlat(atlas_mesh_t mesh, const void *f, int32_t nlev,
                                         atlas_dtype dtype, void *out, hipStream_t stream);
/* Divergence and curl of the same (u, v) field in one pass (Section 4.7:
 * both operators of one Nabla object applied to one field): the field is
 * read once and each output is bitwise the result of its own entry point.
 * out_div and out_curl: [V][nlev] each, caller-owned, disjoint from each
 * other and from uv.  Short columns (nlev < 48) and meshes outside the
 * level-vector form run the two operators one after the other.  Errors: as
 * atlas_nabla_divergence, and ATLAS_EINVAL for overlapping outputs. */
atlas_status atlas_nabla_div_curl(atlas_mesh_t mesh, const void *uv, int32_t nlev,
                                  atlas_dtype dtype, void *out_div, void *out_curl,
                                  hipStream_t stream);
/* workspace: device buffer of atlas_laplacian_workspace_bytes() bytes, or
 * NULL to use a workspace the mesh keeps (grown on first use with
 * hipMalloc; calls that share it on different streams must be ordered by
 * the caller).  The fused one-pass form (the FP64 default on large meshes,
 * ATLAS_VARIANT_FUSED) writes no gradient and uses no workspace. */
atlas_status atlas_nabla_laplacian(atlas_mesh_t mesh, const void *f, int32_t nlev,
                                   atlas_dtype dtype, void *out, void *workspace,
                                   hipStream_t stream);
size_t atlas_laplacian_workspace_bytes(atlas_mesh_t mesh, int32_t nlev,
                                       atlas_dtype dtype);

/* ---------------------------------------------------------------------- */
/* Launch shapes.  Every shape gives bitwise-identical results.            */
/* ---------------------------------------------------------------------- */
typedef enum {
  ATLAS_VARIANT_AUTO = 0,   /* autotuned choice (or built-in default)      */
  ATLAS_VARIANT_COLUMN = 1, /* one wavefront per node, lanes over levels   */
  ATLAS_VARIANT_FLAT = 2,   /* lanes over flattened (node, level) pairs    */
  ATLAS_VARIANT_FLUX = 3,   /* two kernels: edge fluxes into an [E][nlev]
                               buffer (EdgeColumns-like), then the gather  */
  ATLAS_VARIANT_SWEEP = 4,  /* one workgroup per (tile, level chunk) walks
                               its band parallel by parallel, keeping three
                               consecutive parallels' columns in LDS       */
  ATLAS_VARIANT_FUSED = 5   /* Laplacian only: one pass over a two-ring
                               plan -- the workgroup forms the gradients of
                               its tile and their neighbours in LDS and
                               their divergence at once, reading the field
                               once and writing no gradient to memory.  On
                               meshes without the plan (or rows outside 4..6
                               incidences) the two passes run instead.  No
                               workspace is needed.                         */
} atlas_variant;

typedef struct {
  int32_t variant;          /* atlas_variant                                */
  int32_t block_threads;    /* 64, 128, 256, 512 or 1024                    */
  int32_t nodes_per_block;  /* column/flat: processing positions per block;
                               0 = the mesh's tiles.  Fused form,
                               wave-specialised: 4 or 5 = slots of its ring
                               of field runs (4: each run is loaded one step
                               before use instead of one and a half, and a
                               longer level chunk fits in LDS); 0 = five, or
                               four where five would need one more level
                               chunk; other values run the register-staged
                               form                                         */
  int32_t level_chunk;      /* column: levels per unit of work (1..64); the
                               units run chunk by chunk over the whole mesh
                               so a parallel's columns are still cached when
                               the next parallel reads them; 0 = all levels
                               in one unit.  Sweep and fused forms: at most
                               this many levels per workgroup (0 = as many
                               as LDS holds)                                */
  int32_t blocks_per_cu;    /* column/flat: > 0 launches a persistent grid of
                               this many workgroups per compute unit; each
                               XCD's wavefronts then walk that XCD's share of
                               the processing order together, one position
                               per wavefront per step, so the set of columns
                               in flight stays small enough for the L2;
                               0 = one workgroup per tile.  Sweep form: 0 =
                               wave-specialised workgroups (two waves load
                               the next parallels straight into LDS, the
                               others compute and store; 16-byte lane
                               vectors, at least 256 threads, level_vec 0
                               or the 16-byte width); > 0 = every wave
                               stages loads through registers.  Fused
                               form: 0 = wave-specialised (four wavefronts
                               load the next parallels straight into LDS,
                               the others compute and store; at least 320
                               threads, 16-byte lanes); 1..3 = every wave
                               stages loads through registers, each lane
                               taking that many lane vectors of a node  */
  int32_t level_vec;        /* column, sweep and fused forms: levels per
                               lane.  0 = the level-vector kernels at the
                               automatic width: FP64 16-byte lanes (2
                               levels of a scalar, 1 of a vector); FP32 the
                               width (1..4 levels, at most 32 bytes per
                               lane) that needs the fewest level slots per
                               lane, then the fewest loads (3 at 137
                               levels); 2..4 = that width (capped at 32
                               bytes); 1 = the one-level-per-lane kernels.
                               Lanes past the column make no memory access.
                               The level-vector kernels need a mesh of
                               degree 4..6 and at most 256 lane vectors per
                               column; otherwise the one-level-per-lane
                               kernels run.                                */
} atlas_launch;

/* Apply `op` with an explicit launch shape (tests, autotuner).  For
 * ATLAS_VARIANT_FLUX, `workspace` must hold atlas_flux_workspace_bytes();
 * a two-pass Laplacian with ATLAS_VARIANT_FLUX keeps the gradient at the
 * start of the workspace and the fluxes after it, so it needs the SUM
 * atlas_laplacian_workspace_bytes() + atlas_flux_workspace_bytes(mesh,
 * ATLAS_OP_LAPLACIAN, ...).  workspace == NULL: the mesh's own workspace,
 * grown to what the call needs.  shape == NULL is the same as the named
 * entry points. */
atlas_status atlas_nabla_apply(atlas_mesh_t mesh, atlas_op op, const void *in,
                               int32_t nlev, atlas_dtype dtype, void *out,
                               void *workspace, const atlas_launch *shape,
                               hipStream_t stream);
size_t atlas_flux_workspace_bytes(atlas_mesh_t mesh, atlas_op op, int32_t nlev,
                                  atlas_dtype dtype);

/* The launch shape the named entry point of `op` runs with `nlev` levels and
 * `dtype` on this mesh (the autotuned shape if one is stored, else the
 * built-in one).  For the Laplacian, variant ATLAS_VARIANT_FUSED means the
 * one-pass form runs; otherwise the two passes run and `out` is the
 * gradient pass's shape (the divergence pass is what ATLAS_OP_DIVERGENCE
 * reports).  `out`: host struct, written on success.  Errors: ATLAS_EINVAL
 * for a NULL argument, an unknown op or dtype, nlev < 1. */
atlas_status atlas_nabla_get_shape(atlas_mesh_t mesh, atlas_op op, int32_t nlev,
                                   atlas_dtype dtype, atlas_launch *out);

/* Streaming reference with the gradient's byte pattern: reads n elements of
 * `in` and writes each twice into `out` (2n elements), fully coalesced.
 * Used to report the practically reachable HBM bandwidth next to the
 * operators' roofline.  elem_bytes: 4 or 8.  Device pointers, 16-byte
 * aligned, n even.  Errors: ATLAS_EINVAL, ATLAS_EDEVICE. */
atlas_status atlas_bandwidth_probe(const void *in, void *out, int64_t n, int32_t elem_bytes,
                                   hipStream_t stream);

/* Thread-local description of the last failure on this thread. */
const char *atlas_last_error(void);

/* Library version string. */
const char *atlas_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ATLAS_NABLA_H */
