/*
 * atlas_remap.h -- interpolation of nodal fields from one mesh to other
 * points (another grid's nodes, or any list of points).
 *
 * Section 1 of the paper lists remapping / interpolation of fields defined
 * on different grids among the mathematical operations the library offers;
 * it gives no method.  The method implemented: the value at a target point
 * is the piecewise-linear (P1) interpolant of the source field on the
 * source mesh's triangles in the (lon, lat) plane,
 *   out(t) = sum over the three vertices k of the triangle containing t of
 *            w_k(t) * in(vertex k),
 * w_k the barycentric coordinates of t (longitudes unwrapped round t).  A
 * point on the boundary of several triangles takes the first of them in the
 * strip's triangle order.  A target poleward of the first (last) parallel
 * takes the linear interpolant along that parallel at its longitude (two
 * nonzero weights).  Levels are independent (Section 4.3: the mesh is
 * extruded vertically), so one set of weights serves every level.
 *
 * Source meshes: a mesh of parallels triangulated strip by strip as the
 * library's own generators do (atlas_mesh_desc_octahedral,
 * atlas_mesh_desc_reduced_gaussian: between two parallels, the next
 * triangle takes whichever next point lies further west, ties to the
 * parallel with more points, the lower one if counts are equal), with the
 * first point of every parallel at lon 0.  atlas_mesh_upload recognises
 * such meshes; others are refused by atlas_remap_create.
 *
 * Fields are [nnodes][ncol] (ncol values per node: the levels of a scalar,
 * or levels x 2 interleaved components of a vector, each column
 * interpolated on its own), device pointers owned by the caller.
 */
#ifndef ATLAS_REMAP_H
#define ATLAS_REMAP_H

#include "atlas_nabla.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct atlas_remap_s *atlas_remap_t;

typedef struct {
  int64_t nsource;         /* nodes of the source mesh                       */
  int64_t ntarget;         /* target points                                  */
  int64_t nsource_touched; /* source nodes with a nonzero weight             */
  int64_t npolar;          /* targets poleward of the polar parallels        */
  size_t device_bytes;     /* device memory held by the remap                */
  double values_per_column; /* values one column of one apply must move at
                               least: nsource_touched reads + ntarget writes;
                               an apply of ncol columns of w-byte values moves
                               values_per_column * ncol * w + table_bytes   */
  double table_bytes;      /* weight-table bytes one apply reads at least
                              (3 node ids and 3 FP64 weights per target)     */
} atlas_remap_info;

/* Locate `ntarget` points (host arrays lon, lat in radians; lon any finite
 * value, lat in [-pi/2, pi/2]) on the source mesh and store their weights
 * on the device (a location kernel on the current device, which must be the
 * mesh's; synchronous).  The host arrays may be freed on return.  The remap
 * does not refer to the mesh afterwards.
 * Errors: ATLAS_EINVAL (NULL argument, ntarget < 1 or >= 2^31, a
 * non-finite coordinate or a latitude outside [-pi/2, pi/2], a source mesh
 * that is not triangulated between parallels as described above, the mesh
 * on another device), ATLAS_ENOMEM, ATLAS_EDEVICE. */
atlas_status atlas_remap_create(atlas_mesh_t source, int64_t ntarget, const double *lon,
                                const double *lat, atlas_remap_t *out);

/* The same with the nodes of another uploaded mesh as targets (in its node
 * order), taken from that mesh's device store. */
atlas_status atlas_remap_create_to_mesh(atlas_mesh_t source, atlas_mesh_t target,
                                        atlas_remap_t *out);

/* out[t][c] = w0 in[i0][c] + w1 in[i1][c] + w2 in[i2][c] for the ntarget
 * targets and ncol columns, summed in that order.  ATLAS_F64: FP64
 * throughout.  ATLAS_F32: FP32 fields; the weights stay FP64 and the sum is
 * formed in FP64, then rounded once.  in: device [nsource][ncol]; out:
 * device [ntarget][ncol], not overlapping in.  Enqueued on `stream` only.
 * Errors (nothing enqueued): ATLAS_EINVAL (NULL or misaligned pointer,
 * ncol < 1, ntarget * ncol >= 2^40, unknown dtype, overlap), ATLAS_EDEVICE. */
atlas_status atlas_remap_apply(atlas_remap_t remap, const void *in, int32_t ncol,
                               atlas_dtype dtype, void *out, hipStream_t stream);

/* Copy the weights to the host: idx [ntarget][3] source node ids, w
 * [ntarget][3] weights (a polar target's third weight is 0).  Synchronous.
 * Errors: ATLAS_EINVAL (NULL argument), ATLAS_EDEVICE. */
atlas_status atlas_remap_get_weights(atlas_remap_t remap, int32_t *idx, double *w);

atlas_status atlas_remap_get_info(atlas_remap_t remap, atlas_remap_info *info);

/* Release the weights.  Work already enqueued that uses them must have
 * completed. */
atlas_status atlas_remap_free(atlas_remap_t remap);

#ifdef __cplusplus
}
#endif
#endif /* ATLAS_REMAP_H */
