/*
 * atlas_diag.h -- on-device diagnostics of operator results.
 *
 * The discrete divergence and curl of Section 4.7 are built from edge
 * fluxes that enter the two end nodes of every edge with opposite signs, so
 * their volume integrals sum_i V_i div_i and sum_i V_i curl_i vanish up to
 * rounding; the volume integral below checks that on the device.  The error
 * norms compare a result with a reference without copying either to the
 * host.
 *
 * Both reductions are deterministic: fixed partition of the rows, each
 * partial summed in row order, partials summed in partition order, all in
 * FP64.  They are not on the operators' timed path.
 */
#ifndef ATLAS_DIAG_H
#define ATLAS_DIAG_H

#include "atlas_nabla.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[k * ncomp + c] = sum_i V_i * field[i][k][c] over all nodes i, with V_i
 * the dual volume (R^2 cos(lat_i) A_i) of the mesh.  field: device,
 * [nnodes][nlev][ncomp] of `dtype`, ncomp 1 (scalar) or 2 (vector).  out:
 * device, nlev * ncomp doubles, written on `stream`.  A temporary of
 * 1024 * nlev * ncomp doubles is allocated and freed stream-ordered.
 * Errors: ATLAS_EINVAL (NULL or misaligned pointer, nlev < 1, ncomp not 1 or
 * 2, bad dtype), ATLAS_ENOMEM, ATLAS_EDEVICE. */
atlas_status atlas_diag_volume_integral(atlas_mesh_t mesh, const void *field, int32_t nlev,
                                        int32_t ncomp, atlas_dtype dtype, double *out,
                                        hipStream_t stream);

/* The most columns (nlev * ncomp) the variant below takes. */
#define ATLAS_DIAG_NOALLOC_MAX_COLS 512

/* The volume integral above for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, kernels and result bits, but the partials live
 * in one static device array of 1024 * ATLAS_DIAG_NOALLOC_MAX_COLS doubles
 * (4 MiB) that the library holds on every GPU it runs on until the process
 * ends.  No hipMalloc, hipFree or allocating library call is made.  The first
 * call on a device looks up that device's copy of the array (the device that
 * is current, which must be the mesh's).
 * Calls on one GPU share its array: calls that overlap on that GPU (on
 * different streams, or from different threads without ordering) race and
 * may return wrong sums.  Calls ordered on one stream are safe.  Every
 * partial is written before it is read, so nothing carries over between
 * calls.
 * Errors: those of atlas_diag_volume_integral, plus ATLAS_EINVAL when
 * nlev * ncomp exceeds ATLAS_DIAG_NOALLOC_MAX_COLS or the current device is
 * not the mesh's, ATLAS_EDEVICE when the array's address cannot be found. */
atlas_status atlas_diag_volume_integral_noalloc(atlas_mesh_t mesh, const void *field,
                                                int32_t nlev, int32_t ncomp, atlas_dtype dtype,
                                                double *out, hipStream_t stream);

/* Error norms of `got` against `ref`, n rows of ncomp interleaved
 * components (both device arrays, each of its own dtype).  out (device,
 * 4 * ncomp doubles): for component c,
 *   out[4c + 0] = max_i |got - ref|,   out[4c + 1] = sum_i (got - ref)^2,
 *   out[4c + 2] = max_i |ref|,         out[4c + 3] = sum_i ref^2,
 * differences formed in FP64; a NaN in either input makes the affected
 * entries NaN.  Errors: ATLAS_EINVAL (NULL or misaligned pointer, n < 1, ncomp not
 * 1 or 2, bad dtype), ATLAS_ENOMEM, ATLAS_EDEVICE. */
atlas_status atlas_diag_error_norms(const void *got, atlas_dtype got_dtype, const void *ref,
                                    atlas_dtype ref_dtype, int64_t n, int32_t ncomp,
                                    double *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ATLAS_DIAG_H */
