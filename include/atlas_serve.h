/*
 * atlas_serve.h -- a request server for the nabla operators.
 *
 * Meshes stay resident on the device (Section 5: data structures live on
 * the accelerator and are copied once); requests (mesh, operator, dtype,
 * levels, field) arrive at any time.  Besides the four operators a request
 * can remap a field from one grid to another (atlas_remap.h) with weights
 * registered once.  A scheduler thread admits requests in
 * arrival order while their device footprint fits an HBM budget, and each
 * time one of its launch slots (HIP streams) frees up it launches the
 * admitted requests: small ones merged into one persistent batch launch
 * (continuous batching, see atlas_batch.h), large ones alone.  Results are
 * bitwise identical to the same request run alone.
 *
 * Footprint of a request while in the server: its input, its output and, for
 * the Laplacian, its [V][nlev][2] workspace (none for a Laplacian that
 * launches alone in the fused one-pass form).  A request whose footprint alone
 * exceeds the budget is rejected at submit with ATLAS_ENOMEM.  A server-owned
 * output stays in the footprint until atlas_serve_release.  Server-owned
 * outputs and workspaces are ranges of one arena reserved at creation, so
 * serving makes no device allocation; a request whose ranges do not fit the
 * arena yet waits at the head of the queue, as one over the budget does.
 *
 * Ordering: the server launches on streams of its own that do not wait for
 * any other stream.  A request's input and caller-owned output must be ready
 * (no pending device work on them) when it is submitted, and may be used
 * again once atlas_serve_wait has reported the request finished.
 *
 * Threads: every call may come from any thread; one scheduler thread per
 * server makes all device calls.  Meshes and fields live on the device that
 * was current at atlas_serve_create.
 */
#ifndef ATLAS_SERVE_H
#define ATLAS_SERVE_H

#include "atlas_nabla.h"
#include "atlas_remap.h"

/* Request operator value of a remap (the atlas_op values name the four
 * nabla operators). */
#define ATLAS_SERVE_OP_REMAP 4

#ifdef __cplusplus
extern "C" {
#endif

typedef struct atlas_server_s *atlas_server_t;

typedef struct {
  size_t hbm_budget_bytes;  /* bound on the summed footprint in flight; a
                               device server reserves this much device memory
                               at creation as the arena its outputs and
                               workspaces are carved from                    */
  int32_t nstreams;         /* launch slots (1..16)                          */
  int32_t max_batch;        /* most requests merged into one launch (>= 1)   */
  int64_t batch_max_elems;  /* requests with nnodes*nlev above this launch
                               alone (0 = default 2^22)                     */
  int32_t simulate;         /* 1: no device work at all -- launches complete
                               after bytes / sim_bytes_per_us microseconds
                               (host-side tests of the scheduler)            */
  double sim_bytes_per_us;
  int32_t fail_alloc_every; /* fault injection: every k-th server allocation
                               fails (0 = never)                             */
} atlas_serve_config;

typedef struct {
  int32_t mesh_id;  /* from atlas_serve_register_mesh; for a remap, the id
                       from atlas_serve_register_remap                    */
  int32_t op;       /* atlas_op, or ATLAS_SERVE_OP_REMAP: input
                       [nsource][nlev], output [ntarget][nlev] (nlev: the
                       columns per node, 2 x levels for a vector field)   */
  int32_t dtype;    /* atlas_dtype                                        */
  int32_t nlev;
  const void *in;   /* device input, caller-owned, valid until done      */
  void *out;        /* device output, or NULL: the server allocates it;
                       hand it back with atlas_serve_release              */
} atlas_request;

typedef struct {
  int32_t status;     /* atlas_status of the request: ATLAS_OK, ATLAS_ENOMEM
                         (allocation failed), ATLAS_EDEVICE (launch failed),
                         ATLAS_ECANCELLED                                 */
  int32_t batch_size; /* requests launched together with this one         */
  void *out;          /* where the result is                              */
  double queue_us;    /* submit -> launch                                 */
  double run_us;      /* launch -> completion observed                    */
  double total_us;    /* submit -> completion observed                    */
} atlas_result;

typedef struct {
  uint64_t submitted, completed, rejected, failed, cancelled;
  uint64_t launches, batched_launches;
  size_t inflight_bytes, peak_inflight_bytes;
} atlas_serve_stats;

/* Starts a server on the current device (a simulation server touches no
 * device).  Errors: ATLAS_EINVAL (a config field out of range), ATLAS_ENOMEM
 * (the budget's arena or the batch tables cannot be allocated),
 * ATLAS_EDEVICE. */
atlas_status atlas_serve_create(const atlas_serve_config *cfg, atlas_server_t *out);

/* Make a resident mesh known to the server (the server keeps it from being
 * freed until atlas_serve_destroy).  Errors: ATLAS_EINVAL. */
atlas_status atlas_serve_register_mesh(atlas_server_t srv, atlas_mesh_t mesh,
                                       int32_t *mesh_id);

/* Simulation servers only: a mesh of `nnodes` nodes that exists on paper. */
atlas_status atlas_serve_register_sim_mesh(atlas_server_t srv, int64_t nnodes,
                                           int32_t *mesh_id);

/* Make a remap's weights known to the server; remap requests then name
 * the returned id.  The remap cannot be freed (ATLAS_EBUSY) until
 * atlas_serve_destroy.  Remaps always launch alone (no batching).
 * Errors: ATLAS_EINVAL (NULL argument, a simulation server, the remap on
 * another device). */
atlas_status atlas_serve_register_remap(atlas_server_t srv, atlas_remap_t remap,
                                        int32_t *remap_id);

/* Simulation servers only: a remap from `nsource` to `ntarget` nodes that
 * exists on paper. */
atlas_status atlas_serve_register_sim_remap(atlas_server_t srv, int64_t nsource,
                                            int64_t ntarget, int32_t *remap_id);

/* Non-blocking.  Errors: ATLAS_EINVAL (unknown mesh or remap, bad op/dtype/nlev,
 * NULL input), ATLAS_ENOMEM (footprint above the whole budget),
 * ATLAS_ESTATE (server shutting down). */
atlas_status atlas_serve_submit(atlas_server_t srv, const atlas_request *req,
                                uint64_t *ticket);

/* Wait for a request: ATLAS_OK with *res filled (res->status says whether
 * the request itself succeeded), ATLAS_ETIMEOUT if it is not done after
 * timeout_us microseconds (< 0: wait forever), ATLAS_EINVAL for an unknown
 * ticket. */
atlas_status atlas_serve_wait(atlas_server_t srv, uint64_t ticket, int64_t timeout_us,
                              atlas_result *res);

/* Cancel a request that has not been launched yet (ATLAS_ESTATE if it
 * already has). */
atlas_status atlas_serve_cancel(atlas_server_t srv, uint64_t ticket);

/* Forget a finished request; frees its output if the server allocated it
 * (stream-ordered on the server's stream: reads of that output by the caller
 * must have completed).  Errors: ATLAS_EINVAL (unknown ticket), ATLAS_ESTATE
 * (not finished). */
atlas_status atlas_serve_release(atlas_server_t srv, uint64_t ticket);

atlas_status atlas_serve_get_stats(atlas_server_t srv, atlas_serve_stats *st);

/* Drain every admitted request, cancel queued ones that cannot be admitted
 * any more (their footprint waits for releases), stop the scheduler, free
 * server memory (the arena included: server-owned outputs not yet released
 * become invalid). */
atlas_status atlas_serve_destroy(atlas_server_t srv);

#ifdef __cplusplus
}
#endif
#endif /* ATLAS_SERVE_H */
