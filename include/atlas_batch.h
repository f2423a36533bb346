/*
 * atlas_batch.h -- many operator applications in one launch sequence.
 *
 * The paper groups fields into a FieldSet (Section 4.6) and applies the
 * Nabla operators of Section 4.7 field by field.  Here a batch is a table
 * of work items -- (mesh, operator, nlev, input, output) with uneven meshes
 * and level counts.  Small items are executed by one persistent kernel that
 * pulls work units (item, block of nodes, phase) from per-XCD queues; no
 * workgroup ever waits for another.  The Laplacian's second pass
 * (divergence of the gradient) is a second launch of the same kernel after
 * the first (two graph nodes: the launch order is the dependency).  Items
 * large enough to fill the device alone (nnodes * nlev >= solo_min_elems)
 * run after it as their own launches with their own (tuned) shapes.  The
 * whole sequence can be captured once in a hipGraph and replayed.
 *
 * Every item's output is bitwise identical to the same operator launched
 * alone (same per-element operation sequence).
 */
#ifndef ATLAS_BATCH_H
#define ATLAS_BATCH_H

#include "atlas_nabla.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct atlas_batch_s *atlas_batch_t;

/* One work item.  Device pointers owned by the caller; scalar fields
 * [V][nlev], vector fields [V][nlev][2] (as for the single operators).
 * workspace: Laplacian only, [V][nlev][2] elements of the batch dtype, or
 * NULL to let the batch own one. */
typedef struct {
  atlas_mesh_t mesh;
  int32_t op;        /* atlas_op */
  int32_t nlev;
  const void *in;
  void *out;
  void *workspace;
} atlas_work_item;

typedef struct {
  int32_t dtype;         /* atlas_dtype shared by all items               */
  int32_t use_graph;     /* 1: capture the launch in a hipGraph at build  */
  int32_t autotune;      /* 1: time candidate tile shapes per item class
                            with the items' own buffers at build time    */
  int32_t block_threads; /* persistent workgroup size, 0 = 256           */
  int32_t blocks_per_cu; /* 0 = as many as fit (occupancy)               */
  int64_t solo_min_elems; /* items with nnodes * nlev at or above this run
                             as their own launches (0 = 2^22; -1 = never) */
} atlas_batch_config;

typedef struct {
  int32_t nitems, nunits, grid_blocks, block_threads;
  int32_t graph;           /* 1 if replayed from a hipGraph              */
  int32_t form_column;     /* items using the column tile form           */
  int32_t form_flat;       /* items using the flat tile form             */
  size_t owned_bytes;      /* device memory owned by the batch           */
  int32_t solo_items;      /* items run as their own launches            */
} atlas_batch_info;

/* Validate every item (as the single operators do), choose a tile shape
 * per item class (autotuned if cfg->autotune), build the unit queues and
 * the device tables, and capture the graph.  `stream` is used for
 * autotuning and graph capture only.
 * Errors: ATLAS_EINVAL (bad item, mixed dtypes, n < 1), ATLAS_ENOMEM,
 * ATLAS_EDEVICE. */
atlas_status atlas_batch_build(const atlas_work_item *items, int32_t n,
                               const atlas_batch_config *cfg, hipStream_t stream,
                               atlas_batch_t *out);

/* Enqueue the whole batch on `stream` (graph replay or direct launch). */
atlas_status atlas_batch_launch(atlas_batch_t batch, hipStream_t stream);

/* Wait for the batch's last launch; ATLAS_EDEVICE if it failed. */
atlas_status atlas_batch_check(atlas_batch_t batch);

atlas_status atlas_batch_get_info(atlas_batch_t batch, atlas_batch_info *info);
atlas_status atlas_batch_free(atlas_batch_t batch);

/* Autotuner for the single operators: times the candidate launch shapes
 * (column / flat / sweep forms, block sizes, tile sizes) for this
 * (mesh, op, dtype, nlev) on the given buffers, remembers the fastest in
 * the mesh (later calls with the same key use it) and returns it.  The
 * Laplacian is tuned pass by pass (gradient into `workspace` -- device,
 * atlas_laplacian_workspace_bytes() bytes -- or a temporary one when NULL,
 * then its divergence into `out`), and the two tuned passes are timed
 * against the fused one-pass form (ATLAS_VARIANT_FUSED, 1024 and 768
 * threads) where the mesh has its plan.  Later Laplacian calls run the
 * winner: *best is the fused shape if it won, else the gradient pass's
 * shape; *best_ms the winner's time (both passes summed).
 * Errors: as atlas_nabla_apply; ATLAS_ENOMEM if the temporary workspace
 * cannot be allocated. */
atlas_status atlas_autotune(atlas_mesh_t mesh, atlas_op op, const void *in, int32_t nlev,
                            atlas_dtype dtype, void *out, void *workspace,
                            hipStream_t stream, atlas_launch *best, float *best_ms);

#ifdef __cplusplus
}
#endif
#endif /* ATLAS_BATCH_H */
