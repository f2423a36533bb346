// batch.cpp -- batched persistent launch (atlas_batch.h) and the autotuner.
//
// A batch is the device-side analogue of applying the Nabla operators
// (Section 4.7) to every field of a FieldSet (Section 4.6) in one go: one
// persistent kernel pulls (item, block of nodes, phase) units from per-XCD
// queues; the launch can be captured once in a hipGraph and replayed.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <new>
#include <vector>

#include "atlas_batch.h"
#include "internal.h"

namespace atlasx {

atlas_status check_call(atlas_mesh_t mesh, atlas_op op, const void *in, int nlev,
                        atlas_dtype dt, void *out);
atlas_status apply(atlas_mesh_t mesh, atlas_op op, const void *in, int32_t nlev,
                   atlas_dtype dt, void *out, void *workspace, const atlas_launch *shape,
                   hipStream_t stream);

// Untuned batch shape of an item (op: the OP code of its first pass); the
// column form's lane width follows the single-launch default.
ItemShape heuristic_shape(int op, atlas_dtype dt, int nlev) {
  if (nlev >= 48) return {FORM_COLUMN, 16, (dt == ATLAS_F32 && op == 0) ? 1 : 0};
  const int npb = std::max(16, std::min(1024, 4096 / std::max(1, nlev)));
  return {FORM_FLAT, npb, 0};
}

constexpr int kMinColumnUnit = 64;  // positions per column-form unit (16 per wavefront)

// Units of a batch: every item's nodes in blocks of its npb, each item's
// blocks split into 8 contiguous runs, one per queue (XCD); pass 0 holds
// every unit of phase 0, pass 1 the divergence units of the Laplacians.
// qbeg[9 * pass + x] is where queue x of that pass starts in `units`.
void plan_units(const std::vector<BatchItem> &items, const std::vector<ItemShape> &shapes,
                std::vector<BatchUnit> &units, std::vector<int> &qbeg) {
  std::vector<std::vector<BatchUnit>> q0(8), q1(8);
  for (size_t i = 0; i < items.size(); ++i) {
    // a unit costs the workgroup an atomic and a barrier: column-form units
    // hold at least kMinColumnUnit positions (the tile size tuned for a
    // single launch may be smaller)
    const int V = items[i].m.V;
    const int npb = std::max(1, shapes[i].form == FORM_COLUMN
                                    ? std::max(shapes[i].npb, kMinColumnUnit)
                                    : shapes[i].npb);
    const int nu = (V + npb - 1) / npb;
    for (int x = 0; x < 8; ++x) {
      const int u0 = (int)((int64_t)nu * x / 8), u1 = (int)((int64_t)nu * (x + 1) / 8);
      for (int u = u0; u < u1; ++u) {
        const BatchUnit un{(int)i, u * npb, std::min(V, (u + 1) * npb), 0};
        q0[x].push_back(un);
        if (items[i].lapl) q1[x].push_back({(int)i, un.p0, un.p1, 1});
      }
    }
  }
  units.clear();
  qbeg.assign(18, 0);
  for (int pass = 0; pass < 2; ++pass) {
    auto &q = pass ? q1 : q0;
    for (int x = 0; x < 8; ++x) {
      qbeg[9 * pass + x] = (int)units.size();
      units.insert(units.end(), q[x].begin(), q[x].end());
    }
    qbeg[9 * pass + 8] = (int)units.size();
  }
}

namespace {

// An item that runs as its own launch (large enough to fill the device).
struct SoloItem {
  const MeshStore *m;
  atlas_op op;
  const void *in;
  int nlev;
  void *out, *ws;
  LaunchShape sh;
};

struct Batch {
  atlas_dtype dtype = ATLAS_F32;
  int nitems = 0, nunits = 0, grid = 0, block = 256;
  int nbatched = 0;             // items in the persistent launch
  std::vector<SoloItem> solo;   // the others, launched after it in order
  bool two_pass = false;
  int form_column = 0, form_flat = 0;
  BatchItem *d_items = nullptr;
  BatchUnit *d_units = nullptr;
  int *d_qbeg = nullptr;  // [18]: queue starts of pass 0, then of pass 1
  int *d_heads = nullptr; // [16]: queue heads of pass 0, then of pass 1
  std::vector<void *> owned;  // batch-owned Laplacian workspaces
  size_t owned_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  hipEvent_t last = nullptr;
  // solo items on parallel branches: side streams joined back by events
  // (used when no item writes memory another item touches)
  static constexpr int kSide = 3;
  int nside = 0;
  hipStream_t side[kSide] = {};
  hipEvent_t fork = nullptr, join[kSide] = {};
  std::vector<int> solo_lane;   // branch of each solo item (0: the stream)
  ~Batch() {
    for (int i = 0; i < kSide; ++i) {
      if (side[i]) (void)hipStreamDestroy(side[i]);
      if (join[i]) (void)hipEventDestroy(join[i]);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    if (last) (void)hipEventDestroy(last);
    for (void *p : owned) (void)hipFree(p);
    if (d_items) (void)hipFree(d_items);
    if (d_units) (void)hipFree(d_units);
    if (d_qbeg) (void)hipFree(d_qbeg);
    if (d_heads) (void)hipFree(d_heads);
  }
};

// Enqueues a batch on `st`: the persistent launch of the small items (two
// launches if any is a Laplacian), then every solo item in item order.
atlas_status enqueue(Batch &b, hipStream_t st) {
  if (b.nbatched > 0) {
    atlas_status s = launch_batch(b.dtype, b.d_items, b.d_units, b.d_qbeg, b.d_qbeg + 9,
                                  b.two_pass, b.d_heads, b.grid, b.block, st);
    if (s != ATLAS_OK) return s;
  }
  if (b.nside == 0) {
    for (const SoloItem &x : b.solo) {
      atlas_status s = launch_op(*x.m, x.op, b.dtype, x.in, x.nlev, x.out, x.ws, x.sh, st);
      if (s != ATLAS_OK) return s;
    }
    return ATLAS_OK;
  }
  ATLASX_HIP(hipEventRecord(b.fork, st));
  for (int i = 0; i < b.nside; ++i) ATLASX_HIP(hipStreamWaitEvent(b.side[i], b.fork, 0));
  for (size_t k = 0; k < b.solo.size(); ++k) {
    const SoloItem &x = b.solo[k];
    const int lane = b.solo_lane[k];
    atlas_status s = launch_op(*x.m, x.op, b.dtype, x.in, x.nlev, x.out, x.ws, x.sh,
                               lane ? b.side[lane - 1] : st);
    if (s != ATLAS_OK) return s;
  }
  for (int i = 0; i < b.nside; ++i) {
    ATLASX_HIP(hipEventRecord(b.join[i], b.side[i]));
    ATLASX_HIP(hipStreamWaitEvent(st, b.join[i], 0));
  }
  return ATLAS_OK;
}

// Whether any item writes memory that another item reads or writes (then
// the solo items keep their order on one stream).
bool items_overlap(const atlas_work_item *items, int n, atlas_dtype dt) {
  if (n > 4096) return true;
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  struct R { uintptr_t a, b; int item; bool write; };
  std::vector<R> r;
  for (int i = 0; i < n; ++i) {
    const atlas_work_item &it = items[i];
    const size_t V = (size_t)it.mesh->store->d.V, L = (size_t)it.nlev;
    const bool vin = it.op == ATLAS_OP_DIVERGENCE || it.op == ATLAS_OP_CURL;
    const size_t ib = V * L * w * (vin ? 2 : 1), ob = V * L * w * (it.op == ATLAS_OP_GRADIENT ? 2 : 1);
    r.push_back({(uintptr_t)it.in, (uintptr_t)it.in + ib, i, false});
    r.push_back({(uintptr_t)it.out, (uintptr_t)it.out + ob, i, true});
    if (it.op == ATLAS_OP_LAPLACIAN && it.workspace)
      r.push_back({(uintptr_t)it.workspace, (uintptr_t)it.workspace + V * L * w * 2, i, true});
  }
  for (size_t x = 0; x < r.size(); ++x)
    for (size_t y = x + 1; y < r.size(); ++y)
      if (r[x].item != r[y].item && (r[x].write || r[y].write) && r[x].a < r[y].b && r[y].a < r[x].b)
        return true;
  return false;
}

}  // namespace

// Times one launch shape (median of three after a warm-up) on `st`.
static float time_shape(atlas_mesh_t mesh, atlas_op op, const void *in, int nlev,
                        atlas_dtype dt, void *out, void *ws, const atlas_launch &l,
                        hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (apply(mesh, op, in, nlev, dt, out, ws, &l, st) != ATLAS_OK) return -1.0f;
  float best = 1e30f;
  for (int r = 0; r < 3; ++r) {
    (void)hipEventRecord(e0, st);
    if (apply(mesh, op, in, nlev, dt, out, ws, &l, st) != ATLAS_OK) return -1.0f;
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0f;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms);
  }
  return best;
}

static std::vector<atlas_launch> candidates(const MeshStore &m, atlas_op op, atlas_dtype dt,
                                            int nlev) {
  std::vector<atlas_launch> c;
  auto add = [&](int v, int b, int npb, int kc, int bpc, int lv) {
    c.push_back({v, b, npb, kc, bpc, lv});
  };
  // the built-in shape first, so that a tuned shape is never one that lost
  // to it
  {
    const LaunchShape d = default_shape(m, op, nlev, dt);
    add(d.variant, d.block, d.nodes_per_block, d.level_chunk, d.blocks_per_cu, d.level_vec);
  }
  if (nlev >= 32) {
    for (int lv : {0, 1, 2, 3}) add(ATLAS_VARIANT_COLUMN, 256, 16, 0, 0, lv);
    add(ATLAS_VARIANT_COLUMN, 256, 0, 0, 0, 0);
    add(ATLAS_VARIANT_COLUMN, 128, 16, 0, 0, 0);
    add(ATLAS_VARIANT_COLUMN, 256, 4, 0, 0, 0);
    add(ATLAS_VARIANT_COLUMN, 256, 0, 0, 4, 0);
    if (m.d.sweep_ok) {
      // wave-specialised (blocks_per_cu 0) and register-staged (1) sweeps
      for (int b : {768, 1024}) add(ATLAS_VARIANT_SWEEP, b, 0, 0, 0, 0);
      for (int b : {512, 768, 1024}) add(ATLAS_VARIANT_SWEEP, b, 0, 0, 1, 0);
      add(ATLAS_VARIANT_SWEEP, 768, 0, 0, 1, 2);
    }
  }
  const int fl = std::max(16, std::min(1024, 4096 / std::max(1, nlev)));
  add(ATLAS_VARIANT_FLAT, 256, fl, 0, 0, 0);
  add(ATLAS_VARIANT_FLAT, 256, std::max(1, fl / 4), 0, 0, 0);
  add(ATLAS_VARIANT_FLAT, 256, 0, 0, 0, 0);
  add(ATLAS_VARIANT_FLAT, 256, 32, 0, 0, 0);
  add(ATLAS_VARIANT_FLAT, 512, 64, 0, 0, 0);
  add(ATLAS_VARIANT_FLAT, 1024, 128, 0, 0, 0);
  if (nlev < 32) {
    add(ATLAS_VARIANT_COLUMN, 256, 16, 0, 0, 0);
    add(ATLAS_VARIANT_COLUMN, 256, 16, 0, 0, 1);
  }
  return c;
}

// Times every candidate for one operator on the given buffers and remembers
// the fastest in the mesh.
static atlas_status tune_one(atlas_mesh_t mesh, atlas_op op, const void *in, int nlev,
                             atlas_dtype dt, void *out, hipStream_t st, atlas_launch *best,
                             float *best_ms) {
  MeshStore &m = *mesh->store;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ATLASX_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ATLAS_EDEVICE, "hipEventCreate failed");
  }
  float bt = 1e30f;
  atlas_launch bl{};
  for (const atlas_launch &c : candidates(m, op, dt, nlev)) {
    const float t = time_shape(mesh, op, in, nlev, dt, out, nullptr, c, st, e0, e1);
    if (t >= 0.0f && t < bt) {
      bt = t;
      bl = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (bt >= 1e29f) return fail(ATLAS_EDEVICE, "no launch shape ran");
  {
    std::lock_guard<std::mutex> g(m.tune_mu);
    LaunchShape sh;
    sh.variant = bl.variant;
    sh.block = bl.block_threads;
    sh.nodes_per_block = bl.nodes_per_block;
    sh.level_chunk = bl.level_chunk;
    sh.blocks_per_cu = bl.blocks_per_cu;
    sh.level_vec = bl.level_vec;
    m.tuned[TuneKey{(int)op, (int)dt, nlev}] = sh;
  }
  *best = bl;
  *best_ms = bt;
  return ATLAS_OK;
}

// The Laplacian is tuned pass by pass (gradient into the workspace, then
// its divergence); it then runs each pass with that pass's tuned shape.
atlas_status autotune(atlas_mesh_t mesh, atlas_op op, const void *in, int nlev, atlas_dtype dt,
                      void *out, void *ws, hipStream_t st, atlas_launch *best, float *best_ms) {
  atlas_status s = check_call(mesh, op, in, nlev, dt, out);
  if (s != ATLAS_OK) return s;
  atlas_launch bl{};
  float bt = 0.0f;
  if (op != ATLAS_OP_LAPLACIAN) {
    s = tune_one(mesh, op, in, nlev, dt, out, st, &bl, &bt);
  } else {
    const size_t bytes = (size_t)mesh->store->d.V * nlev * 2 * (dt == ATLAS_F64 ? 8 : 4);
    void *grad = ws, *owned = nullptr;
    if (!grad) {
      if (hipMalloc(&owned, bytes) != hipSuccess) return fail(ATLAS_ENOMEM, "autotune workspace");
      grad = owned;
    }
    atlas_launch bd{};
    float td = 0.0f;
    s = tune_one(mesh, ATLAS_OP_GRADIENT, in, nlev, dt, grad, st, &bl, &bt);
    if (s == ATLAS_OK) s = tune_one(mesh, ATLAS_OP_DIVERGENCE, grad, nlev, dt, out, st, &bd, &td);
    bt += td;
    if (s == ATLAS_OK) {
      // the two tuned passes against the fused one-pass form
      MeshStore &m = *mesh->store;
      LaunchShape win;
      win.variant = ATLAS_VARIANT_COLUMN;
      win.per_pass = 1;
      if (m.d.l2_ok) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
          for (int b : {1024, 768}) {
            const atlas_launch c{ATLAS_VARIANT_FUSED, b, 0, 0, 0, 0};
            const float t = time_shape(mesh, op, in, nlev, dt, out, grad, c, st, e0, e1);
            if (t >= 0.0f && t < bt) {
              bt = t;
              bl = c;
              win = LaunchShape();
              win.variant = ATLAS_VARIANT_FUSED;
              win.block = b;
              win.nodes_per_block = 0;
            }
          }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
      }
      std::lock_guard<std::mutex> g(m.tune_mu);
      m.tuned[TuneKey{(int)op, (int)dt, nlev}] = win;
    }
    if (owned) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(owned);
    }
  }
  if (s != ATLAS_OK) return s;
  if (best) *best = bl;
  if (best_ms) *best_ms = bt;
  return ATLAS_OK;
}

// The form a batch uses for an item class after autotuning: the fastest of
// the column / flat candidates with their tile sizes and, for the column
// form, the automatic lane width or one level per lane.
static ItemShape tuned_item_shape(atlas_mesh_t mesh, atlas_op op, const void *in, int nlev,
                                  atlas_dtype dt, void *out, void *ws, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int opc = op == ATLAS_OP_DIVERGENCE ? 1 : op == ATLAS_OP_CURL ? 2 : 0;
  ItemShape best = heuristic_shape(opc, dt, nlev);
  if (hipEventCreate(&e0) != hipSuccess) return best;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return best;
  }
  float bt = 1e30f;
  const int fl = std::max(16, std::min(1024, 4096 / std::max(1, nlev)));
  const ItemShape cands[] = {{FORM_COLUMN, 8, 0},  {FORM_COLUMN, 32, 0},
                             {FORM_COLUMN, 8, 1},  {FORM_COLUMN, 32, 1},
                             {FORM_FLAT, fl, 0},   {FORM_FLAT, std::max(1, fl / 4), 0}};
  for (const ItemShape &c : cands) {
    const atlas_launch l{c.form == FORM_COLUMN ? ATLAS_VARIANT_COLUMN : ATLAS_VARIANT_FLAT, 256,
                         c.npb, 0, 0, c.level_vec};
    const float t = time_shape(mesh, op, in, nlev, dt, out, ws, l, st, e0, e1);
    if (t >= 0.0f && t < bt) {
      bt = t;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

}  // namespace atlasx

using namespace atlasx;

struct atlas_batch_s {
  Batch *b;
};

extern "C" {

atlas_status atlas_autotune(atlas_mesh_t mesh, atlas_op op, const void *in, int32_t nlev,
                            atlas_dtype dtype, void *out, void *workspace, hipStream_t stream,
                            atlas_launch *best, float *best_ms) {
  return autotune(mesh, op, in, nlev, dtype, out, workspace, stream, best, best_ms);
}

atlas_status atlas_batch_build(const atlas_work_item *items, int32_t n,
                               const atlas_batch_config *cfg, hipStream_t stream,
                               atlas_batch_t *out) {
  if (!out) return fail(ATLAS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!items || n < 1) return fail(ATLAS_EINVAL, "a batch needs at least one item");
  if (n > (1 << 20)) return fail(ATLAS_EINVAL, "too many items");
  const atlas_batch_config c = cfg ? *cfg : atlas_batch_config{ATLAS_F32, 0, 0, 0, 0, 0};
  if (c.dtype != ATLAS_F32 && c.dtype != ATLAS_F64) return fail(ATLAS_EINVAL, "unknown dtype");
  const int block = c.block_threads ? c.block_threads : 256;
  if (block < 64 || block > 256 || (block & 63))
    return fail(ATLAS_EINVAL, "block_threads must be 64, 128, 192 or 256");
  if (c.blocks_per_cu < 0 || c.blocks_per_cu > 32 || c.solo_min_elems < -1)
    return fail(ATLAS_EINVAL, "bad batch configuration");
  const int64_t solo_min = c.solo_min_elems == 0 ? ((int64_t)1 << 22) : c.solo_min_elems;
  const atlas_dtype dt = (atlas_dtype)c.dtype;
  const size_t w = dt == ATLAS_F64 ? 8 : 4;
  // validate every item before allocating anything
  for (int i = 0; i < n; ++i) {
    const atlas_work_item &it = items[i];
    atlas_status s = check_call(it.mesh, (atlas_op)it.op, it.in, it.nlev, dt, it.out);
    if (s != ATLAS_OK) return s;
    if (it.op == ATLAS_OP_LAPLACIAN && it.workspace &&
        ((uintptr_t)it.workspace % (2 * w)) != 0)
      return fail(ATLAS_EINVAL, "workspace misaligned");
  }
  Batch *b = new (std::nothrow) Batch();
  if (!b) return fail(ATLAS_ENOMEM, "out of host memory");
  b->dtype = dt;
  b->nitems = n;
  b->block = block;
  auto bail = [&](atlas_status s) {
    delete b;
    return s;
  };
  std::vector<BatchItem> h_items;
  std::vector<ItemShape> h_shapes;
  std::map<std::tuple<const void *, int, int>, ItemShape> shapes;
  std::map<std::tuple<const void *, int, int>, bool> tuned;  // solo classes
  for (int i = 0; i < n; ++i) {
    const atlas_work_item &it = items[i];
    MeshStore &m = *it.mesh->store;
    BatchItem bi;
    std::memset(&bi, 0, sizeof(bi));
    bi.m = m.d;
    bi.lapl = it.op == ATLAS_OP_LAPLACIAN ? 1 : 0;
    bi.op = it.op == ATLAS_OP_DIVERGENCE ? 1 : it.op == ATLAS_OP_CURL ? 2 : 0;
    bi.nlev = it.nlev;
    bi.in = it.in;
    bi.out = it.out;
    bi.ws = it.workspace;
    // a Laplacian's gradient workspace, owned by the batch when the item
    // brings none (the fused one-pass form needs none)
    auto own_ws = [&]() -> atlas_status {
      if (bi.ws) return ATLAS_OK;
      void *p = nullptr;
      const size_t bytes = (size_t)m.d.V * it.nlev * 2 * w;
      if (hipMalloc(&p, bytes) != hipSuccess) return fail(ATLAS_ENOMEM, "batch workspace");
      b->owned.push_back(p);
      b->owned_bytes += bytes;
      bi.ws = p;
      return ATLAS_OK;
    };
    const auto key = std::make_tuple((const void *)&m, it.op, it.nlev);
    if (solo_min >= 0 && (int64_t)m.d.V * it.nlev >= solo_min) {
      // its own launch, with the shape a single call would use (tuned
      // first if asked; the tuner stores the winner in the mesh and brings
      // its own workspace when given none)
      if (c.autotune && !tuned[key]) {
        atlas_status s = autotune(it.mesh, (atlas_op)it.op, it.in, it.nlev, dt, it.out, bi.ws,
                                  stream, nullptr, nullptr);
        if (s != ATLAS_OK) return bail(s);
        tuned[key] = true;
      }
      LaunchShape sh = shape_from(nullptr, m, (atlas_op)it.op, it.nlev, dt);
      if (sh.variant == ATLAS_VARIANT_FLUX) sh = default_shape(m, (atlas_op)it.op, it.nlev, dt);
      if (bi.lapl && !lapl_fused_runs(m, it.nlev, dt, sh)) {
        atlas_status s = own_ws();
        if (s != ATLAS_OK) return bail(s);
      }
      b->solo.push_back({&m, (atlas_op)it.op, it.in, it.nlev, it.out, bi.ws, sh});
      continue;
    }
    if (bi.lapl) {
      atlas_status s = own_ws();
      if (s != ATLAS_OK) return bail(s);
    }
    auto f = shapes.find(key);
    ItemShape sh;
    if (f != shapes.end()) {
      sh = f->second;
    } else {
      sh = c.autotune ? tuned_item_shape(it.mesh, (atlas_op)(bi.lapl ? ATLAS_OP_GRADIENT : it.op),
                                         it.in, it.nlev, dt, bi.lapl ? bi.ws : it.out, nullptr,
                                         stream)
                      : heuristic_shape(bi.lapl ? 0 : bi.op, dt, it.nlev);
      shapes[key] = sh;
    }
    bi.form = sh.form;
    bi.level_vec = sh.level_vec;
    (sh.form == FORM_COLUMN ? b->form_column : b->form_flat) += 1;
    h_items.push_back(bi);
    h_shapes.push_back(sh);
    b->two_pass = b->two_pass || bi.lapl;
  }
  b->nbatched = (int)h_items.size();
  std::vector<BatchUnit> h_units;
  std::vector<int> qbeg;
  plan_units(h_items, h_shapes, h_units, qbeg);
  b->nunits = (int)h_units.size();
  const size_t nb = std::max<size_t>(1, h_items.size());
  if (hipMalloc(&b->d_items, sizeof(BatchItem) * nb) != hipSuccess ||
      hipMalloc(&b->d_units, sizeof(BatchUnit) * std::max<size_t>(1, h_units.size())) != hipSuccess ||
      hipMalloc(&b->d_qbeg, sizeof(int) * 18) != hipSuccess ||
      hipMalloc(&b->d_heads, sizeof(int) * 16) != hipSuccess)
    return bail(fail(ATLAS_ENOMEM, "batch tables"));
  b->owned_bytes += sizeof(BatchItem) * nb + sizeof(BatchUnit) * h_units.size() + 4 * (18 + 16);
  if ((!h_items.empty() && hipMemcpy(b->d_items, h_items.data(), sizeof(BatchItem) * h_items.size(),
                                     hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(b->d_units, h_units.data(), sizeof(BatchUnit) * h_units.size(),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_qbeg, qbeg.data(), sizeof(int) * 18, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(ATLAS_EDEVICE, "batch table upload"));
  const int bpc = c.blocks_per_cu ? c.blocks_per_cu : batch_blocks_per_cu(dt, block);
  // a full persistent grid, or fewer workgroups when there are few units
  b->grid = std::min(std::max(8, (device_cu_count() * bpc + 7) / 8 * 8),
                     std::max(8, (b->nunits + 7) / 8 * 8));
  if (hipEventCreateWithFlags(&b->last, hipEventDisableTiming) != hipSuccess)
    return bail(fail(ATLAS_EDEVICE, "event"));
  // solo items on parallel branches, largest first onto the least loaded
  // (by nnodes * nlev), when the items are independent
  if (b->solo.size() > 1 && !items_overlap(items, n, dt)) {
    b->nside = (int)std::min<size_t>(Batch::kSide, b->solo.size() - 1);
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
      return bail(fail(ATLAS_EDEVICE, "event"));
    for (int i = 0; i < b->nside; ++i)
      if (hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess)
        return bail(fail(ATLAS_EDEVICE, "side stream"));
    std::vector<size_t> order(b->solo.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    auto cost = [&](size_t k) { return (int64_t)b->solo[k].m->d.V * b->solo[k].nlev; };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost(x) > cost(y); });
    std::vector<int64_t> load(b->nside + 1, 0);
    b->solo_lane.assign(b->solo.size(), 0);
    for (size_t k : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->solo_lane[k] = l;
      load[l] += cost(k);
    }
  }
  if (c.use_graph) {
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(ATLAS_EDEVICE, "capture stream"));
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bail(fail(ATLAS_EDEVICE, "hipStreamBeginCapture"));
    atlas_status s = enqueue(*b, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (s != ATLAS_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return bail(s != ATLAS_OK ? s : fail(ATLAS_EDEVICE, "hipStreamEndCapture"));
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
      return bail(fail(ATLAS_EDEVICE, "hipGraphInstantiate"));
  }
  atlas_batch_t h = new (std::nothrow) atlas_batch_s{b};
  if (!h) return bail(fail(ATLAS_ENOMEM, "out of host memory"));
  *out = h;
  return ATLAS_OK;
}

atlas_status atlas_batch_launch(atlas_batch_t batch, hipStream_t stream) {
  if (!batch || !batch->b) return fail(ATLAS_EINVAL, "batch is NULL");
  Batch &b = *batch->b;
  if (b.exec) {
    ATLASX_HIP(hipGraphLaunch(b.exec, stream));
  } else {
    atlas_status s = enqueue(b, stream);
    if (s != ATLAS_OK) return s;
  }
  ATLASX_HIP(hipEventRecord(b.last, stream));
  return ATLAS_OK;
}

atlas_status atlas_batch_check(atlas_batch_t batch) {
  if (!batch || !batch->b) return fail(ATLAS_EINVAL, "batch is NULL");
  ATLASX_HIP(hipEventSynchronize(batch->b->last));
  return ATLAS_OK;
}

atlas_status atlas_batch_get_info(atlas_batch_t batch, atlas_batch_info *info) {
  if (!batch || !batch->b || !info) return fail(ATLAS_EINVAL, "NULL argument");
  const Batch &b = *batch->b;
  info->nitems = b.nitems;
  info->nunits = b.nunits;
  info->grid_blocks = b.grid;
  info->block_threads = b.block;
  info->graph = b.exec ? 1 : 0;
  info->form_column = b.form_column;
  info->form_flat = b.form_flat;
  info->owned_bytes = b.owned_bytes;
  info->solo_items = (int32_t)b.solo.size();
  return ATLAS_OK;
}

atlas_status atlas_batch_free(atlas_batch_t batch) {
  if (!batch) return ATLAS_OK;
  if (batch->b && batch->b->last) (void)hipEventSynchronize(batch->b->last);
  delete batch->b;
  delete batch;
  return ATLAS_OK;
}

}  // extern "C"
