// serve.cpp -- request server for the nabla operators: HBM-budget admission,
// resident meshes, continuous batching over a few HIP streams.
//
// One scheduler thread owns every device call.  Requests queue in arrival
// order; the front one is admitted when its footprint (input + output +
// Laplacian workspace) fits the budget.  Whenever a launch slot (a stream
// with its own batch tables and completion event) is idle, the admitted
// requests are launched on it: a large request alone through the single
// operator path, small ones merged into one persistent batch launch (the
// batch kernel of batch.cpp).  Every launch form computes each output element
// with the same operation sequence, so a result does not depend on what it
// was launched with.
//
// Device memory for outputs and workspaces comes from one arena of the HBM
// budget, reserved at creation: a request's ranges are carved out when it is
// admitted and handed back only after the work that used them has completed
// (a workspace when its request's event has fired, a server-owned output
// when the caller has released it), so reuse needs no stream ordering and
// the steady state makes no hipMalloc or hipFree call (hipFree waits for the
// whole device).  A request whose ranges do not fit the arena yet (it is
// fragmented) waits at the head of the queue like one over the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "atlas_serve.h"
#include "internal.h"

namespace atlasx {

namespace {

using Clock = std::chrono::steady_clock;

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

enum ReqState { QUEUED, ADMITTED, RUNNING, DONE };

struct Req {
  uint64_t ticket = 0;
  atlas_request r{};
  MeshStore *m = nullptr;  // NULL on a simulation server
  RemapPlan *rp = nullptr; // a remap request's weights (NULL when simulated)
  bool remap = false;
  int64_t V = 0;
  size_t in_b = 0, out_b = 0, ws_b = 0;
  size_t out_off = SIZE_MAX, ws_off = SIZE_MAX;  // arena ranges (SIZE_MAX: none)
  LaunchShape sh;      // a large Laplacian's shape, fixed at submit
  bool sh_set = false;
  bool own_out = false;
  bool out_charged = false;  // out_b still counted in flight (a server-owned
                             // output stays counted until it is released)
  void *ws = nullptr;
  int state = QUEUED;
  int status = ATLAS_OK;
  int batch_size = 0;
  int slot = -1;
  Clock::time_point t_sub, t_launch, t_done;
  size_t footprint() const { return in_b + out_b + ws_b; }
};

// A launch slot: one stream, one completion event and the batch tables the
// launch on it reads (device copy plus the pinned staging it is copied from).
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> reqs;
  bool busy = false;
  Clock::time_point sim_done;
  char *d_tab = nullptr, *h_tab = nullptr;
  size_t tab_bytes = 0;
};

struct MeshEntry {
  atlas_mesh_t mesh;  // NULL for a simulated mesh
  int64_t V;
};

struct RemapEntry {
  atlas_remap_t remap;  // NULL for a simulated remap
  int64_t nsrc, nt;
};

constexpr size_t kTabAlign = 256;
size_t align_up(size_t x) { return (x + kTabAlign - 1) / kTabAlign * kTabAlign; }

// Offsets into one device range: best fit over a free list kept sorted by
// offset, neighbours merged when a range comes back.  Sizes are rounded to
// kAlign so every range starts aligned.
struct Arena {
  static constexpr size_t kAlign = 4096;
  char *base = nullptr;  // NULL on a simulation server (offsets only)
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes

  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  void init(char *b, size_t bytes) {  // bytes: a multiple of kAlign
    base = b;
    size = bytes;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool take(size_t bytes, size_t *off) {
    const size_t b = round(bytes);
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= b && (best == free_.end() || it->second < best->second)) best = it;
    if (best == free_.end()) return false;
    *off = best->first;
    const size_t rest = best->second - b, at = best->first + b;
    free_.erase(best);
    if (rest) free_[at] = rest;
    return true;
  }
  void give(size_t off, size_t bytes) {
    size_t b = round(bytes);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + b == next->first) {
      b += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += b;
        return;
      }
    }
    free_[off] = b;
  }
};

}  // namespace

struct Server {
  static constexpr int kBlock = 256;  // batch workgroup size
  atlas_serve_config cfg{};
  int device = 0;
  int grid_full[2] = {8, 8};  // persistent batch grid per dtype (F32, F64)
  std::vector<MeshEntry> meshes;
  std::vector<RemapEntry> remaps;
  std::vector<Slot> slots;
  Arena arena;  // outputs and workspaces (under mu)

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;     // submitted, not admitted (arrival order)
  std::deque<uint64_t> admitted;  // admitted, not launched (arrival order)
  uint64_t next_ticket = 1;
  uint64_t alloc_count = 0;
  uint64_t wake_gen = 0;  // bumped by every call that can unblock admission
  bool stopping = false;
  atlas_serve_stats st{};
  std::thread thread;

  void charge(size_t b) {
    st.inflight_bytes += b;
    st.peak_inflight_bytes = std::max(st.peak_inflight_bytes, st.inflight_bytes);
  }
  void uncharge(size_t b) { st.inflight_bytes -= std::min(b, st.inflight_bytes); }

  // Carves a request's server-owned output and workspace out of the arena.
  // Returns 1 when placed, 0 when a range does not fit yet (nothing is
  // kept), -1 on an injected failure (every cfg.fail_alloc_every-th
  // allocation fails on purpose: fault injection for the error paths).
  int place(Req &q) {
    const size_t need[2] = {q.own_out ? q.out_b : 0, q.ws_b};
    size_t off[2] = {SIZE_MAX, SIZE_MAX};
    for (int i = 0; i < 2; ++i) {
      if (!need[i]) continue;
      ++alloc_count;
      const bool injected =
          cfg.fail_alloc_every > 0 && alloc_count % (uint64_t)cfg.fail_alloc_every == 0;
      if (injected || !arena.take(need[i], &off[i])) {
        if (i == 1 && off[0] != SIZE_MAX) arena.give(off[0], need[0]);
        return injected ? -1 : 0;
      }
    }
    q.out_off = off[0];
    q.ws_off = off[1];
    if (arena.base) {
      if (off[0] != SIZE_MAX) q.r.out = arena.base + off[0];
      if (off[1] != SIZE_MAX) q.ws = arena.base + off[1];
    }
    return 1;
  }
  void give_out(Req &q) {
    if (q.out_off != SIZE_MAX) arena.give(q.out_off, q.out_b);
    q.out_off = SIZE_MAX;
    if (q.own_out) q.r.out = nullptr;
  }
  void give_ws(Req &q) {
    if (q.ws_off != SIZE_MAX) arena.give(q.ws_off, q.ws_b);
    q.ws_off = SIZE_MAX;
    q.ws = nullptr;
  }

  // A request leaves the device: release what it holds except an output the
  // caller still has to read (released by atlas_serve_release).
  // Called once the request's device work (if any) has completed.
  void finish(Req &q, int status, Clock::time_point now) {
    q.status = status;
    q.state = DONE;
    q.t_done = now;
    give_ws(q);
    size_t b = q.in_b + q.ws_b;
    if (!(q.own_out && status == ATLAS_OK)) {
      if (q.out_charged) b += q.out_b;
      q.out_charged = false;
      give_out(q);
    }
    uncharge(b);
    if (status == ATLAS_OK) ++st.completed;
    else if (status == ATLAS_ECANCELLED) ++st.cancelled;
    else ++st.failed;
  }

  void poll(Clock::time_point now) {
    for (Slot &s : slots) {
      if (!s.busy) continue;
      int status = ATLAS_OK;
      if (cfg.simulate) {
        if (now < s.sim_done) continue;
      } else {
        const hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) status = ATLAS_EDEVICE;
      }
      for (uint64_t t : s.reqs) {
        auto it = reqs.find(t);
        if (it != reqs.end()) finish(it->second, status, now);
      }
      s.reqs.clear();
      s.busy = false;
      cv_done.notify_all();
    }
  }

  // Admits queued requests in arrival order while they fit the budget and
  // their ranges fit the arena; an injected allocation failure finishes its
  // request with ATLAS_ENOMEM.
  void admit(Clock::time_point now) {
    while (!queue.empty()) {
      Req &q = reqs.at(queue.front());
      if (st.inflight_bytes + q.footprint() > cfg.hbm_budget_bytes) break;
      const int placed = place(q);
      if (placed == 0) break;
      charge(q.footprint());
      q.out_charged = true;
      queue.pop_front();
      if (placed < 0) {
        finish(q, ATLAS_ENOMEM, now);
        cv_done.notify_all();
        continue;
      }
      q.state = ADMITTED;
      admitted.push_back(q.ticket);
    }
  }

  // Large requests and remaps launch alone.
  bool is_large(const Req &q) const {
    return q.remap || q.V * (int64_t)q.r.nlev > cfg.batch_max_elems || cfg.max_batch <= 1;
  }

  // Takes the next launch group from the admitted list: the front request,
  // and if it is small, the following small requests of the same dtype.
  std::vector<uint64_t> next_group() {
    std::vector<uint64_t> g;
    const Req &a = reqs.at(admitted.front());
    g.push_back(a.ticket);
    admitted.pop_front();
    if (is_large(a)) return g;
    for (auto it = admitted.begin(); it != admitted.end() && (int)g.size() < cfg.max_batch;) {
      const Req &b = reqs.at(*it);
      if (!is_large(b) && b.r.dtype == a.r.dtype) {
        g.push_back(b.ticket);
        it = admitted.erase(it);
      } else {
        ++it;
      }
    }
    return g;
  }

  // Enqueues one group of admitted requests (their memory placed) on slot
  // `si`.
  void launch(int si, std::vector<uint64_t> run, Clock::time_point now) {
    Slot &s = slots[si];
    for (uint64_t t : run) reqs.at(t).slot = si;
    const int n = (int)run.size();
    int status = ATLAS_OK;
    if (cfg.simulate) {
      double bytes = 0;
      for (uint64_t t : run) {
        const Req &q = reqs.at(t);
        bytes += (double)q.in_b + q.out_b + 2.0 * q.ws_b;
      }
      s.sim_done = now + std::chrono::microseconds(
                             (int64_t)(bytes / std::max(1e-9, cfg.sim_bytes_per_us)));
    } else if (n == 1 && reqs.at(run[0]).remap) {
      Req &q = reqs.at(run[0]);
      status = remap_launch(*q.rp, q.r.in, q.r.nlev, (atlas_dtype)q.r.dtype, q.r.out, s.stream);
    } else if (n == 1) {
      Req &q = reqs.at(run[0]);
      const atlas_op op = (atlas_op)q.r.op;
      const atlas_dtype dt = (atlas_dtype)q.r.dtype;
      LaunchShape sh = q.sh_set ? q.sh : shape_from(nullptr, *q.m, op, q.r.nlev, dt);
      if (sh.variant == ATLAS_VARIANT_FLUX) sh = default_shape(*q.m, op, q.r.nlev, dt);
      status = launch_op(*q.m, op, dt, q.r.in, q.r.nlev, q.r.out, q.ws, sh, s.stream);
    } else {
      status = launch_batch_group(s, run);
    }
    if (status == ATLAS_OK && !cfg.simulate && hipEventRecord(s.done, s.stream) != hipSuccess)
      status = ATLAS_EDEVICE;
    if (status != ATLAS_OK) {
      // part of the group's work may be enqueued: let it drain before its
      // ranges go back to the arena
      if (!cfg.simulate) (void)hipStreamSynchronize(s.stream);
      for (uint64_t t : run) finish(reqs.at(t), status, now);
      cv_done.notify_all();
      return;
    }
    ++st.launches;
    if (n > 1) ++st.batched_launches;
    for (uint64_t t : run) {
      Req &q = reqs.at(t);
      q.state = RUNNING;
      q.t_launch = now;
      q.batch_size = n;
    }
    s.reqs = run;
    s.busy = true;
  }

  // Builds the batch tables of a group in the slot's pinned staging, copies
  // them to the slot's device tables and launches the batch kernel.
  atlas_status launch_batch_group(Slot &s, const std::vector<uint64_t> &run) {
    const int n = (int)run.size();
    const atlas_dtype dt = (atlas_dtype)reqs.at(run[0]).r.dtype;
    std::vector<BatchItem> items(n);
    std::vector<ItemShape> shapes(n);
    bool two_pass = false;
    for (int i = 0; i < n; ++i) {
      const Req &q = reqs.at(run[i]);
      BatchItem &bi = items[i];
      std::memset(&bi, 0, sizeof(bi));
      bi.m = q.m->d;
      bi.lapl = q.r.op == ATLAS_OP_LAPLACIAN ? 1 : 0;
      bi.op = q.r.op == ATLAS_OP_DIVERGENCE ? 1 : q.r.op == ATLAS_OP_CURL ? 2 : 0;
      bi.nlev = q.r.nlev;
      bi.in = q.r.in;
      bi.out = q.r.out;
      bi.ws = q.ws;
      shapes[i] = heuristic_shape(bi.op, dt, q.r.nlev);
      bi.form = shapes[i].form;
      bi.level_vec = shapes[i].level_vec;
      two_pass = two_pass || bi.lapl;
    }
    std::vector<BatchUnit> units;
    std::vector<int> qbeg;
    plan_units(items, shapes, units, qbeg);
    const size_t off_q = align_up(sizeof(BatchItem) * n);
    const size_t off_h = off_q + align_up(sizeof(int) * 18);
    const size_t off_u = off_h + align_up(sizeof(int) * 16);
    const size_t need = off_u + sizeof(BatchUnit) * units.size();
    if (need > s.tab_bytes) {
      // the slot is idle, so its old tables are no longer read
      const size_t bytes = std::max(need, s.tab_bytes * 2);
      if (s.d_tab) (void)hipFree(s.d_tab);
      if (s.h_tab) (void)hipHostFree(s.h_tab);
      s.d_tab = s.h_tab = nullptr;
      s.tab_bytes = 0;
      if (hipMalloc(&s.d_tab, bytes) != hipSuccess) return fail(ATLAS_ENOMEM, "batch tables");
      if (hipHostMalloc(&s.h_tab, bytes, hipHostMallocDefault) != hipSuccess)
        return fail(ATLAS_ENOMEM, "batch staging");
      s.tab_bytes = bytes;
    }
    std::memcpy(s.h_tab, items.data(), sizeof(BatchItem) * n);
    std::memcpy(s.h_tab + off_q, qbeg.data(), sizeof(int) * 18);
    std::memcpy(s.h_tab + off_u, units.data(), sizeof(BatchUnit) * units.size());
    ATLASX_HIP(hipMemcpyAsync(s.d_tab, s.h_tab, need, hipMemcpyHostToDevice, s.stream));
    const int full = grid_full[dt == ATLAS_F64 ? 1 : 0];
    const int grid = std::min(full, std::max(8, ((int)units.size() + 7) / 8 * 8));
    const int *qb = (const int *)(s.d_tab + off_q);
    return launch_batch(dt, (const BatchItem *)s.d_tab, (const BatchUnit *)(s.d_tab + off_u), qb,
                        qb + 9, two_pass, (int *)(s.d_tab + off_h), grid, kBlock, s.stream);
  }

  bool any_busy() const {
    for (const Slot &s : slots)
      if (s.busy) return true;
    return false;
  }

  void run() {
    if (!cfg.simulate) (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      Clock::time_point now = Clock::now();
      poll(now);
      admit(now);
      for (int si = 0; si < (int)slots.size() && !admitted.empty(); ++si) {
        if (slots[si].busy) continue;
        launch(si, next_group(), Clock::now());
      }
      const bool busy = any_busy();
      if (stopping && admitted.empty() && !busy) {
        // a request still queued now can only wait for releases that a
        // caller destroying the server will not make: cancel it
        for (uint64_t t : queue) {
          Req &q = reqs.at(t);
          q.status = ATLAS_ECANCELLED;
          q.state = DONE;
          q.t_done = Clock::now();
          ++st.cancelled;
        }
        queue.clear();
        cv_done.notify_all();
        break;
      }
      if (busy) {
        Clock::time_point until = Clock::now() + std::chrono::microseconds(20);
        if (cfg.simulate) {
          until = Clock::time_point::max();
          for (const Slot &s : slots)
            if (s.busy) until = std::min(until, s.sim_done);
        }
        cv_sched.wait_until(lk, until);
      } else {
        // idle: every slot is free, so nothing is admitted-but-unlaunched;
        // a queued request left over does not fit until a submit, cancel,
        // release or destroy changes the picture
        const uint64_t gen = wake_gen;
        cv_sched.wait(lk, [&] { return stopping || wake_gen != gen; });
      }
    }
  }
};

}  // namespace atlasx

struct atlas_server_s {
  atlasx::Server *s;
};

using namespace atlasx;

namespace {

atlas_status release_server(Server *sv) {
  for (Slot &s : sv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
  }
  if (sv->arena.base) (void)hipFree(sv->arena.base);
  sv->arena.base = nullptr;
  for (Slot &s : sv->slots) {
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.d_tab) (void)hipFree(s.d_tab);
    if (s.h_tab) (void)hipHostFree(s.h_tab);
  }
  for (MeshEntry &e : sv->meshes)
    if (e.mesh && e.mesh->store) e.mesh->store->serve_refs -= 1;
  for (RemapEntry &e : sv->remaps)
    if (e.remap && e.remap->plan) e.remap->plan->serve_refs -= 1;
  delete sv;
  return ATLAS_OK;
}

}  // namespace

extern "C" {

atlas_status atlas_serve_create(const atlas_serve_config *cfg, atlas_server_t *out) {
  if (!cfg || !out) return fail(ATLAS_EINVAL, "NULL argument");
  if (cfg->nstreams < 1 || cfg->nstreams > 16) return fail(ATLAS_EINVAL, "nstreams must be in [1, 16]");
  if (cfg->max_batch < 1 || cfg->max_batch > 4096) return fail(ATLAS_EINVAL, "max_batch must be in [1, 4096]");
  if (cfg->batch_max_elems < 0) return fail(ATLAS_EINVAL, "batch_max_elems must be >= 0");
  if (cfg->hbm_budget_bytes == 0 || cfg->hbm_budget_bytes > ((size_t)1 << 50))
    return fail(ATLAS_EINVAL, "hbm_budget_bytes must be in (0, 2^50]");
  if (cfg->simulate && !(cfg->sim_bytes_per_us > 0))
    return fail(ATLAS_EINVAL, "sim_bytes_per_us must be > 0");
  if (cfg->fail_alloc_every < 0) return fail(ATLAS_EINVAL, "fail_alloc_every must be >= 0");
  Server *sv = new (std::nothrow) Server();
  if (!sv) return fail(ATLAS_ENOMEM, "out of host memory");
  sv->cfg = *cfg;
  if (sv->cfg.batch_max_elems == 0) sv->cfg.batch_max_elems = (int64_t)1 << 22;
  sv->slots.resize(cfg->nstreams);
  // the budget plus one alignment granule for each of a request's two
  // ranges: every admissible request fits an empty arena
  const size_t arena_bytes = Arena::round(cfg->hbm_budget_bytes) + 2 * Arena::kAlign;
  if (cfg->simulate) sv->arena.init(nullptr, arena_bytes);
  if (!cfg->simulate) {
    if (hipGetDevice(&sv->device) != hipSuccess) {
      delete sv;
      return fail(ATLAS_EDEVICE, "hipGetDevice");
    }
    void *base = nullptr;
    if (hipMalloc(&base, arena_bytes) != hipSuccess) {
      (void)hipGetLastError();
      delete sv;
      return fail(ATLAS_ENOMEM, "cannot reserve the HBM budget on the device");
    }
    sv->arena.init(static_cast<char *>(base), arena_bytes);
    for (int d = 0; d < 2; ++d)
      sv->grid_full[d] = std::max(
          8, (device_cu_count() * batch_blocks_per_cu(d ? ATLAS_F64 : ATLAS_F32, Server::kBlock) +
              7) / 8 * 8);
    // tables for a full batch of small items; grown on demand
    const size_t tab0 = align_up(sizeof(BatchItem) * cfg->max_batch) + 2 * kTabAlign +
                        sizeof(BatchUnit) * 65536;
    for (Slot &s : sv->slots) {
      if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
        release_server(sv);
        return fail(ATLAS_EDEVICE, "stream or event creation");
      }
      if (hipMalloc(&s.d_tab, tab0) != hipSuccess ||
          hipHostMalloc(&s.h_tab, tab0, hipHostMallocDefault) != hipSuccess) {
        release_server(sv);
        return fail(ATLAS_ENOMEM, "batch tables");
      }
      s.tab_bytes = tab0;
    }
  }
  atlas_server_t h = new (std::nothrow) atlas_server_s{sv};
  if (!h) {
    release_server(sv);
    return fail(ATLAS_ENOMEM, "out of host memory");
  }
  try {
    sv->thread = std::thread([sv] { sv->run(); });
  } catch (...) {
    delete h;
    release_server(sv);
    return fail(ATLAS_ENOMEM, "cannot start the scheduler thread");
  }
  *out = h;
  return ATLAS_OK;
}

atlas_status atlas_serve_register_mesh(atlas_server_t srv, atlas_mesh_t mesh, int32_t *mesh_id) {
  if (!srv || !srv->s || !mesh || !mesh->store || !mesh_id) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  if (sv.cfg.simulate) return fail(ATLAS_EINVAL, "simulation server: use atlas_serve_register_sim_mesh");
  if (mesh->store->device != sv.device) return fail(ATLAS_EINVAL, "mesh lives on another device");
  std::lock_guard<std::mutex> g(sv.mu);
  mesh->store->serve_refs += 1;
  sv.meshes.push_back({mesh, mesh->store->d.V});
  *mesh_id = (int32_t)sv.meshes.size() - 1;
  return ATLAS_OK;
}

atlas_status atlas_serve_register_sim_mesh(atlas_server_t srv, int64_t nnodes, int32_t *mesh_id) {
  if (!srv || !srv->s || !mesh_id) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  if (!sv.cfg.simulate) return fail(ATLAS_EINVAL, "not a simulation server");
  if (nnodes < 1 || nnodes >= ((int64_t)1 << 31)) return fail(ATLAS_EINVAL, "nnodes out of range");
  std::lock_guard<std::mutex> g(sv.mu);
  sv.meshes.push_back({nullptr, nnodes});
  *mesh_id = (int32_t)sv.meshes.size() - 1;
  return ATLAS_OK;
}

atlas_status atlas_serve_register_remap(atlas_server_t srv, atlas_remap_t remap,
                                        int32_t *remap_id) {
  if (!srv || !srv->s || !remap || !remap->plan || !remap_id)
    return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  if (sv.cfg.simulate)
    return fail(ATLAS_EINVAL, "simulation server: use atlas_serve_register_sim_remap");
  if (remap->plan->device != sv.device) return fail(ATLAS_EINVAL, "remap lives on another device");
  std::lock_guard<std::mutex> g(sv.mu);
  remap->plan->serve_refs += 1;
  sv.remaps.push_back({remap, remap->plan->nsrc, remap->plan->nt});
  *remap_id = (int32_t)sv.remaps.size() - 1;
  return ATLAS_OK;
}

atlas_status atlas_serve_register_sim_remap(atlas_server_t srv, int64_t nsource,
                                            int64_t ntarget, int32_t *remap_id) {
  if (!srv || !srv->s || !remap_id) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  if (!sv.cfg.simulate) return fail(ATLAS_EINVAL, "not a simulation server");
  if (nsource < 1 || nsource >= ((int64_t)1 << 31) || ntarget < 1 ||
      ntarget >= ((int64_t)1 << 31))
    return fail(ATLAS_EINVAL, "nsource and ntarget must be in [1, 2^31)");
  std::lock_guard<std::mutex> g(sv.mu);
  sv.remaps.push_back({nullptr, nsource, ntarget});
  *remap_id = (int32_t)sv.remaps.size() - 1;
  return ATLAS_OK;
}

atlas_status atlas_serve_submit(atlas_server_t srv, const atlas_request *req, uint64_t *ticket) {
  if (!srv || !srv->s || !req || !ticket) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  std::lock_guard<std::mutex> g(sv.mu);
  auto reject = [&](atlas_status s, const char *msg) {
    ++sv.st.rejected;
    return fail(s, msg);
  };
  if (sv.stopping) return reject(ATLAS_ESTATE, "server is shutting down");
  const bool remap = req->op == ATLAS_SERVE_OP_REMAP;
  if (remap) {
    if (req->mesh_id < 0 || req->mesh_id >= (int32_t)sv.remaps.size())
      return reject(ATLAS_EINVAL, "unknown remap id");
  } else if (req->mesh_id < 0 || req->mesh_id >= (int32_t)sv.meshes.size()) {
    return reject(ATLAS_EINVAL, "unknown mesh_id");
  }
  if (!remap && (req->op < ATLAS_OP_GRADIENT || req->op > ATLAS_OP_LAPLACIAN))
    return reject(ATLAS_EINVAL, "unknown operator");
  if (req->dtype != ATLAS_F32 && req->dtype != ATLAS_F64) return reject(ATLAS_EINVAL, "unknown dtype");
  if (req->nlev < 1) return reject(ATLAS_EINVAL, "nlev must be >= 1");
  if (!sv.cfg.simulate && !req->in) return reject(ATLAS_EINVAL, "input pointer is NULL");
  const size_t w = req->dtype == ATLAS_F64 ? 8 : 4;
  const bool vin = req->op == ATLAS_OP_DIVERGENCE || req->op == ATLAS_OP_CURL;
  Req q;
  q.ticket = sv.next_ticket;
  q.r = *req;
  if (remap) {
    const RemapEntry &re = sv.remaps[req->mesh_id];
    if (std::max(re.nsrc, re.nt) * req->nlev >= ((int64_t)1 << 40))
      return reject(ATLAS_EINVAL, "nodes * columns too large");
    q.remap = true;
    q.rp = re.remap ? re.remap->plan : nullptr;
    q.V = re.nt;
    q.in_b = (size_t)re.nsrc * req->nlev * w;
    q.out_b = (size_t)re.nt * req->nlev * w;
  } else {
    const MeshEntry &me = sv.meshes[req->mesh_id];
    if (std::string why; me.mesh ? !levels_fit(*me.mesh->store, req->nlev, &why)
                                  : me.V * req->nlev * 2 >= ((int64_t)1 << 40))
      return reject(ATLAS_EINVAL, why.empty() ? "nnodes * nlev too large" : why.c_str());
    const size_t base = (size_t)me.V * req->nlev * w;
    q.m = me.mesh ? me.mesh->store : nullptr;
    q.V = me.V;
    q.in_b = base * (vin ? 2 : 1);
    q.out_b = base * (req->op == ATLAS_OP_GRADIENT ? 2 : 1);
    q.ws_b = req->op == ATLAS_OP_LAPLACIAN ? 2 * base : 0;
    if (q.m && req->op == ATLAS_OP_LAPLACIAN &&
        (me.V * req->nlev > sv.cfg.batch_max_elems || sv.cfg.max_batch <= 1)) {
      // a large Laplacian launches alone: if its shape is the fused one-pass
      // form it needs no workspace (the shape is kept for the launch)
      LaunchShape sh = shape_from(nullptr, *q.m, ATLAS_OP_LAPLACIAN, req->nlev,
                                  (atlas_dtype)req->dtype);
      if (lapl_fused_runs(*q.m, req->nlev, (atlas_dtype)req->dtype, sh)) {
        q.ws_b = 0;
        q.sh = sh;
        q.sh_set = true;
      }
    }
  }
  q.own_out = req->out == nullptr;
  if (!sv.cfg.simulate) {
    const size_t iw = vin ? 2 * w : w, ow = req->op == ATLAS_OP_GRADIENT ? 2 * w : w;
    // (a remap's op is neither: element-aligned input and output)
    if ((uintptr_t)req->in % iw || (req->out && (uintptr_t)req->out % ow))
      return reject(ATLAS_EINVAL, "field pointer not aligned to its element size");
    if (req->out) {
      const char *a = (const char *)req->in, *b = (const char *)req->out;
      if (a < b + q.out_b && b < a + q.in_b) return reject(ATLAS_EINVAL, "input and output overlap");
    }
  }
  if (q.footprint() > sv.cfg.hbm_budget_bytes)
    return reject(ATLAS_ENOMEM, "request footprint exceeds the whole HBM budget");
  q.t_sub = Clock::now();
  sv.next_ticket += 1;
  ++sv.st.submitted;
  sv.reqs.emplace(q.ticket, q);
  sv.queue.push_back(q.ticket);
  *ticket = q.ticket;
  ++sv.wake_gen;
  sv.cv_sched.notify_one();
  return ATLAS_OK;
}

atlas_status atlas_serve_wait(atlas_server_t srv, uint64_t ticket, int64_t timeout_us,
                              atlas_result *res) {
  if (!srv || !srv->s || !res) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  std::unique_lock<std::mutex> lk(sv.mu);
  auto it = sv.reqs.find(ticket);
  if (it == sv.reqs.end()) return fail(ATLAS_EINVAL, "unknown ticket");
  auto done = [&] {
    auto f = sv.reqs.find(ticket);
    return f == sv.reqs.end() || f->second.state == DONE;
  };
  if (timeout_us < 0) {
    sv.cv_done.wait(lk, done);
  } else if (!sv.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
    return fail(ATLAS_ETIMEOUT, "request not finished within the timeout");
  }
  it = sv.reqs.find(ticket);
  if (it == sv.reqs.end()) return fail(ATLAS_EINVAL, "ticket released while waiting");
  const Req &q = it->second;
  res->status = q.status;
  res->batch_size = q.batch_size;
  res->out = q.r.out;
  const bool launched = q.batch_size > 0;
  res->queue_us = launched ? us_between(q.t_sub, q.t_launch) : us_between(q.t_sub, q.t_done);
  res->run_us = launched ? us_between(q.t_launch, q.t_done) : 0.0;
  res->total_us = us_between(q.t_sub, q.t_done);
  return ATLAS_OK;
}

atlas_status atlas_serve_cancel(atlas_server_t srv, uint64_t ticket) {
  if (!srv || !srv->s) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  std::lock_guard<std::mutex> g(sv.mu);
  auto it = sv.reqs.find(ticket);
  if (it == sv.reqs.end()) return fail(ATLAS_EINVAL, "unknown ticket");
  Req &q = it->second;
  if (q.state == QUEUED) {
    sv.queue.erase(std::find(sv.queue.begin(), sv.queue.end(), ticket));
    q.out_charged = false;
    q.status = ATLAS_ECANCELLED;
    q.state = DONE;
    q.t_done = Clock::now();
    ++sv.st.cancelled;
  } else if (q.state == ADMITTED) {
    sv.admitted.erase(std::find(sv.admitted.begin(), sv.admitted.end(), ticket));
    sv.finish(q, ATLAS_ECANCELLED, Clock::now());
  } else {
    return fail(ATLAS_ESTATE, "request already launched");
  }
  sv.cv_done.notify_all();
  ++sv.wake_gen;
  sv.cv_sched.notify_one();
  return ATLAS_OK;
}

atlas_status atlas_serve_release(atlas_server_t srv, uint64_t ticket) {
  if (!srv || !srv->s) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  std::lock_guard<std::mutex> g(sv.mu);
  auto it = sv.reqs.find(ticket);
  if (it == sv.reqs.end()) return fail(ATLAS_EINVAL, "unknown ticket");
  Req &q = it->second;
  if (q.state != DONE) return fail(ATLAS_ESTATE, "request not finished");
  sv.give_out(q);  // the caller has finished reading it
  if (q.out_charged) sv.uncharge(q.out_b);
  sv.reqs.erase(it);
  ++sv.wake_gen;
  sv.cv_sched.notify_one();  // budget freed
  return ATLAS_OK;
}

atlas_status atlas_serve_get_stats(atlas_server_t srv, atlas_serve_stats *st) {
  if (!srv || !srv->s || !st) return fail(ATLAS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(srv->s->mu);
  *st = srv->s->st;
  return ATLAS_OK;
}

atlas_status atlas_serve_destroy(atlas_server_t srv) {
  if (!srv) return ATLAS_OK;
  Server *sv = srv->s;
  if (sv) {
    {
      std::lock_guard<std::mutex> g(sv->mu);
      sv->stopping = true;
      ++sv->wake_gen;
    }
    sv->cv_sched.notify_all();
    if (sv->thread.joinable()) sv->thread.join();
    release_server(sv);
  }
  delete srv;
  return ATLAS_OK;
}

}  // extern "C"
