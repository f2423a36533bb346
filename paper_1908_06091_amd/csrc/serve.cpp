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
// Device memory for outputs and workspaces comes from a small caching
// allocator: blocks are hipMalloc'ed once per size class and handed out
// again only after the work that used them has completed (a workspace when
// its request's event has fired, a server-owned output when the caller has
// released it), so reuse needs no stream ordering.  Cached plus used bytes
// stay within the HBM budget; cached blocks are freed only when a new size
// would not fit otherwise.
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

LaunchShape shape_from(const atlas_launch *l, const MeshStore &m, atlas_op op, int nlev,
                       atlas_dtype dt);

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
  int64_t V = 0;
  size_t in_b = 0, out_b = 0, ws_b = 0;
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

constexpr size_t kTabAlign = 256;
size_t align_up(size_t x) { return (x + kTabAlign - 1) / kTabAlign * kTabAlign; }

}  // namespace

struct Server {
  static constexpr int kBlock = 256;  // batch workgroup size
  atlas_serve_config cfg{};
  int device = 0;
  int grid_full[2] = {8, 8};  // persistent batch grid per dtype (F32, F64)
  std::vector<MeshEntry> meshes;
  std::vector<Slot> slots;
  // caching allocator (scheduler thread and release, under mu)
  std::multimap<size_t, void *> cache;        // free blocks by size
  std::map<void *, size_t> block_bytes;       // every block the server holds
  size_t held_bytes = 0;                      // used + cached

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;     // submitted, not admitted (arrival order)
  std::deque<uint64_t> admitted;  // admitted, not launched (arrival order)
  uint64_t next_ticket = 1;
  uint64_t alloc_count = 0;
  bool stopping = false;
  atlas_serve_stats st{};
  std::thread thread;

  void charge(size_t b) {
    st.inflight_bytes += b;
    st.peak_inflight_bytes = std::max(st.peak_inflight_bytes, st.inflight_bytes);
  }
  void uncharge(size_t b) { st.inflight_bytes -= std::min(b, st.inflight_bytes); }

  static size_t size_class(size_t bytes) {
    const size_t g = (size_t)2 << 20;  // 2 MiB granules
    return (bytes + g - 1) / g * g;
  }

  // Device block of at least `bytes`; every cfg.fail_alloc_every-th call
  // fails on purpose (fault injection for the scheduler's error paths).
  bool alloc(void **p, size_t bytes) {
    ++alloc_count;
    if (cfg.fail_alloc_every > 0 && alloc_count % (uint64_t)cfg.fail_alloc_every == 0) return false;
    if (cfg.simulate) {
      *p = nullptr;
      return true;
    }
    const size_t want = size_class(bytes);
    auto it = cache.lower_bound(want);
    if (it != cache.end() && it->first <= want + want / 4) {  // close fit
      *p = it->second;
      cache.erase(it);
      return true;
    }
    // make room within the budget by dropping cached blocks, largest first
    while (held_bytes + want > cfg.hbm_budget_bytes && !cache.empty()) {
      auto last = std::prev(cache.end());
      (void)hipFree(last->second);
      held_bytes -= last->first;
      block_bytes.erase(last->second);
      cache.erase(last);
    }
    void *q = nullptr;
    if (hipMalloc(&q, want) != hipSuccess) return false;
    block_bytes[q] = want;
    held_bytes += want;
    *p = q;
    return true;
  }
  // Returns a block whose device work has completed to the cache.
  void recycle(void *p) {
    if (!p || cfg.simulate) return;
    auto it = block_bytes.find(p);
    if (it != block_bytes.end()) cache.insert({it->second, p});
  }

  // A request leaves the device: release what it holds except an output the
  // caller still has to read (released by atlas_serve_release).
  // Called once the request's device work (if any) has completed.
  void finish(Req &q, int status, Clock::time_point now) {
    q.status = status;
    q.state = DONE;
    q.t_done = now;
    recycle(q.ws);
    q.ws = nullptr;
    size_t b = q.in_b + q.ws_b;
    if (!(q.own_out && status == ATLAS_OK)) {
      if (q.out_charged) b += q.out_b;
      q.out_charged = false;
      if (q.own_out && q.r.out) recycle(q.r.out);
      if (q.own_out) q.r.out = nullptr;
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

  void admit() {
    while (!queue.empty()) {
      Req &q = reqs.at(queue.front());
      if (st.inflight_bytes + q.footprint() > cfg.hbm_budget_bytes) break;
      charge(q.footprint());
      q.out_charged = true;
      q.state = ADMITTED;
      admitted.push_back(q.ticket);
      queue.pop_front();
    }
  }

  bool is_large(const Req &q) const {
    return q.V * (int64_t)q.r.nlev > cfg.batch_max_elems || cfg.max_batch <= 1;
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

  // Enqueues one group on slot `si`.  Requests whose allocation fails are
  // finished with ATLAS_ENOMEM; the rest run.
  void launch(int si, std::vector<uint64_t> group, Clock::time_point now) {
    Slot &s = slots[si];
    std::vector<uint64_t> run;
    for (uint64_t t : group) {
      Req &q = reqs.at(t);
      q.slot = si;
      bool ok = true;
      if (!q.r.out && q.own_out) ok = alloc(&q.r.out, q.out_b);
      if (ok && q.ws_b) ok = alloc(&q.ws, q.ws_b);
      if (!ok) {
        recycle(q.ws);  // nothing was enqueued on it
        q.ws = nullptr;
        finish(q, ATLAS_ENOMEM, now);
        continue;
      }
      run.push_back(t);
    }
    if (run.empty()) {
      cv_done.notify_all();
      return;
    }
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
    } else if (n == 1) {
      Req &q = reqs.at(run[0]);
      const atlas_op op = (atlas_op)q.r.op;
      const atlas_dtype dt = (atlas_dtype)q.r.dtype;
      LaunchShape sh = shape_from(nullptr, *q.m, op, q.r.nlev, dt);
      if (sh.variant == ATLAS_VARIANT_FLUX) sh = default_shape(*q.m, op, q.r.nlev, dt);
      status = launch_op(*q.m, op, dt, q.r.in, q.r.nlev, q.r.out, q.ws, sh, s.stream);
    } else {
      status = launch_batch_group(s, run);
    }
    if (status == ATLAS_OK && !cfg.simulate && hipEventRecord(s.done, s.stream) != hipSuccess)
      status = ATLAS_EDEVICE;
    if (status != ATLAS_OK) {
      // part of the group's work may be enqueued: let it drain before the
      // blocks go back to the cache
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
      shapes[i] = heuristic_shape(q.r.nlev);
      bi.form = shapes[i].form;
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
      admit();
      for (int si = 0; si < (int)slots.size() && !admitted.empty(); ++si) {
        if (slots[si].busy) continue;
        launch(si, next_group(), Clock::now());
      }
      const bool busy = any_busy();
      if (stopping && queue.empty() && admitted.empty() && !busy) break;
      if (busy) {
        Clock::time_point until = Clock::now() + std::chrono::microseconds(20);
        if (cfg.simulate) {
          until = Clock::time_point::max();
          for (const Slot &s : slots)
            if (s.busy) until = std::min(until, s.sim_done);
        }
        cv_sched.wait_until(lk, until);
      } else {
        cv_sched.wait(lk, [&] {
          return stopping || !queue.empty() || !admitted.empty();
        });
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
  for (auto &kv : sv->block_bytes) (void)hipFree(kv.first);  // used and cached blocks
  sv->block_bytes.clear();
  sv->cache.clear();
  for (Slot &s : sv->slots) {
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.d_tab) (void)hipFree(s.d_tab);
    if (s.h_tab) (void)hipHostFree(s.h_tab);
  }
  for (MeshEntry &e : sv->meshes)
    if (e.mesh && e.mesh->store) e.mesh->store->serve_refs -= 1;
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
  if (cfg->hbm_budget_bytes == 0) return fail(ATLAS_EINVAL, "hbm_budget_bytes must be > 0");
  if (cfg->simulate && !(cfg->sim_bytes_per_us > 0))
    return fail(ATLAS_EINVAL, "sim_bytes_per_us must be > 0");
  if (cfg->fail_alloc_every < 0) return fail(ATLAS_EINVAL, "fail_alloc_every must be >= 0");
  Server *sv = new (std::nothrow) Server();
  if (!sv) return fail(ATLAS_ENOMEM, "out of host memory");
  sv->cfg = *cfg;
  if (sv->cfg.batch_max_elems == 0) sv->cfg.batch_max_elems = (int64_t)1 << 22;
  sv->slots.resize(cfg->nstreams);
  if (!cfg->simulate) {
    if (hipGetDevice(&sv->device) != hipSuccess) {
      delete sv;
      return fail(ATLAS_EDEVICE, "hipGetDevice");
    }
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

atlas_status atlas_serve_submit(atlas_server_t srv, const atlas_request *req, uint64_t *ticket) {
  if (!srv || !srv->s || !req || !ticket) return fail(ATLAS_EINVAL, "NULL argument");
  Server &sv = *srv->s;
  std::lock_guard<std::mutex> g(sv.mu);
  auto reject = [&](atlas_status s, const char *msg) {
    ++sv.st.rejected;
    return fail(s, msg);
  };
  if (sv.stopping) return reject(ATLAS_ESTATE, "server is shutting down");
  if (req->mesh_id < 0 || req->mesh_id >= (int32_t)sv.meshes.size())
    return reject(ATLAS_EINVAL, "unknown mesh_id");
  if (req->op < ATLAS_OP_GRADIENT || req->op > ATLAS_OP_LAPLACIAN)
    return reject(ATLAS_EINVAL, "unknown operator");
  if (req->dtype != ATLAS_F32 && req->dtype != ATLAS_F64) return reject(ATLAS_EINVAL, "unknown dtype");
  if (req->nlev < 1) return reject(ATLAS_EINVAL, "nlev must be >= 1");
  const MeshEntry &me = sv.meshes[req->mesh_id];
  if (me.V * req->nlev * 2 >= ((int64_t)1 << 31)) return reject(ATLAS_EINVAL, "nnodes * nlev too large");
  if (!sv.cfg.simulate && !req->in) return reject(ATLAS_EINVAL, "input pointer is NULL");
  const size_t w = req->dtype == ATLAS_F64 ? 8 : 4;
  const bool vin = req->op == ATLAS_OP_DIVERGENCE || req->op == ATLAS_OP_CURL;
  const size_t base = (size_t)me.V * req->nlev * w;
  Req q;
  q.ticket = sv.next_ticket;
  q.r = *req;
  q.m = me.mesh ? me.mesh->store : nullptr;
  q.V = me.V;
  q.in_b = base * (vin ? 2 : 1);
  q.out_b = base * (req->op == ATLAS_OP_GRADIENT ? 2 : 1);
  q.ws_b = req->op == ATLAS_OP_LAPLACIAN ? 2 * base : 0;
  q.own_out = req->out == nullptr;
  if (!sv.cfg.simulate) {
    const size_t iw = vin ? 2 * w : w, ow = req->op == ATLAS_OP_GRADIENT ? 2 * w : w;
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
  if (q.own_out && q.r.out) sv.recycle(q.r.out);  // the caller has finished reading it
  if (q.out_charged) sv.uncharge(q.out_b);
  sv.reqs.erase(it);
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
    }
    sv->cv_sched.notify_all();
    if (sv->thread.joinable()) sv->thread.join();
    release_server(sv);
  }
  delete srv;
  return ATLAS_OK;
}

}  // extern "C"
