"""Host-side tests of the request server's scheduler (atlas_serve.h) in
simulation mode: admission by HBM budget, continuous batching, cancellation,
time-outs and allocation-failure handling.  No device is touched: a launch
completes after bytes / sim_bytes_per_us microseconds."""
import time

import pytest

import paper_1908_06091_amd as P
from paper_1908_06091_amd import AtlasError

F64, F32 = P.ATLAS_F64, P.ATLAS_F32
GRAD, DIV, LAPL = P.ATLAS_OP_GRADIENT, P.ATLAS_OP_DIVERGENCE, P.ATLAS_OP_LAPLACIAN


def footprint(V, nlev, op, w):
    base = V * nlev * w
    inb = base * (2 if op in (P.ATLAS_OP_DIVERGENCE, P.ATLAS_OP_CURL) else 1)
    outb = base * (2 if op == GRAD else 1)
    ws = 2 * base if op == LAPL else 0
    return inb + outb + ws


def until_launched(s, n, limit_s=5.0):
    """Waits until the server has made n launches (the scheduler runs on its
    own thread)."""
    t0 = time.time()
    while s.stats()["launches"] < n:
        assert time.time() - t0 < limit_s, "scheduler made no launch"
        time.sleep(1e-4)


def make(**kw):
    cfg = dict(hbm_budget_bytes=1 << 40, nstreams=2, max_batch=16, simulate=True,
               sim_bytes_per_us=1e5)
    cfg.update(kw)
    return P.Server(**cfg)


def test_all_requests_complete_and_budget_returns_to_zero():
    s = make()
    m = s.register_sim_mesh(10000)
    ts = [s.submit(m, op, nlev=nl, dtype=dt)
          for op in (GRAD, DIV, P.ATLAS_OP_CURL, LAPL) for nl in (1, 37) for dt in (F32, F64)]
    for t in ts:
        r = s.wait(t)
        assert r["status"] == P.ATLAS_OK and r["batch_size"] >= 1
        assert r["total_us"] >= r["queue_us"] >= 0
    st = s.stats()
    # server-owned outputs stay charged until released
    assert st["inflight_bytes"] > 0
    for t in ts:
        s.release(t)
    st = s.stats()
    assert st["submitted"] == st["completed"] == len(ts)
    assert st["inflight_bytes"] == 0 and st["failed"] == 0
    s.close()


def test_budget_bounds_inflight_and_admits_in_order():
    V, nlev = 50000, 10
    fp = footprint(V, nlev, GRAD, 8)
    s = make(hbm_budget_bytes=3 * fp, nstreams=4, sim_bytes_per_us=2e4)
    m = s.register_sim_mesh(V)
    ts = [s.submit(m, GRAD, nlev=nlev, dtype=F64) for _ in range(12)]
    launch_at = []
    for t in ts:
        r = s.wait(t)
        launch_at.append(r["queue_us"])
        s.release(t)  # the budget frees once the output is handed back
    st = s.stats()
    assert st["peak_inflight_bytes"] == 3 * fp
    assert st["completed"] == 12
    # admission in arrival order: the i-th request never waits less than an
    # earlier one by more than the submission spread
    assert st["launches"] >= 4
    for i in range(3, 12):
        assert launch_at[i] + 5e3 >= max(launch_at[:3])
    s.close()


def test_request_larger_than_budget_is_rejected():
    s = make(hbm_budget_bytes=1000)
    m = s.register_sim_mesh(1000)
    with pytest.raises(AtlasError, match="ENOMEM"):
        s.submit(m, GRAD, nlev=1, dtype=F64)
    assert s.stats()["rejected"] == 1
    s.close()


@pytest.mark.parametrize("bad", [dict(op=7), dict(nlev=0), dict(dtype=5), dict(mesh_id=3)])
def test_invalid_requests_are_rejected(bad):
    s = make()
    m = s.register_sim_mesh(100)
    a = dict(mesh_id=m, op=GRAD, nlev=2, dtype=F64)
    a.update(bad)
    with pytest.raises(AtlasError, match="EINVAL"):
        s.submit(a["mesh_id"], a["op"], nlev=a["nlev"], dtype=a["dtype"])
    s.close()


def test_invalid_configs():
    with pytest.raises(AtlasError, match="EINVAL"):
        make(nstreams=0)
    with pytest.raises(AtlasError, match="EINVAL"):
        make(max_batch=0)
    with pytest.raises(AtlasError, match="EINVAL"):
        make(hbm_budget_bytes=0)
    with pytest.raises(AtlasError, match="EINVAL"):
        make(sim_bytes_per_us=0.0)
    s = make()
    with pytest.raises(AtlasError, match="EINVAL"):
        s.register_sim_mesh(0)
    s.close()


def test_continuous_batching_merges_arrivals_while_busy():
    V = 20000
    s = make(nstreams=1, max_batch=8, sim_bytes_per_us=2e3)
    m = s.register_sim_mesh(V)
    first = s.submit(m, GRAD, nlev=37, dtype=F64)
    until_launched(s, 1)  # the first request is on the (only) slot
    rest = [s.submit(m, GRAD, nlev=37, dtype=F64) for _ in range(20)]
    r0 = s.wait(first)
    sizes = [s.wait(t)["batch_size"] for t in rest]
    assert r0["batch_size"] == 1
    assert max(sizes) == 8 and all(1 <= b <= 8 for b in sizes)
    st = s.stats()
    assert st["batched_launches"] >= 2
    assert st["launches"] == 1 + 3  # 20 arrivals in groups of at most 8
    s.close()


def test_large_requests_launch_alone_and_dtypes_do_not_mix():
    s = make(nstreams=1, max_batch=16, batch_max_elems=1000, sim_bytes_per_us=1e3)
    m_small = s.register_sim_mesh(10)
    m_large = s.register_sim_mesh(5000)
    blocker = s.submit(m_small, GRAD, nlev=1000, dtype=F64)
    until_launched(s, 1)
    ts = [s.submit(m_large, GRAD, nlev=1, dtype=F64),
          s.submit(m_small, GRAD, nlev=1, dtype=F64),
          s.submit(m_small, GRAD, nlev=1, dtype=F32),
          s.submit(m_small, GRAD, nlev=1, dtype=F64),
          s.submit(m_large, GRAD, nlev=1, dtype=F64)]
    s.wait(blocker)
    res = [s.wait(t) for t in ts]
    assert res[0]["batch_size"] == 1 and res[4]["batch_size"] == 1
    assert res[1]["batch_size"] == res[3]["batch_size"] == 2  # same dtype merged
    assert res[2]["batch_size"] == 1  # the F32 request runs on its own
    s.close()


def test_cancel_queued_and_refuse_cancel_of_running():
    V = 100000
    s = make(nstreams=1, max_batch=1, sim_bytes_per_us=1e3)
    m = s.register_sim_mesh(V)
    running = s.submit(m, GRAD, nlev=10, dtype=F64)
    until_launched(s, 1)
    queued = s.submit(m, GRAD, nlev=10, dtype=F64)
    s.cancel(queued)
    r = s.wait(queued)
    assert r["status"] == P.ATLAS_ECANCELLED and r["batch_size"] == 0
    with pytest.raises(AtlasError, match="ESTATE"):
        s.cancel(running)
    assert s.wait(running)["status"] == P.ATLAS_OK
    assert s.stats()["cancelled"] == 1
    s.close()


def test_wait_timeout_then_completion():
    s = make(nstreams=1, sim_bytes_per_us=10.0)
    m = s.register_sim_mesh(1000)
    t = s.submit(m, GRAD, nlev=10, dtype=F64)   # 240 kB at 10 B/us: ~24 ms
    with pytest.raises(AtlasError, match="ETIMEOUT"):
        s.wait(t, timeout_us=1000)
    assert s.wait(t, timeout_us=5_000_000)["status"] == P.ATLAS_OK
    with pytest.raises(AtlasError, match="ESTATE"):
        t2 = s.submit(m, GRAD, nlev=10, dtype=F64)
        s.release(t2)  # not finished yet
    s.close()


def test_release_unknown_ticket_and_wait_unknown():
    s = make()
    with pytest.raises(AtlasError, match="EINVAL"):
        s.wait(12345)
    with pytest.raises(AtlasError, match="EINVAL"):
        s.release(12345)
    s.close()


def test_injected_allocation_failures_fail_only_their_requests():
    V, nlev = 2000, 4
    s = make(nstreams=2, max_batch=4, fail_alloc_every=3, sim_bytes_per_us=1e4)
    m = s.register_sim_mesh(V)
    ts = [s.submit(m, GRAD, nlev=nlev, dtype=F64) for _ in range(30)]
    status = [s.wait(t)["status"] for t in ts]
    for t in ts:
        s.release(t)
    st = s.stats()
    assert status.count(P.ATLAS_ENOMEM) == st["failed"] == 10
    assert status.count(P.ATLAS_OK) == st["completed"] == 20
    assert st["inflight_bytes"] == 0
    s.close()


def test_destroy_drains_pending_requests():
    s = make(nstreams=1, sim_bytes_per_us=1e4)
    m = s.register_sim_mesh(1000)
    for _ in range(10):
        s.submit(m, LAPL, nlev=3, dtype=F32)
    s.close()  # returns once every admitted request has run
    with pytest.raises(AtlasError):
        P.Server(hbm_budget_bytes=1, nstreams=1, max_batch=1, simulate=True,
                 sim_bytes_per_us=1.0).register_mesh(type("M", (), {"handle": None})())


def test_fragmented_arena_holds_the_head_until_a_release():
    """Server-owned outputs are ranges of one arena of the budget (plus one
    4 KiB granule per range).  Four small outputs fill it in order; releasing
    the first and third leaves free space that the budget allows but no
    contiguous range for a larger output, which is admitted once the second
    is released too (the freed ranges merge)."""
    X = 4096 * 100
    s = make(hbm_budget_bytes=3 * X, nstreams=4, max_batch=1, sim_bytes_per_us=1e4)
    small = s.register_sim_mesh(X // 4 // 8)      # F64, 1 level: output X/2
    big = s.register_sim_mesh(6 * X // 10 // 8)   # output 1.2 X
    ts = [s.submit(small, GRAD, nlev=1, dtype=F64) for _ in range(4)]
    assert all(s.wait(t)["status"] == P.ATLAS_OK for t in ts)
    s.release(ts[0])
    s.release(ts[2])
    assert s.stats()["inflight_bytes"] == X
    tb = s.submit(big, GRAD, nlev=1, dtype=F64)
    assert footprint(6 * X // 10 // 8, 1, GRAD, 8) + X <= 3 * X  # within budget
    with pytest.raises(AtlasError, match="ETIMEOUT"):
        s.wait(tb, timeout_us=200_000)
    s.release(ts[1])
    assert s.wait(tb, timeout_us=5_000_000)["status"] == P.ATLAS_OK
    s.release(tb)
    s.release(ts[3])
    assert s.stats()["inflight_bytes"] == 0
    s.close()


@pytest.mark.timeout(60)
def test_destroy_cancels_requests_that_can_no_longer_be_admitted():
    """A request queued behind server-owned outputs that are never released
    cannot be admitted; destroying the server cancels it instead of waiting
    forever."""
    V = 1000
    fp = footprint(V, 1, GRAD, 8)
    s = make(hbm_budget_bytes=fp, nstreams=1, sim_bytes_per_us=1e4)
    m = s.register_sim_mesh(V)
    t0 = s.submit(m, GRAD, nlev=1, dtype=F64)
    assert s.wait(t0)["status"] == P.ATLAS_OK
    t1 = s.submit(m, GRAD, nlev=1, dtype=F64)  # blocked: t0's output is held
    with pytest.raises(AtlasError, match="ETIMEOUT"):
        s.wait(t1, timeout_us=100_000)
    s.close()


def test_remap_requests_launch_alone_and_charge_their_sizes():
    """Remap requests (ATLAS_SERVE_OP_REMAP) footprint: source rows in,
    target rows out, no workspace; they never merge into a batch, while the
    operator requests around them still do."""
    REMAP = P.ATLAS_SERVE_OP_REMAP
    s = make(max_batch=64, nstreams=1, sim_bytes_per_us=2.0)  # the blocker: 1.6 s
    m = s.register_sim_mesh(1000)
    r = s.register_sim_remap(4000, 1000)
    blocker = s.submit(m, GRAD, nlev=137, dtype=F64)
    until_launched(s, 1)
    ts = [s.submit(r, REMAP, nlev=10, dtype=F64) for _ in range(3)]
    ts += [s.submit(m, GRAD, nlev=1, dtype=F32) for _ in range(3)]
    want = footprint(1000, 137, GRAD, 8) + 3 * (4000 + 1000) * 10 * 8 + \
        3 * footprint(1000, 1, GRAD, 4)
    t0 = time.time()  # admission runs on the scheduler thread
    while s.stats()["inflight_bytes"] != want and time.time() - t0 < 1.0:
        time.sleep(1e-3)
    assert s.stats()["inflight_bytes"] == want
    for t in [blocker] + ts:
        assert s.wait(t)["status"] == P.ATLAS_OK
    for t in ts[:3]:
        assert s.wait(t)["batch_size"] == 1
    assert max(s.wait(t)["batch_size"] for t in ts[3:]) > 1
    for t in [blocker] + ts:
        s.release(t)
    assert s.stats()["inflight_bytes"] == 0
    with pytest.raises(AtlasError):
        s.submit(r + 1, REMAP, nlev=1, dtype=F64)  # unknown remap id
    with pytest.raises(AtlasError):
        s.submit(m, 5, nlev=1, dtype=F64)  # unknown operator
    with pytest.raises(AtlasError):
        s.register_sim_remap(0, 10)
    s.close()
