"""GPU tests of the request server (atlas_serve.h): a request's result is the
same, bit for bit, whether it runs alone or is admitted, batched and
overlapped with others; server-owned outputs and a tight HBM budget keep
that property; a served FP64 result matches the oracle."""
import ctypes
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPS = ("grad", "div", "curl", "lapl")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06091_amd as P
    return P


@pytest.fixture(scope="module")
def meshes(P):
    return {N: P.Mesh(N) for N in (8, 16, 24, 48)}


def _code(P, op):
    return {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}[op]


def _requests(P, meshes, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        N = int(rng.choice(list(meshes)))
        gm = meshes[N]
        nlev = int(rng.choice([1, 37, 137]))
        op = OPS[int(rng.integers(0, 4))]
        dt = torch.float32 if rng.integers(0, 2) else torch.float64
        shape = (gm.nnodes, nlev, 2) if op in ("div", "curl") else (gm.nnodes, nlev)
        x = torch.from_numpy(rng.standard_normal(shape)).to(dtype=dt, device="cuda")
        reqs.append((N, op, x))
    return reqs


def _out_like(gm, op, x):
    shape = (gm.nnodes, x.shape[1], 2) if op == "grad" else (gm.nnodes, x.shape[1])
    return torch.full(shape, float("nan"), dtype=x.dtype, device="cuda")


@pytest.mark.parametrize("nstreams,max_batch", [(4, 16), (1, 64), (2, 1)])
def test_results_same_alone_and_in_mix(P, meshes, nstreams, max_batch):
    print(f"serve mix nstreams={nstreams} max_batch={max_batch}", flush=True)
    reqs = _requests(P, meshes, 48, seed=5 + nstreams)
    solo = [meshes[N].apply(_code(P, op), x) for N, op, x in reqs]
    torch.cuda.synchronize()
    srv = P.Server(hbm_budget_bytes=1 << 32, nstreams=nstreams, max_batch=max_batch,
                   batch_max_elems=1 << 20)
    ids = {N: srv.register_mesh(gm) for N, gm in meshes.items()}
    rng = np.random.default_rng(1)
    outs = [_out_like(meshes[N], op, x) for N, op, x in reqs]
    torch.cuda.synchronize()  # the server's streams do not wait for torch's
    tickets = []
    for i, ((N, op, x), out) in enumerate(zip(reqs, outs)):
        tickets.append(srv.submit(ids[N], _code(P, op), x, out))
        if i % 8 == 7:
            time.sleep(float(rng.exponential(2e-4)))  # bursts of arrivals
    sizes = []
    for t in tickets:
        r = srv.wait(t, timeout_us=60_000_000)
        assert r["status"] == P.ATLAS_OK
        sizes.append(r["batch_size"])
        srv.release(t)
    st = srv.stats()
    srv.close()
    for (N, op, x), out, ref in zip(reqs, outs, solo):
        assert torch.equal(out, ref), (N, op, tuple(x.shape), x.dtype)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    if max_batch > 1:
        assert st["batched_launches"] >= 1 and max(sizes) > 1
    else:
        assert max(sizes) == 1


def test_server_owned_outputs(P, meshes):
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    reqs = _requests(P, meshes, 12, seed=3)
    srv = P.Server(hbm_budget_bytes=1 << 32, nstreams=2, max_batch=8)
    ids = {N: srv.register_mesh(gm) for N, gm in meshes.items()}
    torch.cuda.synchronize()
    tickets = [srv.submit(ids[N], _code(P, op), x) for N, op, x in reqs]
    for (N, op, x), t in zip(reqs, tickets):
        r = srv.wait(t, timeout_us=60_000_000)
        assert r["status"] == P.ATLAS_OK and r["out"] != 0
        ref = meshes[N].apply(_code(P, op), x)
        got = torch.empty_like(ref)
        torch.cuda.synchronize()
        assert hip.hipMemcpy(got.data_ptr(), r["out"], ref.numel() * ref.element_size(), 3) == 0
        assert torch.equal(got, ref)
        srv.release(t)
    assert srv.stats()["inflight_bytes"] == 0
    srv.close()


def test_tight_budget_on_device(P, meshes):
    gm = meshes[48]
    x = torch.randn(gm.nnodes, 137, dtype=torch.float64, device="cuda")
    fp = 4 * x.numel() * 8   # Laplacian: input, output, [V][nlev][2] workspace
    srv = P.Server(hbm_budget_bytes=2 * fp, nstreams=4, max_batch=8)
    mid = srv.register_mesh(gm)
    outs = [torch.empty_like(x) for _ in range(10)]
    torch.cuda.synchronize()
    ts = [srv.submit(mid, P.ATLAS_OP_LAPLACIAN, x, o) for o in outs]
    for t in ts:
        assert srv.wait(t, timeout_us=60_000_000)["status"] == P.ATLAS_OK
        srv.release(t)
    st = srv.stats()
    srv.close()
    assert st["peak_inflight_bytes"] <= 2 * fp
    ref = gm.laplacian(x)
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref)


def test_served_result_matches_oracle(P, meshes):
    import oracle
    from gpu_util import TOL, make_inputs, normwise_error
    om = oracle.Mesh(16)
    gm = meshes[16]
    nlev = 37
    f, uv = make_inputs(om, nlev)
    srv = P.Server(hbm_budget_bytes=1 << 30, nstreams=2, max_batch=8)
    mid = srv.register_mesh(gm)
    cases = []
    for op, host in (("grad", f), ("div", uv), ("curl", uv), ("lapl", f)):
        x = torch.from_numpy(np.ascontiguousarray(host)).to("cuda")
        out = _out_like(gm, op, x)
        torch.cuda.synchronize()
        cases.append((op, host, x, out, srv.submit(mid, _code(P, op), x, out)))
    for op, host, _, out, t in cases:
        assert srv.wait(t, timeout_us=60_000_000)["status"] == P.ATLAS_OK
        srv.release(t)
        ref = {"grad": om.gradient, "div": om.divergence, "curl": om.curl,
               "lapl": om.laplacian}[op](host, nlev)
        emax, _ = normwise_error(out.cpu().numpy(), ref)
        assert emax <= TOL["f64"], (op, emax)
    srv.close()


def test_remap_requests_in_the_mix(P, meshes):
    """Remap requests (ATLAS_SERVE_OP_REMAP) between O48 and O16, FP64 and
    FP32, submitted among operator requests: each result equals the same
    remap run alone, bit for bit, and the FP64 one matches the oracle's
    interpolation."""
    import oracle
    gs, gd = meshes[48], meshes[16]
    r = P.Remap(gs, gd)
    srv = P.Server(hbm_budget_bytes=1 << 30, nstreams=3, max_batch=16)
    rid = srv.register_remap(r)
    mid = srv.register_mesh(gd)
    x64 = torch.randn(gs.nnodes, 37, dtype=torch.float64, device="cuda")
    x32 = torch.randn(gs.nnodes, 5, 2, dtype=torch.float32, device="cuda")
    y = torch.randn(gd.nnodes, 7, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ts = []
    for _ in range(4):
        ts.append(("r64", srv.submit(rid, P.ATLAS_SERVE_OP_REMAP, x64)))
        ts.append(("g", srv.submit(mid, P.ATLAS_OP_GRADIENT, y)))
        ts.append(("r32", srv.submit(rid, P.ATLAS_SERVE_OP_REMAP, x32)))
    alone = {"r64": r.apply(x64), "r32": r.apply(x32), "g": gd.gradient(y)}
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    for kind, t in ts:
        res = srv.wait(t, timeout_us=60_000_000)
        assert res["status"] == P.ATLAS_OK
        ref = alone[kind]
        got = torch.empty_like(ref)
        torch.cuda.synchronize()
        assert hip.hipMemcpy(got.data_ptr(), res["out"], ref.numel() * ref.element_size(), 3) == 0
        assert torch.equal(got, ref), kind
        srv.release(t)
    with pytest.raises(P.AtlasError):
        r.close()  # registered with a live server
    srv.close()
    om_s, om_d = oracle.Mesh(48), oracle.Mesh(16)
    want = om_s.remap(x64.cpu().numpy(), 37, om_d.lon, om_d.lat)
    got = alone["r64"].cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    r.close()
