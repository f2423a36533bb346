"""GPU tests of the batched persistent launch: every item of a batch equals
the same operator launched alone, bit for bit; graph replays interleaved
with other work stay identical."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06091_amd as P
    return P


@pytest.fixture(scope="module")
def meshes(P):
    return {N: P.Mesh(N) for N in (8, 16, 24)}


OPS = ("grad", "div", "curl", "lapl")


def _op_code(P, op):
    return {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}[op]


def _make_items(P, meshes, n, dtype, seed):
    rng = np.random.default_rng(seed)
    items = []
    for i in range(n):
        N = int(rng.choice(list(meshes)))
        gm = meshes[N]
        # 300 levels: two lane vectors per lane in FP32, one level per lane
        # past three chunks in FP64
        nlev = int(rng.choice([1, 10, 91, 137, 300]))
        op = OPS[int(rng.integers(0, 4))]
        vec_in = op in ("div", "curl")
        shape = (gm.nnodes, nlev, 2) if vec_in else (gm.nnodes, nlev)
        x = torch.from_numpy(rng.standard_normal(shape)).to(dtype=dtype, device="cuda")
        oshape = (gm.nnodes, nlev, 2) if op == "grad" else (gm.nnodes, nlev)
        out = torch.full(oshape, float("nan"), dtype=dtype, device="cuda")
        items.append((gm, _op_code(P, op), x, out))
    return items


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("autotune", [False, True])
@pytest.mark.parametrize("solo_min", [0, 20000, 1])
def test_batch_items_equal_solo(P, meshes, dtype, use_graph, autotune, solo_min):
    """solo_min 0: every item of these small meshes in the persistent
    launch; 20000: items of 20000+ elements as their own launches; 1: all."""
    print(f"batch dtype={dtype} graph={use_graph} autotune={autotune} solo_min={solo_min}",
          flush=True)
    items = _make_items(P, meshes, 24, dtype, seed=7)
    b = P.Batch(items, use_graph=use_graph, autotune=autotune, solo_min_elems=solo_min)
    assert b.info.nitems == 24 and b.info.graph == int(use_graph)
    nsolo = sum(1 for gm, op, x, out in items if gm.nnodes * x.shape[1] >= solo_min) if solo_min else 0
    assert b.info.solo_items == nsolo
    if solo_min == 20000:
        assert 0 < nsolo < 24
    b.launch()
    b.check()
    for gm, op, x, out in items:
        ref = gm.apply(op, x)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (op, x.shape)


@pytest.mark.parametrize("solo_min", [0, 1])
def test_graph_replays_with_eager_work_between(P, meshes, solo_min):
    print(f"graph replays solo_min={solo_min}", flush=True)
    items = _make_items(P, meshes, 16, torch.float32, seed=11)
    b = P.Batch(items, use_graph=True, solo_min_elems=solo_min)
    b.launch()
    b.check()
    first = [out.clone() for _, _, _, out in items]
    gm = meshes[16]
    y = torch.randn(gm.nnodes, 7, device="cuda")
    for _ in range(3):
        for _, _, _, out in items:
            out.fill_(float("nan"))
        gm.laplacian(y)           # unrelated eager work between replays
        torch.cuda.synchronize()
        b.launch()
        b.check()
        for (_, _, _, out), ref in zip(items, first):
            assert torch.equal(out, ref)


def test_laplacian_items_two_passes(P, meshes):
    """Laplacian items run as gradient then divergence passes of the batch;
    mixed with other operators they still equal the single operator."""
    gm = meshes[16]
    x = torch.randn(gm.nnodes, 10, device="cuda")
    y = torch.randn(gm.nnodes, 10, 2, device="cuda")
    o1 = torch.empty_like(x)
    o2 = torch.empty_like(x)
    ws = torch.empty(gm.nnodes, 10, 2, device="cuda")
    b = P.Batch([(gm, P.ATLAS_OP_LAPLACIAN, x, o1, ws), (gm, P.ATLAS_OP_DIVERGENCE, y, o2)],
                use_graph=False)
    b.launch()
    b.check()
    assert torch.equal(o1, gm.laplacian(x))
    assert torch.equal(o2, gm.divergence(y))


def test_batch_validation(P, meshes):
    gm = meshes[8]
    x32 = torch.randn(gm.nnodes, 3, device="cuda")
    x64 = x32.double()
    with pytest.raises(TypeError):
        P.Batch([(gm, P.ATLAS_OP_GRADIENT, x32, torch.empty(gm.nnodes, 3, 2, device="cuda")),
                 (gm, P.ATLAS_OP_GRADIENT, x64,
                  torch.empty(gm.nnodes, 3, 2, device="cuda", dtype=torch.float64))])
    with pytest.raises(P.AtlasError):
        P.Batch([(gm, 9, x32, torch.empty(gm.nnodes, 3, device="cuda"))])
    with pytest.raises(P.AtlasError):  # input and output overlap
        P.Batch([(gm, P.ATLAS_OP_LAPLACIAN, x32, x32)])


def _mixed_grid_items(P, meshes, n, seed):
    """n seeded FP32 items over O80/O160/O320 with nlev from {1, 10, 91,
    137} and operators from {grad, div, lapl}: each level a harmonic field
    of degree <= 16 (four per grid, cycled over the levels, times
    (1 + k/137)); divergence inputs are gradients of such fields."""
    import synthetic as sy
    rng = np.random.default_rng(seed)
    fields, items = {}, []
    for _ in range(n):
        N = int(rng.choice([80, 160, 320]))
        nlev = int(rng.choice([1, 10, 91, 137]))
        op = ("grad", "div", "lapl")[int(rng.integers(0, 3))]
        gm = meshes[N]
        if N not in fields:
            d = P.mesh_desc_octahedral(N)
            co = sy.random_coeffs(16, [sy.seed_rng(4, N, j) for j in range(4)])
            fields[N] = (torch.from_numpy(sy.synthesize(d["lon"], d["lat"], co)).cuda(),
                         torch.from_numpy(sy.synthesize_gradient(d["lon"], d["lat"], co)).cuda())
        H, G = fields[N]
        k = torch.arange(nlev, device="cuda", dtype=torch.float64)
        fac = 1.0 + k / 137.0
        if op == "div":
            x = (G[k.long() % 4].permute(1, 0, 2) * fac[None, :, None]).float().contiguous()
            out = torch.full((gm.nnodes, nlev), float("nan"), device="cuda")
        else:
            x = (H[k.long() % 4].t() * fac[None, :]).float().contiguous()
            shape = (gm.nnodes, nlev, 2) if op == "grad" else (gm.nnodes, nlev)
            out = torch.full(shape, float("nan"), device="cuda")
        items.append((gm, _op_code(P, op), x, out, N, op))
    return items


def test_mixed_grid_batch_forms_match_oracle(P):
    """The 64-item FP32 batch over O80/O160/O320 and 1-137 levels in three
    forms -- large items as their own launches beside the persistent kernel
    (the default), every item inside the persistent kernel, and autotuned
    tile shapes -- gives the same bits in each form and for each item alone,
    and every item matches the FP64 oracle on its own (FP32) inputs at
    sampled nodes within 1e-5 of the output scale."""
    import oracle
    from gpu_util import TOL, normwise_error, oracle_apply_at
    meshes = {N: P.Mesh(N) for N in (80, 160, 320)}
    items = _mixed_grid_items(P, meshes, 64, seed=64)
    kinds = [("hybrid", dict()), ("persistent", dict(solo_min_elems=-1)),
             ("autotuned", dict(autotune=True))]
    results = {}
    for name, kw in kinds:
        print(f"mixed-grid batch form {name}", flush=True)
        for it in items:
            it[3].fill_(float("nan"))
        b = P.Batch([it[:4] for it in items], use_graph=True, **kw)
        if name == "persistent":
            assert b.info.solo_items == 0
        b.launch()
        b.check()
        torch.cuda.synchronize()
        results[name] = [it[3].clone() for it in items]
        b.close()
    for name in ("persistent", "autotuned"):
        for a, c in zip(results["hybrid"], results[name]):
            assert torch.equal(a, c), name
    oms = {N: oracle.Mesh(N) for N in meshes}
    rng = np.random.default_rng(4)
    worst = 0.0
    for (gm, code, x, out, N, op), got_all in zip(items, results["hybrid"]):
        solo = gm.apply(code, x)
        torch.cuda.synchronize()
        assert torch.equal(solo, got_all), (N, op, x.shape)
        om = oms[N]
        nodes = np.sort(rng.choice(om.V, size=256, replace=False)).astype(np.int64)
        nodes[:8] = np.arange(8)  # a polar cap
        nodes = np.unique(nodes)
        nlev = x.shape[1]
        ref = oracle_apply_at(om, op, x.double().cpu().numpy(), nlev, nodes)
        got = got_all.double().cpu().numpy()[nodes]
        emax, _ = normwise_error(got, ref)
        worst = max(worst, emax)
        assert emax <= TOL["f32"], (N, op, nlev, emax)
    print(f"mixed-grid batch: worst max_rel vs oracle {worst:.3e}", flush=True)


@pytest.mark.parametrize("use_graph", [True, False])
def test_dependent_solo_items_keep_their_order(P, meshes, use_graph):
    """Items launched on their own run on parallel branches only when no
    item writes memory another touches.  Here item 1 reads item 0's output
    (a gradient, then its divergence) and items 2 and 3 write the same
    buffer, so the batch keeps the items' order: the results are those of
    the calls made one after another."""
    print(f"dependent solo items graph={use_graph}", flush=True)
    gm = meshes[24]
    f = torch.randn(gm.nnodes, 10, dtype=torch.float64, device="cuda")
    g = torch.full((gm.nnodes, 10, 2), float("nan"), dtype=torch.float64, device="cuda")
    d = torch.full((gm.nnodes, 10), float("nan"), dtype=torch.float64, device="cuda")
    uv = torch.randn(gm.nnodes, 10, 2, dtype=torch.float64, device="cuda")
    shared = torch.full((gm.nnodes, 10), float("nan"), dtype=torch.float64, device="cuda")
    items = [(gm, P.ATLAS_OP_GRADIENT, f, g), (gm, P.ATLAS_OP_DIVERGENCE, g, d),
             (gm, P.ATLAS_OP_DIVERGENCE, uv, shared), (gm, P.ATLAS_OP_CURL, uv, shared)]
    b = P.Batch(items, use_graph=use_graph, solo_min_elems=1)
    assert b.info.solo_items == 4
    for _ in range(2):
        b.launch()
        b.check()
        assert torch.equal(g, gm.gradient(f))
        assert torch.equal(d, gm.divergence(gm.gradient(f)))
        assert torch.equal(shared, gm.curl(uv))
        g.fill_(float("nan"))
        d.fill_(float("nan"))
        shared.fill_(float("nan"))
