"""Full-size parity: O1280 (6,599,680 nodes, 19,799,000 edges), 137 levels, in
the launch configuration the benchmark times (default shapes).  The oracle
evaluates each sampled node on its own (all levels), so the comparison covers
random nodes plus the places where the mesh is special: both polar caps,
ring starts and ends, and the octahedral seams."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

N, NLEV = 1280, 137


def _build(N, nrandom):
    import oracle
    import paper_1908_06091_amd as P
    import synthetic as sy
    print(f"fullsize: building O{N} meshes", flush=True)
    om = oracle.Mesh(N)
    gm = P.Mesh(N)
    dev = torch.device("cuda")
    co = sy.random_coeffs(128, [sy.seed_rng(3, 0, j) for j in range(8)], amplitude=1e2)
    H = torch.from_numpy(sy.synthesize(om.lon, om.lat, co)).to(dev)       # [8, V]
    G = torch.from_numpy(sy.synthesize_gradient(om.lon, om.lat, co)).to(dev)  # [8, V, 2]
    k = torch.arange(NLEV, device=dev, dtype=torch.float64)
    fac = 1.0 + k / NLEV
    idx = (k.long() % 8)
    f = (H[idx].t() * fac[None, :]).contiguous()
    # divergence input: a gradient field (its divergence is the Laplacian);
    # curl input: the rotated gradient k x grad (its curl is the Laplacian),
    # so that neither output is a cancellation to rounding level
    uv = (G[idx].permute(1, 0, 2) * fac[None, :, None]).contiguous()
    Gr = torch.stack((-G[..., 1], G[..., 0]), dim=-1)
    uvr = (Gr[idx].permute(1, 0, 2) * fac[None, :, None]).contiguous()
    del H, G, Gr
    g = torch.Generator(device=dev)
    g.manual_seed(N)
    for t in (f, uv, uvr):
        t += 1e-2 * (2.0 * torch.rand(t.shape, dtype=torch.float64, device=dev, generator=g) - 1.0)
    torch.cuda.synchronize()
    f_h, uv_h, uvr_h = f.cpu().numpy(), uv.cpu().numpy(), uvr.cpu().numpy()
    # sampled nodes: random, polar caps, ring starts/ends, seams
    rng = np.random.default_rng(137)
    pick = set(rng.choice(om.V, size=nrandom, replace=False).tolist())
    pick.update(range(0, 64))
    pick.update(range(om.V - 64, om.V))
    ro, nx = np.asarray(om.ring_off), np.asarray(om.nx)
    for j in range(0, len(nx), 37):
        for q in range(4):
            pick.add(int(ro[j] + q * nx[j] // 4))
        pick.add(int(ro[j] + nx[j] - 1))
    nodes = np.array(sorted(pick), dtype=np.int64)
    print(f"fullsize: O{N}, {len(nodes)} sampled nodes", flush=True)
    return dict(N=N, P=P, om=om, gm=gm, f=f, uv=uv, uvr=uvr, f_h=f_h, uv_h=uv_h, uvr_h=uvr_h,
                nodes=nodes, nodes_d=torch.from_numpy(nodes).to(dev), refs={})


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _build(N, 3000)


def _ref(big, op, dtype="f64"):
    """Oracle values at the sampled nodes.  FP32 runs are compared with the
    oracle on their own inputs (the FP32-rounded field, promoted exactly to
    FP64): the rounding of the inputs is not an error of the operator."""
    key = (op, dtype)
    if key not in big["refs"]:
        om, nodes = big["om"], big["nodes"]
        fn = {"grad": om.gradient_at, "div": om.divergence_at, "curl": om.curl_at,
              "lapl": om.laplacian_at}[op]
        name = {"grad": "f", "div": "uv", "curl": "uvr", "lapl": "f"}[op]
        if dtype == "f64":
            x = big[name + "_h"]
        else:
            x = big[name].float().double().cpu().numpy()
        big["refs"][key] = fn(x, NLEV, nodes)
        del x
    return big["refs"][key]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", ["grad", "div", "curl", "lapl"])
def test_o1280_l137_sampled(big, op, dtype):
    from gpu_util import TOL, normwise_error
    gm = big["gm"]
    dt = torch.float64 if dtype == "f64" else torch.float32
    x = big[{"grad": "f", "div": "uv", "curl": "uvr", "lapl": "f"}[op]].to(dt)
    fn = {"grad": gm.gradient, "div": gm.divergence, "curl": gm.curl,
          "lapl": gm.laplacian}[op]
    out = fn(x)
    got = out.index_select(0, big["nodes_d"]).double().cpu().numpy()
    del out, x
    torch.cuda.empty_cache()
    emax, erms = normwise_error(got, _ref(big, op, dtype))
    msg = f"O1280 L137 {op} {dtype}: max_rel={emax:.3e} rms_rel={erms:.3e}"
    if dtype == "f32":  # information: against the oracle on the FP64 inputs
        e64, r64 = normwise_error(got, _ref(big, op, "f64"))
        msg += f" (vs FP64 inputs: max_rel={e64:.3e} rms_rel={r64:.3e})"
    print(msg, flush=True)
    assert np.isfinite(got).all()
    assert emax <= TOL[dtype], (op, dtype, emax)
    if dtype == "f64" and op != "lapl":
        _assert_local(big, op, got, _ref(big, op, dtype), NLEV)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_o1280_l137_laplacian_forms_and_div_curl(big, dtype):
    """At full size, in the shapes the benchmark times: the fused one-pass
    Laplacian equals the two passes bit for bit, and the one-pass divergence
    and curl equal the separate operators bit for bit (each of which the
    sampled test above pins to the oracle)."""
    P, gm = big["P"], big["gm"]
    dt = torch.float64 if dtype == "f64" else torch.float32
    print(f"fullsize forms {dtype}", flush=True)
    f = big["f"].to(dt)
    one = gm.apply(P.ATLAS_OP_LAPLACIAN, f, launch=P.Launch(P.VARIANT_FUSED, 1024, 0, 0, 0, 0))
    two = gm.apply(P.ATLAS_OP_LAPLACIAN, f, launch=P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0))
    torch.cuda.synchronize()
    assert torch.equal(one, two)
    del one
    # the field ring forced to five slots (the automatic choice takes four
    # where that saves a level chunk: FP64 here) and to four
    for fslots in (4, 5):
        one = gm.apply(P.ATLAS_OP_LAPLACIAN, f, launch=P.Launch(P.VARIANT_FUSED, 1024, fslots, 0, 0, 0))
        torch.cuda.synchronize()
        assert torch.equal(one, two), fslots
        del one
    del two, f
    uv = big["uv"].to(dt)
    d, c = gm.div_curl(uv)
    torch.cuda.synchronize()
    assert torch.equal(d, gm.divergence(uv))
    assert torch.equal(c, gm.curl(uv))
    del d, c, uv
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_o1280_256_levels(big, dtype):
    """O1280 with 256 levels (27 GB per FP64 vector field: every field and
    column base is past 2^31 elements).  Levels are independent, so a field
    whose level k is level k mod 137 of the benchmark field must give,
    level for level, the bits of the 137-level results (pinned to the
    oracle by the sampled test above).  The mesh reports the most levels
    it takes: the byte offsets inside one parallel of FP64 vector columns
    (5136 nodes at O1280, 16 bytes per level) stay below 2^31."""
    P, gm = big["P"], big["gm"]
    dt = torch.float64 if dtype == "f64" else torch.float32
    assert gm.max_levels == (2 ** 31 - 1) // (16 * (4 * 1280 + 16))
    L = 256
    assert 2 * gm.nnodes * L > 2 ** 31
    print(f"fullsize 256 levels {dtype}", flush=True)
    kk = torch.arange(L, device="cuda") % NLEV
    for op, name in (("grad", "f"), ("div", "uv"), ("curl", "uvr"), ("lapl", "f")):
        x = big[name].to(dt)
        xl = x.index_select(1, kk).contiguous()
        fn = {"grad": gm.gradient, "div": gm.divergence, "curl": gm.curl,
              "lapl": gm.laplacian}[op]
        ref = fn(x).index_select(1, kk)
        got = fn(xl)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (op, dtype)
        del ref, got
        if op == "div":
            d, c = gm.div_curl(xl)
            torch.cuda.synchronize()
            assert torch.equal(d, gm.divergence(xl))
            assert torch.equal(c, gm.curl(xl))
            del d, c
        del x, xl
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nlev", [1, 2, 3, 4, 5, 6, 8, 11, 12, 16, 17, 24, 32, 33, 37, 40, 41, 48,
                                  64, 65, 72, 79, 80, 87, 88, 91, 96, 97, 100, 128, 129])
def test_o1280_short_columns_sampled(big, nlev, dtype):
    """O1280 with the first nlev levels of the benchmark fields, in the
    default shapes of those sizes, against the oracle at the sampled nodes.
    The sizes cover every built-in shape switch: the flat form (1 to 11
    levels depending on the operator; 17 is one GPU's slab when 137 levels
    are split over eight GPUs), the wave-specialised sweep of the FP64
    divergence and curl from 2 levels (in chunks of 16 lane vectors from
    33) and of the FP64 gradient from 4, of the FP32 divergence and curl
    from 6 to 64 (chunks of 16 from 41; to 96 on this mesh) and of the FP32
    gradient from 12 (chunks of 16 from 88), with 8, 5, 4, 3, 2 and 1
    positions per wavefront as the level chunk narrows (768 and 1024
    threads), and the column forms; 137 (the test above) and 256 levels
    take the FP64 gradient's chunk count that fills the most lanes.  The
    oracle treats every level on its own, so its values for the first nlev
    levels are the first nlev levels of its 137-level values."""
    _sampled(big, nlev, dtype)


def _sampled(big, nlev, dtype):
    from gpu_util import TOL, normwise_error
    gm = big["gm"]
    dt = torch.float64 if dtype == "f64" else torch.float32
    print(f"fullsize O{big['N']} nlev={nlev} {dtype}", flush=True)
    for op, name in (("grad", "f"), ("div", "uv"), ("curl", "uvr"), ("lapl", "f")):
        x = big[name][:, :nlev].contiguous().to(dt)
        fn = {"grad": gm.gradient, "div": gm.divergence, "curl": gm.curl,
              "lapl": gm.laplacian}[op]
        got = fn(x).index_select(0, big["nodes_d"]).double().cpu().numpy()
        del x
        ref = _ref(big, op, dtype)[:, :nlev]
        emax, erms = normwise_error(got, ref)
        print(f"O{big['N']} L{nlev} {op} {dtype}: max_rel={emax:.3e} rms_rel={erms:.3e}",
              flush=True)
        assert np.isfinite(got).all()
        assert emax <= TOL[dtype], (op, nlev, dtype, emax)
        if dtype == "f64" and op != "lapl":
            _assert_local(big, op, got, ref, nlev)
    torch.cuda.empty_cache()


def _assert_local(big, op, got, ref, nlev):
    """FP64 error node by node: each sampled node's error stays within a
    bound set by the size of that node's own terms (sum over its edges of
    |S| times the edge values, times its scale), so a wrong term at a node
    whose result is small cannot hide under the normwise bar."""
    bound = _local_scale(big, op, nlev)
    d = np.abs(got - ref)
    if d.ndim == 3:
        d = d.max(axis=2)
    worst = float((d / bound).max())
    assert worst <= 64 * 2.0 ** -52, (op, nlev, worst)


def _local_scale(big, op, nlev):
    """alpha_i (R / V_i, the larger of the node's two scales) times the sum
    over its edges of (|S_lon| + |S_lat|) (|x_a| + |x_b|), plus the polar
    face's |S| (|x_i| + |x_partner|) at polar nodes: the size of the terms
    the node sums, level by level (|x| the larger component of a vector)."""
    key = ("local", op)
    if key not in big["refs"]:
        om, nodes = big["om"], big["nodes"]
        inc = big.get("incidences")
        if inc is None:  # each node's edges, from the oracle's edge table
            E = om.E
            ends = np.concatenate([om.edge[:, 0], om.edge[:, 1]]).astype(np.int64)
            order = np.argsort(ends, kind="stable")
            eid = (order % E).astype(np.int64)
            lo = np.searchsorted(ends[order], nodes, "left")
            hi = np.searchsorted(ends[order], nodes, "right")
            inc = big["incidences"] = [eid[a:b] for a, b in zip(lo, hi)]
        e2n = om.edge
        S = np.abs(om.S).sum(axis=1)
        name = {"grad": "f", "div": "uv", "curl": "uvr"}[op]
        x = big[name + "_h"]
        partner = {}
        for (a, b), sn in zip(om.pole_edge, om.pole_normal):
            partner[int(a)] = (int(b), abs(sn))
            partner[int(b)] = (int(a), abs(sn))
        out = np.empty((len(nodes), NLEV))
        for q, i in enumerate(nodes):
            es = inc[q]
            a, b = e2n[es, 0], e2n[es, 1]
            xa, xb = np.abs(x[a]), np.abs(x[b])
            if xa.ndim == 3:
                xa, xb = xa.max(axis=2), xb.max(axis=2)
            t = (S[es][:, None] * (xa + xb)).sum(axis=0)
            if int(i) in partner:
                p_, sn = partner[int(i)]
                xi, xp = np.abs(x[i]), np.abs(x[p_])
                if xi.ndim == 2:
                    xi, xp = xi.max(axis=1), xp.max(axis=1)
                t = t + sn * (xi + xp)
            out[q] = t / om.vol[i] * om.R
        big["refs"][key] = out
    return big["refs"][key][:, :nlev]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_o1280_remap_to_o640_points_sampled(big, dtype):
    """Remap of the 137-level benchmark field from O1280 to the 1,661,440
    nodes of O640 (their coordinates from the oracle's O640 grid), in the
    apply launch the benchmark times: the weights and the remapped values of
    sampled targets (random, both polar caps, ring starts and quarter
    points) against the oracle."""
    import oracle
    P, om, gm = big["P"], big["om"], big["gm"]
    tgt = big.get("o640")
    if tgt is None:
        tgt = big["o640"] = oracle.Mesh(640)
    print(f"fullsize remap O1280 -> O640 points {dtype}", flush=True)
    r = P.Remap(gm, lon=tgt.lon, lat=tgt.lat)
    assert r.ntarget == tgt.V
    dt = torch.float64 if dtype == "f64" else torch.float32
    x = big["f"].to(dt)
    out = r.apply(x)
    rng = np.random.default_rng(640)
    pick = set(rng.choice(tgt.V, size=3000, replace=False).tolist())
    pick.update(range(0, 48))
    pick.update(range(tgt.V - 48, tgt.V))
    ro, nx = np.asarray(tgt.ring_off), np.asarray(tgt.nx)
    for j in range(0, len(nx), 17):
        for q in range(4):
            pick.add(int(ro[j] + q * nx[j] // 4))
    sel = np.array(sorted(pick), dtype=np.int64)
    got = out.index_select(0, torch.from_numpy(sel).cuda()).double().cpu().numpy()
    del out
    torch.cuda.empty_cache()
    oidx, ow = om.remap_weights(tgt.lon[sel], tgt.lat[sel])
    gidx, gw = r.weights()
    from scipy.sparse import csr_matrix
    rows = np.repeat(np.arange(sel.size), 3)
    Wg = csr_matrix((gw[sel].ravel(), (rows, gidx[sel].ravel().astype(np.int64))),
                    shape=(sel.size, om.V))
    Wo = csr_matrix((ow.ravel(), (rows, oidx.ravel().astype(np.int64))), shape=(sel.size, om.V))
    dW = Wg - Wo
    assert (np.abs(dW.data).max() if dW.nnz else 0.0) <= 1e-13
    xh = big["f_h"] if dtype == "f64" else x.double().cpu().numpy()
    ref = oracle.remap_apply(oidx, ow, xh, NLEV, om.V)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"O1280 -> O640 remap L137 {dtype}: max_rel={err:.3e}", flush=True)
    assert err <= (1e-12 if dtype == "f64" else 1e-5)
    del x


@pytest.fixture(scope="module")
def mid():
    """O640 (1,661,440 nodes, 4,984,280 edges)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _build(640, 2000)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nlev", [1, 16, 37, 64, 100, 137])
def test_o640_sampled(mid, nlev, dtype):
    """O640, the serving mix's second largest grid, at its level counts (1,
    37, 137) and at 16, 64 and 100 levels, default shapes, against the
    oracle at the sampled nodes."""
    _sampled(mid, nlev, dtype)
