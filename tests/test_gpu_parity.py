"""GPU parity: the HIP operators against the FP64 CPU oracle, element by
element on the same seeded inputs (Section 4.7 operators; Section 4.5
NodeColumns layout [node][level]).

Bar: FP64 normwise max|gpu - oracle| <= 1e-12 max|oracle| per component;
FP32 (fields rounded to FP32, oracle run on those values promoted to FP64)
<= 1e-5 max|oracle|.  Every launch shape must give identical bits.
"""
import functools

import numpy as np
import pytest

import oracle
from gpu_util import OPS, TOL, make_inputs, normwise_error, oracle_apply

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06091_amd as P
    return P


@functools.lru_cache(maxsize=None)
def _oracle_mesh(N):
    return oracle.Mesh(N)


_gpu_meshes = {}


def _gpu_mesh(P, N):
    if N not in _gpu_meshes:
        _gpu_meshes[N] = P.Mesh(N)
    return _gpu_meshes[N]


@functools.lru_cache(maxsize=None)
def _inputs(N, nlev):
    return make_inputs(_oracle_mesh(N), nlev)


def _run(P, gm, op, x, launch=None, workspace=None):
    code = {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}[op]
    out = gm.apply(code, x, launch=launch, workspace=workspace)
    torch.cuda.synchronize()
    return out


def _device_input(op, f, uv, dtype):
    x = uv if op in ("div", "curl") else f
    return torch.from_numpy(x).to(dtype=dtype, device="cuda").contiguous()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("nlev", [1, 3, 64, 65, 137])
@pytest.mark.parametrize("N", [1, 2, 4, 16])
def test_parity_small_meshes(P, N, nlev, op, dtype):
    print(f"parity N={N} nlev={nlev} op={op} dtype={dtype}", flush=True)
    om, gm = _oracle_mesh(N), _gpu_mesh(P, N)
    f, uv = _inputs(N, nlev)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    x = _device_input(op, f, uv, tdt)
    got = _run(P, gm, op, x).double().cpu().numpy()
    ref = oracle_apply(om, op, x.double().cpu().numpy(), nlev)
    rel_max, rel_rms = normwise_error(got.reshape(ref.shape), ref)
    assert rel_max <= TOL[dtype], (rel_max, rel_rms)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("nlev", [1, 7, 72, 137])
def test_launch_shapes_bitwise_identical(P, nlev, op, dtype):
    print(f"shapes nlev={nlev} op={op} dtype={dtype}", flush=True)
    N = 16
    gm = _gpu_mesh(P, N)
    f, uv = _inputs(N, nlev)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    x = _device_input(op, f, uv, tdt)
    base = _run(P, gm, op, x)
    shapes = []
    for variant in (P.VARIANT_COLUMN, P.VARIANT_FLAT):
        for block in (64, 256, 512):
            for npb in (0, 1, 7, 64):
                shapes.append(P.Launch(variant, block, npb))
    shapes.append(P.Launch(P.VARIANT_FLUX, 256, 0))
    shapes.append(P.Launch(P.VARIANT_FLUX, 64, 0))
    # level chunks of 1..64 levels: 1 to 8 positions per wavefront in the
    # wave-specialised sweep (blocks of at least 512 threads)
    for block in (64, 256, 512, 1024):
        for kc in (0, 1, 5, 20, 32, 40):
            shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc))      # lane vectors
            shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc, 0, 2))
            shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc, 0, 3))
            shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc, 0, 4))
            # register-staged sweep (blocks_per_cu = 1) beside the
            # wave-specialised one (blocks_per_cu = 0)
            shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc, 1))
            shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc, 1, 2))
            if block <= 512:
                shapes.append(P.Launch(P.VARIANT_SWEEP, block, 0, kc, 0, 1))  # one level per lane
    for kc in (1, 7, 64):
        shapes.append(P.Launch(P.VARIANT_COLUMN, 256, 0, kc))
    for block in (64, 256):
        for bpc in (1, 3, 8):
            shapes.append(P.Launch(P.VARIANT_COLUMN, block, 0, 0, bpc))
    # levels per lane: one, or lane vectors of 2 / 4 levels (capped at 16 B)
    for lv in (1, 2, 3, 4):
        shapes.append(P.Launch(P.VARIANT_COLUMN, 256, 0, 0, 0, lv))
        shapes.append(P.Launch(P.VARIANT_COLUMN, 64, 7, 0, 0, lv))
        shapes.append(P.Launch(P.VARIANT_COLUMN, 256, 0, 0, 3, lv))
    for sh in shapes:
        got = _run(P, gm, op, x, launch=sh)
        assert torch.equal(got, base), (sh.variant, sh.block_threads, sh.nodes_per_block,
                                        sh.level_vec)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_repeated_runs_bitwise_identical(P, dtype):
    N, nlev = 16, 65
    gm = _gpu_mesh(P, N)
    f, uv = _inputs(N, nlev)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for op in OPS:
        x = _device_input(op, f, uv, tdt)
        a = _run(P, gm, op, x).clone()
        b = _run(P, gm, op, x)
        assert torch.equal(a, b), op


def test_config1_o16_gradient(P):
    """O16, nlev = 1, FP64 gradient of a degree-4 harmonic field with seeded
    N(0,1) coefficients plus 1e-3 uniform noise."""
    import synthetic as sy
    om, gm = _oracle_mesh(16), _gpu_mesh(P, 16)
    f = sy.config_field(om.lon, om.lat, 4, 1, 0, noise_eps=1e-3)
    x = torch.from_numpy(f).cuda()
    got = gm.gradient(x).cpu().numpy()
    ref = om.gradient(f, 1)
    rel_max, _ = normwise_error(got, ref)
    assert rel_max <= 1e-12


@pytest.mark.parametrize("op", ["grad", "div", "curl", "lapl"])
def test_config2_o320_l137_fp64(P, op):
    """O320, nlev = 137, FP64: each level an independent harmonic field of
    degree <= 32 scaled by its level index; the vector input is the analytic
    gradient of a second seeded field."""
    import synthetic as sy
    print(f"O320 L137 {op}", flush=True)
    om, gm = _oracle_mesh(320), _gpu_mesh(P, 320)
    nlev = 137
    key = ("o320", nlev)
    if key not in _cfg2:
        f = sy.level_field_stack(om.lon, om.lat, nlev, 32, 2, 0)
        co = sy.random_coeffs(32, [sy.seed_rng(2, 1, 0)])
        g = sy.synthesize_gradient(om.lon, om.lat, co)[0]
        uv = np.repeat(g[:, None, :], nlev, axis=1) * (np.arange(nlev) + 1.0)[None, :, None]
        _cfg2[key] = (f, np.ascontiguousarray(uv))
    f, uv = _cfg2[key]
    x = torch.from_numpy(uv if op in ("div", "curl") else f).cuda()
    got = _run(P, gm, op, x).cpu().numpy()
    ref = oracle_apply(om, op, uv if op in ("div", "curl") else f, nlev)
    rel_max, rel_rms = normwise_error(got.reshape(ref.shape), ref)
    print(f"  max rel {rel_max:.3e} rms rel {rel_rms:.3e}", flush=True)
    assert rel_max <= 1e-12


_cfg2 = {}


def test_invalid_arguments_enqueue_nothing(P):
    gm = _gpu_mesh(P, 4)
    x = torch.zeros(gm.nnodes, 3, dtype=torch.float64, device="cuda")
    out = torch.full((gm.nnodes, 3, 2), 7.0, dtype=torch.float64, device="cuda")
    L = P.lib()
    s = torch.cuda.current_stream().cuda_stream
    import ctypes
    # nlev < 1
    assert L.atlas_nabla_gradient(gm.handle, ctypes.c_void_p(x.data_ptr()), 0, 1,
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s)) == -1
    assert b"nlev" in L.atlas_last_error()
    # NULL input
    assert L.atlas_nabla_gradient(gm.handle, None, 3, 1, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(s)) == -1
    # misaligned output
    assert L.atlas_nabla_gradient(gm.handle, ctypes.c_void_p(x.data_ptr()), 3, 1,
                                  ctypes.c_void_p(out.data_ptr() + 8), ctypes.c_void_p(s)) == -1
    # overlapping input and output
    assert L.atlas_nabla_gradient(gm.handle, ctypes.c_void_p(out.data_ptr()), 3, 1,
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s)) == -1
    # unknown dtype
    assert L.atlas_nabla_gradient(gm.handle, ctypes.c_void_p(x.data_ptr()), 3, 7,
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s)) == -1
    # levels per lane outside [0, 4]
    with pytest.raises(P.AtlasError):
        gm.apply(P.ATLAS_OP_GRADIENT, x, out=out, launch=P.Launch(P.VARIANT_COLUMN, 256, 0, 0, 0, 5))
    torch.cuda.synchronize()
    assert torch.all(out == 7.0), "a rejected call must not write anything"
    with pytest.raises(ValueError):
        gm.gradient(x.cpu())  # host tensor
    with pytest.raises(ValueError):
        gm.gradient(torch.zeros(gm.nnodes + 1, device="cuda", dtype=torch.float64))


def test_mesh_upload_from_description(P):
    """Upload through atlas_mesh_upload from the host description (the
    arrays a caller would pass) and from an explicit ring layout."""
    N, nlev = 8, 5
    desc = P.mesh_desc_octahedral(N)
    gm_a = P.Mesh(desc=desc)
    d2 = dict(desc)
    d2.pop("ring_off")
    gm_b = P.Mesh(desc=d2)
    om = _oracle_mesh(N)
    f, _ = make_inputs(om, nlev)
    x = torch.from_numpy(f).cuda()
    a = gm_a.gradient(x)
    b = gm_b.gradient(x)
    c = _gpu_mesh(P, N).gradient(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    bad = dict(desc)
    bad["node2edge_sign"] = -bad["node2edge_sign"]
    with pytest.raises(P.AtlasError):
        P.Mesh(desc=bad)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", OPS)
def test_autotune_keeps_results(P, op, dtype):
    """The autotuner times the candidate shapes, remembers the fastest in the
    mesh, and later calls with that shape give the same bits as before."""
    N, nlev = 24, 137
    gm = P.Mesh(N)
    rng = np.random.default_rng(5)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    shape = (gm.nnodes, nlev, 2) if op in ("div", "curl") else (gm.nnodes, nlev)
    x = torch.from_numpy(rng.standard_normal(shape)).to(dtype=tdt, device="cuda")
    before = _run(P, gm, op, x).clone()
    out = torch.empty_like(before)
    code = {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}[op]
    best, ms = P.autotune(gm, code, x, out)
    assert ms > 0 and best.variant in (P.VARIANT_COLUMN, P.VARIANT_FLAT, P.VARIANT_SWEEP)
    after = _run(P, gm, op, x)
    torch.cuda.synchronize()
    assert torch.equal(after, before)
    assert torch.equal(out, before)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("nlev", [255, 513, 1100])
def test_parity_long_columns(P, nlev, op, dtype):
    """Columns longer than the level-vector forms take (more than 4 chunks
    of 64 lane vectors fall back to one level per lane, beyond 3 chunks to
    the generic loop): every default shape against the oracle on O4, plus
    the fused Laplacian and the one-pass divergence + curl bitwise."""
    print(f"long columns nlev={nlev} {op} {dtype}", flush=True)
    N = 4
    om, gm = _oracle_mesh(N), _gpu_mesh(P, N)
    rng = np.random.default_rng(nlev)
    f = rng.standard_normal((om.V, nlev))
    uv = rng.standard_normal((om.V, nlev, 2))
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
        uv = uv.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    x = _device_input(op, f, uv, tdt)
    got = _run(P, gm, op, x)
    ref = oracle_apply(om, op, uv if op in ("div", "curl") else f, nlev)
    emax, _ = normwise_error(got.double().cpu().numpy().reshape(ref.shape), ref)
    assert emax <= TOL[dtype], (nlev, op, dtype, emax)
    if op == "lapl":
        fused = _run(P, gm, op, x, launch=P.Launch(P.VARIANT_FUSED, 1024, 0, 0, 0, 0))
        assert torch.equal(fused, got)
    if op == "div":
        d, c = gm.div_curl(x)
        torch.cuda.synchronize()
        assert torch.equal(d, got)
        assert torch.equal(c, _run(P, gm, "curl", x))


@pytest.mark.parametrize("N", [16, 48])
@pytest.mark.parametrize("nlev", [1, 7, 137])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gradient_lonlat_matches_oracle(P, N, nlev, dtype):
    """d/dlon and d/dlat (atlas_nabla_gradient_lonlat) against the oracle's
    computational-plane derivatives."""
    import oracle
    om = oracle.Mesh(N)
    gm = _gpu_mesh(P, N)
    f, _ = _inputs(N, nlev)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    x = torch.from_numpy(np.ascontiguousarray(f)).to(device="cuda", dtype=tdt)
    got = gm.gradient_lonlat(x).double().cpu().numpy()
    ref = om.gradient_lonlat(x.double().cpu().numpy(), nlev)
    emax, _ = normwise_error(got, ref)
    assert emax <= TOL[dtype], emax
