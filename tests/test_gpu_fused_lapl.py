"""GPU tests of the fused one-pass Laplacian (ATLAS_VARIANT_FUSED): the
gradients of a tile and of its neighbours are formed in LDS and their
divergence taken at once, on the two-ring plan.  Every gradient and every
divergence goes through the same per-element operation sequence as the
two-pass form (Section 4.7: the Laplacian as the divergence of the
gradient), so the results must be bitwise those of the two passes; they
are also checked against the FP64 oracle."""
import functools

import numpy as np
import pytest

import oracle
from gpu_util import TOL, make_inputs, normwise_error, oracle_apply

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


_meshes = {}


def _mesh(P, N, layout=None):
    key = (N, layout)
    if key not in _meshes:
        _meshes[key] = P.Mesh(N, layout=layout)
    return _meshes[key]


def _fused(P, block=1024, level_chunk=0):
    return P.Launch(P.VARIANT_FUSED, block, 0, level_chunk, 0, 0)


def _lapl(P, gm, x, launch=None):
    out = gm.apply(P.ATLAS_OP_LAPLACIAN, x, launch=launch)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nlev", [1, 2, 3, 37, 137, 300])
@pytest.mark.parametrize("N", [1, 2, 8, 24, 48])
def test_fused_equals_two_pass_and_oracle(P, N, nlev, dtype):
    print(f"fused lapl O{N} nlev={nlev} {dtype}", flush=True)
    gm = _mesh(P, N)
    om = _oracle_mesh(N)
    f, _ = make_inputs(om, nlev)
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    x = torch.from_numpy(f).to(dtype=dtype, device="cuda").contiguous()
    two = _lapl(P, gm, x, P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0))
    one = _lapl(P, gm, x, _fused(P))
    assert torch.equal(one, two)
    ref = oracle_apply(om, "lapl", f, nlev)
    err, _ = normwise_error(one.double().cpu().numpy().reshape(ref.shape), ref)
    assert err <= TOL["f64" if dtype == torch.float64 else "f32"], err


@pytest.mark.parametrize("layout", [(1, 1), (2, 3), (4, 4), (16, 24), (64, 64)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_any_layout(P, layout, dtype):
    """Tiles of one node, thin bands, tiles wider than the mesh: windows
    clipped at both poles, g-runs covering whole parallels."""
    print(f"fused lapl layout={layout} {dtype}", flush=True)
    gm = _mesh(P, 16, layout)
    x = torch.randn(gm.nnodes, 45, dtype=dtype, device="cuda")
    two = _lapl(P, gm, x, P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0))
    assert torch.equal(_lapl(P, gm, x, _fused(P)), two)


@pytest.mark.parametrize("block", [256, 512, 768, 1024])
@pytest.mark.parametrize("level_chunk", [0, 2, 8, 40])
def test_fused_blocks_and_chunks(P, block, level_chunk):
    """Workgroup sizes and level chunks (several chunks per column, a ragged
    last chunk); a block too small for the staging falls back to the two
    passes with the same bits."""
    print(f"fused lapl block={block} level_chunk={level_chunk}", flush=True)
    gm = _mesh(P, 48)
    x = torch.randn(gm.nnodes, 137, dtype=torch.float64, device="cuda")
    two = _lapl(P, gm, x, P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0))
    assert torch.equal(_lapl(P, gm, x, _fused(P, block, level_chunk)), two)


@pytest.mark.parametrize("fslots", [4, 5])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nlev", [2, 37, 137, 300])
@pytest.mark.parametrize("N", [8, 24, 48])
def test_fused_field_ring_slots(P, N, nlev, dtype, fslots):
    """The wave-specialised kernel with its field ring forced to four slots
    (each field run loaded one step ahead) or five (one and a half): the
    bits of the two passes, and the oracle's values."""
    print(f"fused lapl ring={fslots} O{N} nlev={nlev} {dtype}", flush=True)
    gm = _mesh(P, N)
    om = _oracle_mesh(N)
    f, _ = make_inputs(om, nlev)
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    x = torch.from_numpy(f).to(dtype=dtype, device="cuda").contiguous()
    two = _lapl(P, gm, x, P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0))
    one = _lapl(P, gm, x, P.Launch(P.VARIANT_FUSED, 1024, fslots, 0, 0, 0))
    assert torch.equal(one, two)
    ref = oracle_apply(om, "lapl", f, nlev)
    err, _ = normwise_error(one.double().cpu().numpy().reshape(ref.shape), ref)
    assert err <= TOL["f64" if dtype == torch.float64 else "f32"], err


@pytest.mark.parametrize("layout", [(1, 1), (2, 3), (64, 64)])
@pytest.mark.parametrize("level_chunk", [0, 8])
def test_fused_four_slot_ring_layouts_and_chunks(P, layout, level_chunk):
    """Four field slots on tiles of one node, thin bands and tiles wider
    than the mesh, with one and several level chunks."""
    print(f"fused lapl ring=4 layout={layout} level_chunk={level_chunk}", flush=True)
    gm = _mesh(P, 16, layout)
    x = torch.randn(gm.nnodes, 45, dtype=torch.float64, device="cuda")
    two = _lapl(P, gm, x, P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0))
    assert torch.equal(_lapl(P, gm, x, P.Launch(P.VARIANT_FUSED, 1024, 4, level_chunk, 0, 0)), two)


def test_fused_repeated_and_into_nan_output(P):
    gm = _mesh(P, 24)
    x = torch.randn(gm.nnodes, 91, dtype=torch.float64, device="cuda")
    ref = _lapl(P, gm, x, _fused(P))
    for _ in range(3):
        out = torch.full_like(ref, float("nan"))
        gm.apply(P.ATLAS_OP_LAPLACIAN, x, out=out, launch=_fused(P))
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_fused_is_for_the_laplacian_only(P):
    gm = _mesh(P, 8)
    x = torch.randn(gm.nnodes, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(P.AtlasError, match="Laplacian only"):
        gm.apply(P.ATLAS_OP_GRADIENT, x, launch=_fused(P))


# ---- divergence and curl in one pass (atlas_nabla_div_curl)

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nlev", [1, 47, 48, 64, 137, 300])
@pytest.mark.parametrize("N", [2, 16, 48])
def test_div_curl_equals_separate_calls(P, N, nlev, dtype):
    """One read of (u, v), two outputs, each bitwise the separate operator's
    result (which the parity tests pin to the oracle)."""
    print(f"div_curl O{N} nlev={nlev} {dtype}", flush=True)
    gm = _mesh(P, N)
    uv = torch.randn(gm.nnodes, nlev, 2, dtype=dtype, device="cuda")
    d, c = gm.div_curl(uv)
    torch.cuda.synchronize()
    assert torch.equal(d, gm.divergence(uv))
    assert torch.equal(c, gm.curl(uv))


def test_div_curl_against_oracle(P):
    N, nlev = 24, 137
    gm, om = _mesh(P, N), _oracle_mesh(N)
    _, uv = make_inputs(om, nlev)
    d, c = gm.div_curl(torch.from_numpy(uv).cuda())
    torch.cuda.synchronize()
    for got, op in ((d, "div"), (c, "curl")):
        ref = oracle_apply(om, op, uv, nlev)
        err, _ = normwise_error(got.cpu().numpy().reshape(ref.shape), ref)
        assert err <= TOL["f64"], (op, err)


def test_div_curl_rejects_overlapping_outputs(P):
    gm = _mesh(P, 8)
    uv = torch.randn(gm.nnodes, 4, 2, dtype=torch.float64, device="cuda")
    o = torch.empty(gm.nnodes, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(P.AtlasError, match="overlap"):
        gm.div_curl(uv, out_div=o, out_curl=o)


@pytest.mark.parametrize("nlev", [24, 37, 48, 64, 91, 137])
def test_div_curl_on_the_sweep_equals_separate_calls(P, nlev):
    """O640 (over a thousand tiles): where the FP64 divergence runs the
    wave-specialised sweep, the curl rides on its loads (one or two
    positions per wavefront, one to three level chunks); both outputs are
    bitwise the separate operators' results."""
    print(f"div_curl sweep O640 nlev={nlev}", flush=True)
    gm = _mesh(P, 640)
    uv = torch.randn(gm.nnodes, nlev, 2, dtype=torch.float64, device="cuda")
    d, c = gm.div_curl(uv)
    torch.cuda.synchronize()
    assert torch.equal(d, gm.divergence(uv))
    assert torch.equal(c, gm.curl(uv))
