"""GPU parity on reduced Gaussian grids other than O<N>: the regular grid
F<N> (Section 4.2.3.6, nx = 4N) and a hand-made reduced grid (Section
4.2.3.7), all operators in both precisions against the FP64 oracle built
from the same points-per-parallel array, every launch form bitwise equal."""
import functools

import numpy as np
import pytest

import oracle
from gpu_util import TOL, make_inputs, normwise_error, oracle_apply

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRIDS = {"F1": oracle.regular_gaussian_nx(1), "F4": oracle.regular_gaussian_nx(4),
         "F24": oracle.regular_gaussian_nx(24),
         "R3": np.array([6, 9, 13, 13, 10, 8], np.int32)}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06091_amd as P
    return P


@functools.lru_cache(maxsize=None)
def _om(name):
    return oracle.Mesh(nx=GRIDS[name])


_gms = {}


def _gm(P, name):
    if name not in _gms:
        _gms[name] = P.Mesh(nx=GRIDS[name])
    return _gms[name]


def _code(P, op):
    return {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}[op]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("op", ["grad", "div", "curl", "lapl"])
@pytest.mark.parametrize("nlev", [1, 7, 137])
@pytest.mark.parametrize("name", sorted(GRIDS))
def test_parity_reduced_grids(P, name, nlev, op, dtype):
    print(f"reduced grid {name} nlev={nlev} {op} {dtype}", flush=True)
    om, gm = _om(name), _gm(P, name)
    assert gm.nnodes == om.V and gm.nedges == om.E
    f, uv = make_inputs(om, nlev)
    x = uv if op in ("div", "curl") else f
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    xd = torch.from_numpy(x).to(dtype=tdt, device="cuda").contiguous()
    got = gm.apply(_code(P, op), xd)
    torch.cuda.synchronize()
    ref = oracle_apply(om, op, x, nlev)
    emax, _ = normwise_error(got.double().cpu().numpy().reshape(ref.shape), ref)
    assert emax <= TOL[dtype], (name, op, dtype, emax)


@pytest.mark.parametrize("op", ["grad", "div", "lapl"])
def test_launch_forms_bitwise_on_f24(P, op):
    gm = _gm(P, "F24")
    vec = op == "div"
    x = torch.randn((gm.nnodes, 137, 2) if vec else (gm.nnodes, 137), dtype=torch.float64,
                    device="cuda")
    ref = gm.apply(_code(P, op), x, launch=P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 1))
    shapes = [P.Launch(P.VARIANT_COLUMN, 256, 16, 0, 0, 0), P.Launch(P.VARIANT_FLAT, 256, 64, 0, 0, 0),
              P.Launch(P.VARIANT_SWEEP, 1024, 0, 0, 0, 0)]
    if op == "lapl":
        shapes.append(P.Launch(P.VARIANT_FUSED, 1024, 0, 0, 0, 0))
    for sh in shapes:
        try:
            out = gm.apply(_code(P, op), x, launch=sh)
        except P.AtlasError as e:  # a sweep tile too large for LDS is refused
            assert "too large" in str(e), e
            continue
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (op, sh.variant)
    if vec:
        d, c = gm.div_curl(x)
        torch.cuda.synchronize()
        assert torch.equal(d, ref)
        assert torch.equal(c, gm.curl(x))
