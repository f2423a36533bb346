"""GPU parity on meshes with quadrilateral elements (Section 4.3: the
blocked quadrilaterals of regular grids; a mesh with two element blocks,
Figure 27) and on the regular longitude-latitude grids without points on
the poles (Section 4.2.3.8: SLAT and S): every operator, both dtypes,
against the FP64 oracle built independently on the same grid; every launch
form gives the same bits."""
import numpy as np
import pytest

from gpu_util import OPS, TOL, make_inputs, normwise_error, oracle_apply

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06091_amd as P
    return P


def _pair(P, case):
    import oracle
    if case in ("SLAT32x16", "S24x12"):
        shifted = case == "S24x12"
        nlon, nlat = (32, 16) if case == "SLAT32x16" else (24, 12)
        nx, lat = P.lonlat_grid(nlon, nlat)
        return (oracle.Mesh(nx=nx, lat=lat, shift=shifted, quads=True),
                P.Mesh(nx=nx, lat=lat, shifted=shifted, quads=True))
    if case == "O16q":
        return oracle.Mesh(16, quads=True), P.Mesh(16, quads=True)
    nx = np.full(16, 32, np.int32)  # F8
    return oracle.Mesh(nx=nx, quads=True), P.Mesh(nx=nx, quads=True)


def _run(P, gm, op, x, launch=None):
    code = {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}[op]
    out = gm.apply(code, x, launch=launch)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("case", ["SLAT32x16", "S24x12", "O16q", "F8q"])
@pytest.mark.parametrize("nlev", [1, 7, 137])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_parity_quadrilateral_meshes(P, case, nlev, dtype):
    om, gm = _pair(P, case)
    assert om.V == gm.nnodes and om.E == gm.nedges
    print(f"quads {case} nlev={nlev} {dtype}", flush=True)
    f, uv = make_inputs(om, nlev, lmax=6, config=97)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for op in OPS:
        host = uv if op in ("div", "curl") else f
        x = torch.from_numpy(np.ascontiguousarray(host)).to(device="cuda", dtype=tdt)
        got = _run(P, gm, op, x).double().cpu().numpy()
        ref = oracle_apply(om, op, x.double().cpu().numpy(), nlev)
        emax, _ = normwise_error(got, ref)
        assert emax <= TOL[dtype], (case, op, emax)


@pytest.mark.parametrize("op", OPS)
def test_launch_forms_bitwise_on_quads(P, op):
    om, gm = _pair(P, "SLAT32x16")
    f, uv = make_inputs(om, 72, lmax=6, config=98)
    x = torch.from_numpy(np.ascontiguousarray(uv if op in ("div", "curl") else f)).cuda()
    base = _run(P, gm, op, x)
    shapes = [P.Launch(P.VARIANT_COLUMN, 256, 16), P.Launch(P.VARIANT_COLUMN, 64, 0),
              P.Launch(P.VARIANT_FLAT, 256, 64), P.Launch(P.VARIANT_FLUX, 256, 0),
              P.Launch(P.VARIANT_SWEEP, 512, 0), P.Launch(P.VARIANT_SWEEP, 1024, 0, 0, 1),
              P.Launch(P.VARIANT_COLUMN, 256, 0, 0, 0, 1)]
    for sh in shapes:
        got = _run(P, gm, op, x, launch=sh)
        assert torch.equal(got, base), (op, sh.variant, sh.block_threads)
