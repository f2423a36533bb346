"""The most levels a mesh takes, on a mesh where that limit is cheap to
reach: two parallels of 65,536 nodes each (a reduced Gaussian grid of two
latitudes, Section 4.2.3.4).  The sweep kernels address one parallel of
columns through one buffer resource with 32-bit byte offsets, so a mesh
takes fields of at most (2^31 - 1) / (16 * longest parallel) levels (16
bytes per level: an FP64 vector column); here 2047.

At that limit every operator must give, level for level, the bits it gives
on a 7-level field whose level k mod 7 the long field repeats, and the
7-level results match the FP64 oracle; one level more is refused before
any launch (real buffers of the refused size are passed).

The dual cells of this mesh are about 10^4 times taller than wide, so a
field that is smooth along the parallels makes the zonal edge terms cancel
to 1 part in 10^4 and FP32 rounding of the terms grows by that factor.
The inputs are therefore zonal waves of 8 to 32 nodes per wavelength,
where each edge term carries an O(1) part of the result and the FP32 bar
of the reduced Gaussian grids applies unchanged."""
import numpy as np
import pytest

import oracle
import synthetic as sy
from gpu_util import OPS, TOL, normwise_error, oracle_apply

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NX = 65536


@pytest.fixture(scope="module")
def meshes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06091_amd as P
    nx = np.full(2, NX, np.int32)
    return P, oracle.Mesh(nx=nx), P.Mesh(nx=nx)


def _waves(om, nlev, seed):
    """Scalar [V][nlev] and vector [V][nlev][2] fields: zonal waves of
    wavenumber NX/8, NX/16, NX/32 by level, random phases, latitude
    profiles that differ between the two parallels."""
    rng = sy.seed_rng(seed, 0, 0)
    f = np.empty((om.V, nlev))
    uv = np.empty((om.V, nlev, 2))
    for k in range(nlev):
        m = NX // (8 << (k % 3))
        ph = rng.uniform(0.0, 2.0 * np.pi, 3)
        f[:, k] = np.cos(m * om.lon + ph[0]) * (1.5 + np.sin(om.lat))
        uv[:, k, 0] = np.sin(m * om.lon + ph[1]) * (1.0 + 0.5 * np.cos(om.lat))
        uv[:, k, 1] = np.cos(m * om.lon + ph[2]) * (1.0 - 0.5 * np.sin(om.lat))
    return f, uv


def _fn(gm, op):
    return {"grad": gm.gradient, "div": gm.divergence, "curl": gm.curl,
            "lapl": gm.laplacian}[op]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_longest_parallel_at_the_level_limit(meshes, dtype):
    P, om, gm = meshes
    assert gm.nnodes == om.V == 2 * NX
    L = gm.max_levels
    assert L == (2 ** 31 - 1) // (16 * NX) == 2047
    tdt = torch.float64 if dtype == "f64" else torch.float32
    f, uv = _waves(om, 7, 131)
    kk = torch.arange(L, device="cuda") % 7
    for op in OPS:
        print(f"level limit {op} {dtype} nlev={L}", flush=True)
        host = uv if op in ("div", "curl") else f
        x = torch.from_numpy(np.ascontiguousarray(host)).to(device="cuda", dtype=tdt)
        short = _fn(gm, op)(x)
        torch.cuda.synchronize()
        ref = oracle_apply(om, op, x.double().cpu().numpy(), 7)
        emax, _ = normwise_error(short.double().cpu().numpy(), ref)
        assert emax <= TOL[dtype], (op, emax)
        xl = x.index_select(1, kk).contiguous()
        got = _fn(gm, op)(xl)
        torch.cuda.synchronize()
        assert torch.equal(got, short.index_select(1, kk)), (op, dtype)
        del got
        over = torch.cat((xl, xl[:, :1]), dim=1).contiguous()
        del xl
        with pytest.raises(P.AtlasError):
            _fn(gm, op)(over)
        del over
        torch.cuda.empty_cache()
