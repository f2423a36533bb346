"""GPU tests of the diagnostics (atlas_diag.h): the deterministic volume
integral and error norms against numpy, and the telescoping invariant
sum_i V_i div_i = sum_i V_i curl_i = 0 (every edge flux enters its two end
nodes with opposite signs; pole edges do not enter) measured on the device."""
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


@pytest.mark.parametrize("N,nlev", [(4, 3), (16, 137), (48, 37)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_volume_integral_matches_numpy(P, N, nlev, dtype):
    import oracle
    om, gm = oracle.Mesh(N), P.Mesh(N)
    rng = np.random.default_rng(N + nlev)
    x = rng.standard_normal((om.V, nlev)).astype(np.float32 if dtype == torch.float32 else np.float64)
    uv = rng.standard_normal((om.V, nlev, 2)).astype(x.dtype)
    xs = gm.volume_integral(torch.from_numpy(x).cuda()).cpu().numpy()
    xv = gm.volume_integral(torch.from_numpy(uv).cuda()).cpu().numpy()
    ref_s = (om.vol[:, None] * x.astype(np.float64)).sum(axis=0)
    ref_v = (om.vol[:, None, None] * uv.astype(np.float64)).sum(axis=0)
    scale_s = (om.vol[:, None] * np.abs(x)).sum(axis=0)
    scale_v = (om.vol[:, None, None] * np.abs(uv)).sum(axis=0)
    assert np.all(np.abs(xs - ref_s) <= 1e-13 * scale_s)
    assert np.all(np.abs(xv - ref_v) <= 1e-13 * scale_v)
    # deterministic: a second call gives the same bits
    again = gm.volume_integral(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(again, xs)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
@pytest.mark.parametrize("op", ["div", "curl"])
def test_volume_integral_of_div_and_curl_vanishes(P, op, dtype, tol):
    gm = P.Mesh(64)
    rng = np.random.default_rng(7)
    uv = torch.from_numpy(rng.standard_normal((gm.nnodes, 37, 2))).to(dtype=dtype, device="cuda")
    d = gm.divergence(uv) if op == "div" else gm.curl(uv)
    total = gm.volume_integral(d).cpu().numpy()
    absint = gm.volume_integral(d.abs()).cpu().numpy()
    assert np.all(np.abs(total) <= tol * absint), (np.abs(total) / absint).max()
    # a gradient does not integrate to zero: the check has teeth
    g = gm.gradient(uv[..., 0].contiguous())
    gt = gm.volume_integral(g).cpu().numpy()
    ga = gm.volume_integral(g.abs()).cpu().numpy()
    assert np.abs(gt).max() > 10 * tol * ga.max()


@pytest.mark.parametrize("gdt,rdt", [(torch.float64, torch.float64), (torch.float32, torch.float64),
                                     (torch.float64, torch.float32), (torch.float32, torch.float32)])
@pytest.mark.parametrize("shape", [(1,), (1000, 3), (5000, 7, 2)])
def test_error_norms_match_numpy(P, gdt, rdt, shape):
    rng = np.random.default_rng(3)
    ref = rng.standard_normal(shape)
    got = ref + 1e-3 * rng.standard_normal(shape)
    g = torch.from_numpy(got).to(dtype=gdt, device="cuda")
    r = torch.from_numpy(ref).to(dtype=rdt, device="cuda")
    res = P.error_norms(g, r)
    gh, rh = g.double().cpu().numpy(), r.double().cpu().numpy()
    comps = [(gh[..., c], rh[..., c]) for c in range(2)] if len(shape) == 3 else [(gh, rh)]
    for (a, b), rec in zip(comps, res["components"]):
        d = a - b
        assert rec["max_abs"] == np.abs(d).max()
        assert rec["ref_max"] == np.abs(b).max()
        assert abs(rec["rms"] - np.sqrt((d ** 2).mean())) <= 1e-12 * np.sqrt((d ** 2).mean())
        assert abs(rec["ref_rms"] - np.sqrt((b ** 2).mean())) <= 1e-12 * np.sqrt((b ** 2).mean())


def test_error_norms_propagate_nan(P):
    ref = torch.zeros(4096, dtype=torch.float64, device="cuda")
    got = ref.clone()
    got[1234] = float("nan")
    res = P.error_norms(got, ref)
    assert np.isnan(res["components"][0]["max_abs"])
    assert np.isnan(res["components"][0]["rms"])
