"""CPU-side checks of the C ABI: the library loads, exports every symbol the
headers declare, and its host-side mesh setup agrees with the oracle's
(topology bit for bit, geometry to rounding).  No GPU call is made."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(atlas_[a-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def P():
    import paper_1908_06091_amd as P
    return P


def test_library_exports_every_declared_symbol(P):
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1908_06091_amd import _abi
    assert set(_abi.SIGNATURES) <= names


@pytest.mark.parametrize("N", [1, 2, 16, 160])
def test_host_mesh_matches_oracle(P, N):
    d = P.mesh_desc_octahedral(N)
    m = oracle.Mesh(N)
    np.testing.assert_array_equal(d["edge2node"], m.edge)
    np.testing.assert_array_equal(d["pole_edges"], m.pole_edge)
    np.testing.assert_allclose(d["lat"], m.lat, rtol=0, atol=4e-16)
    np.testing.assert_array_equal(d["lon"], m.lon)
    np.testing.assert_allclose(d["dual_normals"], m.S, rtol=0, atol=1e-15)
    np.testing.assert_allclose(d["dual_volumes"], m.vol, rtol=1e-13)
    np.testing.assert_array_equal(d["pole_normals"], m.pole_normal)
    # the CSR lists each node's edges in ascending id with the right sign
    ptr, e, s = d["node2edge_ptr"], d["node2edge"], d["node2edge_sign"]
    for i in range(0, m.V, max(1, m.V // 200)):
        row = e[ptr[i]:ptr[i + 1]]
        assert np.all(np.diff(row) > 0)
        ends = m.edge[row]
        np.testing.assert_array_equal(np.where(ends[:, 0] == i, 1, -1), s[ptr[i]:ptr[i + 1]])
        assert np.all((ends[:, 0] == i) | (ends[:, 1] == i))


def test_host_errors_without_gpu(P):
    L = P.lib()
    p = ctypes.POINTER(P._abi.MeshDesc)()
    assert L.atlas_mesh_desc_octahedral(0, 1.0, ctypes.byref(p)) == -1
    assert b"N must be" in L.atlas_last_error()
    assert L.atlas_mesh_desc_octahedral(4, -1.0, ctypes.byref(p)) == -1
    # malformed descriptions are rejected before any device call
    d = P.mesh_desc_octahedral(4)
    for key, mutate in [
        ("edge2node", lambda a: a[::-1].copy()),
        ("node2edge_sign", lambda a: -a),
        ("dual_volumes", lambda a: -a),
        ("node2edge", lambda a: np.roll(a, 1)),
    ]:
        bad = dict(d)
        bad[key] = mutate(np.asarray(d[key]))
        desc, keep = P._abi.numpy_to_desc(bad)
        h = ctypes.c_void_p()
        assert L.atlas_mesh_upload(ctypes.byref(desc), ctypes.byref(h)) == -1, key
        assert not h.value
    h = ctypes.c_void_p()
    assert L.atlas_mesh_upload(None, ctypes.byref(h)) == -1
    assert L.atlas_nabla_gradient(None, None, 1, 1, None, None) == -1
    assert L.atlas_mesh_desc_free(ctypes.cast(ctypes.c_void_p(16), ctypes.POINTER(P._abi.MeshDesc))) == -1


def test_product_package_has_no_cpu_fallback():
    """The package never imports the oracle and never computes operators on
    the host: grep its Python sources."""
    pkg = os.path.join(ROOT, "paper_1908_06091_amd")
    for py in glob.glob(os.path.join(pkg, "*.py")):
        text = open(py).read()
        assert "import oracle" not in text and "from oracle" not in text, py
        assert "synthetic" not in text, py


@pytest.mark.parametrize("nx", [[4] * 2, [8] * 4, [64] * 32, [6, 9, 13, 13, 10, 8]])
def test_host_reduced_gaussian_matches_oracle(P, nx):
    """Regular (F<N>) and hand-made reduced Gaussian grids: the library's
    host description against the oracle's, topology bit for bit."""
    nx = np.array(nx, np.int32)
    d = P.mesh_desc_reduced_gaussian(nx)
    m = oracle.Mesh(nx=nx)
    np.testing.assert_array_equal(d["edge2node"], m.edge)
    np.testing.assert_array_equal(d["pole_edges"], m.pole_edge)
    np.testing.assert_allclose(d["lat"], m.lat, rtol=0, atol=4e-16)
    np.testing.assert_array_equal(d["lon"], m.lon)
    np.testing.assert_allclose(d["dual_normals"], m.S, rtol=0, atol=1e-15)
    np.testing.assert_allclose(d["dual_volumes"], m.vol, rtol=1e-13)
    np.testing.assert_array_equal(d["pole_normals"], m.pole_normal)


def test_host_reduced_gaussian_rejects_bad_grids(P):
    for nx in ([5, 8, 8, 6], [6, 8, 8], [6, 3, 8, 6]):
        with pytest.raises(P.AtlasError):
            P.mesh_desc_reduced_gaussian(np.array(nx, np.int32))
    # O<N> through the general builder is O<N>
    o = P.mesh_desc_octahedral(3)
    r = P.mesh_desc_reduced_gaussian(np.array([20, 24, 28, 28, 24, 20], np.int32))
    for k in ("edge2node", "lon", "lat", "dual_normals", "dual_volumes", "pole_edges"):
        np.testing.assert_array_equal(o[k], r[k])


@pytest.mark.parametrize("case", ["SLAT16x8", "S12x6", "O6q", "F4q", "R3q"])
def test_host_grids_with_quadrilaterals_match_oracle(P, case):
    """Regular longitude-latitude grids (latitude-shifted and shifted) and
    Gaussian grids meshed with quadrilaterals where two parallels have equal
    counts: the library's host description (element blocks included)
    against the oracle's, topology bit for bit."""
    if case.startswith(("SLAT", "S")):
        shifted = not case.startswith("SLAT")
        nlon, nlat = (16, 8) if case == "SLAT16x8" else (12, 6)
        nx, lat = P.lonlat_grid(nlon, nlat)
        d = P.mesh_desc_grid(nx, lat, shifted=shifted, quads=True)
        m = oracle.Mesh(nx=nx, lat=lat, shift=shifted, quads=True)
    else:
        nx = {"O6q": np.array([20 + 4 * j for j in range(6)] + [20 + 4 * j for j in range(5, -1, -1)]),
              "F4q": np.full(8, 16), "R3q": np.array([6, 9, 9, 13, 10, 8])}[case].astype(np.int32)
        d = P.mesh_desc_grid(nx, quads=True)
        m = oracle.Mesh(nx=nx, quads=True)
    np.testing.assert_array_equal(d["edge2node"], m.edge)
    np.testing.assert_array_equal(d["triangles"], m.tri)
    np.testing.assert_array_equal(d["quads"], m.quad)
    np.testing.assert_array_equal(d["pole_edges"], m.pole_edge)
    np.testing.assert_array_equal(d["lon"], m.lon)
    np.testing.assert_allclose(d["lat"], m.lat, rtol=0, atol=4e-16)
    np.testing.assert_allclose(d["dual_normals"], m.S, rtol=0, atol=1e-15)
    np.testing.assert_allclose(d["dual_volumes"], m.vol, rtol=1e-13)
    np.testing.assert_array_equal(d["pole_normals"], m.pole_normal)
    assert len(m.quad) > 0


def test_host_grid_arguments_refused(P):
    nx = np.full(4, 8, np.int32)
    for lat in (np.array([1.0, 0.5, 0.5, -1.0]), np.array([1.6, 0.5, 0.0, -1.0]),
                np.array([np.nan, 0.5, 0.0, -1.0])):
        with pytest.raises(P.AtlasError):
            P.mesh_desc_grid(nx, lat)
    with pytest.raises(P.AtlasError):  # shifted needs equal counts
        P.mesh_desc_grid(np.array([8, 12, 12, 8], np.int32), shifted=True)
