"""FP64 CPU oracle for the median-dual finite-volume nabla operators.

TEST INFRASTRUCTURE ONLY.  This package is the correctness reference the GPU
library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import it; the GPU library never does, and
this package never imports the GPU library.

The arithmetic lives in ``nabla_oracle.c`` (plain C, FP64, OpenMP over
disjoint level chunks); this module only builds it with gcc and marshals
numpy arrays through ctypes.  Paper anchors (Atlas, ESCAPE D1.3):
Section 4.2.3.5 and 4.2.3.7 / Listing 6 for the octahedral Gaussian grid,
Section 4.3 for the mesh, Section 4.5 / Figure 31 for the [node][level]
field layout and Section 4.7 / Figure 33 / Listing 12 for the operators.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nabla_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_nabla.so")
_lock = threading.Lock()
_lib = None

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no fast-math, no FMA
    contraction).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_gauss_mu.argtypes = [ctypes.c_int, _c_dp]
        lib.orc_mesh_build.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.orc_mesh_build.restype = ctypes.c_void_p
        lib.orc_mesh_build_pl.argtypes = [ctypes.c_int, _c_i32p, ctypes.c_double]
        lib.orc_mesh_build_pl.restype = ctypes.c_void_p
        lib.orc_mesh_build_ex.argtypes = [ctypes.c_int, _c_i32p, _c_dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double]
        lib.orc_mesh_build_ex.restype = ctypes.c_void_p
        lib.orc_mesh_copy_quads.argtypes = [ctypes.c_void_p, _c_i32p]
        lib.orc_mesh_free.argtypes = [ctypes.c_void_p]
        lib.orc_mesh_sizes.argtypes = [ctypes.c_void_p, _c_i64p]
        lib.orc_mesh_copy.argtypes = [ctypes.c_void_p, _c_i32p, _c_i64p, _c_dp,
                                      _c_dp, _c_i32p, _c_i32p, _c_dp, _c_dp,
                                      _c_dp, _c_i32p, _c_dp]
        lib.orc_threads_used.argtypes = [ctypes.c_int]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        for name in ("orc_gradient", "orc_gradient_lonlat", "orc_divergence", "orc_curl",
                     "orc_laplacian"):
            getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_int, _c_dp, _c_dp]
        for name in ("orc_gradient_at", "orc_divergence_at", "orc_curl_at",
                     "orc_laplacian_at"):
            getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_int, _c_dp,
                                           ctypes.c_int64, _c_i64p, _c_dp]
        lib.orc_remap_weights.argtypes = [ctypes.c_void_p, ctypes.c_int64, _c_dp, _c_dp,
                                          _c_i32p, _c_dp]
        lib.orc_remap_apply.argtypes = [ctypes.c_int64, ctypes.c_int64, _c_i32p, _c_dp,
                                        ctypes.c_int, _c_dp, _c_dp]
        _lib = lib
        return lib


def _dp(a):
    return a.ctypes.data_as(_c_dp)


def gauss_mu(N: int) -> np.ndarray:
    """The 2N Gaussian latitudes as mu = sin(lat), descending (Sec. 4.2.3.5)."""
    out = np.empty(2 * N, dtype=np.float64)
    if _load().orc_gauss_mu(int(N), _dp(out)) != 0:
        raise ValueError("N must be >= 1")
    return out


def threads_used(nlev: int) -> int:
    """Number of OpenMP threads the dense operators use for ``nlev`` levels."""
    return int(_load().orc_threads_used(int(nlev)))


def set_threads(n: int) -> int:
    """Threads the oracle's later calls may use (timing only: results do not
    depend on it); returns the previous maximum."""
    return int(_load().orc_set_threads(int(n)))


def shifted_lonlat(nlon: int, nlat: int):
    """Points per parallel and latitudes of the regular lon-lat grid with
    nlat parallels at lat = 90 deg - (j + 1/2) 180 deg / nlat (no point on
    a pole) and nlon points on each (Section 4.2.3.8: the latitude-shifted
    grid SLAT<nlon>x<nlat>; with ``shift=True`` in Mesh, the shifted grid
    S<nlon>x<nlat>)."""
    lat = 0.5 * np.pi - (np.arange(nlat) + 0.5) * np.pi / nlat
    return np.full(nlat, int(nlon), np.int32), lat


def regular_gaussian_nx(N: int) -> np.ndarray:
    """Points per parallel of the regular Gaussian grid F<N> (Section
    4.2.3.6: nx = 4N on each of the 2N parallels)."""
    return np.full(2 * int(N), 4 * int(N), dtype=np.int32)


class Mesh:
    """A grid of parallels, its mesh, edges and median-dual geometry, built
    by the oracle: O<N> from (N, R) alone (Section 4.2.3.7, Listing 6), or
    any grid from its points per parallel ``nx`` (at the Gaussian latitudes
    of degree len(nx), or at explicit latitudes ``lat``; ``shift`` puts the
    first point of every parallel half a spacing east of lon 0, as the
    shifted regular grids of Section 4.2.3.8; ``quads`` makes every strip
    between two parallels of equal counts a row of quadrilaterals instead of
    triangles, so the elements come in two blocks, ``tri`` and ``quad``)."""

    def __init__(self, N: int = 0, R: float = 1.0, nx=None, *, lat=None, shift=False,
                 quads=False):
        lib = _load()
        self._lib = lib
        if nx is None and lat is None and not shift and not quads:
            self._h = lib.orc_mesh_build(int(N), float(R))
            what = f"O{N}"
        else:
            if nx is None:
                nx = np.array([20 + 4 * j for j in range(N)] +
                              [20 + 4 * j for j in range(N - 1, -1, -1)], np.int32)
            nx = np.ascontiguousarray(nx, dtype=np.int32)
            N = len(nx) // 2
            if lat is None and not shift and not quads:
                self._h = lib.orc_mesh_build_pl(len(nx), nx.ctypes.data_as(_c_i32p), float(R))
            else:
                la = None if lat is None else np.ascontiguousarray(lat, dtype=np.float64)
                self._h = lib.orc_mesh_build_ex(len(nx), nx.ctypes.data_as(_c_i32p),
                                                None if la is None else _dp(la), int(bool(shift)),
                                                int(bool(quads)), float(R))
            what = f"the grid with nx={nx.tolist()[:4]}..."
        if not self._h:
            raise ValueError(f"cannot build {what} with R={R}")
        sz = np.zeros(8, dtype=np.int64)
        lib.orc_mesh_sizes(self._h, sz.ctypes.data_as(_c_i64p))
        self.N = int(N)
        self.R = float(R)
        self.V, self.E, self.F, self.npole, self.nrings = (int(x) for x in sz[:5])
        self.Q = int(sz[6])
        self.nx = np.empty(self.nrings, np.int32)
        self.ring_off = np.empty(self.nrings + 1, np.int64)
        self.lon = np.empty(self.V, np.float64)
        self.lat = np.empty(self.V, np.float64)
        self.tri = np.empty((self.F, 3), np.int32)
        self.quad = np.empty((self.Q, 4), np.int32)
        self.edge = np.empty((self.E, 2), np.int32)
        self.S = np.empty((self.E, 2), np.float64)
        self.A = np.empty(self.V, np.float64)
        self.vol = np.empty(self.V, np.float64)
        self.pole_edge = np.empty((self.npole, 2), np.int32)
        self.pole_normal = np.empty(self.npole, np.float64)
        lib.orc_mesh_copy(self._h, self.nx.ctypes.data_as(_c_i32p),
                          self.ring_off.ctypes.data_as(_c_i64p), _dp(self.lon),
                          _dp(self.lat), self.tri.ctypes.data_as(_c_i32p),
                          self.edge.ctypes.data_as(_c_i32p), _dp(self.S),
                          _dp(self.A), _dp(self.vol),
                          self.pole_edge.ctypes.data_as(_c_i32p),
                          _dp(self.pole_normal))
        lib.orc_mesh_copy_quads(self._h, self.quad.ctypes.data_as(_c_i32p))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_mesh_free(h)
            self._h = None

    # -- dense operators ---------------------------------------------------
    def _scalar_in(self, f, nlev):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.size != self.V * nlev:
            raise ValueError("scalar field must be [V][nlev]")
        return f

    def _vector_in(self, uv, nlev):
        uv = np.ascontiguousarray(uv, dtype=np.float64)
        if uv.size != self.V * nlev * 2:
            raise ValueError("vector field must be [V][nlev][2]")
        return uv

    def gradient(self, f, nlev: int = 1) -> np.ndarray:
        f = self._scalar_in(f, nlev)
        out = np.empty((self.V, nlev, 2), np.float64)
        if self._lib.orc_gradient(self._h, nlev, _dp(f), _dp(out)) != 0:
            raise ValueError("orc_gradient failed")
        return out

    def gradient_lonlat(self, f, nlev: int = 1) -> np.ndarray:
        """(d f/d lon, d f/d lat) at the nodes, [V][nlev][2]: the gradient's
        edge sums divided by the dual area in the (lon, lat) plane."""
        f = self._scalar_in(f, nlev)
        out = np.empty((self.V, nlev, 2), np.float64)
        if self._lib.orc_gradient_lonlat(self._h, nlev, _dp(f), _dp(out)) != 0:
            raise ValueError("orc_gradient_lonlat failed")
        return out

    def divergence(self, uv, nlev: int = 1) -> np.ndarray:
        uv = self._vector_in(uv, nlev)
        out = np.empty((self.V, nlev), np.float64)
        if self._lib.orc_divergence(self._h, nlev, _dp(uv), _dp(out)) != 0:
            raise ValueError("orc_divergence failed")
        return out

    def curl(self, uv, nlev: int = 1) -> np.ndarray:
        uv = self._vector_in(uv, nlev)
        out = np.empty((self.V, nlev), np.float64)
        if self._lib.orc_curl(self._h, nlev, _dp(uv), _dp(out)) != 0:
            raise ValueError("orc_curl failed")
        return out

    def laplacian(self, f, nlev: int = 1) -> np.ndarray:
        f = self._scalar_in(f, nlev)
        out = np.empty((self.V, nlev), np.float64)
        if self._lib.orc_laplacian(self._h, nlev, _dp(f), _dp(out)) != 0:
            raise ValueError("orc_laplacian failed")
        return out

    # -- sampled operators (bitwise equal to the dense ones) ---------------
    def _sel(self, nodes):
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        if nodes.size and (nodes.min() < 0 or nodes.max() >= self.V):
            raise ValueError("node index out of range")
        return nodes

    def gradient_at(self, f, nlev: int, nodes) -> np.ndarray:
        f = self._scalar_in(f, nlev)
        sel = self._sel(nodes)
        out = np.empty((sel.size, nlev, 2), np.float64)
        rc = self._lib.orc_gradient_at(self._h, nlev, _dp(f), sel.size,
                                       sel.ctypes.data_as(_c_i64p), _dp(out))
        if rc != 0:
            raise ValueError("orc_gradient_at failed")
        return out

    def _vec_at(self, name, uv, nlev, nodes):
        uv = self._vector_in(uv, nlev)
        sel = self._sel(nodes)
        out = np.empty((sel.size, nlev), np.float64)
        rc = getattr(self._lib, name)(self._h, nlev, _dp(uv), sel.size,
                                      sel.ctypes.data_as(_c_i64p), _dp(out))
        if rc != 0:
            raise ValueError(f"{name} failed")
        return out

    def divergence_at(self, uv, nlev: int, nodes) -> np.ndarray:
        return self._vec_at("orc_divergence_at", uv, nlev, nodes)

    def curl_at(self, uv, nlev: int, nodes) -> np.ndarray:
        return self._vec_at("orc_curl_at", uv, nlev, nodes)

    def laplacian_at(self, f, nlev: int, nodes) -> np.ndarray:
        f = self._scalar_in(f, nlev)
        sel = self._sel(nodes)
        out = np.empty((sel.size, nlev), np.float64)
        rc = self._lib.orc_laplacian_at(self._h, nlev, _dp(f), sel.size,
                                        sel.ctypes.data_as(_c_i64p), _dp(out))
        if rc != 0:
            raise ValueError("orc_laplacian_at failed")
        return out

    # -- remap to other points (Section 1: interpolation between grids) -----
    def remap_weights(self, lon, lat):
        """Source nodes and weights of the P1 interpolant on this mesh's
        triangles at the target points (lon, lat in radians): two arrays of
        shape [nt][3] (int32 node ids, FP64 weights).  Targets poleward of
        the polar parallels take the linear interpolant along that parallel
        (two nonzero weights)."""
        lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
        lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
        if lon.size != lat.size:
            raise ValueError("lon and lat must have the same size")
        idx = np.empty((lon.size, 3), np.int32)
        w = np.empty((lon.size, 3), np.float64)
        rc = self._lib.orc_remap_weights(self._h, lon.size, _dp(lon), _dp(lat),
                                         idx.ctypes.data_as(_c_i32p), _dp(w))
        if rc == -3:
            raise ValueError("remap needs a triangulated mesh with parallels starting at lon 0")
        if rc != 0:
            raise ValueError("a target latitude is outside [-pi/2, pi/2] or not finite")
        return idx, w

    def remap(self, x, ncol: int, lon, lat) -> np.ndarray:
        """Field x [V][ncol] of this mesh (ncol values per node: levels, or
        levels x components) interpolated to the target points: [nt][ncol]."""
        idx, w = self.remap_weights(lon, lat)
        return remap_apply(idx, w, x, ncol, self.V)


def remap_apply(idx, w, x, ncol: int, nsrc: int) -> np.ndarray:
    """out[t] = sum_k w[t][k] x[idx[t][k]] (k = 0, 1, 2 in that order), for
    x of nsrc nodes with ncol values each."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.size != nsrc * ncol or idx.shape != w.shape or idx.ndim != 2 or idx.shape[1] != 3:
        raise ValueError("shapes: idx, w [nt][3]; x [nsrc][ncol]")
    out = np.empty((idx.shape[0], ncol), np.float64)
    rc = _load().orc_remap_apply(nsrc, idx.shape[0], idx.ctypes.data_as(_c_i32p), _dp(w),
                                 int(ncol), _dp(x), _dp(out))
    if rc != 0:
        raise ValueError("source index out of range")
    return out
