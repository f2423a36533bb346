"""Python binding of ``libatlas_nabla.so`` (MI355X / gfx950).

Argument marshalling only: every operator runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  There is no CPU
fallback: without the built library every call raises.

Names follow the C ABI in ``include/atlas_nabla.h`` (Atlas, Section 4.7 /
Listing 12: ``Nabla.gradient(in, out)`` and friends on NodeColumns fields,
Section 4.5 / Figure 31 layout [node][level]).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import numpy as np

from . import _abi
from ._abi import (ATLAS_ECANCELLED, ATLAS_ENOMEM, ATLAS_OK,  # noqa: F401
                   ATLAS_F32, ATLAS_F64, ATLAS_OP_CURL, ATLAS_OP_DIVERGENCE,  # noqa: F401
                   ATLAS_OP_GRADIENT, ATLAS_OP_LAPLACIAN, VARIANT_AUTO, VARIANT_COLUMN,
                   VARIANT_FLAT, VARIANT_FLUX, VARIANT_FUSED, VARIANT_SWEEP, AtlasError, Launch, Layout, MeshDesc,
                   MeshInfo)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libatlas_nabla.so")

_lock = threading.Lock()
_lib = None


def build(verbose: bool = False) -> str:
    from .build import build as _build
    return _build(verbose=verbose)


def lib():
    """The loaded library (built first if no library is present)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            _lib = _abi.bind(ctypes.CDLL(LIB_PATH))
        return _lib


def _check(rc):
    if rc != 0:
        raise AtlasError(rc, lib().atlas_last_error().decode())


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return ATLAS_F64
    if t.dtype == torch.float32:
        return ATLAS_F32
    raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float64")


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, what):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _out_ptr(t, like, numel, what):
    """Device pointer of a caller-supplied output, checked to hold exactly
    the `numel` elements of `like`'s dtype the library will write."""
    if t.dtype != like.dtype:
        raise TypeError(f"{what} dtype must match the input dtype")
    if t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, the operator writes {numel}")
    return _dev_ptr(t, what)


def _ws_ptr(t, need):
    """Device pointer of a caller-supplied workspace of at least `need` bytes
    (None: the mesh's own workspace)."""
    if t is None:
        return ctypes.c_void_p()
    if t.numel() * t.element_size() < need:
        raise ValueError(f"workspace holds {t.numel() * t.element_size()} bytes, "
                         f"the call needs {need}")
    return _dev_ptr(t, "workspace")


def mesh_desc_octahedral(N: int, radius: float = 1.0) -> dict:
    """The library's host description of O<N> (grid, triangulation, edges,
    signed node->edge table, median-dual geometry), copied into numpy."""
    L = lib()
    p = ctypes.POINTER(MeshDesc)()
    _check(L.atlas_mesh_desc_octahedral(int(N), float(radius), ctypes.byref(p)))
    try:
        return _abi.desc_to_numpy(p.contents)
    finally:
        L.atlas_mesh_desc_free(p)


def mesh_desc_reduced_gaussian(nx, radius: float = 1.0) -> dict:
    """The library's host description of the reduced Gaussian grid with
    nx[j] points on parallel j (2N parallels); ``regular_gaussian_nx(N)``
    gives F<N>."""
    import numpy as _np
    L = lib()
    arr = _np.ascontiguousarray(nx, dtype=_np.int32)
    p = ctypes.POINTER(MeshDesc)()
    _check(L.atlas_mesh_desc_reduced_gaussian(len(arr),
                                              arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              float(radius), ctypes.byref(p)))
    try:
        return _abi.desc_to_numpy(p.contents)
    finally:
        L.atlas_mesh_desc_free(p)


ATLAS_MESH_SHIFTED, ATLAS_MESH_QUADS = 1, 2


def mesh_desc_grid(nx, lat=None, *, shifted=False, quads=False, radius: float = 1.0) -> dict:
    """The library's host description of any grid of parallels
    (``atlas_mesh_desc_grid``): nx[j] points on parallel j at latitude lat[j]
    (radians; None: Gaussian latitudes), optionally shifted half a spacing
    east, optionally with quadrilaterals between parallels of equal counts.
    ``lonlat_grid(nlon, nlat)`` gives the regular longitude-latitude grids."""
    import numpy as _np
    L = lib()
    arr = _np.ascontiguousarray(nx, dtype=_np.int32)
    la = None if lat is None else _np.ascontiguousarray(lat, dtype=_np.float64)
    flags = (ATLAS_MESH_SHIFTED if shifted else 0) | (ATLAS_MESH_QUADS if quads else 0)
    p = ctypes.POINTER(MeshDesc)()
    _check(L.atlas_mesh_desc_grid(len(arr), arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  None if la is None else la.ctypes.data_as(
                                      ctypes.POINTER(ctypes.c_double)),
                                  flags, float(radius), ctypes.byref(p)))
    try:
        return _abi.desc_to_numpy(p.contents)
    finally:
        L.atlas_mesh_desc_free(p)


def lonlat_grid(nlon: int, nlat: int):
    """(nx, lat) of the regular longitude-latitude grid with nlat parallels
    at lat = pi/2 - (j + 1/2) pi / nlat (none on a pole) and nlon points on
    each: SLAT<nlon>x<nlat>, or S<nlon>x<nlat> with shifted=True."""
    import numpy as _np
    lat = 0.5 * _np.pi - (_np.arange(nlat) + 0.5) * _np.pi / nlat
    return _np.full(nlat, int(nlon), _np.int32), lat


def regular_gaussian_nx(N: int):
    """Points per parallel of F<N> (nx = 4N on each of the 2N parallels)."""
    import numpy as _np
    return _np.full(2 * int(N), 4 * int(N), dtype=_np.int32)


def bandwidth_probe(x, out, stream=None):
    """Streaming reference: read x (n elements), write 2n elements to out."""
    n = x.numel()
    if out.numel() < 2 * n or out.dtype != x.dtype:
        raise ValueError("out must hold 2 * x.numel() elements of x's dtype")
    _check(lib().atlas_bandwidth_probe(_dev_ptr(x, "x"), _dev_ptr(out, "out"), n - (n & 1),
                                       x.element_size(), _stream(stream)))
    return out


class Mesh:
    """A mesh resident on the current device (``atlas_mesh_upload``)."""

    def __init__(self, N: int | None = None, radius: float = 1.0, *, desc: dict | None = None,
                 layout: tuple[int, int] | None = None, nx=None, lat=None, shifted=False,
                 quads=False):
        """O<N> by default; ``nx`` (points per parallel) gives any reduced
        Gaussian grid, with ``lat`` any grid of parallels (``shifted``,
        ``quads`` as in mesh_desc_grid); ``desc`` any mesh description."""
        L = lib()
        self._lib = L
        self._h = ctypes.c_void_p()
        if desc is None and (lat is not None or shifted or quads):
            if nx is None:
                nx = [20 + 4 * j for j in range(N)] + [20 + 4 * j for j in range(N - 1, -1, -1)]
            desc = mesh_desc_grid(nx, lat, shifted=shifted, quads=quads, radius=radius)
            N = len(nx) // 2
        if nx is not None and desc is None:
            desc = mesh_desc_reduced_gaussian(nx, radius)
            N = len(nx) // 2
        if layout is not None and desc is None:
            desc = mesh_desc_octahedral(N, radius)
        if desc is not None:
            c_desc, keep = _abi.numpy_to_desc(desc)
            lay = ctypes.byref(Layout(*layout)) if layout is not None else None
            _check(L.atlas_mesh_upload_ex(ctypes.byref(c_desc), lay, ctypes.byref(self._h)))
            del keep
        else:
            _check(L.atlas_mesh_create_octahedral(int(N), float(radius), ctypes.byref(self._h)))
        info = MeshInfo()
        _check(L.atlas_mesh_get_info(self._h, ctypes.byref(info)))
        self.info = info
        self.nnodes = int(info.nnodes)
        self.nedges = int(info.nedges)
        self.max_levels = int(info.max_levels)
        self.N = N

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(self._lib.atlas_mesh_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def volume_integral(self, x, stream=None):
        """sum_i V_i x[i][k] (scalar [V][nlev]) or sum_i V_i x[i][k][c]
        (vector [V][nlev][2]) per level, as a float64 device tensor."""
        torch = _torch()
        if x.dim() == 3 and x.shape[2] == 2:
            nlev, ncomp = self._nlev_vector(x), 2
            out = torch.empty(nlev, 2, dtype=torch.float64, device=x.device)
        else:
            nlev, ncomp = self._nlev_scalar(x), 1
            out = torch.empty(nlev, dtype=torch.float64, device=x.device)
        _check(self._lib.atlas_diag_volume_integral(self._h, _dev_ptr(x, "x"), nlev, ncomp,
                                                    _dtype_code(x), _dev_ptr(out, "out"),
                                                    _stream(stream)))
        return out

    # -- shape helpers ------------------------------------------------------
    def _nlev_scalar(self, t):
        if t.dim() == 1:
            n = 1
        elif t.dim() == 2:
            n = t.shape[1]
        else:
            raise ValueError("scalar field must be [V] or [V, nlev]")
        if t.shape[0] != self.nnodes:
            raise ValueError(f"field has {t.shape[0]} nodes, mesh has {self.nnodes}")
        return int(n)

    def _nlev_vector(self, t):
        if t.dim() == 2 and t.shape[1] == 2:
            n = 1
        elif t.dim() == 3 and t.shape[2] == 2:
            n = t.shape[1]
        else:
            raise ValueError("vector field must be [V, 2] or [V, nlev, 2]")
        if t.shape[0] != self.nnodes:
            raise ValueError(f"field has {t.shape[0]} nodes, mesh has {self.nnodes}")
        return int(n)

    # -- operators ------------------------------------------------------------
    def apply(self, op: int, x, out=None, *, workspace=None, launch: Launch | None = None,
              stream=None):
        torch = _torch()
        vec_in = op in (ATLAS_OP_DIVERGENCE, ATLAS_OP_CURL)
        nlev = self._nlev_vector(x) if vec_in else self._nlev_scalar(x)
        shape = (self.nnodes, nlev, 2) if op == ATLAS_OP_GRADIENT else (self.nnodes, nlev)
        if out is None:
            out = torch.empty(shape, dtype=x.dtype, device=x.device)
        op_ = _out_ptr(out, x, math.prod(shape), "output")
        need = 0
        if workspace is not None:
            dc = _dtype_code(x)
            if op == ATLAS_OP_LAPLACIAN:
                need += self.laplacian_workspace_bytes(nlev, dc)
            if launch is not None and launch.variant == VARIANT_FLUX:
                need += self.flux_workspace_bytes(op, nlev, dc)
        ws = _ws_ptr(workspace, need)
        lp = ctypes.byref(launch) if launch is not None else None
        _check(self._lib.atlas_nabla_apply(self._h, int(op), _dev_ptr(x, "input"), nlev,
                                           _dtype_code(x), op_, ws, lp, _stream(stream)))
        return out

    def gradient(self, f, out=None, stream=None):
        nlev = self._nlev_scalar(f)
        if out is None:
            out = _torch().empty((self.nnodes, nlev, 2), dtype=f.dtype, device=f.device)
        op_ = _out_ptr(out, f, self.nnodes * nlev * 2, "out")
        _check(self._lib.atlas_nabla_gradient(self._h, _dev_ptr(f, "f"), nlev, _dtype_code(f),
                                              op_, _stream(stream)))
        return out

    def gradient_lonlat(self, f, out=None, stream=None):
        """(d f/d lon, d f/d lat) in the computational plane, [V][nlev][2]
        (``atlas_nabla_gradient_lonlat``)."""
        nlev = self._nlev_scalar(f)
        if out is None:
            out = _torch().empty((self.nnodes, nlev, 2), dtype=f.dtype, device=f.device)
        op_ = _out_ptr(out, f, self.nnodes * nlev * 2, "out")
        _check(self._lib.atlas_nabla_gradient_lonlat(self._h, _dev_ptr(f, "f"), nlev,
                                                     _dtype_code(f), op_, _stream(stream)))
        return out

    def divergence(self, uv, out=None, stream=None):
        nlev = self._nlev_vector(uv)
        if out is None:
            out = _torch().empty((self.nnodes, nlev), dtype=uv.dtype, device=uv.device)
        op_ = _out_ptr(out, uv, self.nnodes * nlev, "out")
        _check(self._lib.atlas_nabla_divergence(self._h, _dev_ptr(uv, "uv"), nlev,
                                                _dtype_code(uv), op_, _stream(stream)))
        return out

    def curl(self, uv, out=None, stream=None):
        nlev = self._nlev_vector(uv)
        if out is None:
            out = _torch().empty((self.nnodes, nlev), dtype=uv.dtype, device=uv.device)
        op_ = _out_ptr(out, uv, self.nnodes * nlev, "out")
        _check(self._lib.atlas_nabla_curl(self._h, _dev_ptr(uv, "uv"), nlev, _dtype_code(uv),
                                          op_, _stream(stream)))
        return out

    def div_curl(self, uv, out_div=None, out_curl=None, stream=None):
        """Divergence and curl of one (u, v) field in one pass."""
        nlev = self._nlev_vector(uv)
        if out_div is None:
            out_div = _torch().empty((self.nnodes, nlev), dtype=uv.dtype, device=uv.device)
        if out_curl is None:
            out_curl = _torch().empty((self.nnodes, nlev), dtype=uv.dtype, device=uv.device)
        od = _out_ptr(out_div, uv, self.nnodes * nlev, "out_div")
        oc = _out_ptr(out_curl, uv, self.nnodes * nlev, "out_curl")
        _check(self._lib.atlas_nabla_div_curl(self._h, _dev_ptr(uv, "uv"), nlev, _dtype_code(uv),
                                              od, oc, _stream(stream)))
        return out_div, out_curl

    def laplacian(self, f, out=None, workspace=None, stream=None):
        nlev = self._nlev_scalar(f)
        if out is None:
            out = _torch().empty((self.nnodes, nlev), dtype=f.dtype, device=f.device)
        op_ = _out_ptr(out, f, self.nnodes * nlev, "out")
        need = (self.laplacian_workspace_bytes(nlev, _dtype_code(f))
                if workspace is not None else 0)
        ws = _ws_ptr(workspace, need)
        _check(self._lib.atlas_nabla_laplacian(self._h, _dev_ptr(f, "f"), nlev, _dtype_code(f),
                                               op_, ws, _stream(stream)))
        return out

    def laplacian_workspace_bytes(self, nlev: int, dtype_code: int) -> int:
        return int(self._lib.atlas_laplacian_workspace_bytes(self._h, int(nlev), int(dtype_code)))

    def shape_of(self, op: int, nlev: int, like) -> dict:
        """The launch shape the named entry point of `op` runs for `nlev`
        levels in the dtype of tensor `like` (or a dtype code)."""
        dc = like if isinstance(like, int) else _dtype_code(like)
        sh = Launch()
        _check(self._lib.atlas_nabla_get_shape(self._h, int(op), int(nlev), int(dc),
                                               ctypes.byref(sh)))
        return {k: getattr(sh, k) for k, _ in Launch._fields_}

    def flux_workspace_bytes(self, op: int, nlev: int, dtype_code: int) -> int:
        return int(self._lib.atlas_flux_workspace_bytes(self._h, int(op), int(nlev),
                                                        int(dtype_code)))


class Remap:
    """Interpolation of nodal fields from `source` (a Mesh) to other points
    (``atlas_remap.h``): the nodes of another Mesh (`target`) or the points
    (lon, lat) in radians.  P1 interpolation on the source triangles;
    targets poleward of the polar parallels interpolate along them."""

    def __init__(self, source: Mesh, target: Mesh | None = None, *, lon=None, lat=None):
        import numpy as _np
        L = lib()
        self._lib = L
        self._h = ctypes.c_void_p()
        if target is not None:
            _check(L.atlas_remap_create_to_mesh(source.handle, target.handle,
                                                ctypes.byref(self._h)))
        else:
            lo = _np.ascontiguousarray(lon, dtype=_np.float64).ravel()
            la = _np.ascontiguousarray(lat, dtype=_np.float64).ravel()
            if lo.size != la.size:
                raise ValueError("lon and lat must have the same size")
            _check(L.atlas_remap_create(source.handle, lo.size,
                                        lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        la.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        ctypes.byref(self._h)))
        info = _abi.RemapInfo()
        _check(L.atlas_remap_get_info(self._h, ctypes.byref(info)))
        self.info = info
        self.nsource = int(info.nsource)
        self.ntarget = int(info.ntarget)

    @property
    def handle(self):
        return self._h

    def weights(self):
        """(idx [nt][3] int32, w [nt][3] float64), copied to the host."""
        import numpy as _np
        idx = _np.empty((self.ntarget, 3), _np.int32)
        w = _np.empty((self.ntarget, 3), _np.float64)
        _check(self._lib.atlas_remap_get_weights(
            self._h, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return idx, w

    def apply(self, x, out=None, stream=None):
        """x: device [nsource, ...] (any trailing shape: levels, components);
        returns [ntarget, ...] of x's dtype."""
        if x.shape[0] != self.nsource:
            raise ValueError(f"field has {x.shape[0]} nodes, the source mesh has {self.nsource}")
        ncol = math.prod(x.shape[1:]) if x.dim() > 1 else 1
        shape = (self.ntarget,) + tuple(x.shape[1:])
        if out is None:
            out = _torch().empty(shape, dtype=x.dtype, device=x.device)
        op_ = _out_ptr(out, x, self.ntarget * ncol, "out")
        _check(self._lib.atlas_remap_apply(self._h, _dev_ptr(x, "x"), int(ncol), _dtype_code(x),
                                           op_, _stream(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(self._lib.atlas_remap_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(mesh, op: int, x, out, workspace=None, stream=None):
    """Time the candidate launch shapes for (mesh, op, dtype, nlev) on these
    buffers; the mesh remembers the fastest.  Returns (Launch, ms)."""
    vec_in = op in (ATLAS_OP_DIVERGENCE, ATLAS_OP_CURL)
    nlev = mesh._nlev_vector(x) if vec_in else mesh._nlev_scalar(x)
    best = Launch()
    ms = ctypes.c_float()
    nout = mesh.nnodes * nlev * (2 if op == ATLAS_OP_GRADIENT else 1)
    o = _out_ptr(out, x, nout, "out")
    need = mesh.laplacian_workspace_bytes(nlev, _dtype_code(x)) if op == ATLAS_OP_LAPLACIAN else 0
    ws = _ws_ptr(workspace, need) if workspace is not None else ctypes.c_void_p()
    _check(lib().atlas_autotune(mesh.handle, int(op), _dev_ptr(x, "x"), nlev, _dtype_code(x),
                                o, ws, _stream(stream), ctypes.byref(best),
                                ctypes.byref(ms)))
    return best, ms.value


class Batch:
    """Many operator applications in one launch sequence (atlas_batch.h):
    small items in one persistent launch, items with nnodes * nlev at or
    above solo_min_elems (0: 2^22, -1: never) as their own launches.
    items: list of (mesh, op, x, out) or (mesh, op, x, out, workspace)."""

    def __init__(self, items, *, use_graph=True, autotune=False, block_threads=0,
                 blocks_per_cu=0, solo_min_elems=0, stream=None):
        if not items:
            raise ValueError("a batch needs at least one item")
        self._keep = []
        arr = (_abi.WorkItem * len(items))()
        dtype = None
        for i, it in enumerate(items):
            mesh, op, x, out = it[:4]
            ws = it[4] if len(it) > 4 else None
            vec_in = op in (ATLAS_OP_DIVERGENCE, ATLAS_OP_CURL)
            nlev = mesh._nlev_vector(x) if vec_in else mesh._nlev_scalar(x)
            d = _dtype_code(x)
            if dtype is None:
                dtype = d
            elif d != dtype:
                raise TypeError("all items of a batch share one dtype")
            arr[i].mesh = mesh.handle
            arr[i].op = int(op)
            arr[i].nlev = nlev
            arr[i].in_ = _dev_ptr(x, "input").value
            nout = mesh.nnodes * nlev * (2 if op == ATLAS_OP_GRADIENT else 1)
            arr[i].out = _out_ptr(out, x, nout, "output").value
            if ws is not None:
                need = mesh.laplacian_workspace_bytes(nlev, d) if op == ATLAS_OP_LAPLACIAN else 0
                arr[i].workspace = _ws_ptr(ws, need).value
            else:
                arr[i].workspace = None
            self._keep.append((mesh, x, out, ws))
        cfg = _abi.BatchConfig(dtype, int(use_graph), int(autotune), int(block_threads),
                               int(blocks_per_cu), int(solo_min_elems))
        self._lib = lib()
        self._h = ctypes.c_void_p()
        _check(self._lib.atlas_batch_build(arr, len(items), ctypes.byref(cfg), _stream(stream),
                                           ctypes.byref(self._h)))
        info = _abi.BatchInfo()
        _check(self._lib.atlas_batch_get_info(self._h, ctypes.byref(info)))
        self.info = info

    def launch(self, stream=None):
        _check(self._lib.atlas_batch_launch(self._h, _stream(stream)))

    def check(self):
        """Wait for the last launch."""
        _check(self._lib.atlas_batch_check(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(self._lib.atlas_batch_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def error_norms(got, ref, stream=None) -> dict:
    """Error of `got` against `ref` computed on the device (atlas_diag.h):
    per component (last axis of a [..][2] field, else one component) the
    max |got - ref|, the RMS of got - ref, max |ref| and RMS of ref, and the
    normwise ratios max_rel = max|d| / max|ref|, rms_rel = rms(d) / rms(ref)."""
    torch = _torch()
    if got.shape != ref.shape:
        raise ValueError("got and ref must have the same shape")
    ncomp = 2 if got.dim() == 3 and got.shape[-1] == 2 else 1
    n = got.numel() // ncomp
    out = torch.empty(4 * ncomp, dtype=torch.float64, device=got.device)
    _check(lib().atlas_diag_error_norms(_dev_ptr(got, "got"), _dtype_code(got), _dev_ptr(ref, "ref"),
                                        _dtype_code(ref), n, ncomp, _dev_ptr(out, "out"),
                                        _stream(stream)))
    v = out.cpu().numpy().reshape(ncomp, 4)
    comps = []
    for c in range(ncomp):
        dmax, dss, rmax, rss = (float(t) for t in v[c])
        comps.append({"max_abs": dmax, "rms": (dss / n) ** 0.5, "ref_max": rmax,
                      "ref_rms": (rss / n) ** 0.5,
                      "max_rel": dmax / rmax if rmax > 0 else dmax,
                      "rms_rel": (dss / rss) ** 0.5 if rss > 0 else dss ** 0.5})
    return {"components": comps, "max_rel": max(c["max_rel"] for c in comps),
            "rms_rel": max(c["rms_rel"] for c in comps)}


ATLAS_SERVE_OP_REMAP = 4


class Server:
    """Request server (atlas_serve.h): HBM-budget admission, resident meshes,
    continuous batching over `nstreams` HIP streams.  With simulate=True no
    device is touched (launch durations follow bytes / sim_bytes_per_us)."""

    def __init__(self, *, hbm_budget_bytes, nstreams=4, max_batch=64, batch_max_elems=0,
                 simulate=False, sim_bytes_per_us=1e6, fail_alloc_every=0):
        cfg = _abi.ServeConfig(int(hbm_budget_bytes), int(nstreams), int(max_batch),
                               int(batch_max_elems), int(bool(simulate)), float(sim_bytes_per_us),
                               int(fail_alloc_every))
        self._lib = lib()
        self._h = ctypes.c_void_p()
        self._keep = {}
        self._meshes = []
        self._remaps = []
        self._nnodes = {}  # mesh id -> nodes, to check request buffers
        self._remap_nodes = {}  # remap id -> (source nodes, target nodes)
        _check(self._lib.atlas_serve_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self.simulate = bool(simulate)

    def register_mesh(self, mesh) -> int:
        mid = ctypes.c_int32()
        _check(self._lib.atlas_serve_register_mesh(self._h, mesh.handle, ctypes.byref(mid)))
        self._meshes.append(mesh)
        self._nnodes[mid.value] = mesh.nnodes
        return mid.value

    def register_sim_mesh(self, nnodes: int) -> int:
        mid = ctypes.c_int32()
        _check(self._lib.atlas_serve_register_sim_mesh(self._h, int(nnodes), ctypes.byref(mid)))
        self._nnodes[mid.value] = int(nnodes)
        return mid.value

    def register_remap(self, remap) -> int:
        """A Remap whose weights remap requests (op ATLAS_SERVE_OP_REMAP) use."""
        rid = ctypes.c_int32()
        _check(self._lib.atlas_serve_register_remap(self._h, remap.handle, ctypes.byref(rid)))
        self._remaps.append(remap)
        self._remap_nodes[rid.value] = (remap.nsource, remap.ntarget)
        return rid.value

    def register_sim_remap(self, nsource: int, ntarget: int) -> int:
        rid = ctypes.c_int32()
        _check(self._lib.atlas_serve_register_sim_remap(self._h, int(nsource), int(ntarget),
                                                        ctypes.byref(rid)))
        self._remap_nodes[rid.value] = (int(nsource), int(ntarget))
        return rid.value

    def submit(self, mesh_id: int, op: int, x=None, out=None, *, nlev=None, dtype=None) -> int:
        """Device request: x (and out, or None for a server-owned output) are
        device tensors [V][nlev] or [V][nlev][2].  Simulation request: x is
        None and nlev, dtype (ATLAS_F32/ATLAS_F64) are given.  A remap
        request (op ATLAS_SERVE_OP_REMAP, mesh_id a remap id): x is
        [nsource, ...], out [ntarget, ...] with the same trailing shape."""
        if x is None:
            req = _abi.Request(int(mesh_id), int(op), int(dtype), int(nlev), None, None)
        elif op == ATLAS_SERVE_OP_REMAP:
            ns, nt = self._remap_nodes[int(mesh_id)]
            if x.shape[0] != ns:
                raise ValueError(f"input has {x.shape[0]} nodes, remap {mesh_id} reads {ns}")
            ncol = x.numel() // ns
            o = None
            if out is not None:
                o = _out_ptr(out, x, nt * ncol, "output").value
            req = _abi.Request(int(mesh_id), int(op), _dtype_code(x), int(ncol),
                               _dev_ptr(x, "input").value, o)
        else:
            vec_in = op in (ATLAS_OP_DIVERGENCE, ATLAS_OP_CURL)
            lev = x.shape[1] if x.dim() >= 2 else 1
            if vec_in and (x.dim() != 3 or x.shape[2] != 2):
                raise ValueError("vector input must be [V][nlev][2]")
            V = self._nnodes.get(int(mesh_id))
            if V is not None and x.shape[0] != V:
                raise ValueError(f"input has {x.shape[0]} nodes, mesh {mesh_id} has {V}")
            if V is not None and x.numel() != V * lev * (2 if vec_in else 1):
                raise ValueError("input must be [V][nlev] (scalar) or [V][nlev][2] (vector)")
            o = None
            if out is not None:
                nout = (V or x.shape[0]) * lev * (2 if op == ATLAS_OP_GRADIENT else 1)
                o = _out_ptr(out, x, nout, "output").value
            req = _abi.Request(int(mesh_id), int(op), _dtype_code(x), int(lev),
                               _dev_ptr(x, "input").value, o)
        t = ctypes.c_uint64()
        _check(self._lib.atlas_serve_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (x, out)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> dict:
        r = _abi.Result()
        _check(self._lib.atlas_serve_wait(self._h, int(ticket), int(timeout_us), ctypes.byref(r)))
        return {"status": r.status, "batch_size": r.batch_size, "out": r.out or 0,
                "queue_us": r.queue_us, "run_us": r.run_us, "total_us": r.total_us}

    def cancel(self, ticket: int):
        _check(self._lib.atlas_serve_cancel(self._h, int(ticket)))

    def release(self, ticket: int):
        _check(self._lib.atlas_serve_release(self._h, int(ticket)))
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        s = _abi.ServeStats()
        _check(self._lib.atlas_serve_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _abi.ServeStats._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(self._lib.atlas_serve_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["error_norms", "Server", "Batch", "autotune", "Mesh", "mesh_desc_octahedral",
           "mesh_desc_reduced_gaussian", "regular_gaussian_nx", "lib", "build", "Launch", "AtlasError",
           "ATLAS_F32", "ATLAS_F64", "ATLAS_OP_GRADIENT", "ATLAS_OP_DIVERGENCE",
           "ATLAS_OP_CURL", "ATLAS_OP_LAPLACIAN", "VARIANT_AUTO", "VARIANT_COLUMN",
           "VARIANT_FLAT", "VARIANT_FLUX", "VARIANT_FUSED", "VARIANT_SWEEP"]
