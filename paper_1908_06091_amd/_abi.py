"""ctypes declarations mirroring ``include/atlas_nabla.h``."""
from __future__ import annotations

import ctypes

import numpy as np

ATLAS_F32, ATLAS_F64 = 0, 1
ATLAS_OP_GRADIENT, ATLAS_OP_DIVERGENCE, ATLAS_OP_CURL, ATLAS_OP_LAPLACIAN = 0, 1, 2, 3
VARIANT_AUTO, VARIANT_COLUMN, VARIANT_FLAT, VARIANT_FLUX, VARIANT_SWEEP, VARIANT_FUSED = 0, 1, 2, 3, 4, 5

STATUS = {0: "ATLAS_OK", -1: "ATLAS_EINVAL", -2: "ATLAS_ENOMEM", -3: "ATLAS_EDEVICE",
          -4: "ATLAS_EBUSY", -5: "ATLAS_ESTATE", -6: "ATLAS_ETIMEOUT", -7: "ATLAS_ECANCELLED"}
ATLAS_OK, ATLAS_EINVAL, ATLAS_ENOMEM, ATLAS_EDEVICE = 0, -1, -2, -3
ATLAS_EBUSY, ATLAS_ESTATE, ATLAS_ETIMEOUT, ATLAS_ECANCELLED = -4, -5, -6, -7


class AtlasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i8p = ctypes.POINTER(ctypes.c_int8)


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("nnodes", ctypes.c_int64), ("lon", _dp), ("lat", _dp), ("cos_lat", _dp),
        ("nrings", ctypes.c_int32), ("ring_off", _i64p),
        ("nedges", ctypes.c_int64), ("edge2node", _i32p),
        ("node2edge_ptr", _i64p), ("node2edge", _i32p), ("node2edge_sign", _i8p),
        ("dual_volumes", _dp), ("dual_normals", _dp),
        ("npole_edges", ctypes.c_int64), ("pole_edges", _i32p), ("pole_normals", _dp),
        ("radius", ctypes.c_double),
        ("ntriangles", ctypes.c_int64), ("triangles", _i32p),
        ("nquads", ctypes.c_int64), ("quads", _i32p),
    ]


class MeshInfo(ctypes.Structure):
    _fields_ = [
        ("nnodes", ctypes.c_int64), ("nedges", ctypes.c_int64),
        ("nincidences", ctypes.c_int64), ("npole_edges", ctypes.c_int64),
        ("ntiles", ctypes.c_int64), ("nrings", ctypes.c_int32),
        ("max_degree", ctypes.c_int32), ("device_bytes", ctypes.c_size_t),
        ("geometry_bytes_per_call", ctypes.c_double), ("max_levels", ctypes.c_int64),
    ]


class Layout(ctypes.Structure):
    _fields_ = [("band_rings", ctypes.c_int32), ("sector_nodes", ctypes.c_int32)]


class Launch(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("nodes_per_block", ctypes.c_int32), ("level_chunk", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("level_vec", ctypes.c_int32)]


class WorkItem(ctypes.Structure):
    _fields_ = [("mesh", ctypes.c_void_p), ("op", ctypes.c_int32), ("nlev", ctypes.c_int32),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("solo_min_elems", ctypes.c_int64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("nitems", ctypes.c_int32), ("nunits", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("form_column", ctypes.c_int32),
                ("form_flat", ctypes.c_int32), ("owned_bytes", ctypes.c_size_t),
                ("solo_items", ctypes.c_int32)]


class RemapInfo(ctypes.Structure):
    _fields_ = [("nsource", ctypes.c_int64), ("ntarget", ctypes.c_int64),
                ("nsource_touched", ctypes.c_int64), ("npolar", ctypes.c_int64),
                ("device_bytes", ctypes.c_size_t), ("values_per_column", ctypes.c_double),
                ("table_bytes", ctypes.c_double)]


# name -> (restype, argtypes); every symbol the headers declare
class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("nstreams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("batch_max_elems", ctypes.c_int64),
                ("simulate", ctypes.c_int32), ("sim_bytes_per_us", ctypes.c_double),
                ("fail_alloc_every", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("mesh_id", ctypes.c_int32), ("op", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("nlev", ctypes.c_int32), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("queue_us", ctypes.c_double),
                ("run_us", ctypes.c_double), ("total_us", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("batched_launches", ctypes.c_uint64), ("inflight_bytes", ctypes.c_size_t),
                ("peak_inflight_bytes", ctypes.c_size_t)]


SIGNATURES = {
    "atlas_last_error": (ctypes.c_char_p, []),
    "atlas_version": (ctypes.c_char_p, []),
    "atlas_mesh_desc_octahedral": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double,
                                                  ctypes.POINTER(ctypes.POINTER(MeshDesc))]),
    "atlas_mesh_desc_reduced_gaussian": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                        ctypes.c_double,
                                                        ctypes.POINTER(ctypes.POINTER(MeshDesc))]),
    "atlas_mesh_desc_grid": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _dp,
                                            ctypes.c_int32, ctypes.c_double,
                                            ctypes.POINTER(ctypes.POINTER(MeshDesc))]),
    "atlas_mesh_desc_free": (ctypes.c_int, [ctypes.POINTER(MeshDesc)]),
    "atlas_mesh_upload": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_mesh_upload_ex": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(Layout),
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_mesh_create_octahedral": (ctypes.c_int, [ctypes.c_int32, ctypes.c_double,
                                                    ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_mesh_free": (ctypes.c_int, [ctypes.c_void_p]),
    "atlas_mesh_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MeshInfo)]),
    "atlas_nabla_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "atlas_nabla_gradient_lonlat": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_int32, ctypes.c_int, ctypes.c_void_p,
                                                   ctypes.c_void_p]),
    "atlas_nabla_divergence": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "atlas_nabla_curl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "atlas_nabla_div_curl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "atlas_nabla_laplacian": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "atlas_laplacian_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int32,
                                                          ctypes.c_int]),
    "atlas_nabla_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(Launch),
                                         ctypes.c_void_p]),
    "atlas_bandwidth_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_int32, ctypes.c_void_p]),
    "atlas_batch_build": (ctypes.c_int, [ctypes.POINTER(WorkItem), ctypes.c_int32,
                                         ctypes.POINTER(BatchConfig), ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "atlas_batch_check": (ctypes.c_int, [ctypes.c_void_p]),
    "atlas_batch_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchInfo)]),
    "atlas_batch_free": (ctypes.c_int, [ctypes.c_void_p]),
    "atlas_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_int32, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Launch),
                                      ctypes.POINTER(ctypes.c_float)]),
    "atlas_flux_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int,
                                                     ctypes.c_int32, ctypes.c_int]),
    "atlas_nabla_get_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int32,
                                             ctypes.c_int, ctypes.POINTER(Launch)]),
    "atlas_diag_volume_integral": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "atlas_diag_volume_integral_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                          ctypes.c_int32, ctypes.c_int32,
                                                          ctypes.c_int, ctypes.c_void_p,
                                                          ctypes.c_void_p]),
    "atlas_diag_error_norms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                              ctypes.c_int, ctypes.c_int64, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "atlas_remap_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _dp, _dp,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_remap_create_to_mesh": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_remap_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "atlas_remap_get_weights": (ctypes.c_int, [ctypes.c_void_p, _i32p, _dp]),
    "atlas_remap_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RemapInfo)]),
    "atlas_remap_free": (ctypes.c_int, [ctypes.c_void_p]),
    "atlas_serve_create": (ctypes.c_int, [ctypes.POINTER(ServeConfig),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "atlas_serve_register_mesh": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.POINTER(ctypes.c_int32)]),
    "atlas_serve_register_sim_mesh": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                                     ctypes.POINTER(ctypes.c_int32)]),
    "atlas_serve_register_remap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_int32)]),
    "atlas_serve_register_sim_remap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                                      ctypes.c_int64,
                                                      ctypes.POINTER(ctypes.c_int32)]),
    "atlas_serve_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "atlas_serve_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                        ctypes.POINTER(Result)]),
    "atlas_serve_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "atlas_serve_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "atlas_serve_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServeStats)]),
    "atlas_serve_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}


def bind(lib):
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def desc_to_numpy(d: MeshDesc) -> dict:
    V, E, NP = int(d.nnodes), int(d.nedges), int(d.npole_edges)

    def arr(ptr, n, dt):
        return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dt, copy=True)

    out = {
        "lon": arr(d.lon, V, np.float64), "lat": arr(d.lat, V, np.float64),
        "cos_lat": arr(d.cos_lat, V, np.float64),
        "edge2node": arr(d.edge2node, 2 * E, np.int32).reshape(E, 2),
        "node2edge_ptr": arr(d.node2edge_ptr, V + 1, np.int64),
        "node2edge": arr(d.node2edge, 2 * E, np.int32),
        "node2edge_sign": arr(d.node2edge_sign, 2 * E, np.int8),
        "dual_volumes": arr(d.dual_volumes, V, np.float64),
        "dual_normals": arr(d.dual_normals, 2 * E, np.float64).reshape(E, 2),
        "pole_edges": arr(d.pole_edges, 2 * NP, np.int32).reshape(NP, 2),
        "pole_normals": arr(d.pole_normals, NP, np.float64),
        "radius": float(d.radius),
    }
    if d.nrings > 0 and d.ring_off:
        out["ring_off"] = arr(d.ring_off, int(d.nrings) + 1, np.int64)
    nt, nq = int(d.ntriangles), int(d.nquads)
    out["triangles"] = (arr(d.triangles, 3 * nt, np.int32).reshape(nt, 3) if nt and d.triangles
                        else np.zeros((0, 3), np.int32))
    out["quads"] = (arr(d.quads, 4 * nq, np.int32).reshape(nq, 4) if nq and d.quads
                    else np.zeros((0, 4), np.int32))
    return out


def numpy_to_desc(a: dict):
    """Build a MeshDesc pointing at (contiguous copies of) numpy arrays;
    returns (desc, keepalive)."""
    keep = {}

    def ptr(name, dt, ctype):
        x = np.ascontiguousarray(a[name], dtype=dt)
        keep[name] = x
        return x.ctypes.data_as(ctype)

    d = MeshDesc()
    d.nnodes = len(a["lon"])
    d.lon = ptr("lon", np.float64, _dp)
    d.lat = ptr("lat", np.float64, _dp)
    d.cos_lat = ptr("cos_lat", np.float64, _dp)
    if a.get("ring_off") is not None:
        d.nrings = len(a["ring_off"]) - 1
        d.ring_off = ptr("ring_off", np.int64, _i64p)
    d.nedges = len(np.asarray(a["edge2node"]).reshape(-1, 2))
    d.edge2node = ptr("edge2node", np.int32, _i32p)
    d.node2edge_ptr = ptr("node2edge_ptr", np.int64, _i64p)
    d.node2edge = ptr("node2edge", np.int32, _i32p)
    d.node2edge_sign = ptr("node2edge_sign", np.int8, _i8p)
    d.dual_volumes = ptr("dual_volumes", np.float64, _dp)
    d.dual_normals = ptr("dual_normals", np.float64, _dp)
    d.npole_edges = len(np.asarray(a["pole_normals"]))
    d.pole_edges = ptr("pole_edges", np.int32, _i32p)
    d.pole_normals = ptr("pole_normals", np.float64, _dp)
    d.radius = float(a["radius"])
    for name, n_name, width in (("triangles", "ntriangles", 3), ("quads", "nquads", 4)):
        el = a.get(name)
        if el is not None and len(el):
            setattr(d, name, ptr(name, np.int32, _i32p))
            setattr(d, n_name, len(np.asarray(el).reshape(-1, width)))
    return d, keep
