#!/usr/bin/env python3
"""Benchmark of the MI355X nabla operators (one GPU).

Default workload: gradient on the O1280 mesh (6,599,680 nodes, 19,799,000
edges), 137 levels, FP64 fields -- the headline configuration.  A step is
one gradient application over the resident [node][level] field; the other
operators (divergence, Laplacian) and the FP32 + Kahan form are timed in the
same run and reported under "ops".

Printed: ONE JSON line with edge*level updates per second, the HBM roofline
of the dominant kernel (algorithmic bytes / average kernel duration measured
with HIP events on the launch stream, against the 8 TB/s HBM3E peak), the
measured streaming ceiling for the same byte pattern, and the FP64 CPU oracle
timed on this host on a bounded sample of the same workload.

Inputs are seeded synthetic fields: 8 real spherical-harmonic fields of
degree <= 128 with amplitude 1e2, cycled over the levels with a factor
(1 + k/137), plus 1e-2 uniform noise per node and level.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILE = os.path.join(ROOT, "profiles", "gradient_o1280_l137_f64_counters.md")


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=1280, help="octahedral grid O<N>")
    ap.add_argument("--nlev", type=int, default=137)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-ops", action="store_true")
    ap.add_argument("--cpu-levels", type=int, default=16,
                    help="levels of the workload the CPU oracle sample covers")
    return ap.parse_args()


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("nabla_kernels.hip", "mesh_store.cpp"):
        with open(os.path.join(ROOT, "paper_1908_06091_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_for(kernel_sha):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    if not os.path.exists(PROFILE):
        return None
    text = open(PROFILE).read()
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", text, re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_sha") != kernel_sha:
        return None
    return rec


def make_field(om_lon, om_lat, nlev, dtype, device, torch):
    """Seeded harmonic levels on the host, level factors and noise on the
    device (seeded generator)."""
    import numpy as np
    import synthetic as sy
    co = sy.random_coeffs(128, [sy.seed_rng(3, 0, j) for j in range(8)], amplitude=1e2)
    H = torch.from_numpy(sy.synthesize(om_lon, om_lat, co)).to(device)  # [8, V]
    V = H.shape[1]
    f = torch.empty(V, nlev, dtype=torch.float64, device=device)
    for k in range(nlev):
        f[:, k] = H[k % 8] * (1.0 + k / nlev)
    g = torch.Generator(device=device)
    g.manual_seed(20170331)
    f += 1e-2 * (2.0 * torch.rand(V, nlev, dtype=torch.float64, device=device, generator=g) - 1.0)
    grad = sy.synthesize_gradient(om_lon, om_lat, co)  # [8, V, 2]
    G = torch.from_numpy(grad).to(device)
    uv = torch.empty(V, nlev, 2, dtype=torch.float64, device=device)
    for k in range(nlev):
        uv[:, k, :] = G[k % 8] * (1.0 + k / nlev)
    del G, H
    return f.to(dtype), uv.to(dtype), np


def time_op(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per launch sequence


def cpu_baseline(N, nlev_total, levels, f_host):
    """The FP64 oracle on this host: dense gradient over all edges for the
    first `levels` levels of the same field (a bounded sample)."""
    import numpy as np
    import oracle
    om = oracle.Mesh(N)
    fs = np.ascontiguousarray(f_host[:, :levels])
    t0 = time.perf_counter()
    om.gradient(fs, levels)
    dt = time.perf_counter() - t0
    return {
        "value": om.E * levels / dt,
        "unit": "edge*level updates/s",
        "cores": oracle.threads_used(levels),
        "kind": "oracle",
        "sample": f"O{N} FP64 gradient, all {om.E} edges, first {levels} of {nlev_total} levels "
                  f"({dt:.1f} s)",
    }


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(levels and mesh bands shard across GPUs by design, not built here)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1908_06091_amd as P
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, nlev = args.N, args.nlev
    gm = P.Mesh(N)
    desc_lonlat = P.mesh_desc_octahedral(N)
    f64, uv64, np = make_field(desc_lonlat["lon"], desc_lonlat["lat"], nlev, torch.float64, dev, torch)
    V, E = gm.nnodes, gm.nedges
    geo = gm.info.geometry_bytes_per_call

    def alg_bytes(op, w):
        if op == "lapl":
            return 6 * V * nlev * w + 2 * geo
        return 3 * V * nlev * w + geo

    # headline: FP64 gradient
    out = torch.empty(V, nlev, 2, dtype=torch.float64, device=dev)
    ms = time_op(lambda: gm.gradient(f64, out=out), args.steps, args.warmup, torch)
    value = E * nlev / (ms * 1e-3)
    achieved = alg_bytes("grad", 8) / (ms * 1e-3) / 1e9

    # streaming ceiling for the same byte pattern (read n, write 2n)
    ceil_ms = time_op(lambda: P.bandwidth_probe(f64, out), 10, 2, torch)
    ceiling = 3 * V * nlev * 8 / (ceil_ms * 1e-3) / 1e9

    ops = {}
    if not args.no_extra_ops:
        f32, uv32 = f64.float(), uv64.float()
        for name, dt, fn_in, w in (("div_f64", "f64", uv64, 8), ("lapl_f64", "f64", f64, 8),
                                   ("curl_f64", "f64", uv64, 8), ("grad_f32", "f32", f32, 4),
                                   ("div_f32", "f32", uv32, 4), ("lapl_f32", "f32", f32, 4)):
            opname = name.split("_")[0]
            if opname == "grad":
                o = torch.empty(V, nlev, 2, dtype=fn_in.dtype, device=dev)
                fn = lambda o=o, x=fn_in: gm.gradient(x, out=o)
            elif opname == "div":
                o = torch.empty(V, nlev, dtype=fn_in.dtype, device=dev)
                fn = lambda o=o, x=fn_in: gm.divergence(x, out=o)
            elif opname == "curl":
                o = torch.empty(V, nlev, dtype=fn_in.dtype, device=dev)
                fn = lambda o=o, x=fn_in: gm.curl(x, out=o)
            else:
                o = torch.empty(V, nlev, dtype=fn_in.dtype, device=dev)
                fn = lambda o=o, x=fn_in: gm.laplacian(x, out=o)
            t = time_op(fn, max(5, args.steps // 2), 2, torch)
            b = alg_bytes(opname, w)
            ops[name] = {"ms": round(t, 4), "edge_level_per_s": E * nlev / (t * 1e-3),
                         "GBps": round(b / (t * 1e-3) / 1e9, 1),
                         "hbm_frac": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del o

    sha = kernel_source_sha()
    rec = counters_for(sha)
    traffic = None
    if rec is not None:
        traffic = rec["fetch_bytes"] + rec["write_bytes"]

    cpu = None
    if not args.no_cpu_baseline:
        f_host = f64[:, :args.cpu_levels].cpu().numpy()
        cpu = cpu_baseline(N, nlev, args.cpu_levels, np.ascontiguousarray(f_host))

    line = {
        "metric": "edge*level updates/s (gradient, O1280 L137) + % HBM peak",
        "value": value,
        "unit": "edge*level updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded spherical harmonics degree<=128 + noise)",
        "config": {"workload": f"O{N} L{nlev} FP64 gradient", "grid": f"O{N}", "nodes": V,
                   "edges": E, "nlev": nlev, "op": "gradient"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "stream_ceiling_GBps": round(ceiling, 1),
                     "frac_of_stream_ceiling": round(achieved / ceiling, 4),
                     "algorithmic_bytes": alg_bytes("grad", 8)},
        "cpu_baseline": cpu,
        "ops": ops,
        "kernel_source_sha": sha,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
