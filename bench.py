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
    ap.add_argument("--ops", type=str, default="",
                    help="comma list of the extra operators to time (default: all)")
    ap.add_argument("--no-other-grids", action="store_true")
    ap.add_argument("--cpu-levels", type=int, default=137,
                    help="levels of the workload the CPU oracle sample covers")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-remap", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the GPU and oracle timings of the O16 L1 and O320 L137 configs")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=str, default="0.5,0.9,1.5",
                    help="offered rates as multiples of the sequential FP64 service rate")
    return ap.parse_args()


def kernel_source_sha():
    """Identity of what sets the dominant kernel's memory traffic: the source
    of the wave-specialised sweep (the FP64 gradient's kernel) and of its
    geometry packing, and the default tile layout of the processing order."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1908_06091_amd", "csrc", "nabla_kernels.hip")) as fh:
        src = fh.read()
    for start, end in (("// Wave-specialised sweep.", "// Fused Laplacian: one pass"),
                       ("__global__ void k_pack_sgeo(", "\n}\n")):
        i = src.find(start)
        j = src.find(end, i + 1)
        h.update(src[i:j].encode() if i >= 0 and j > i else src.encode())
    with open(os.path.join(ROOT, "paper_1908_06091_amd", "csrc", "internal.h")) as fh:
        layout = "\n".join(l for l in fh.read().splitlines() if re.search(r"kDefault(Band|Width)", l))
    h.update(layout.encode())
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


def time_op(fn, steps, warmup, torch, stats=None):
    """Mean ms per call over `steps` back-to-back calls, bracketed by two
    events on the launch stream.  With `stats` (a dict), each call is also
    timed on its own between two events, and the median, min and max of
    those per-call times are stored in it."""
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
    mean = start.elapsed_time(end) / steps  # ms per launch sequence
    if stats is not None:
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(max(steps, 20))]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        per = sorted(a.elapsed_time(b) for a, b in ev)
        stats.update({"median_ms": round(per[len(per) // 2], 4), "min_ms": round(per[0], 4),
                      "max_ms": round(per[-1], 4), "reps": len(per)})
    return mean


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, nlev_total, levels, f_host, runs=5):
    """The FP64 oracle on this host: dense gradient over all edges for the
    first `levels` levels of the same field, median of `runs` runs (a bounded
    sample: about 13 s at O1280 with all 137 levels on 16 threads)."""
    import numpy as np
    import oracle
    om = oracle.Mesh(N)
    fs = np.ascontiguousarray(f_host[:, :levels])
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        om.gradient(fs, levels)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    return {
        "value": om.E * levels / dt,
        "unit": "edge*level updates/s",
        "cores": oracle.threads_used(levels),
        "kind": "oracle",
        "sample": f"O{N} FP64 gradient, all {om.E} edges, {levels} of {nlev_total} levels, "
                  f"median of {runs} runs ({dt:.2f} s each)",
        "nproc": os.cpu_count(),
        "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
        "cpu_model": _cpu_model(),
    }, om


def accuracy(gm, om, f64, uv64, torch, np, nsample=2000):
    """Max and RMS error of the FP64 and FP32 paths against the FP64 oracle on
    sampled nodes (all levels), normwise per output component.  FP32 results
    are compared with the oracle on their own inputs (the FP32-rounded fields
    promoted exactly to FP64); the error against the FP64 inputs is reported
    beside it."""
    nlev = f64.shape[1]
    rng = np.random.default_rng(1280)
    nodes = np.sort(rng.choice(gm.nnodes, size=nsample, replace=False)).astype(np.int64)
    idx = torch.from_numpy(nodes).to(f64.device)

    def refs_for(f, uv):
        f_h, uv_h = f.double().cpu().numpy(), uv.double().cpu().numpy()
        r = {"grad": om.gradient_at(f_h, nlev, nodes), "div": om.divergence_at(uv_h, nlev, nodes),
             "lapl": om.laplacian_at(f_h, nlev, nodes)}
        del f_h, uv_h
        return r

    def err(got, ref):
        comps = [(got[..., c], ref[..., c]) for c in range(2)] if got.ndim == 3 else [(got, ref)]
        emax = max(float(np.abs(g - r).max() / np.abs(r).max()) for g, r in comps)
        erms = max(float(np.sqrt(((g - r) ** 2).mean() / (r ** 2).mean())) for g, r in comps)
        return emax, erms

    refs64 = refs_for(f64, uv64)
    res = {}
    for dt, tag in ((torch.float64, "f64"), (torch.float32, "f32")):
        f, uv = f64.to(dt), uv64.to(dt)
        refs = refs64 if tag == "f64" else refs_for(f, uv)
        for op, fn, x in (("grad", gm.gradient, f), ("div", gm.divergence, uv),
                          ("lapl", gm.laplacian, f)):
            got = fn(x).index_select(0, idx).double().cpu().numpy()
            emax, erms = err(got, refs[op])
            rec = {"max_rel": emax, "rms_rel": erms}
            if tag == "f32":
                m64, r64 = err(got, refs64[op])
                rec["vs_f64_inputs"] = {"max_rel": m64, "rms_rel": r64}
            res[f"{op}_{tag}"] = rec
        del f, uv
        torch.cuda.empty_cache()
    res["sample"] = f"{nsample} random nodes x {nlev} levels, oracle evaluated per node"
    return res


def batch_items(P, torch, np, dev, grids, nlevs, seed):
    """64 seeded FP32 work items: grid from `grids`, nlev from `nlevs`,
    operator from {grad, div, lapl}."""
    import synthetic as sy
    rng = np.random.default_rng(seed)
    meshes = {N: P.Mesh(N) for N in grids}
    lonlat = {N: P.mesh_desc_octahedral(N) for N in meshes}
    fields = {}
    items, edges_levels = [], 0
    for i in range(64):
        N = int(rng.choice(list(grids)))
        nlev = int(rng.choice(list(nlevs)))
        op = ["grad", "div", "lapl"][int(rng.integers(0, 3))]
        gm = meshes[N]
        if N not in fields:
            co = sy.random_coeffs(16, [sy.seed_rng(4, N, j) for j in range(4)])
            d = lonlat[N]
            fields[N] = (torch.from_numpy(sy.synthesize(d["lon"], d["lat"], co)).to(dev),
                         torch.from_numpy(sy.synthesize_gradient(d["lon"], d["lat"], co)).to(dev))
        H, G = fields[N]
        k = torch.arange(nlev, device=dev, dtype=torch.float64)
        fac = 1.0 + k / 137.0
        if op == "div":
            x = (G[(k.long() % 4)].permute(1, 0, 2) * fac[None, :, None]).float().contiguous()
            out = torch.empty(gm.nnodes, nlev, dtype=torch.float32, device=dev)
            code = P.ATLAS_OP_DIVERGENCE
        else:
            x = (H[(k.long() % 4)].t() * fac[None, :]).float().contiguous()
            shape = (gm.nnodes, nlev, 2) if op == "grad" else (gm.nnodes, nlev)
            out = torch.empty(shape, dtype=torch.float32, device=dev)
            code = P.ATLAS_OP_GRADIENT if op == "grad" else P.ATLAS_OP_LAPLACIAN
        items.append((gm, code, x, out))
        edges_levels += gm.nedges * nlev * (2 if op == "lapl" else 1)
    torch.cuda.synchronize()
    return items, meshes, edges_levels, rng


def batch_small_items(P, torch, np, dev):
    """64 small FP32 items (O80, nlev in {1, 10}): launch overhead dominates,
    which one persistent launch replayed from a graph removes."""
    items, _, _, _ = batch_items(P, torch, np, dev, (80,), (1, 10), 65)
    b = P.Batch(items, use_graph=True)
    ms_batch = time_op(lambda: b.launch(), 20, 3, torch)
    out_b = [it[3].clone() for it in items]
    ms_seq = time_op(lambda: [gm.apply(c, x, out=o) for gm, c, x, o in items], 20, 3, torch)
    same = all(torch.equal(a, it[3]) for a, it in zip(out_b, items))
    b.close()
    return {"items": 64, "mix": "O80, nlev 1/10, grad/div/lapl, f32", "ms_batch": round(ms_batch, 4),
            "ms_one_by_one": round(ms_seq, 4), "speedup": round(ms_seq / ms_batch, 3),
            "bitwise_equal_to_solo": bool(same)}


def batch_bench(P, torch, np, dev):
    """64 FP32 work items over O80/O160/O320 with nlev in {1,10,91,137} and
    operators in {grad, div, lapl}, autotuned and captured in a hipGraph
    (items of 2^22+ elements as their own launches, the rest in the
    persistent launch): replay time against the same items launched one by
    one."""
    items, meshes, edges_levels, rng = batch_items(P, torch, np, dev, (80, 160, 320),
                                                   (1, 10, 91, 137), 64)
    t0 = time.perf_counter()
    b = P.Batch(items, use_graph=True, autotune=True)
    build_s = time.perf_counter() - t0
    ms_batch = time_op(lambda: b.launch(), 20, 3, torch)
    hybrid = [it[3].clone() for it in items]
    # every item inside the one persistent kernel (no item launched on its own)
    bp = P.Batch(items, use_graph=True, autotune=True, solo_min_elems=-1)
    ms_persistent = time_op(lambda: bp.launch(), 20, 3, torch)
    same_persistent = all(torch.equal(a, it[3]) for a, it in zip(hybrid, items))
    info_p = bp.info
    bp.close()
    solo = [it[3].clone() for it in items]
    ms_seq = time_op(lambda: [gm.apply(c, x, out=o) for gm, c, x, o in items], 20, 3, torch)
    same = all(torch.equal(a, it[3]) for a, it in zip(solo, items))
    info = b.info
    b.close()
    # each item against the FP64 oracle on its (FP32) inputs, sampled nodes
    import oracle
    oms = {N: oracle.Mesh(N) for N in meshes}
    worst = 0.0
    for gm, c, x, out in items:
        N = next(k for k, v in meshes.items() if v is gm)
        om = oms[N]
        nodes = np.sort(rng.choice(om.V, size=min(256, om.V), replace=False)).astype(np.int64)
        xh = x.double().cpu().numpy()
        nlev = x.shape[1]
        fn = {P.ATLAS_OP_GRADIENT: om.gradient_at, P.ATLAS_OP_DIVERGENCE: om.divergence_at,
              P.ATLAS_OP_LAPLACIAN: om.laplacian_at}[c]
        ref = fn(xh, nlev, nodes)
        got = out.double().cpu().numpy()[nodes]
        comps = [(got[..., k], ref[..., k]) for k in range(2)] if ref.ndim == 3 else [(got, ref)]
        for g_, r_ in comps:
            worst = max(worst, float(np.abs(g_ - r_).max() / np.abs(r_).max()))
    return {"items": 64, "dtype": "f32", "graph": bool(info.graph), "units": info.nunits,
            "solo_items": info.solo_items,
            "grid_blocks": info.grid_blocks, "form_column": info.form_column,
            "form_flat": info.form_flat, "build_s_incl_autotune": round(build_s, 2),
            "ms_batch": round(ms_batch, 4), "ms_one_by_one": round(ms_seq, 4),
            "speedup": round(ms_seq / ms_batch, 3),
            "persistent_only": {"ms": round(ms_persistent, 4), "units": info_p.nunits,
                                "grid_blocks": info_p.grid_blocks,
                                "bitwise_equal": bool(same_persistent)},
            "edge_level_per_s": edges_levels / (ms_batch * 1e-3),
            "bitwise_equal_to_solo": bool(same),
            "max_rel_error_vs_oracle": worst,
            "oracle_sample": "256 random nodes per item, all levels"}


def serve_bench(P, torch, np, dev, gm1280, nreq, qps_factors):
    """Poisson arrivals of seeded requests over {O48,O160,O320,O640,O1280} x
    nlev {1,37,137} x {grad,div,curl,lapl} x {FP32,FP64}: the server
    (admission by HBM budget, continuous batching over 4 streams) against the
    same arrival schedule served by sequential plain FP64 calls.  The offered
    rates are multiples of the sequential FP64 service rate mu_seq, measured
    first on the same request mix."""
    import threading
    grids = (48, 160, 320, 640, 1280)
    meshes = {N: (gm1280 if N == 1280 else P.Mesh(N)) for N in grids}
    rng = np.random.default_rng(2000)
    reqs = []
    for _ in range(nreq):
        reqs.append((int(rng.choice(grids)), int(rng.choice([1, 37, 137])),
                     ["grad", "div", "curl", "lapl"][int(rng.integers(0, 4))],
                     "f32" if rng.integers(0, 2) else "f64"))
    gaps = rng.exponential(1.0, size=nreq)  # unit-rate inter-arrival times
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    inputs = {}

    def field(N, nlev, vec, dt):
        key = (N, nlev, vec, dt)
        if key not in inputs:
            shape = (meshes[N].nnodes, nlev, 2) if vec else (meshes[N].nnodes, nlev)
            inputs[key] = torch.randn(shape, generator=g, device=dev,
                                      dtype=torch.float64 if dt == "f64" else torch.float32)
        return inputs[key]

    code = {"grad": P.ATLAS_OP_GRADIENT, "div": P.ATLAS_OP_DIVERGENCE,
            "curl": P.ATLAS_OP_CURL, "lapl": P.ATLAS_OP_LAPLACIAN}
    for N, nlev, op, dt in reqs:
        field(N, nlev, op in ("div", "curl"), dt)
        field(N, nlev, op in ("div", "curl"), "f64")
    work = sum(meshes[N].nedges * nlev * (2 if op == "lapl" else 1) for N, nlev, op, _ in reqs)
    outs = {}
    for N, nlev, op, _ in reqs:
        shape = (meshes[N].nnodes, nlev, 2) if op == "grad" else (meshes[N].nnodes, nlev)
        outs.setdefault((N, nlev, op), torch.empty(shape, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()

    def seq_call(i):
        N, nlev, op, _ = reqs[i]
        meshes[N].apply(code[op], field(N, nlev, op in ("div", "curl"), "f64"),
                        out=outs[(N, nlev, op)])
        torch.cuda.synchronize()

    for i in range(20):  # warm-up
        seq_call(i)
    t0 = time.perf_counter()
    for i in range(nreq):
        seq_call(i)
    mu_seq = nreq / (time.perf_counter() - t0)

    def pct(lat):
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    def run_sequential(arrivals):
        lat = []
        t0 = time.perf_counter()
        for i, ta in enumerate(arrivals):
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            seq_call(i)
            lat.append((time.perf_counter() - t0 - ta) * 1e6)
        return lat, time.perf_counter() - t0

    budget = 64 << 30

    def run_server(arrivals):
        srv = P.Server(hbm_budget_bytes=budget, nstreams=4, max_batch=64)
        ids = {N: srv.register_mesh(meshes[N]) for N in grids}
        tickets = [None] * nreq
        lat, sizes, status = [0.0] * nreq, [0] * nreq, [0] * nreq
        ready = threading.Semaphore(0)

        def waiter():
            for i in range(nreq):
                ready.acquire()
                r = srv.wait(tickets[i])
                lat[i], sizes[i], status[i] = r["total_us"], r["batch_size"], r["status"]
                srv.release(tickets[i])

        th = threading.Thread(target=waiter, daemon=True)
        th.start()
        t0 = time.perf_counter()
        for i, ((N, nlev, op, dt), ta) in enumerate(zip(reqs, arrivals)):
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            tickets[i] = srv.submit(ids[N], code[op], field(N, nlev, op in ("div", "curl"), dt))
            ready.release()
        th.join()
        span = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return lat, span, st, sizes, status

    runs = []
    for f in qps_factors:
        qps = f * mu_seq
        arrivals = np.cumsum(gaps / qps)
        lat_seq, span_seq = run_sequential(arrivals)
        lat_srv, span_srv, st, sizes, status = run_server(arrivals)
        p50s, p99s = pct(lat_seq)
        p50v, p99v = pct(lat_srv)
        runs.append({
            "qps_offered": round(qps, 1), "load_vs_mu_seq": f,
            "server": {"p50_us": round(p50v, 1), "p99_us": round(p99v, 1),
                       "req_per_s": round(nreq / span_srv, 1),
                       "edge_level_per_s": work / span_srv,
                       "launches": st["launches"], "batched_launches": st["batched_launches"],
                       "mean_batch": round(float(np.mean(sizes)), 2),
                       "failed": int(sum(1 for x in status if x != 0)),
                       "peak_inflight_GB": round(st["peak_inflight_bytes"] / 1e9, 2)},
            "sequential_f64": {"p50_us": round(p50s, 1), "p99_us": round(p99s, 1),
                               "req_per_s": round(nreq / span_seq, 1),
                               "edge_level_per_s": work / span_seq}})
        print(f"# serving at {f} x mu_seq done", file=sys.stderr, flush=True)
    return {
        "requests": nreq,
        "mix": "grids O48/O160/O320/O640/O1280, nlev 1/37/137, grad/div/curl/lapl, f32/f64",
        "mu_seq_req_per_s": round(mu_seq, 1),
        "hbm_budget_GB": round(budget / 1e9, 2), "streams": 4, "max_batch": 64,
        "runs": runs,
    }


def remap_bench(P, torch, dev, gm, f64, steps):
    """Remap (P1 interpolation) of a 137-level field between O1280 and O640
    node sets, FP64 and FP32, apply kernel only (weights built once).  Bytes:
    touched source rows read once, target rows written once, plus 36 B of
    weights per target."""
    nlev = f64.shape[1]
    g640 = P.Mesh(640)
    x640 = torch.randn(g640.nnodes, nlev, dtype=torch.float64, device=dev)
    rows = {}
    for name, src, dst, x in (("O1280_to_O640", gm, g640, f64), ("O640_to_O1280", g640, gm, x640)):
        r = P.Remap(src, dst)
        info = r.info
        for dname, dt, w in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
            xi = x.to(dt)
            o = torch.empty(r.ntarget, nlev, dtype=dt, device=dev)
            st = {}
            t = time_op(lambda: r.apply(xi, out=o), max(10, steps // 2), 3, torch, st)
            b = info.values_per_column * nlev * w + info.table_bytes
            rows[f"{name}_{dname}"] = {
                "ms": round(t, 4), **st, "targets": r.ntarget,
                "sources_touched": int(info.nsource_touched),
                "target_values_per_s": r.ntarget * nlev / (t * 1e-3),
                "GBps": round(b / (t * 1e-3) / 1e9, 1),
                "hbm_frac": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "bytes_model": "(touched + targets) * L * w + 36 * targets"}
            del xi, o
        r.close()
        torch.cuda.empty_cache()
    del x640
    g640.close()
    torch.cuda.empty_cache()
    return rows


def config_bench(P, torch, np, dev, steps):
    """The O16 L1 FP64 gradient and the O320 L137 FP64 gradient, divergence
    and Laplacian: GPU time per call (median of >= 20, min, max) next to the
    FP64 oracle on all host threads and, for O320, on one thread (median of
    3 runs, one run if a run takes over 30 s)."""
    import oracle
    import synthetic as sy
    rows = {}
    for cfg, N, nlev, lmax, ops in ((1, 16, 1, 4, ("grad",)),
                                    (2, 320, 137, 32, ("grad", "div", "lapl"))):
        om, gm = oracle.Mesh(N), P.Mesh(N)
        if cfg == 1:
            f = sy.level_field_stack(om.lon, om.lat, 1, lmax, 1, 0, noise_eps=1e-3)
            co2 = sy.random_coeffs(lmax, [sy.seed_rng(1, 1, 0)])
        else:  # eight seeded degree-32 fields cycled over the levels, scaled
            co = sy.random_coeffs(lmax, [sy.seed_rng(2, 0, j) for j in range(8)])
            H = sy.synthesize(om.lon, om.lat, co)
            f = np.stack([H[k % 8] * (k + 1) for k in range(nlev)], axis=1)
            co2 = sy.random_coeffs(lmax, [sy.seed_rng(2, 1, j) for j in range(8)])
        G = sy.synthesize_gradient(om.lon, om.lat, co2)
        uv = np.stack([G[k % G.shape[0]] for k in range(nlev)], axis=1)
        f = np.ascontiguousarray(f)
        uv = np.ascontiguousarray(uv)
        xf, xuv = torch.from_numpy(f).to(dev), torch.from_numpy(uv).to(dev)
        for op in ops:
            x = xuv if op == "div" else xf
            shape = (gm.nnodes, nlev, 2) if op == "grad" else (gm.nnodes, nlev)
            o = torch.empty(shape, dtype=torch.float64, device=dev)
            fn = {"grad": lambda: gm.gradient(x, out=o), "div": lambda: gm.divergence(x, out=o),
                  "lapl": lambda: gm.laplacian(x, out=o)}[op]
            st = {}
            t = time_op(fn, max(20, steps), 3, torch, st)
            ofn = {"grad": om.gradient, "div": om.divergence, "lapl": om.laplacian}[op]
            xh = uv if op == "div" else f

            def cpu_time(threads):
                old = oracle.set_threads(threads)
                try:
                    times = []
                    for _ in range(3):
                        t0 = time.perf_counter()
                        ofn(xh, nlev)
                        times.append(time.perf_counter() - t0)
                        if times[-1] > 30.0:
                            break
                finally:
                    oracle.set_threads(old)
                return float(np.median(times)), len(times)

            t_all, n_all = cpu_time(os.cpu_count() or 1)
            row = {"gpu_ms": round(t, 4), **{"gpu_" + k: v for k, v in st.items()},
                   "gpu_edge_level_per_s": gm.nedges * nlev / (t * 1e-3),
                   "oracle_ms": round(t_all * 1e3, 3), "oracle_runs": n_all,
                   "oracle_threads": oracle.threads_used(nlev),
                   "oracle_edge_level_per_s": om.E * nlev / t_all}
            if cfg == 2:
                t1, n1 = cpu_time(1)
                row.update({"oracle_1thread_ms": round(t1 * 1e3, 3), "oracle_1thread_runs": n1,
                            "oracle_1thread_edge_level_per_s": om.E * nlev / t1})
            rows[f"cfg{cfg}_O{N}_L{nlev}_{op}_f64"] = row
            del o
        del xf, xuv
        gm.close()
        torch.cuda.empty_cache()
    return rows


def cpu_ops_o1280(om, f_host, uv_host, nlev):
    """The oracle's divergence and Laplacian at O1280 on all host threads,
    one run each (the gradient is the cpu_baseline figure)."""
    import numpy as np
    import oracle
    rows = {}
    for op, fn, x in (("div", om.divergence, uv_host), ("lapl", om.laplacian, f_host)):
        t0 = time.perf_counter()
        fn(x, nlev)
        dt = time.perf_counter() - t0
        rows[f"O1280_L{nlev}_{op}_f64"] = {"oracle_ms": round(dt * 1e3, 1), "runs": 1,
                                           "threads": oracle.threads_used(nlev),
                                           "edge_level_per_s": om.E * nlev / dt}
    del np
    return rows


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
        if op == "divcurl":  # (u, v) read once, two scalar outputs
            return 4 * V * nlev * w + geo
        return 3 * V * nlev * w + geo

    # headline: FP64 gradient
    out = torch.empty(V, nlev, 2, dtype=torch.float64, device=dev)
    head_stats = {}
    ms = time_op(lambda: gm.gradient(f64, out=out), args.steps, args.warmup, torch, head_stats)
    value = E * nlev / (ms * 1e-3)
    achieved = alg_bytes("grad", 8) / (ms * 1e-3) / 1e9

    # streaming ceiling for the same byte pattern (read n, write 2n)
    ceil_ms = time_op(lambda: P.bandwidth_probe(f64, out), 10, 2, torch)
    ceiling = 3 * V * nlev * 8 / (ceil_ms * 1e-3) / 1e9

    ops = {}
    want = set(x for x in args.ops.split(",") if x)
    if not args.no_extra_ops:
        f32, uv32 = f64.float(), uv64.float()
        for name, dt, fn_in, w in (("div_f64", "f64", uv64, 8), ("lapl_f64", "f64", f64, 8),
                                   ("curl_f64", "f64", uv64, 8), ("divcurl_f64", "f64", uv64, 8),
                                   ("grad_f32", "f32", f32, 4), ("div_f32", "f32", uv32, 4),
                                   ("lapl_f32", "f32", f32, 4), ("divcurl_f32", "f32", uv32, 4)):
            if want and name not in want:
                continue
            opname = name.split("_")[0]
            if opname == "divcurl":
                o = (torch.empty(V, nlev, dtype=fn_in.dtype, device=dev),
                     torch.empty(V, nlev, dtype=fn_in.dtype, device=dev))
                fn = lambda o=o, x=fn_in: gm.div_curl(x, out_div=o[0], out_curl=o[1])
            elif opname == "grad":
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
            st = {}
            t = time_op(fn, max(5, args.steps // 2), 2, torch, st)
            napp = 2 if opname == "divcurl" else 1  # operator applications per call
            fused = opname == "lapl" and gm.shape_of(P.ATLAS_OP_LAPLACIAN, nlev, fn_in)["variant"] \
                == P.VARIANT_FUSED
            # the bytes of the form that runs: the fused Laplacian reads the
            # field once and writes the result (2 V L w + G)
            b = 2 * V * nlev * w + geo if fused else alg_bytes(opname, w)
            ops[name] = {"ms": round(t, 4), **st,
                         "edge_level_per_s": napp * E * nlev / (t * 1e-3),
                         "GBps": round(b / (t * 1e-3) / 1e9, 1),
                         "hbm_frac": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            if opname == "lapl":
                ops[name]["form"] = "fused one pass" if fused else "two passes"
                ops[name]["bytes_model"] = ("2*V*L*w + G" if fused else "6*V*L*w + 2*G")
                if fused:
                    b2 = alg_bytes("lapl", w)
                    ops[name]["two_pass_equiv_frac"] = round(b2 / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            del o

    # another reduced Gaussian grid: the regular grid F640 (nx = 2560 on all
    # 1280 parallels, 3.28 M nodes), default shapes
    grids = {}
    if not args.no_extra_ops and not args.no_other_grids:
        nxF = P.regular_gaussian_nx(640)
        gF = P.Mesh(nx=nxF)
        VF, EF, geoF = gF.nnodes, gF.nedges, gF.info.geometry_bytes_per_call
        xF = torch.randn(VF, nlev, dtype=torch.float64, device=dev)
        for name, op, shape, nbytes in (
                ("F640_grad_f64", "grad", (VF, nlev, 2), 3 * VF * nlev * 8 + geoF),
                ("F640_lapl_f64", "lapl", (VF, nlev), 6 * VF * nlev * 8 + 2 * geoF)):
            o = torch.empty(shape, dtype=torch.float64, device=dev)
            fn = (lambda o=o: gF.gradient(xF, out=o)) if op == "grad" else \
                 (lambda o=o: gF.laplacian(xF, out=o))
            t = time_op(fn, max(5, args.steps // 2), 2, torch)
            grids[name] = {"ms": round(t, 4), "nodes": VF, "edges": EF,
                           "edge_level_per_s": EF * nlev / (t * 1e-3),
                           "GBps": round(nbytes / (t * 1e-3) / 1e9, 1),
                           "hbm_frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del o
        del xF, gF
        torch.cuda.empty_cache()

    # one GPU's share when the levels are split over eight GPUs (the larger
    # share: ceil(nlev / 8) levels, 18 of 137), FP64 gradient, default shape
    slab = {}
    if not args.no_extra_ops and not args.no_other_grids:
        ls = (nlev + 7) // 8
        xs = f64[:, :ls].contiguous()
        os_ = torch.empty(V, ls, 2, dtype=torch.float64, device=dev)
        t = time_op(lambda: gm.gradient(xs, out=os_), max(5, args.steps // 2), 2, torch)
        b = 3 * V * ls * 8 + geo
        slab = {"gpus": 8, "nlev": ls, "grad_f64_ms": round(t, 4),
                "edge_level_per_s": E * ls / (t * 1e-3),
                "GBps": round(b / (t * 1e-3) / 1e9, 1),
                "hbm_frac": round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del xs, os_
        torch.cuda.empty_cache()

    remap = None
    if not args.no_remap:
        remap = remap_bench(P, torch, dev, gm, f64, args.steps)
        print("# remap done", file=sys.stderr, flush=True)
    configs = None
    if not args.no_configs:
        configs = config_bench(P, torch, np, dev, args.steps)
        print("# configs done", file=sys.stderr, flush=True)

    sha = kernel_source_sha()
    rec = counters_for(sha)
    traffic = None
    if rec is not None:
        traffic = rec["fetch_bytes"] + rec["write_bytes"]

    cpu = None
    om = None
    if not args.no_cpu_baseline:
        f_host = f64[:, :args.cpu_levels].cpu().numpy()
        cpu, om = cpu_baseline(N, nlev, args.cpu_levels, np.ascontiguousarray(f_host))
        print(f"# cpu baseline done: {cpu['sample']}", file=sys.stderr, flush=True)
        if not args.no_configs and args.cpu_levels == nlev:
            cpu["other_ops"] = cpu_ops_o1280(om, np.ascontiguousarray(f_host),
                                             np.ascontiguousarray(uv64.cpu().numpy()), nlev)
            print("# cpu div/lapl done", file=sys.stderr, flush=True)
        del f_host
    acc = None
    if not args.no_accuracy:
        if om is None:
            import oracle
            om = oracle.Mesh(N)
        acc = accuracy(gm, om, f64, uv64, torch, np)
        print("# accuracy done", file=sys.stderr, flush=True)
    del om
    batch = None
    if not args.no_batch:
        batch = batch_bench(P, torch, np, dev)
        batch["small_items"] = batch_small_items(P, torch, np, dev)
        print("# batch done", file=sys.stderr, flush=True)
    serving = None
    if not args.no_serve:
        del f64, uv64
        torch.cuda.empty_cache()
        serving = serve_bench(P, torch, np, dev, gm, args.serve_requests,
                              [float(v) for v in args.serve_load.split(",")])
        print("# serving done", file=sys.stderr, flush=True)

    line = {
        "metric": "edge*level updates/s (gradient, O1280 L137) + % HBM peak",
        "value": value,
        "unit": "edge*level updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "per_launch_ms": head_stats,
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
        "other_grids": grids,
        "level_slab_share": slab,
        "remap": remap,
        "configs": configs,
        "accuracy_vs_oracle": acc,
        "batch": batch,
        "serving": serving,
        "kernel_source_sha": sha,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
