#!/usr/bin/env python3
"""Benchmark of the MI355X TPC sector tracker.

Workload: 256 independent sector instances of very uneven occupancy (cluster
counts log-uniform 1e3..4e5 per instance, noise 0-20 %, 15.65 M clusters,
seeded synthetic helix events).  One step = the whole hot path (grid build,
neighbours, cleaner, start hits, tracklet construction, selection) over the
batch, with the clusters already resident in HBM.  Reported:

  value        clusters/s of the batched deterministic path (one launch chain
               for all 256 instances, captured in a HIP graph, launch
               parameters from the autotuner); batched_eager without the graph
  plain        clusters/s of 256 per-instance launch chains on one stream,
               eager and graph-captured
  prod         clusters/s of the batched production path, the det/prod ratio,
               its quality and the fraction of clusters it assigns
               differently from the deterministic path
  quality      efficiency, fake and clone rates against the MC truth
  roofline     the dominant kernel's algorithmic bytes per launch divided by
               its average launch time (HIP events recorded on the kernel's
               stream over a timed pass), against the 8 TB/s HBM peak;
               traffic from the committed counter summary when it matches
  copy_ceiling a 1 GiB device copy in the same run (practical HBM ceiling)
  h2d          the upload of the inputs (outside the timed region)
  cpu_baseline the CPU oracle on a sample of the instances, on a pool of
               host threads (and on one thread)
  refit        the differentiable Kalman refit of 200k found tracks (forward
               and reverse pass) in tracks/s, with its own roofline and CPU
               baseline

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPC clusters/sec tracked, batched vs plain (deterministic FP32); refit grad tracks/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "chain_config4_traffic.md")
KERNEL_SOURCES = ["paper_2511_17018_amd/csrc/tpc_kernels.hip", "paper_2511_17018_amd/csrc/tpc_kalman.h",
                  "paper_2511_17018_amd/csrc/tpc_internal.h", "include/tpcca.h",
                  "paper_2511_17018_amd/build.py"]


def kernel_code_digest() -> str:
    """SHA-256 of the kernel sources with comments and white space removed,
    so that a committed profile stays valid across changes of comments only."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        if f.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()


def _profiled(path: str, field: str, kernel: str, occ: float, chunk: int) -> int | None:
    """Per-launch figure `field` of `kernel` from a committed rocprofv3
    summary, or None when the kernel sources or the launch parameters differ
    from the ones it was taken on."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != kernel_code_digest():
        return None
    # one block of figures per profiled launch configuration
    for block in re.split(r"^launch: ", text, flags=re.M)[1:]:
        ml = re.match(r"([0-9.]+),(\d+)", block)
        if not ml or float(ml.group(1)) != float(occ) or int(ml.group(2)) != int(chunk):
            continue
        mt = re.search(rf"^{re.escape(field)} {re.escape(kernel)}: (\d+)", block, flags=re.M)
        return int(mt.group(1)) if mt else None
    return None


def measured_traffic(kernel: str, occ: float, chunk: int) -> int | None:
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return _profiled(TRAFFIC_PROFILE, "traffic_bytes", kernel, occ, chunk)


def kernel_bytes(name: str, c: dict) -> float | None:
    """Algorithmic bytes one launch of `name` must move (per-unit figures
    times the units of the launch; see the design notes)."""
    N, S, Ht, E = c["N"], c["S"], c["Ht"], c["E"]
    R = 152
    table = {
        "grid_stats": 14 * N,                 # y, z, row in; segment id out
        "grid_part": 24 * N,                  # segment id, y, z in; index, y, z out
        "grid_seg": 28 * N + 4 * c.get("bins", 0),  # partitioned in; position data, bins out
        "neighbours": 24 * N + 8 * N,         # own + two neighbour rows' y,z; links out
        "clean": 16 * N + 8 * N,
        "tracklets": 4 * S + 16 * Ht + 8 * E + 88 * S,
        # every hit slot of every row, the keys of the hits, ownership bytes
        # out, the rows' owner keys out
        "sel_rows": 4 * R * S + 8 * Ht + R * S + 8 * N,
        "sel_count": Ht,
        # per position: owner, segment, input index; per owned hit of a
        # track: the track record, hit list entry and cluster->track entry
        "sel_hits": 12 * N + 40 * c.get("Hs", 0),
        # refit, per track-hit: hit index 4, cluster x,y,z 12, row 2, sector 1,
        # checkpoint 80 (written forward, read backward), gradient x,y,z 12
        "refit_fwd": 99 * c.get("Hr", 0),
        "refit_bwd": 111 * c.get("Hr", 0),
    }
    return table.get(name)


def run(args) -> dict:
    import torch

    import paper_2511_17018_amd as tpc
    import synth
    from paper_2511_17018_amd import autotune
    from paper_2511_17018_amd.runtime import Chain, GraphChain, plain_chains
    from synth.quality import track_quality

    t0 = time.time()
    ev = synth.config4(scale=args.scale)
    N, n_inst = ev.n, ev.n_inst
    sha = hashlib.sha256(np.concatenate([ev.y.view(np.uint8), ev.z.view(np.uint8),
                                         ev.row.view(np.uint8)]).tobytes()).hexdigest()
    log(f"generated {N} clusters in {n_inst} instances ({time.time() - t0:.1f}s)")
    dev = "cuda:0"
    torch.cuda.set_device(0)
    L = tpc.lib()
    geom = synth.geometry()
    torch.cuda.synchronize()
    t_h2d = time.perf_counter()
    batch = tpc.upload(ev.x, ev.y, ev.z, ev.row, ev.charge, ev.inst_off, dev)
    torch.cuda.synchronize()
    t_h2d = time.perf_counter() - t_h2d
    stream = torch.cuda.Stream(dev)

    def timed(fn, steps, warmup, label):
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                fn()
        stream.synchronize()
        t = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(steps):
                fn()
        stream.synchronize()
        dt = (time.perf_counter() - t) / steps
        log(f"{label}: {dt * 1e3:.3f} ms/step, {N / dt / 1e9:.3f} G clusters/s")
        return dt

    out = {}
    # ---- autotuned launch parameters (performance-only; outputs checked identical)
    if args.fixed:
        occ, chunk = args.fixed.split(",")
        tuned = {"grid_occupancy": float(occ), "tl_chunk": int(chunk), "ms": None,
                 "default_ms": None}
    else:
        tuned = autotune.tune(geom, batch, stream=stream, use_cache=not args.retune, log=log)
    tp = dict(grid_occupancy=tuned["grid_occupancy"], tl_chunk=tuned["tl_chunk"])
    out["autotune"] = {k: tuned[k] for k in ("grid_occupancy", "tl_chunk", "ms",
                                             "default_ms")}
    out["autotune"]["fixed"] = bool(args.fixed)
    # ---- batched, deterministic
    det_c = Chain(geom, batch, True, stream, **tp)
    dt_eager = timed(det_c.enqueue, args.steps, args.warmup, "batched det (eager)")
    res = det_c.result()
    if int(res["overflow"]) or int(res["n_bad"]):
        raise RuntimeError(f"unexpected status {res}")
    # the same chain with the generic kernels (settings as kernel arguments)
    # instead of those compiled for the standard configuration
    gen_c = Chain(geom, batch, True, stream, generic=True, **tp)
    dt_gen = timed(gen_c.enqueue, args.steps, args.warmup, "batched det, generic kernels")
    out["standard_kernels"] = {"used": tpc.standard_configuration(geom, det_c.params),
                               "generic_ms_per_step": dt_gen * 1e3,
                               "standard_ms_per_step": dt_eager * 1e3,
                               "generic_over_standard_time": dt_gen / dt_eager}
    del gen_c
    graph = GraphChain([det_c], stream)
    dt_det = timed(graph.replay, args.steps, args.warmup, "batched det (graph)")
    out["batched_eager"] = {"value": N / dt_eager, "ms_per_step": dt_eager * 1e3}
    # per-kernel times with HIP events (a second timed pass of the same steps, eager)
    assert L.tpc_profile_enable(1) == 0
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            det_c.enqueue()
    stream.synchronize()
    rows = (tpc_kernel_time * 64)()
    nk = L.tpc_profile_read(rows, 64)
    L.tpc_profile_enable(0)
    ktimes = {rows[i].name.decode(): (rows[i].total_ms, rows[i].launches) for i in range(nk)}
    # counts for the byte model
    ws = det_c.ws
    cap = ws.layout.cap_tracklets
    S = int(min(res["n_start"], cap))
    i32 = torch.int32
    nhit = ws.view("tl_nhit", i32, cap)[:S].to(torch.int64).sum().item()
    # E: clusters inside the extension searches' window boxes, counted by the
    # instrumented tracklet kernel in an untimed run (same results)
    cnt_c = Chain(geom, batch, True, stream, count=True, **tp)
    with torch.cuda.stream(stream):
        cnt_c.enqueue()
    stream.synchronize()
    if int(cnt_c.result()["n_tracks"]) != int(res["n_tracks"]):
        raise RuntimeError("instrumented run differs")
    ncand = cnt_c.ws.view("tl_ncand", i32, cap)[:S].to(torch.int64).sum().item()
    del cnt_c
    counts = dict(N=N, S=S, Ht=nhit, E=ncand, bins=int(res["n_bins"]), Hs=int(res["n_hits"]))
    dom = max(ktimes.items(), key=lambda kv: kv[1][0])
    name, (tot_ms, launches) = dom
    avg_s = tot_ms / launches / 1e3
    kb = kernel_bytes(name, counts)
    achieved = kb / avg_s / 1e9 if kb else None
    traffic = measured_traffic(name, tp["grid_occupancy"], tp["tl_chunk"])
    roofline = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": traffic, "traffic_source": os.path.relpath(TRAFFIC_PROFILE, ROOT)
                if traffic else None, "avg_launch_ms": avg_s * 1e3,
                "alg_bytes_per_launch": kb, "counts": counts}
    out["kernels_ms_per_step"] = {k: round(v[0] / args.steps, 4) for k, v in
                                  sorted(ktimes.items(), key=lambda kv: -kv[1][0])}
    out["kernels_sum_ms_per_step"] = round(sum(v[0] for v in ktimes.values()) / args.steps, 4)
    out["result"] = {k: int(res[k]) for k in ("n_valid", "n_start", "n_tracklets_kept",
                                              "n_tracks", "n_hits")}
    det_out = det_c.outputs()
    out["quality"] = track_quality(ev.label, ev.inst_off, det_out["hit_off"], det_out["hit_clu"])
    out["h2d"] = {"seconds": t_h2d, "bytes": 16 * N, "GB_per_s": 16 * N / t_h2d / 1e9,
                  "note": "pageable host arrays -> device SoA, outside the timed region"}
    out["copy_ceiling"] = copy_bandwidth(torch, stream)
    del graph, det_c
    # ---- batched, production
    if not args.no_prod:
        prod_c = Chain(geom, batch, False, stream, **tp)
        dt_prod = timed(prod_c.enqueue, args.steps, args.warmup, "batched prod (eager)")
        assert L.tpc_profile_enable(1) == 0
        with torch.cuda.stream(stream):
            for _ in range(args.steps):
                prod_c.enqueue()
        stream.synchronize()
        nk = L.tpc_profile_read(rows, 64)
        L.tpc_profile_enable(0)
        prod_out = prod_c.outputs()
        out["prod"] = {"value": N / dt_prod, "ms_per_step": dt_prod * 1e3,
                       "det_eager_over_prod_eager_time": dt_eager / dt_prod,
                       "quality": track_quality(ev.label, ev.inst_off, prod_out["hit_off"],
                                                prod_out["hit_clu"]),
                       "differently_assigned_vs_det": differently_assigned(det_out, prod_out, N),
                       "kernels_ms_per_step": {
                           rows[i].name.decode(): round(rows[i].total_ms / args.steps, 4)
                           for i in sorted(range(nk), key=lambda i: -rows[i].total_ms)[:8]}}
        del prod_c
    # ---- plain: one launch chain per instance, eager and graph-captured
    if not args.no_plain:
        plain = plain_chains(geom, batch, True, stream)
        ps = max(1, min(args.steps, 3))

        def run_plain():
            for c in plain:
                c.enqueue()

        dt_plain = timed(run_plain, ps, 1, "plain det (eager)")
        pg = GraphChain(plain, stream)
        dt_plain_g = timed(pg.replay, ps, 1, "plain det (graph)")
        out["plain"] = {"value": N / dt_plain, "ms_per_step": dt_plain * 1e3, "steps": ps,
                        "graph_value": N / dt_plain_g, "graph_ms_per_step": dt_plain_g * 1e3,
                        "batched_over_plain": dt_plain / dt_det,
                        "batched_over_plain_graph": dt_plain_g / dt_det}
        del pg, plain
    out.update(dt_det=dt_det, N=N, n_inst=n_inst, sha=sha, roofline=roofline)
    return out, ev


def run_refit(args) -> dict:
    """Refit forward + reverse pass over 200k found tracks (config 5)."""
    import torch

    import paper_2511_17018_amd as tpc
    import synth

    t0 = time.time()
    ev = synth.config5()
    ho, hc, seed = ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"]
    n_trk, n_hits = len(ho) - 1, int(ho[-1])
    log(f"refit: generated {n_trk} tracks, {n_hits} hits ({time.time() - t0:.1f}s)")
    dev = "cuda:0"
    L = tpc.lib()
    xyz = torch.from_numpy(np.stack([ev.x, ev.y, ev.z]).astype(np.float32)).to(dev)
    row = torch.from_numpy(ev.row.view(np.int16)).to(dev)
    trk = tpc.upload_refit_tracks(ho, hc, ev.sector, seed, dev)
    dmap = torch.zeros((152, 18), dtype=torch.float32, device=dev)   # start of a map fit
    chi2 = torch.empty(n_trk, dtype=torch.float32, device=dev)
    status = torch.empty(n_trk, dtype=torch.int32, device=dev)
    ckpt = torch.empty((n_hits, 20), dtype=torch.float32, device=dev)
    gmap = torch.empty((152, 18), dtype=torch.float32, device=dev)
    gxyz = torch.empty((3, xyz.shape[1]), dtype=torch.float32, device=dev)
    ones = torch.ones(n_trk, dtype=torch.float32, device=dev)
    L.tpc_refit_workspace_bytes.restype = C.c_size_t
    ws = torch.empty(int(L.tpc_refit_workspace_bytes()), dtype=torch.uint8, device=dev)
    geom = tpc.make_geometry(synth.geometry())
    par = tpc.make_params(True)
    cl = tpc._xyz_struct(xyz, row)
    ts = trk.struct()
    sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    fa = (C.byref(geom), C.byref(par), C.c_int64(xyz.shape[1]), cl, ts, tpc._ptr(dmap), None,
          tpc._ptr(chi2), tpc._ptr(status), tpc._ptr(ckpt), sp)
    ba = (C.byref(geom), C.byref(par), C.c_int64(xyz.shape[1]), cl, ts, tpc._ptr(dmap), None,
          tpc._ptr(ckpt), tpc._ptr(status), tpc._ptr(ones), tpc._ptr(gmap), tpc._ptr(gxyz[0]),
          tpc._ptr(gxyz[1]), tpc._ptr(gxyz[2]), tpc._ptr(ws), C.c_size_t(ws.numel()), sp)

    def step():
        if L.tpc_refit(*fa) or L.tpc_refit_backward(*ba):
            raise RuntimeError("refit call failed")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    log(f"refit fwd+bwd: {dt * 1e3:.3f} ms/step, {n_trk / dt / 1e6:.3f} M tracks/s")
    assert L.tpc_profile_enable(1) == 0
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    rows = (tpc_kernel_time * 64)()
    nk = L.tpc_profile_read(rows, 64)
    L.tpc_profile_enable(0)
    kt = {rows[i].name.decode(): (rows[i].total_ms, rows[i].launches) for i in range(nk)}
    out = {"value": n_trk / dt, "unit": "tracks/s", "ms_per_step": dt * 1e3,
           "workload": f"{n_trk} found tracks, {n_hits} hits, map 152x18 at zero, "
                       "forward + reverse pass, sum of chi2",
           "n_tracks": n_trk, "n_hits": n_hits,
           "failed_tracks": int((status != 0).sum().item()),
           "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items()}}
    rl = {}
    for name in ("refit_fwd", "refit_bwd"):
        if name in kt:
            avg_s = kt[name][0] / kt[name][1] / 1e3
            kb = kernel_bytes(name, dict(N=0, S=0, Ht=0, E=0, Hr=n_hits))
            rl[name] = {"bound": "hbm", "achieved": kb / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": kb / avg_s / 1e9 / HBM_PEAK_GBS,
                        "avg_launch_ms": avg_s * 1e3, "alg_bytes_per_launch": kb}
    out["roofline"] = rl
    # the same tracks through a field map (25 z bins per row) and the gas's
    # material (multiple scattering and energy loss), forward + reverse pass
    gm = tpc.upload_material(bz=synth.field_map(), ix0=synth.material_map()[0],
                             eloss=synth.material_map()[1], device=dev)
    ms = gm.struct()
    fam = fa[:6] + (C.byref(ms),) + fa[7:]
    bam = ba[:6] + (C.byref(ms),) + ba[7:]

    def step_mat():
        if L.tpc_refit(*fam) or L.tpc_refit_backward(*bam):
            raise RuntimeError("refit call with material failed")

    for _ in range(args.warmup):
        step_mat()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step_mat()
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - t) / args.steps
    log(f"refit fwd+bwd with field map and material: {dtm * 1e3:.3f} ms/step, "
        f"{n_trk / dtm / 1e6:.3f} M tracks/s")
    km = _prof_pass(L, torch, step_mat, args.steps)
    out["material"] = {"value": n_trk / dtm, "unit": "tracks/s", "ms_per_step": dtm * 1e3,
                       "workload": "the same tracks and map with a 0.5 T field map varying by "
                                   "up to 4.5 % (152 rows x 25 z bins), multiple scattering and "
                                   "energy loss of the gas per row",
                       "kernels_ms_per_step": {k: round(v[0], 4) for k, v in km.items()}}
    if not args.no_cpu:
        from concurrent.futures import ThreadPoolExecutor

        import oracle
        sub = 8000
        workers = cpu_workers()
        chunk = sub // workers

        def part(i):
            a, b = i * chunk, (i + 1) * chunk if i + 1 < workers else sub
            hs = ho[a:b + 1] - ho[a]
            oracle.refit_grad(synth.geometry(), oracle.DEFAULT_PARAMS, ev, hs,
                              hc[ho[a]:ho[b]], seed[a:b], np.zeros((152, 18), np.float32))
            return b - a

        t = time.perf_counter()
        part_one = sub // 4
        hs = ho[:part_one + 1]
        oracle.refit_grad(synth.geometry(), oracle.DEFAULT_PARAMS, ev, hs, hc[:hs[-1]],
                          seed[:part_one], np.zeros((152, 18), np.float32))
        t1 = time.perf_counter() - t
        t = time.perf_counter()
        with ThreadPoolExecutor(workers) as ex:
            done = sum(ex.map(part, range(workers)))
        tc = time.perf_counter() - t
        out["cpu_baseline"] = {"value": done / tc, "unit": "tracks/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"first {sub} tracks, binary64 forward + reverse pass, "
                                         f"in {workers} chunks on {workers} threads",
                               "single_thread": {"value": part_one / t1, "cores": 1,
                                                 "sample": f"first {part_one} tracks"},
                               "host": host_info()}
    return out


def _prof_pass(L, torch, fn, steps):
    """Per-kernel HIP-event times (ms per step) of `steps` calls of fn."""
    assert L.tpc_profile_enable(1) == 0
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    rows = (tpc_kernel_time * 64)()
    nk = L.tpc_profile_read(rows, 64)
    L.tpc_profile_enable(0)
    return {rows[i].name.decode(): (rows[i].total_ms / steps, rows[i].launches // steps)
            for i in range(nk)}


def run_transform(args, ev) -> dict:
    """Cluster coordinate transformation with both correction maps over the
    benchmark's clusters (raw readout coordinates of the same 15.65 M
    clusters, displaced by a smooth distortion)."""
    import torch

    import paper_2511_17018_amd as tpc
    import synth

    tg = synth.transform_geometry()
    dist = synth.Distortion(amp=1.0)
    raw = synth.encode_raw(ev, tg, dist=dist)
    rmap = synth.calibration_map(tg, dist)
    D = np.random.default_rng(3).uniform(-0.8, 0.8, (152, 18)).astype(np.float32)
    dev = "cuda:0"
    L = tpc.lib()
    s = torch.from_numpy(raw["sector"]).to(dev)
    r = torch.from_numpy(raw["row"].view(np.int16)).to(dev)
    pd = torch.from_numpy(raw["pad"]).to(dev)
    tm = torch.from_numpy(raw["time"]).to(dev)
    Dd = torch.from_numpy(D).to(dev)
    rm = torch.from_numpy(rmap).to(dev)
    n = len(raw["row"])
    out = tuple(torch.empty(n, dtype=dt, device=dev) for dt in (torch.float32, torch.float32,
                                                               torch.float32, torch.int16))

    def step():
        tpc.cluster_transform(tg, s, r, pd, tm, Dd, rm, det=True, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    kt = _prof_pass(L, torch, step, args.steps)
    avg_s = kt["transform"][0] / 1e3
    kb = 25 * n        # sector 1 + row 2 + pad 4 + time 4 in, x y z 12 + row 2 out
    res = {"value": n / dt, "unit": "clusters/s", "ms_per_step": dt * 1e3,
           "workload": f"{n} raw clusters (the benchmark's, displaced by a 1 cm distortion), "
                       "radial map 152x18 and residual map 36x16x9x26, deterministic build",
           "roofline": {"bound": "hbm", "kernel": "transform", "achieved": kb / avg_s / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": kb / avg_s / 1e9 / HBM_PEAK_GBS, "avg_launch_ms": avg_s * 1e3,
                        "alg_bytes_per_launch": kb}}
    if not args.no_cpu:
        import oracle
        t = time.perf_counter()
        oracle.transform(tg, raw["sector"], raw["row"], raw["pad"], raw["time"], D, rmap)
        tc = time.perf_counter() - t
        res["cpu_baseline"] = {"value": n / tc, "unit": "clusters/s", "cores": 1,
                               "kind": "oracle", "sample": f"all {n} clusters, binary32 oracle, "
                                                           "one thread"}
    log(f"transform: {dt * 1e3:.3f} ms/step, kernel {avg_s * 1e3:.3f} ms, "
        f"{kb / avg_s / 1e9:.0f} GB/s")
    return res


def run_config1(args, tp: dict) -> dict:
    """Config 1 (one sector wedge, 50 tracks, about 7 k clusters): the
    chain is bound by its launches' latency, not by work; graph-captured and
    eager times per step."""
    import torch

    import paper_2511_17018_amd as tpc
    import synth
    from paper_2511_17018_amd.runtime import Chain, GraphChain

    ev = synth.config1()
    dev = "cuda:0"
    stream = torch.cuda.Stream(dev)
    batch = tpc.upload(ev.x, ev.y, ev.z, ev.row, ev.charge, ev.inst_off, dev)
    ch = Chain(synth.geometry(), batch, True, stream, **tp)
    graph = GraphChain([ch], stream)
    steps = max(10, args.steps * 10)
    out = {"unit": "clusters/s", "workload": "config 1: one sector wedge, 50 tracks",
           "n_clusters": ev.n, "steps": steps}
    for label, fn in (("graph", graph.replay), ("eager", ch.enqueue)):
        with torch.cuda.stream(stream):
            for _ in range(max(1, args.warmup)):
                fn()
        stream.synchronize()
        t = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(steps):
                fn()
        stream.synchronize()
        dt = (time.perf_counter() - t) / steps
        log(f"config 1 tracking ({label}): {dt * 1e6:.1f} us/step")
        out[label] = {"value": ev.n / dt, "ms_per_step": dt * 1e3}
    res = ch.result()
    out["n_tracks"] = int(res["n_tracks"])
    return out


def run_sectors(args, which: int, tp: dict) -> dict:
    """Configs 2 and 3 (36 TPC sectors: one central collision, or 128
    collisions of a time frame in one pass): the batched deterministic chain
    (graph-captured) and the merging of its tracks across sector edges, with
    per-kernel times."""
    import torch

    import paper_2511_17018_amd as tpc
    import synth
    from paper_2511_17018_amd.runtime import Chain, GraphChain

    t0 = time.time()
    ev = synth.config2() if which == 2 else synth.config3()
    N = ev.n
    log(f"config {which}: {N} clusters ({time.time() - t0:.1f}s)")
    geom = synth.geometry()
    L = tpc.lib()
    dev = "cuda:0"
    stream = torch.cuda.Stream(dev)
    batch = tpc.upload(ev.x, ev.y, ev.z, ev.row, ev.charge, ev.inst_off, dev)
    # the tracker also writes each hit's plane, position and sector, which
    # the merging reads instead of gathering the clusters
    ch = Chain(geom, batch, True, stream, hit_data=True, **tp)
    steps = max(1, args.steps if which == 2 else min(args.steps, 5))
    with torch.cuda.stream(stream):
        ch.enqueue()
        merged = tpc.merge_tracks(geom, batch, ch.tracks, ch.ws.result)
    stream.synchronize()
    res = ch.result()
    if int(res["overflow"]):
        raise RuntimeError(f"config {which}: overflow {res}")
    graph = GraphChain([ch], stream)

    def timed(fn, label):
        with torch.cuda.stream(stream):
            for _ in range(max(1, args.warmup)):
                fn()
        stream.synchronize()
        t = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(steps):
                fn()
        stream.synchronize()
        dt = (time.perf_counter() - t) / steps
        log(f"config {which} {label}: {dt * 1e3:.3f} ms/step")
        return dt

    dt = timed(graph.replay, "tracking (graph)")

    def merge():
        tpc.merge_tracks(geom, batch, ch.tracks, ch.ws.result, out=merged)

    dtm = timed(merge, "merging")

    def both():
        with torch.cuda.stream(stream):
            ch.enqueue()
            merge()

    kt = _prof_pass(L, torch, both, steps)
    h = merged.host()
    n_seg = int(res["n_tracks"])
    out = {"value": N / dt, "unit": "clusters/s", "ms_per_step": dt * 1e3, "steps": steps,
           "workload": ("config 2: one central collision, 8000 tracks, 36 sectors"
                        if which == 2 else
                        "config 3: 128 collisions over 3 ms of drift time, 36 sectors, one pass"),
           "n_clusters": N, "n_tracks": n_seg, "n_hits": int(res["n_hits"]),
           "merge": {"ms_per_step": dtm * 1e3, "segments": n_seg, "merged_tracks": h["n"],
                     "links": int((h["next"][:n_seg] >= 0).sum()),
                     "refit_failed": int((h["status"] != 0).sum())},
           "kernels_ms_per_step": {k: round(v[0], 4) for k, v in
                                   sorted(kt.items(), key=lambda kv: -kv[1][0])}}
    del graph, ch, merged
    return out


def copy_bandwidth(torch, stream, reps: int = 5) -> dict:
    """Device-to-device copy of 1 GiB: a practical HBM ceiling for the same run."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    stream.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return {"GB_per_s": 2 * (1 << 30) / (ms / 1e3) / 1e9, "bytes_per_copy": 2 * (1 << 30),
            "ms": ms}


def differently_assigned(a: dict, b: dict, n: int) -> dict:
    """Fraction of clusters assigned differently by two outputs: unassigned in
    one of them only, or on a track of `b` that is not the majority partner of
    its track in `a` (tracks matched by shared clusters)."""
    ca, cb = a["clu2trk"][:n].astype(np.int64), b["clu2trk"][:n].astype(np.int64)
    both = (ca >= 0) & (cb >= 0)
    diff = int(((ca >= 0) != (cb >= 0)).sum())
    if both.any():
        pa, pb = ca[both], cb[both]
        keys, cnt = np.unique(pa * (int(cb.max()) + 1) + pb, return_counts=True)
        ka, kb = keys // (int(cb.max()) + 1), keys % (int(cb.max()) + 1)
        order = np.lexsort((-cnt, ka))
        first = np.ones(len(order), bool)
        first[1:] = ka[order][1:] != ka[order][:-1]
        partner = np.full(int(ca.max()) + 1, -1, np.int64)
        partner[ka[order][first]] = kb[order][first]
        diff += int((partner[pa] != pb).sum())
    return {"clusters": diff, "fraction": diff / max(1, n)}


def host_info() -> dict:
    """The host the CPU baselines ran on: logical CPUs, the ones this process
    may use, and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity": aff, "cpu_model": model,
            "share_note": "a one-GPU share of the host is 16 CPUs; the pools use "
                          "min(16, affinity) threads"}


def cpu_workers() -> int:
    return max(1, min(16, host_info()["affinity"]))


def cpu_baseline(ev, every: int) -> dict:
    """The binary32 oracle (whole chain a1-a6, as it stands) on every
    `every`-th instance: once on one thread, once with the instances dealt to
    a pool of threads (the oracle's C calls release the interpreter lock and
    keep no shared state)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth
    g = synth.geometry()
    sel = list(range(0, ev.n_inst, every))

    def one(i):
        a, b = int(ev.inst_off[i]), int(ev.inst_off[i + 1])
        off = np.array([0, b - a], np.int64)
        oracle.track(g, oracle.DEFAULT_PARAMS, off, ev.y[a:b], ev.z[a:b], ev.row[a:b])
        return b - a

    t = time.perf_counter()
    n_tot = sum(one(i) for i in sel)
    t1 = time.perf_counter() - t
    workers = cpu_workers()
    # largest instances first, so the pool ends together
    order = sorted(sel, key=lambda i: -(ev.inst_off[i + 1] - ev.inst_off[i]))
    t = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:
        n_par = sum(ex.map(one, order))
    tp = time.perf_counter() - t
    log(f"cpu oracle: {n_tot} clusters in {t1:.1f}s on 1 thread, {tp:.2f}s on {workers}")
    return {"value": n_par / tp, "unit": "clusters/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(sel)} of {ev.n_inst} instances (every {every}th), {n_tot} clusters, "
                      f"binary32 oracle, whole chain a1-a6, instances dealt to {workers} threads",
            "single_thread": {"value": n_tot / t1, "cores": 1, "seconds": t1},
            "host": host_info()}


class tpc_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("total_ms", C.c_double), ("launches", C.c_int64)]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="scale of the per-instance sizes")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-prod", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-every", type=int, default=4)
    ap.add_argument("--no-refit", action="store_true")
    ap.add_argument("--no-transform", action="store_true")
    ap.add_argument("--no-sectors", action="store_true",
                    help="skip the config 1 / 2 / 3 lines (tracking; merging for 2 and 3)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--fixed", default="",
                    help="OCC,CHUNK: use these launch parameters instead of tuning "
                         "(profiler runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this tracker runs on one GPU; sector instances shard across "
                                   "GPUs with no exchange, which this benchmark does not run",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    r, ev = run(args)
    if args.copy_calib:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
    line = {
        "metric": METRIC,
        "value": r["N"] / r["dt_det"],
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["dt_det"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256 uneven sector instances (log-uniform 1e3-4e5 clusters, "
                               "noise 0-20%), batched deterministic chain, graph-captured, "
                               "autotuned launch parameters",
                   "n_clusters": r["N"], "n_instances": r["n_inst"], "mode": "deterministic",
                   "path": "batched+graph", "input_sha256": r["sha"]},
        "roofline": r["roofline"],
    }
    for k in ("batched_eager", "autotune", "standard_kernels", "plain", "prod", "result",
              "quality", "h2d", "copy_ceiling", "kernels_ms_per_step", "kernels_sum_ms_per_step"):
        if k in r:
            line[k] = r[k]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(ev, args.cpu_every)
    if not args.no_transform:
        line["transform"] = run_transform(args, ev)
    del ev
    if not args.no_sectors:
        tp = {k: r["autotune"][k] for k in ("grid_occupancy", "tl_chunk")}
        line["config1"] = run_config1(args, tp)
        line["config2"] = run_sectors(args, 2, tp)
        line["config3"] = run_sectors(args, 3, tp)
    if not args.no_refit:
        line["refit"] = run_refit(args)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
