#!/usr/bin/env python
"""Per-frame mapping benchmark of the Gaussian-plus-SDF path on one MI355X.

Workload (synthetic, seeded): a 2.56 m procedural room fused into a 256^3 TSDF
at 1 cm, a smooth camera orbit of 1280x720 RGB-D frames with depth noise
sigma = 1 mm * z^2, and 100,000 Gaussians seeded near the surfaces seen along
the orbit.  One step = one frame: fuse the frame, raycast its view (the cached
SDF base image), then 10 optimisation iterations of render forward (with the
fused L1 colour + depth loss), backward (Gaussians and pose) and Adam.

Prints one JSON line: iterations/s over the timed frames (value), ms per frame,
the whole-iteration algorithmic HBM rate, the roofline of the dominant kernel
(from per-kernel HIP-event times) and the reference implementation timed on
this host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd+Adam iters/s @1280x720,100k Gaussians; ms/frame; HBM GB/s"
ITERS_PER_FRAME = 10
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3

# Algorithmic operation counts of the compositing kernels:
# every evaluated (pixel, instance) pair costs 15 flops for the opacity of Eq. 3,
# every composited pair 11 more in the forward and 66 more in the backward.
FLOPS_EVAL = 15
FLOPS_CONTRIB_FWD = 11
FLOPS_CONTRIB_BWD = 66


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of a kernel comes from rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE),
# recorded in profiles/traffic.json with the SHA-256 of the kernel's source files at
# the time of the measurement; it is reported only while those sources are unchanged.
KERNEL_SOURCES = {
    "composite_bwd": ("composite_bwd.hip", "render_common.h", "gps_internal.h"),
    "composite_fwd": ("composite_fwd.hip", "binning.h", "render_common.h", "gps_internal.h"),
}


def sources_sha256(kernel: str):
    import hashlib
    files = KERNEL_SOURCES.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_11574_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, tile: str, mode: int):
    """HBM bytes per launch of `kernel` at `tile`, or None when not measured for the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return None
    e = table.get(f"{kernel} {tile} mode{mode}")
    if not e or e.get("sources_sha256") != sources_sha256(kernel):
        return None
    return e.get("hbm_bytes_per_launch"), e.get("hbm_bytes_by_request_size")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--gaussians", type=int, default=100_000)
    ap.add_argument("--res", type=str, default="1280x720")
    ap.add_argument("--volume", type=int, default=256)
    ap.add_argument("--tile", type=str, default="16x32x128x2",
                    help="tile_w x tile_h x batch x pixels_per_lane, or 'auto' (autotuned on the first frame; on "
                         "the room workload its pick is 16x32 with a batch of 128 or 256 and 2 pixels per lane, "
                         "within 1 %% of each other, so the default fixes the first to keep profiles and the bench "
                         "line on one kernel)")
    ap.add_argument("--graph", type=int, default=0,
                    help="0: time kernel-by-kernel launches (the default: on the same frames they ran ahead of "
                         "graph replay); 1: time graph replay of each iteration (the view table is uploaded "
                         "once per frame either way); the other mode replays the same frames from the same "
                         "map state")
    ap.add_argument("--mode", type=int, default=0, help="0 sorted over-compositing, 1 the sort-free blend")
    ap.add_argument("--no-sort", action="store_true",
                    help="with --mode 1: no per-tile depth sort at all (the lists in emission order)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--modes", type=int, default=1,
                    help="time the forward and backward passes sorted and sort-free on the room view (Table 7 analogue)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the 8-keyframe batch (one 8-view iteration) against 8 single-view iterations")
    ap.add_argument("--large-frames", type=int, default=6,
                    help="frames timed on the 512^3 / 1M-Gaussian / 4-keyframe workload (0 skips it)")
    ap.add_argument("--maintenance", type=int, default=1,
                    help="time Gaussian removal (Eq. 8) and insertion (Eq. 6) once the timed frames are done")
    ap.add_argument("--other-mode", type=int, default=1,
                    help="also time the other launch mode (graph replay or kernel-by-kernel) on the same frames")
    ap.add_argument("--tracking", type=int, default=1,
                    help="time ICP tracking (Eq. 5) of one frame against the previous frame's raycast")
    ap.add_argument("--hash-frames", type=int, default=30,
                    help="frames fused and raycast over the voxel-block hash and over the dense lattice (0 skips)")
    ap.add_argument("--sh-frames", type=int, default=10,
                    help="frames of the mapping loop with SH bands 1-3 and without, from the same map (0 skips)")
    ap.add_argument("--calibrate-counters", type=int, default=0,
                    help="MiB written 3 times by a write-only kernel, then read 3 times by a read-only kernel, "
                         "before the workload, so that a counter run can scale WRITE_SIZE / FETCH_SIZE to bytes")
    ap.add_argument("--summarize-counters", nargs="+", default=None, metavar="DIR",
                    help="no GPU run: read the rocprofv3 counter CSVs under the given directories (made with "
                         "--calibrate-counters) and print per-dispatch means for the compositing kernels at --tile "
                         "and the calibration kernels; with FETCH_SIZE and WRITE_SIZE present, also the scaled "
                         "HBM bytes per launch (--write-traffic records them in profiles/traffic.json)")
    ap.add_argument("--summarize-trace", nargs="+", default=None, metavar="DIR",
                    help="no GPU run: the gps kernels of the rocprofv3 kernel-trace run under DIR (stats table, "
                         "and the mean of the last --last dispatches of the compositing kernels at --tile)")
    ap.add_argument("--last", type=int, default=300, help="dispatches averaged by --summarize-counters / -trace")
    ap.add_argument("--write-traffic", action="store_true")
    return ap.parse_args()


def _kname(name: str) -> str:
    """A rocprofv3 kernel name without its return type and argument list."""
    name = name.split("(")[0].strip()
    return name[5:] if name.startswith("void ") else name


def _counter_rows(dirs):
    """(dispatch id, kernel name, counter, value) of every rocprofv3 counter CSV under dirs."""
    import csv
    import glob
    rows = []
    for d in dirs:
        for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"],
                                 float(r["Counter_Value"])))
    rows.sort()
    return rows


def summarize_trace(args):
    """The gps kernels of a rocprofv3 --kernel-trace --stats run (its stats table), and the
    mean duration of the last --last dispatches of the compositing kernels at --tile."""
    import csv
    import glob
    for d in args.summarize_trace:
        for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
            print("| kernel | calls | avg µs | min µs | max µs | total µs |")
            print("|---|---|---|---|---|---|")
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    if "gps::" not in r["Name"]:
                        continue
                    print(f"| `{_kname(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                          f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                          f"{float(r['TotalDurationNs']) / 1e3:.0f} |")
        tw, th, b, ppt = args.tile.split("x")
        for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
            per = {}
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    name = _kname(r["Kernel_Name"])
                    per.setdefault(name, []).append((int(r["Start_Timestamp"]),
                                                     int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
            for k in ("fwd", "bwd"):
                name = f"gps::k_composite_{k}<{tw}, {th}, {b}, {ppt}, {args.mode}>"
                v = [dt for _, dt in sorted(per.get(name, []))][-args.last:]
                if v:
                    print(f"{name}: mean of the last {len(v)} of {len(per[name])} dispatches "
                          f"{sum(v) / len(v) / 1e3:.2f} µs")


def summarize_counters(args):
    """Per-dispatch means of the counters of the compositing kernels at --tile (the last
    --last dispatches) and of the calibration kernels; FETCH_SIZE and WRITE_SIZE scaled to
    bytes by what they read for the calibration kernels of known traffic."""
    rows = _counter_rows(args.summarize_counters)
    tw, th, b, ppt = args.tile.split("x")
    want = {f"gps::k_composite_{k}<{tw}, {th}, {b}, {ppt}, {args.mode}>": f"composite_{k}" for k in ("fwd", "bwd")}
    want.update({"gps::k_stream_read": "stream_read", "gps::k_stream_write": "stream_write"})
    vals = {}
    for _, name, ctr, v in rows:
        base = _kname(name)
        if base in want:
            vals.setdefault((want[base], ctr), []).append(v)
    out = {}
    for (k, ctr), v in sorted(vals.items()):
        last = v if k.startswith("stream") else v[-args.last:]
        out.setdefault(k, {})[ctr] = (sum(last) / len(last), len(last), len(v))
    for k, c in out.items():
        print(f"{k}: " + ", ".join(f"{n}={m:.6g} (mean of {u} of {t})" for n, (m, u, t) in sorted(c.items())))
    kib = args.calibrate_counters * 1024.0
    rd, wr = out.get("stream_read", {}), out.get("stream_write", {})
    if kib > 0 and "FETCH_SIZE" in rd and "WRITE_SIZE" in wr:
        fs, ws_ = kib / rd["FETCH_SIZE"][0], kib / wr["WRITE_SIZE"][0]
        print(f"scale: FETCH_SIZE x {fs:.4f} (read-only kernel: {rd['FETCH_SIZE'][0]:.1f} KiB for {kib:.0f} KiB), "
              f"WRITE_SIZE x {ws_:.4f} (write-only kernel: {wr['WRITE_SIZE'][0]:.1f} KiB for {kib:.0f} KiB)")
        table = {}
        path = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(path):
            with open(path) as fh:
                table = json.load(fh)
        rq = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")

        def read_bytes(c):  # read requests counted by size: 32, 64 and 128 bytes
            if not all(n in c for n in rq):
                return None
            return 32.0 * c[rq[0]][0] + 64.0 * c[rq[1]][0] + 128.0 * c[rq[2]][0]

        if read_bytes(rd) is not None:
            print(f"read requests by size, read-only kernel: {read_bytes(rd) / 1024:.1f} KiB for {kib:.0f} KiB")
        for k in ("composite_fwd", "composite_bwd"):
            c = out.get(k, {})
            if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
                continue
            hbm = (c["FETCH_SIZE"][0] * fs + c["WRITE_SIZE"][0] * ws_) * 1024.0
            rb = read_bytes(c)
            by_size = None if rb is None else int(rb + c["WRITE_SIZE"][0] * ws_ * 1024.0)
            print(f"{k} {args.tile} mode{args.mode}: {hbm / 1e6:.2f} MB of HBM traffic per launch (scaled FETCH_SIZE "
                  f"+ WRITE_SIZE)" + ("" if rb is None else
                                      f", {by_size / 1e6:.2f} MB with reads counted by request size "
                                      f"({c[rq[0]][0]:.0f} x 32 B, {c[rq[1]][0]:.0f} x 64 B, {c[rq[2]][0]:.0f} x 128 B)"))
            table[f"{k} {args.tile} mode{args.mode}"] = {
                "hbm_bytes_by_request_size": by_size,
                "kernel": next(n for n, v in want.items() if v == k).replace("gps::", ""),
                "fetch_kib_per_launch": round(c["FETCH_SIZE"][0], 1),
                "write_kib_per_launch": round(c["WRITE_SIZE"][0], 1),
                "fetch_scale": round(fs, 4), "write_scale": round(ws_, 4),
                "hbm_bytes_per_launch": int(hbm), "sources_sha256": sources_sha256(k),
                "dispatches": f"mean of the last {c['FETCH_SIZE'][1]} of {c['FETCH_SIZE'][2]}",
                "calibration": f"read-only and write-only kernels of {args.calibrate_counters} MiB "
                               f"(FETCH_SIZE {rd['FETCH_SIZE'][0]:.1f} KiB, WRITE_SIZE {wr['WRITE_SIZE'][0]:.1f} KiB; "
                               f"cross terms: the read kernel writes {rd.get('WRITE_SIZE', (0.0,))[0]:.1f} KiB, "
                               f"the write kernel fetches {wr.get('FETCH_SIZE', (0.0,))[0]:.1f} KiB)"}
        if args.write_traffic:
            with open(path, "w") as fh:
                json.dump(table, fh, indent=1)
                fh.write("\n")


def main():
    args = parse()
    if args.no_sort and args.mode != 1:
        print("bench.py: --no-sort needs --mode 1 (the sorted mode composites in depth order)", file=sys.stderr)
        sys.exit(2)
    if args.summarize_counters or args.summarize_trace:
        if args.summarize_trace:
            summarize_trace(args)
        if args.summarize_counters:
            summarize_counters(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by view across GPUs by design, but no multi-GPU run is made).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2509_11574_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    W_img, H_img = (int(x) for x in args.res.split("x"))
    K, Wu, M = args.steps, args.warmup, args.gaussians
    # warm-up frames, then K frames for the timed pass (timed again in the other launch mode
    # from the same map state), K new frames for the pass with per-kernel events (each frame
    # new to the map, as in mapping), then one frame that is tracked against the raycast of
    # the last one
    n_frames = Wu + 2 * K + 1

    if args.calibrate_counters > 0:
        n = args.calibrate_counters * (1 << 20) // 4
        buf = torch.empty(n, dtype=torch.float32, device=dev)
        part = torch.empty(P.gps.stream_blocks(), dtype=torch.float32, device=dev)
        for k in range(3):
            P.gps.stream_write(buf, 1.0 + k)
        for _ in range(3):
            P.gps.stream_read(buf, part)
        torch.cuda.synchronize()
        assert float(part.sum()) == 3.0 * n  # the reads saw the last write
        del buf, part

    # ---------------------------------------------------------------- inputs
    t0 = time.time()
    scene = synth.scene_room(args.volume)
    cams = synth.orbit_cameras(0, W_img, H_img, frames=list(range(n_frames)))
    frames = [synth.render_frame(scene, c, noise_sigma_per_m2=1e-3, frame_index=k, device=dev, as_torch=True)
              for k, c in enumerate(cams)]
    seed_cams = synth.orbit_cameras(0, W_img, H_img, frames=list(range(0, 100, 10)))
    seed_depths = [synth.render_frame(scene, c, device=dev, as_torch=True)[0].cpu().numpy() for c in seed_cams]
    gauss_np = synth.seed_gaussians(scene, seed_cams, seed_depths, M)
    params = P.gaussians_to_device(gauss_np, dev)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s: {n_frames} frames {W_img}x{H_img}, {M} Gaussians, "
        f"{args.volume}^3 volume")

    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=dev)
    cfg = P.RenderCfg(mode=args.mode, eps_cull=scene.voxel, no_sort=args.no_sort)
    cam0 = cams[0].as_dict()
    base_depth = torch.empty(H_img, W_img, device=dev)
    base_rgb = torch.empty(3, H_img, W_img, device=dev)
    out_rgb = torch.empty(3, H_img, W_img, device=dev)
    out_depth = torch.empty(H_img, W_img, device=dev)
    loss = torch.zeros(1, device=dev)
    grads = P.zeros_like_gaussians(params)
    dpose = torch.zeros(1, 6, device=dev)
    opt = P.Adam(params)

    def frame_prep(k):
        cam = cams[k].as_dict()
        depth, rgb = frames[k]
        P.fuse(vol, cam, depth, rgb)
        P.raycast(vol, [cam], z_near=cfg.z_near, out=[(base_depth, base_rgb)])
        return P.View(cam, base_rgb, base_depth, rgb, depth, out_rgb=out_rgb, out_depth=out_depth)

    tune_ms = None
    if args.tile == "auto":
        from paper_2509_11574_amd import autotune
        view = frame_prep(0)
        snapshot = {k: v.clone() for k, v in params.items()}  # tuning runs forward+backward only
        cfg, tune_ms = autotune.autotune(cfg, params, [view], reps=5, use_cache=False)
        torch.cuda.synchronize()
        for k in params:
            params[k].copy_(snapshot[k])
        vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=dev)  # start the map afresh
        log(f"autotuned: {cfg.tile_w}x{cfg.tile_h}x{cfg.batch}x{cfg.pix_per_thread} ({tune_ms})")
    else:
        tw, th, tb, ppt = (int(x) for x in args.tile.split("x"))
        cfg = P.RenderCfg(tile_w=tw, tile_h=th, batch=tb, pix_per_thread=ppt, mode=args.mode,
                          eps_cull=scene.voxel, no_sort=args.no_sort)
    ws = P.Workspace(cfg, M, [cam0], device=dev)

    from dataclasses import replace
    cfg_pre = replace(cfg, views_preset=True)

    def frame_step_eager(k):
        # the view table (and its tile depth maxima) is uploaded once per frame; the
        # iterations read it from the workspace, as the captured graph does
        view = frame_prep(k)
        P.gps.views_upload(cfg, params, [view], ws)
        for _ in range(ITERS_PER_FRAME):
            P.render_fwd(cfg_pre, params, [view], ws, out_loss=loss)
            P.render_bwd_adam(cfg_pre, params, [view], ws, opt, dpose=dpose)  # backward with Adam fused in
        return view

    graph = None

    def frame_step_graph(k):
        view = frame_prep(k)
        graph.set_views([view])
        for _ in range(ITERS_PER_FRAME):
            graph.replay()

    last_view = None
    for k in range(Wu):
        last_view = frame_step_eager(k)
    from paper_2509_11574_amd.graph import IterationGraph
    # captured on the last warm-up frame's view (capturing runs nothing on the device)
    graph = IterationGraph(cfg, params, [last_view], ws, grads, opt, loss, dpose, fused_adam=True)
    if args.graph:
        frame_step, mode_name, alt_step, alt_mode = frame_step_graph, "graph", frame_step_eager, "eager"
    else:
        frame_step, mode_name, alt_step, alt_mode = frame_step_eager, "eager", frame_step_graph, "graph"
    torch.cuda.synchronize()
    st0 = ws.stats()
    if st0["status"] != 0:
        raise RuntimeError(f"device status {st0['status']} after warm-up: {st0}")
    first_loss = float(loss.item())

    # the map state before the timed frames: the other launch mode replays the same frames from it
    def snapshot():
        st = {("p", k): v.clone() for k, v in params.items()}
        st.update({("m", k): v.clone() for k, v in opt.m.items()})
        st.update({("v", k): v.clone() for k, v in opt.v.items()})
        st.update({("vol", n): getattr(vol, n).clone() for n in ("tsdf", "weight", "rgb", "rgb_weight")})
        st[("ctr", "")] = opt.counter.clone()
        return st, opt.t

    def restore(snap):
        st, t = snap
        for (kind, k), v in st.items():
            dst = {"p": params, "m": opt.m, "v": opt.v}.get(kind)
            if dst is not None:
                dst[k].copy_(v)
            elif kind == "vol":
                getattr(vol, k).copy_(v)
            else:
                opt.counter.copy_(v)
        opt.t = t

    snap = snapshot() if args.other_mode else None

    # ------------------------------------------------------- timed frames
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_start = time.perf_counter()
    ev0.record()
    fev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    fev[0].record()
    for i, k in enumerate(range(Wu, Wu + K)):
        frame_step(k)
        fev[i + 1].record()
    ev1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start
    ms_event = ev0.elapsed_time(ev1)
    st1 = ws.stats()
    if st1["status"] != 0:
        raise RuntimeError(f"device status {st1['status']}: {st1}")
    ms_per_frame = 1000.0 * t_wall / K
    iters_per_s = ITERS_PER_FRAME * K / t_wall
    last_loss = float(loss.item())
    per_frame = sorted(fev[i].elapsed_time(fev[i + 1]) for i in range(K))
    pct = lambda q: per_frame[min(K - 1, int(round(q * (K - 1))))]
    frame_ms_pct = {"p10": round(pct(0.1), 4), "p50": round(pct(0.5), 4), "p90": round(pct(0.9), 4)}

    log(f"timed {K} frames ({mode_name}): {ms_per_frame:.3f} ms/frame (events {ms_event / K:.3f}), "
        f"{iters_per_s:.1f} iters/s, loss {first_loss:.5f} -> {last_loss:.6f}, instances {st1['n_instances']}")

    # ------------- the same frames from the same map state in the other launch mode
    alt = None
    if snap is not None:
        end_params = {k: v.clone() for k, v in params.items()}
        restore(snap)
        del snap
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(Wu, Wu + K):
            alt_step(k)
        torch.cuda.synchronize()
        te = time.perf_counter() - t1
        same = float(loss.item()) == last_loss and all(torch.equal(params[k], end_params[k]) for k in params)
        del end_params
        alt = {"launch": alt_mode, "ms_per_frame": round(1000.0 * te / K, 4),
               "iters_per_s": round(ITERS_PER_FRAME * K / te, 1),
               "bitwise_same_map": same,
               "frames": "the same %d frames from the same map state (parameters, moments, step counter and "
                         "volume restored), each iteration %s" %
                         (K, "launched kernel by kernel" if alt_mode == "eager"
                          else "replayed as one captured HIP graph")}
        log(f"other launch mode ({alt_mode}) on the same frames: {alt['ms_per_frame']:.3f} ms/frame, "
            f"{alt['iters_per_s']:.1f} iters/s, bitwise the same map: {same}")

    # --------------------------------------- per-kernel times (HIP events)
    kernels, pairs = {}, None
    if not args.no_profile:
        stp0 = ws.stats()
        P.gps.profile_start()
        for k in range(Wu + K, Wu + 2 * K):  # the next frames, launched eagerly so events bracket each kernel
            frame_step_eager(k)
        torch.cuda.synchronize()
        P.gps.profile_stop()
        kernels = P.gps.profile_read()
        stp1 = ws.stats()
        n_fwd = kernels.get("composite_fwd", (1, 0))[0]
        pairs = {"eval_per_launch": (stp1["pairs_eval"] - stp0["pairs_eval"]) / n_fwd,
                 "contrib_per_launch": (stp1["pairs_contrib"] - stp0["pairs_contrib"]) / n_fwd}
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda n: kernels[n][1])
        launches, total = kernels[dom]
        avg_s = total / launches / 1000.0
        if dom in ("composite_fwd", "composite_bwd"):
            per = FLOPS_CONTRIB_FWD if dom == "composite_fwd" else FLOPS_CONTRIB_BWD
            flops = FLOPS_EVAL * pairs["eval_per_launch"] + per * pairs["contrib_per_launch"]
            ach = flops / avg_s / 1e12
            tile_s = f"{cfg.tile_w}x{cfg.tile_h}x{cfg.batch}x{cfg.pix_per_thread}"
            tr = measured_traffic(dom, tile_s, args.mode) or (None, None)
            roofline = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                        "traffic": tr[0], "traffic_by_request_size": tr[1],
                        "avg_launch_ms": round(avg_s * 1e3, 4), "flops_per_launch": flops}
        else:
            roofline = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": None, "traffic": None, "avg_launch_ms": round(avg_s * 1e3, 4)}

    # ------------------------------ whole-iteration algorithmic HBM bytes
    I = st1["n_instances"]
    Pp = W_img * H_img
    bytes_iter = (56 * M + 48 * M + 8 * M            # project: params in, records + counts out
                  + 12 * I + 8 * M + 16 * I          # emit (keys, slots), tile sort (read + write)
                  + 60 * I + 48 * Pp                 # composite fwd: keys/slots/records, base+target+out
                  + 60 * I + 40 * I + 64 * Pp        # composite bwd: instances, partials out, per-pixel in
                  + 40 * I + 56 * M + 8 * M          # per-Gaussian reduce: partials, params in, slot offsets
                  + 336 * M)                         # Adam in its epilogue: 14 scalars x 24 B (p, m, v in + out)
    iter_ms = None
    if kernels:
        it_kernels = ("project", "scan", "count", "scan_tiles", "emit", "tile_sort",
                      "tile_sort_large", "composite_fwd", "loss_reduce", "composite_bwd", "gauss_bwd",
                      "pose_reduce", "adam", "step_incr")
        iter_ms = sum(kernels[n][1] for n in it_kernels if n in kernels) / (K * ITERS_PER_FRAME)
    hbm_gbs = bytes_iter / (iter_ms / 1e3) / 1e9 if iter_ms else None

    # ------------------------ sorted against sort-free passes (Table 7 analogue)
    mview = frame_prep(Wu + K - 1)
    modes = bench_modes(P, cfg, params, mview, M, cam0, reps=40) if args.modes else None

    # ----------------------------------- batched keyframes and the large map
    batched = bench_batched(P, synth, dev, cfg, reps=20) if args.batched else None
    large = bench_large(P, synth, dev, cfg, args.large_frames) if args.large_frames > 0 else None

    # -------------------------------- map maintenance: removal and insertion
    maint = bench_maintenance(P, cfg, mview, params, opt) if args.maintenance else None

    # ------------- the voxel-block hash, and view-dependent colour (SH bands 1-3)
    n_hash, n_sh = min(args.hash_frames, len(frames)), min(args.sh_frames, len(frames) - Wu)
    hashed = bench_hash(P, scene, cams, frames, cfg.z_near, n_hash) if n_hash > 0 else None
    sh = bench_sh(P, scene, cams, frames, gauss_np, cfg, Wu, n_sh) if n_sh > 0 else None

    # ------------- camera tracking of the next frame against the last raycast
    tracking = None
    if args.tracking:
        kl = Wu + 2 * K - 1
        frame_prep(kl)  # base_depth: the SDF raycast of the last frame
        tracking = bench_tracking(P, cams[kl].as_dict(), base_depth, cams[kl + 1].as_dict(), frames[kl + 1][0])

    # ------------------------------- reference implementation on the host
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, cams[Wu], frames[Wu], gauss_np, cfg)

    out = {"metric": METRIC, "value": round(iters_per_s, 2), "unit": "iters/s", "n_gpus": 1, "steps": K,
           "warmup": Wu, "ms_per_step": round(ms_per_frame, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"plain per-frame mapping: {args.volume}^3 TSDF at {scene.voxel * 100:.3g} cm, "
                                  f"{W_img}x{H_img} orbit frames, {M} Gaussians, {ITERS_PER_FRAME} iterations/frame",
                      "tile": f"{cfg.tile_w}x{cfg.tile_h}x{cfg.batch}x{cfg.pix_per_thread}",
                      "autotuned": args.tile == "auto",
                      "mode": "sorted" if args.mode == 0 else ("sort-free, no sort" if args.no_sort else "sort-free"),
                      "graph": bool(args.graph)},
           "autotune_ms_fwd_bwd": tune_ms,
           "ms_per_frame": round(ms_per_frame, 4),
           "ms_per_iteration_kernels": round(iter_ms, 4) if iter_ms else None,
           "hbm_gbs_iteration": round(hbm_gbs, 1) if hbm_gbs else None,
           "instances": I, "pairs": pairs,
           "loss_first_last": [round(first_loss, 6), round(last_loss, 6)],
           "roofline": roofline,
           "frame_ms_p10_p50_p90": frame_ms_pct,
           "other_launch_mode": alt,
           "sorted_vs_sort_free": modes,
           "batched_keyframes": batched,
           "large_map": large,
           "map_maintenance": maint,
           "voxel_block_hash": hashed,
           "sh_degree_3": sh,
           "tracking": tracking,
           "kernels_ms_per_frame": {n: round(v[1] / K, 4) for n, v in sorted(kernels.items(), key=lambda x: -x[1][1])},
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def _window_views(P, synth, scene, vol, cams, frames, dev, cfg):
    """Views of a window of keyframes: each frame fused into `vol`, then every
    keyframe's SDF base image raycast from the fused map (cached for the window)."""
    import torch
    views = []
    for cam, (depth, rgb) in zip(cams, frames):
        P.fuse(vol, cam.as_dict(), depth, rgb)
    for cam, (depth, rgb) in zip(cams, frames):
        bd = torch.empty(cam.height, cam.width, device=dev)
        bc = torch.empty(3, cam.height, cam.width, device=dev)
        P.raycast(vol, [cam.as_dict()], z_near=cfg.z_near, out=[(bd, bc)])
        views.append(P.View(cam.as_dict(), bc, bd, rgb, depth))
    return views


def bench_modes(P, cfg, params, view, M, cam0, reps=40):
    """Forward pass (binning, sort, compositing, fused loss) and backward pass (compositing
    backward, per-Gaussian reduce, pose) of one room view, timed with HIP events: the
    sorted over-compositing (mode 0); the sort-free blend of Eq. 1-4 without any depth
    sort (mode 1 with no_sort: the paper's renderer, its lists in emission order), with
    the tile backward and with the per-Gaussian backward over pixel chunks (App. B); and
    the sort-free blend with the lists sorted (bitwise reproducible).  Median of `reps`
    calls each."""
    import statistics
    from dataclasses import replace
    import torch
    out = {}
    for mode, name, pg, ns in ((0, "sorted", False, False), (1, "sort_free", False, True),
                               (1, "sort_free_per_gaussian_bwd", True, True),
                               (1, "sort_free_sorted_lists", False, False)):
        c = replace(cfg, mode=mode, bwd_per_gaussian=pg, no_sort=ns)
        ws = P.Workspace(c, M, [cam0], device=view.base_depth.device)
        grads = P.zeros_like_gaussians(params)
        dpose = torch.zeros(1, 6, device=view.base_depth.device)
        loss = torch.zeros(1, device=view.base_depth.device)
        for _ in range(3):
            P.render_fwd(c, params, [view], ws, out_loss=loss)
            P.render_bwd(c, params, [view], ws, grads, dpose)
        torch.cuda.synchronize()
        tf, tb = [], []
        for _ in range(reps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            P.render_fwd(c, params, [view], ws, out_loss=loss)
            e1.record()
            P.render_bwd(c, params, [view], ws, grads, dpose)
            e2.record()
            e2.synchronize()
            tf.append(e0.elapsed_time(e1))
            tb.append(e1.elapsed_time(e2))
        st = ws.stats()
        if st["status"] != 0:
            raise RuntimeError(f"device status {st['status']} in mode {mode}")
        out[name] = {"fwd_ms": round(statistics.median(tf), 4), "bwd_ms": round(statistics.median(tb), 4),
                     "loss": round(float(loss.item()), 6)}
        del ws
    out["note"] = ("median over %d calls, eager launches; the paper's Table 7 (RTX 4090, its own scenes): "
                   "with sort 0.97 / 1.87 ms, sort-free 0.87 / 1.51 ms (forward / backward)" % reps)
    return out


def bench_maintenance(P, cfg, view, params, opt, reps=20):
    """Map maintenance of Sec. 3.2.2 on the trained map and a room frame.
    Kernel time per call (HIP events around each launch): removal (Eq. 8) over the
    Gaussians with their two Adam moment sets as companions (3 sets, out of place);
    insertion (Eq. 6, App. A) from the map's own sort-free render of the frame (C* and
    the Gaussian weight W_G of Eq. 2, one forward in mode 1) with a seeded uniform draw.
    Algorithmic bytes: removal reads the 16 B that decide each Gaussian, all 56 B rows
    of every set and writes the kept rows; insertion reads 36 B per pixel and writes
    60 B per new Gaussian (its rows and pixel index).
    Then one whole keyframe cycle on a copy of the map (wall clock, host reads of the
    counts included): sort-free render, insertion and append, ten iterations of forward
    and backward with Adam on the grown map, and removal."""
    from dataclasses import replace

    import torch

    from paper_2509_11574_amd.mapping import GaussianMap, insert_from_render
    dev = params["mean"].device
    M = int(params["opacity_logit"].numel())
    c = P.camera(view.cam)
    W, H = c.width, c.height
    cfg1 = replace(cfg, mode=1, views_preset=False)
    v1 = P.View(view.cam, view.base_rgb, view.base_depth, view.target_rgb, view.target_depth,
                out_aux=torch.empty(H, W, device=dev))
    ws1 = P.Workspace(cfg1, M, [view.cam], device=dev)
    rand = torch.rand(H, W, device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    cd = view.cam

    def once():
        P.render_fwd(cfg1, params, [v1], ws1)
        ins = P.insert_gaussians(cd, v1.out_rgb, v1.target_rgb, v1.out_aux, v1.base_depth, rand)
        rem = P.remove_gaussians(params, [opt.m, opt.v])
        return ins, rem

    for _ in range(2):
        once()
    torch.cuda.synchronize()
    P.gps.profile_start()
    for _ in range(reps):
        (new, _, n_taken), (_, _, kept) = once()
    torch.cuda.synchronize()
    P.gps.profile_stop()
    kt = P.gps.profile_read()
    rem_ms, ins_ms = kt["remove"][1] / reps, kt["insert"][1] / reps
    render_ms = sum(kt[n][1] for n in kt if n not in ("remove", "insert")) / reps
    px = W * H
    rem_bytes = 16 * M + 3 * 56 * (M + kept)
    ins_bytes = 36 * px + 60 * min(n_taken, px)
    out = {"removal": {"gaussians": M, "kept": kept, "sets": 3, "ms_per_call": round(rem_ms, 4),
                       "algorithmic_bytes": rem_bytes, "gbs": round(rem_bytes / (rem_ms / 1e3) / 1e9, 1)},
           "insertion": {"pixels": px, "new": n_taken, "ms_per_call": round(ins_ms, 4),
                         "algorithmic_bytes": ins_bytes, "gbs": round(ins_bytes / (ins_ms / 1e3) / 1e9, 1),
                         "inputs": "C* and W_G of the map's sort-free render of the frame, "
                                   "uniform draw from a seeded generator",
                         "render_ms": round(render_ms, 4)},
           "launches_per_call": {"removal": 3, "insertion": 4}}
    # one keyframe cycle on a copy of the map
    gmap = GaussianMap({k: v.clone() for k, v in params.items()})
    for k in gmap.params:
        gmap.opt.m[k].copy_(opt.m[k])
        gmap.opt.v[k].copy_(opt.v[k])
    gmap.opt.t = opt.t
    gmap.opt.counter.copy_(opt.counter)
    loss = torch.zeros(1, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, n_new = insert_from_render(gmap, cfg, v1, rand)
    ws = P.Workspace(cfg, gmap.count, [view.cam], device=dev)
    P.gps.views_upload(cfg, gmap.params, [view], ws)
    cfg_pre = replace(cfg, views_preset=True)
    first = None
    for it in range(ITERS_PER_FRAME):
        P.render_fwd(cfg_pre, gmap.params, [view], ws, out_loss=loss)
        if it == 0:
            first = loss.clone()
        P.render_bwd_adam(cfg_pre, gmap.params, [view], ws, gmap.opt)
    grown = gmap.count
    n_kept = gmap.prune()
    torch.cuda.synchronize()
    cyc_ms = 1000.0 * (time.perf_counter() - t0)
    out["keyframe_cycle"] = {"ms": round(cyc_ms, 3), "gaussians_before": M, "inserted": n_new, "grown": grown,
                             "kept": n_kept, "loss_first_last": [round(float(first.item()), 6),
                                                                 round(float(loss.item()), 6)],
                             "steps": "sort-free render + insertion + append, %d iterations (forward, backward "
                                      "with Adam) on the grown map, removal; one run, wall clock" % ITERS_PER_FRAME}
    return out


def bench_tracking(P, prev_cam, prev_depth, cur_cam, cur_depth, reps=10):
    """Coarse-to-fine ICP (Eq. 5) of one frame against the SDF raycast of the frame
    before it: three levels (4, 4 and 6 Gauss-Newton steps, coarsest first), the depth
    hierarchy built inside each run; kernel time per tracked frame from HIP events
    around each launch, and the pose error against the frame's true pose."""
    import numpy as np
    import torch
    dev = cur_depth.device
    pose0 = P.pose_tensor(prev_cam, dev)
    pose = pose0.clone()
    ws = P.gps.IcpWorkspace(cur_cam["width"], cur_cam["height"], device=dev)
    P.icp_track(prev_cam, prev_depth, cur_cam, cur_depth, pose, ws=ws)
    torch.cuda.synchronize()
    P.gps.profile_start()
    for _ in range(reps):
        pose.copy_(pose0)
        P.icp_track(prev_cam, prev_depth, cur_cam, cur_depth, pose, ws=ws)
    torch.cuda.synchronize()
    P.gps.profile_stop()
    kt = P.gps.profile_read()
    launches, total = kt["icp"]
    p = pose.cpu().numpy().astype(np.float64)
    R, t = p[:9].reshape(3, 3), p[9:]
    RB, tB = np.asarray(cur_cam["R"], np.float64), np.asarray(cur_cam["t"], np.float64)
    R0 = np.asarray(prev_cam["R"], np.float64)
    t0 = np.asarray(prev_cam["t"], np.float64)
    def err(R_, t_):
        M = R_ @ RB.T
        s = 0.5 * np.linalg.norm([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
        return float(np.linalg.norm(-R_.T @ t_ + RB.T @ tB)), float(np.arctan2(s, 0.5 * (np.trace(M) - 1)))
    e0, e1 = err(R0, t0), err(R, t)
    pairs = int(ws.sys[28].item())
    return {"ms_per_frame": round(total / reps, 4), "launches_per_frame": launches // reps,
            "levels": "%dx%d, %dx%d, %dx%d" % (cur_cam["width"] // 4, cur_cam["height"] // 4, cur_cam["width"] // 2,
                                               cur_cam["height"] // 2, cur_cam["width"], cur_cam["height"]),
            "gauss_newton_steps": [4, 4, 6], "pairs_last_step": pairs,
            "start_error_mm_mrad": [round(e0[0] * 1e3, 3), round(e0[1] * 1e3, 3)],
            "final_error_mm_mrad": [round(e1[0] * 1e3, 3), round(e1[1] * 1e3, 3)]}


def bench_batched(P, synth, dev, cfg, reps=20, n_gauss=300_000):
    """Eight keyframes of mixed resolution (3 x 1280x720, 3 x 640x480, 2 x 320x240 at
    orbit frames 0, 12, ..., 87 of the room) sharing 300,000 Gaussians.  Batched: one
    iteration renders, differentiates and steps all eight views (one forward and one
    backward launch each, one graph).  Per-frame: eight single-view iterations in
    sequence (eight graphs, eight Adam steps).  Both produce the same per-view
    gradients; the batched form averages them into one step."""
    import torch

    from paper_2509_11574_amd.graph import IterationGraph
    scene = synth.scene_room(256)
    cams, frames = [], []
    for (k, W, H) in synth.STANDARD_VIEWS:
        cam = synth.orbit_cameras(0, W, H, frames=[k])[0]
        cams.append(cam)
        frames.append(synth.render_frame(scene, cam, noise_sigma_per_m2=1e-3, frame_index=k, device=dev,
                                         as_torch=True))
    seed_cams = synth.orbit_cameras(0, 1280, 720, frames=list(range(0, 100, 10)))
    seed_depths = [synth.render_frame(scene, c, device=dev, as_torch=True)[0].cpu().numpy() for c in seed_cams]
    params = P.gaussians_to_device(synth.seed_gaussians(scene, seed_cams, seed_depths, n_gauss), dev)
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=dev)
    views = _window_views(P, synth, scene, vol, cams, frames, dev, cfg)
    grads = P.zeros_like_gaussians(params)

    def timed(fn, n):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    init = {k: v.clone() for k, v in params.items()}
    opt_b = P.Adam(params)
    ws_b = P.Workspace(cfg, n_gauss, [v.cam for v in views], device=dev)
    loss_b = torch.zeros(1, device=dev)
    g_b = IterationGraph(cfg, params, views, ws_b, grads, opt_b, loss_b, torch.zeros(len(views), 6, device=dev))
    t_b = timed(g_b.replay, reps)
    st = ws_b.stats()
    if st["status"] != 0:
        raise RuntimeError(f"batched keyframes: device status {st}")
    inst_b = st["n_instances"]
    opt_s = P.Adam(params)
    graphs = []
    for v in views:
        ws = P.Workspace(cfg, n_gauss, [v.cam], device=dev)
        graphs.append((IterationGraph(cfg, params, [v], ws, grads, opt_s, torch.zeros(1, device=dev),
                                      torch.zeros(1, 6, device=dev)), ws))

    def seq():
        for g, _ in graphs:
            g.replay()
    t_s = timed(seq, reps)
    for _, ws in graphs:
        if ws.status() != 0:
            raise RuntimeError("per-frame keyframes: device status")
    nv = len(views)
    log(f"keyframe batch: batched {1e3 * t_b:.3f} ms per 8-view iteration, sequential {1e3 * t_s:.3f} ms "
        f"for 8 single-view iterations")

    # Time to the same accuracy: both forms start from the same map and fresh Adam state;
    # the batched form runs n_acc iterations, then the single-view form runs rounds of 8
    # (one per keyframe) until the mean loss over the 8 keyframes, measured by a separate
    # forward, is at most the batched form's.  Only the optimisation launches are timed.
    ws_e = P.Workspace(cfg, n_gauss, [v.cam for v in views], device=dev)
    le = torch.zeros(1, device=dev)

    def window_loss():
        P.render_fwd(cfg, params, views, ws_e, out_loss=le)
        torch.cuda.synchronize()
        return float(le.item())

    def reset(opt):
        for k in params:
            params[k].copy_(init[k])
        for k in opt.m:
            opt.m[k].zero_()
            opt.v[k].zero_()
        opt.counter.zero_()
        torch.cuda.synchronize()

    n_acc = 40
    reset(opt_b)
    l0 = window_loss()
    t0 = time.perf_counter()
    for _ in range(n_acc):
        g_b.replay()
    torch.cuda.synchronize()
    tb_acc = time.perf_counter() - t0
    target = window_loss()
    reset(opt_s)
    ts_acc, rounds, ls = 0.0, 0, l0
    while ls > target and rounds < 4 * n_acc:
        t0 = time.perf_counter()
        seq()
        torch.cuda.synchronize()
        ts_acc += time.perf_counter() - t0
        rounds += 1
        ls = window_loss()
    accuracy = {"start_loss": round(l0, 6), "target_loss": round(target, 6),
                "batched": {"iterations": n_acc, "view_iterations": n_acc * nv, "ms": round(1e3 * tb_acc, 3)},
                "single_view": {"rounds_of_8": rounds, "view_iterations": rounds * nv, "ms": round(1e3 * ts_acc, 3),
                                "final_loss": round(ls, 6), "reached": bool(ls <= target)},
                "time_to_accuracy_speedup": round(ts_acc / tb_acc, 3) if ls <= target else None,
                "note": "mean fused loss over the 8 keyframes; both forms from the same map and fresh Adam state"}
    log(f"keyframe batch, same accuracy: batched {n_acc} iterations {1e3 * tb_acc:.1f} ms to loss {target:.6f}; "
        f"single-view {rounds} rounds of 8 {1e3 * ts_acc:.1f} ms to loss {ls:.6f}")
    del g_b, ws_b, ws_e
    return {"workload": "8 keyframes (3x1280x720, 3x640x480, 2x320x240), 300000 Gaussians, 256^3 room",
            "instances": inst_b,
            "batched_ms_per_iteration": round(1e3 * t_b, 4),
            "sequential_ms_per_8_iterations": round(1e3 * t_s, 4),
            "batched_view_iters_per_s": round(nv / t_b, 1),
            "sequential_view_iters_per_s": round(nv / t_s, 1),
            "speedup": round(t_s / t_b, 3),
            "same_accuracy": accuracy}


def bench_hash(P, scene, cams, frames, z_near, n_frames, capacity=32768):
    """Per-frame map update over the voxel-block hash against the dense lattice, on the
    same frames from an empty map: fusion (with block allocation) and the raycast of the
    frame's view, eager launches.  Reports the time per frame, the pool in use and the
    largest depth difference of the last raycast where both hit (the hash reads points
    of unallocated blocks as unobserved, so the two may differ at the band's edges)."""
    import numpy as np
    import torch
    dev = frames[0][0].device
    H, W = frames[0][0].shape
    out_d = [(torch.empty(H, W, device=dev), torch.empty(3, H, W, device=dev)) for _ in range(2)]

    def run(fuse, raycast, vol, out):
        for k in range(2):  # warm-up on the first two frames, then the map starts afresh
            fuse(vol, cams[k].as_dict(), *frames[k])
            raycast(vol, [cams[k].as_dict()], z_near=z_near, out=[out])
        return vol

    res = {}
    for name in ("dense", "hash"):
        if name == "dense":
            make = lambda: P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=dev)
            fuse, raycast, out = P.fuse, P.raycast, out_d[0]
        else:
            make = lambda: P.HashVolume(scene.dims, scene.origin, scene.voxel, scene.trunc, capacity=capacity,
                                        device=dev)
            fuse, raycast, out = P.hash_fuse, P.hash_raycast, out_d[1]
        run(fuse, raycast, make(), out)
        vol = make()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_frames):
            cam = cams[k].as_dict()
            fuse(vol, cam, *frames[k])
            raycast(vol, [cam], z_near=z_near, out=[out])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / n_frames
        if name == "dense":
            mem = 24 * int(np.prod(scene.dims))
            res[name] = {"ms_per_frame": round(ms, 4), "volume_mb": round(mem / 1e6, 1)}
        else:
            st = vol.state()
            if st["status"] != 0:
                raise RuntimeError(f"hash volume status {st}")
            blocks = st["allocated"]
            mem = 24 * blocks * P.gps.HASH_BLOCK ** 3
            res[name] = {"ms_per_frame": round(ms, 4), "blocks": blocks, "capacity": capacity,
                         "pool_in_use_mb": round(mem / 1e6, 1),
                         "table_mb": round(12 * vol.n_buckets / 1e6, 2)}
    dd, dh = out_d[0][0], out_d[1][0]
    both = (dd > 0) & (dh > 0)
    diff = (dd - dh).abs()[both]
    res["last_raycast"] = {"hit_agree": round(float(((dd > 0) == (dh > 0)).float().mean()), 6),
                           "depth_equal_frac": round(float((diff == 0).float().mean()), 6),
                           "depth_diff_over_1cm_frac": round(float((diff > 0.01).float().mean()), 6),
                           "max_depth_diff_m": round(float(diff.max()), 6)}
    res["frames"] = n_frames
    log(f"hash: {res['hash']['ms_per_frame']:.3f} ms per frame ({res['hash']['blocks']} blocks, "
        f"{res['hash']['pool_in_use_mb']} MB), dense {res['dense']['ms_per_frame']:.3f} ms "
        f"({res['dense']['volume_mb']} MB)")
    return res


def bench_sh(P, scene, cams, frames, gauss_np, cfg, first, n_frames, degree=3):
    """The per-frame mapping loop with view-dependent colour (SH bands 1..degree, 3
    channels) against the same loop without, on the same frames from the same map:
    fusion, raycast and 10 iterations of forward + backward with Adam per frame."""
    import numpy as np
    import torch
    dev = frames[0][0].device
    H, W = frames[0][0].shape
    K = {1: 3, 2: 8, 3: 15}[degree]
    M = int(gauss_np["opacity_logit"].size)
    rng = np.random.Generator(np.random.PCG64(11))
    res = {}
    for L in (0, degree):
        g = dict(gauss_np)
        if L:
            g["sh"] = (0.05 * rng.standard_normal((3, K, M))).astype(np.float32)
        params = P.gaussians_to_device(g, dev)
        opt = P.Adam(params)
        vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=dev)
        ws = P.Workspace(cfg, M, [cams[first].as_dict()], device=dev)
        bd, br = torch.empty(H, W, device=dev), torch.empty(3, H, W, device=dev)
        orgb, od = torch.empty(3, H, W, device=dev), torch.empty(H, W, device=dev)
        loss, dpose = torch.zeros(1, device=dev), torch.zeros(1, 6, device=dev)
        from dataclasses import replace
        cfg_pre = replace(cfg, views_preset=True)

        def frame(k):
            cam = cams[k].as_dict()
            P.fuse(vol, cam, *frames[k])
            P.raycast(vol, [cam], z_near=cfg.z_near, out=[(bd, br)])
            view = P.View(cam, br, bd, frames[k][1], frames[k][0], out_rgb=orgb, out_depth=od)
            P.gps.views_upload(cfg, params, [view], ws)
            for _ in range(ITERS_PER_FRAME):
                P.render_fwd(cfg_pre, params, [view], ws, out_loss=loss)
                P.render_bwd_adam(cfg_pre, params, [view], ws, opt, dpose=dpose)

        for k in range(first):
            frame(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(first, first + n_frames):
            frame(k)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / n_frames
        if ws.status() != 0:
            raise RuntimeError("SH leg: device status")
        res[f"degree_{L}"] = {"ms_per_frame": round(ms, 4), "iters_per_s": round(1e3 * ITERS_PER_FRAME / ms, 1),
                              "loss_last": round(float(loss.item()), 6)}
    res["frames"] = n_frames
    log(f"SH degree {degree}: {res[f'degree_{degree}']['ms_per_frame']:.3f} ms per frame against "
        f"{res['degree_0']['ms_per_frame']:.3f} without")
    return res


def bench_large(P, synth, dev, cfg, n_frames, n_gauss=1_000_000, warm=2):
    """Large map: the room at 5 mm (512^3 lattice, 3.2 GB of volume), 1280x720 orbit
    frames fused every frame, 1,000,000 Gaussians, and per frame 10 batched
    iterations over the latest 4 keyframes (one keyframe every 10 frames; a new
    keyframe's base image is raycast when it enters the window)."""
    import torch

    from paper_2509_11574_amd.graph import IterationGraph
    scene = synth.scene_room(512)
    W, H = 1280, 720
    total = warm + n_frames
    first = 40  # the window starts full: keyframes at frames 10, 20, 30, 40
    idx = list(range(first - 30, first + 1 + total))  # frames 10 .. 41 + total
    cams = synth.orbit_cameras(0, W, H, frames=idx)
    frames = [synth.render_frame(scene, c, noise_sigma_per_m2=1e-3, frame_index=k, device=dev, as_torch=True)
              for k, c in zip(idx, cams)]
    seed_cams = synth.orbit_cameras(0, W, H, frames=list(range(0, 100, 10)))
    seed_depths = [synth.render_frame(scene, c, device=dev, as_torch=True)[0].cpu().numpy() for c in seed_cams]
    params = P.gaussians_to_device(synth.seed_gaussians(scene, seed_cams, seed_depths, n_gauss), dev)
    vol = P.Volume(scene.dims, scene.origin, scene.voxel, scene.trunc, device=dev)
    kf = [30, 0, 10, 20]  # frames 40, 10, 20, 30: window slot (frame / 10) mod 4 holds that keyframe
    views = _window_views(P, synth, scene, vol, [cams[i] for i in kf], [frames[i] for i in kf], dev, cfg)
    grads = P.zeros_like_gaussians(params)
    opt = P.Adam(params)
    ws = P.Workspace(cfg, n_gauss, [v.cam for v in views], device=dev)
    g = IterationGraph(cfg, params, views, ws, grads, opt, torch.zeros(1, device=dev),
                       torch.zeros(len(views), 6, device=dev))
    ring = [(v.base_depth, v.base_rgb) for v in views]

    def frame(i):
        cam = cams[i]
        depth, rgb = frames[i]
        P.fuse(vol, cam.as_dict(), depth, rgb)
        if idx[i] % 10 == 0:  # new keyframe: raycast its base into the oldest slot
            slot = (idx[i] // 10) % 4
            bd, bc = ring[slot]
            P.raycast(vol, [cam.as_dict()], z_near=cfg.z_near, out=[(bd, bc)])
            views[slot] = P.View(cam.as_dict(), bc, bd, rgb, depth)
            g.set_views(views)
        for _ in range(ITERS_PER_FRAME):
            g.replay()

    for i in range(31, 31 + warm):
        frame(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(31 + warm, 31 + warm + n_frames):
        frame(i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n_frames
    st = ws.stats()
    if st["status"] != 0:
        raise RuntimeError(f"large map: device status {st}")
    log(f"large map: {1e3 * dt:.3f} ms per frame, {ITERS_PER_FRAME / dt:.1f} batched iterations/s")
    return {"workload": "512^3 TSDF at 5 mm, 1280x720 frames fused every frame, 1000000 Gaussians, "
                        "10 batched iterations per frame over the latest 4 keyframes",
            "frames": n_frames, "ms_per_frame": round(1e3 * dt, 3),
            "batched_iters_per_s": round(ITERS_PER_FRAME / dt, 2),
            "view_iters_per_s": round(4 * ITERS_PER_FRAME / dt, 1),
            "instances": st["n_instances"]}


def _host_threads():
    """Threads the host gives this process: the OpenMP setting where it is set, else the
    CPUs this process may run on."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(env))) if env.isdigit() else n


def _oracle_frame(O, scene, cam, frame, gauss_np, cfg):
    """Seconds of the reference on a bounded sample of one frame of the room workload: one
    fusion of the full volume, the raycast of every 8th pixel in each direction and one
    forward + backward of every 16th, Adam over all parameters; scaled to the frame."""
    import numpy as np
    depth = frame[0].cpu().numpy()
    rgb = frame[1].cpu().numpy()
    camd = cam.as_dict()
    H, W = depth.shape
    Pp = W * H
    grid = O.make_grid(scene.dims, scene.origin, scene.voxel, scene.trunc, 100.0)
    vol = O.new_volume(grid)
    t = time.perf_counter()
    O.fuse(grid, vol, camd, depth, rgb)
    t_fuse = time.perf_counter() - t
    t32, c32 = vol["tsdf"].astype(np.float32), vol["rgb"].astype(np.float32)
    jj, ii = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    pix_r = (jj * W + ii).reshape(-1).astype(np.int32)
    t = time.perf_counter()
    rd, rc, _ = O.raycast(grid, t32, c32, camd, z_near=cfg.z_near, pix=pix_r)
    t_ray = (time.perf_counter() - t) * Pp / pix_r.size
    bd = np.zeros(Pp, np.float32)
    bc = np.zeros((3, Pp), np.float32)
    bd[pix_r] = rd
    bc[:, pix_r] = rc
    jj, ii = np.meshgrid(np.arange(0, H, 16), np.arange(0, W, 16), indexing="ij")
    pix_f = (jj * W + ii).reshape(-1).astype(np.int32)
    ocfg = O.RenderCfg(mode=cfg.mode, eps_cull=cfg.eps_cull)
    t = time.perf_counter()
    r = O.render(ocfg, gauss_np, camd, bc, bd, pix=pix_f)
    t_fwd = time.perf_counter() - t
    gC = np.sign(r["rgb"] - rgb.reshape(3, -1)[:, pix_f]) / (3.0 * Pp)
    gD = np.where((depth.reshape(-1)[pix_f] > 0) & (bd[pix_f] > 0), np.sign(r["depth"] - depth.reshape(-1)[pix_f]), 0)
    gD = gD / max(1, int(((depth.reshape(-1) > 0) & (bd > 0)).sum()))
    t = time.perf_counter()
    O.render_bwd(ocfg, gauss_np, camd, bc, bd, gC, gD, pix=pix_f)
    t_bwd = time.perf_counter() - t
    t = time.perf_counter()
    for k, v in gauss_np.items():
        a = v.astype(np.float64).reshape(-1).copy()
        O.adam(a, np.ones_like(a), np.zeros_like(a), np.zeros_like(a), O.PAPER_LR[k], 1)
    t_adam = time.perf_counter() - t
    scale = Pp / pix_f.size
    t_iter = (t_fwd + t_bwd) * scale + t_adam
    t_frame = t_fuse + t_ray + ITERS_PER_FRAME * t_iter
    return {"t_frame": t_frame, "t_iter": t_iter, "t_fuse": t_fuse, "t_fwd_bwd": t_fwd + t_bwd,
            "pix_r": pix_r.size, "pix_f": pix_f.size, "ray_scale": Pp / pix_r.size, "fb_scale": scale}


def _oracle_tiny(O, synth):
    """Seconds of the reference on the whole tiny workload, unsampled: 64^3 fusion, raycast
    of every pixel of the 160x120 frame, forward + backward over 2,000 Gaussians, Adam."""
    import numpy as np
    w = synth.workload_small(M=2000)
    sc, cam = w["scene"], w["cam"]
    camd = cam.as_dict()
    t = time.perf_counter()
    grid = O.make_grid(sc.dims, sc.origin, sc.voxel, sc.trunc, 100.0)
    vol = O.fuse(grid, O.new_volume(grid), camd, w["depth"], w["rgb"])
    rd, rc, _ = O.raycast(grid, vol["tsdf"].astype(np.float32), vol["rgb"].astype(np.float32), camd)
    bd, bc = rd.astype(np.float32), rc.astype(np.float32)
    ocfg = O.RenderCfg(eps_cull=sc.voxel)
    r = O.render(ocfg, w["gauss"], camd, bc, bd)
    L, gC, gD, _ = O.loss(ocfg, cam.width, cam.height, r["rgb"], r["depth"], w["rgb"], w["depth"], bd)
    g = O.render_bwd(ocfg, w["gauss"], camd, bc, bd, gC, gD)
    for k, v in w["gauss"].items():
        a = v.astype(np.float64).reshape(-1).copy()
        O.adam(a, g[k].reshape(-1), np.zeros_like(a), np.zeros_like(a), O.PAPER_LR[k], 1)
    return time.perf_counter() - t


def cpu_baseline(scene, cam, frame, gauss_np, cfg):
    """The reference implementation, as it stands, on this host's cores: a bounded sample of
    one frame of the room workload (see _oracle_frame) at the host's thread count and at
    one thread, and the whole tiny workload unsampled at the host's thread count."""
    import synth
    from oracle import oracle as O

    n = _host_threads()
    O.set_threads(n)
    full = _oracle_frame(O, scene, cam, frame, gauss_np, cfg)
    tiny = _oracle_tiny(O, synth)
    O.set_threads(1)
    one = _oracle_frame(O, scene, cam, frame, gauss_np, cfg)
    O.set_threads(n)
    return {"value": round(ITERS_PER_FRAME / full["t_frame"], 5), "unit": "iters/s", "cores": n, "kind": "oracle",
            "ms_per_frame": round(1e3 * full["t_frame"], 1), "ms_per_iteration": round(1e3 * full["t_iter"], 1),
            "sample": f"FP64 C reference, {n} OpenMP threads: full-volume fusion ({full['t_fuse']:.2f} s), raycast of "
                      f"{full['pix_r']} px scaled x{full['ray_scale']:.0f}, forward+backward of {full['pix_f']} px "
                      f"({full['t_fwd_bwd']:.2f} s) scaled x{full['fb_scale']:.0f}, Adam over all parameters",
            "one_thread": {"value": round(ITERS_PER_FRAME / one["t_frame"], 5), "ms_per_frame": round(1e3 * one["t_frame"], 1),
                           "ms_per_iteration": round(1e3 * one["t_iter"], 1)},
            "tiny_workload_unsampled": {"threads": n, "ms": round(1e3 * tiny, 1),
                                        "steps": "64^3 fusion, raycast of 160x120, forward + backward of 2,000 "
                                                 "Gaussians, Adam"},
            "cpu": _cpu_model(), "host_threads": n}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
