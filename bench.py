#!/usr/bin/env python3
"""Benchmark of the selective multi-scale Gaussian rasteriser on one MI355X.

Workload: the 4-level synthetic scene (531,250 Gaussians; level l holds
400k/4^l Gaussians, log-scale mean -4.5 + 1.4 l, SH degree 3), S^max/S^min
established by the library's own range update over 8 seeded cameras, one
1600x1064 camera at distance 3 (f = 1875).  One step = the whole hot path at
the four downscales 1x, 4x, 16x, 64x with selective rendering: forward render
(projection, coverage, selection, SH, binning, sorts, blending) and the
backward pass against a fixed seeded dL/dRGB.  Inputs are resident in HBM
before timing; the timed region is bracketed by device synchronisation.  The
timed steps replay one captured HIP graph per frame (fixed tile-list capacity
of 1.25x the counted instances, so no host synchronisation inside a frame),
the four frames on four streams; every replayed frame is checked to have done
the counted work.  The eager step (exact tile lists, one host thread and
stream per frame) is timed too and reported beside it.

Metric: Gaussian-pixel blends per second (accumulated contributions of the
forward renders of one step, divided by the step time).  The JSON line also
carries per-downscale frame rates and p50/p99 frame latency for selective and
single-scale (selection off) rendering, the roofline of the dominant kernel
(live HIP-event timing of that kernel's launches) and the CPU oracle's rate on
a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DOWNSCALES = (1, 4, 16, 64)
W_FULL, H_FULL, FOCAL = 1600, 1064, 1875.0
HBM_PEAK_GBS = 8000.0
# fp32 vector peak: 256 CUs x 4 SIMD x 32 fp32 lanes per cycle x 2.4 GHz x 2
# flops per fma = 157.3 TFLOP/s.  The library is compiled with packed fp32
# disabled, but a wave64 fp32 fma still issues every ~2 cycles on gfx950 (a
# probe of eight independent fma chains per thread measured 2.45 cycles), so
# the unpacked rate is this same peak.
ALU_PEAK_TFLOPS = 256 * 4 * 32 * 2.4e9 * 2 / 1e12
# algorithmic fp32 flops of the compositing loop (fma = 2): every evaluated
# (pixel, instance) pair costs the offset and quadratic form (11); every
# accumulated contribution adds exp (19), alpha, transmittance and colour (10).
FLOPS_PER_VISIT = 11
FLOPS_PER_BLEND = 29
# the adjoint per accumulated contribution: exp (19); alpha, 1/(1-alpha) and
# the replayed transmittance (6); colour and alpha partials with the suffix
# colour update (24); partials of sigma, centre and conic (16); and the sum of
# the nine partials over the tile's pixels (9)
FLOPS_PER_BLEND_BWD = 74
# stage name -> index into the library's per-frame stage timings
STAGE_IDX = {"project": 0, "depth_sort": 1, "count_scan": 2, "emit": 3, "tile_sort": 4,
             "ranges": 5, "blend": 6, "zero_bwd": 10, "blend_bwd": 7, "chain_bwd": 8}
STAGES = tuple(STAGE_IDX)


def c2_camera(G):
    import numpy as np
    return G.Camera(R=np.eye(3, dtype=np.float32).reshape(9), t=np.array([0, 0, 3], np.float32),
                    fx=FOCAL, fy=FOCAL, cx=W_FULL / 2.0, cy=H_FULL / 2.0, width=W_FULL,
                    height=H_FULL)


def depth_sort_passes(fr):
    """The depth-sort passes a frame needs: one per 8-bit digit of the 32-bit
    depth keys of its drawable Gaussians that is not the same for all of them
    (the library skips the others)."""
    import numpy as np
    k, _ = fr.keys()
    d = np.unique((k & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    if d.size < 2:
        return 1
    return sum(1 for q in range(4) if np.unique((d >> np.uint32(8 * q)) & np.uint32(255)).size > 1)


def stage_bytes(st, n, sh_degree, passes_depth, passes_tile):
    """Algorithmic HBM bytes of the memory-bound stages of one render."""
    K = (sh_degree + 1) ** 2
    nv, I = st["n_visible"], st["n_instances"]
    ntile = st["tiles_x"] * st["tiles_y"]
    return {
        # read mu, s, q, sigma, level, S^max, S^min; write mask and tile count;
        # visible: read SH, write record, rectangle, depth key, compacted pair
        "project": n * (12 + 12 + 16 + 4 + 1 + 4 + 4) + n * (1 + 4) + nv * (12 * K + 48 + 8 + 4 + 8),
        # one read of the keys for the digit histograms, then per pass the keys
        # and values read and written, except the last pass's keys
        "depth_sort": nv * 4 + passes_depth * nv * 16 - nv * 4,
        "count_scan": nv * (4 + 4 + 4),
        "emit": nv * (4 + 4 + 8 + 4) + I * 8,
        "tile_sort": passes_tile * I * (4 + 16),
        "ranges": I * 4 + ntile * 8,
        # clear of the written-partial bit mask
        "zero_bwd": (I + 31) // 32 * 4,
        # read the partials and tile counts, write/read the per-Gaussian sums,
        # read the parameters again, write every gradient plane
        "chain_bwd": I // 8 + n * 8 + n * 72 + n * (53 + 12 * K) + n * (44 + 12 * K),
    }


def cpu_info():
    """CPU model (lscpu) and core count of the machine that runs the oracle."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline_extra():
    """The oracle at one thread on a smaller sample of the same workload (1024
    random pixels of the 1x frame and the whole 64x frame), and the oracle's
    projection + sort stage (projection of all 531,250 Gaussians, emission and
    std::stable_sort of the 1x frame's tile keys) timed on its own at full size,
    median of 3."""
    import numpy as np
    import oracle as O
    from paper_2311_17089_amd import scenegen as G
    sc = G.four_level_scene()
    cal = O.calibrate(sc, G.calibration_cameras(1002, W_FULL, H_FULL, FOCAL))
    cam = c2_camera(G)
    rng = np.random.default_rng(8)
    idx = rng.choice(W_FULL * H_FULL, size=1024, replace=False)
    pix = np.stack([idx % W_FULL, idx // W_FULL], 1).astype(np.int32)
    t0 = time.perf_counter()
    _, _, nc = O.render_pixels(cal, cam, pix, downscale=1, nthreads=1)
    _, _, _, b64 = O.render(cal, cam, downscale=64, nthreads=1)
    dt1 = time.perf_counter() - t0
    blends1 = int(nc.sum()) + b64
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        k, _ = O.keys(cal, cam, downscale=1)
        ts.append(time.perf_counter() - t0)
    tk = sorted(ts)[1]
    return {"one_thread": {"value": blends1 / dt1, "unit": "blends/s", "cores": 1,
                           "sample": f"1024 random pixels at 1x and the full 64x frame, "
                                     f"{blends1} blends in {dt1:.1f} s"},
            "projection_and_sort_stage": {"ms": tk * 1e3, "instances": int(k.size),
                                          "instances_per_s": k.size / tk,
                                          "what": "projection of all Gaussians (OpenMP), tile-key "
                                                  "emission and one std::stable_sort of the 1x "
                                                  "frame's keys, median of 3"}}


def cpu_baseline(seconds_hint=True):
    """The oracle as it stands, on a bounded sample of the workload: brute-force
    compositing of 131072 random pixels of the 1x frame and of the whole 4x, 16x
    and 64x frames (each call includes the oracle's projection of all
    Gaussians).  Returns blends per second over the sample."""
    import numpy as np
    import oracle as O
    from paper_2311_17089_amd import scenegen as G
    sc = G.four_level_scene()
    cal = O.calibrate(sc, G.calibration_cameras(1002, W_FULL, H_FULL, FOCAL))
    cam = c2_camera(G)
    rng = np.random.default_rng(7)
    blends = 0
    t0 = time.perf_counter()
    for ds in DOWNSCALES:
        W, H = W_FULL // ds, H_FULL // ds
        if ds == 1:
            idx = rng.choice(W * H, size=131072, replace=False)
            pix = np.stack([idx % W, idx // W], 1).astype(np.int32)
            _, _, nc = O.render_pixels(cal, cam, pix, downscale=ds)
            blends += int(nc.sum())
        else:
            _, _, _, b = O.render(cal, cam, downscale=ds)
            blends += b
    dt = time.perf_counter() - t0
    return {"value": blends / dt, "unit": "blends/s", "cores": int(O.lib().or_max_threads()),
            "kind": "oracle",
            "sample": "brute-force compositing of 131072 random pixels at 1x and of the full "
                      "4x, 16x and 64x frames of the same scene and camera, selective, "
                      f"{blends} blends in {dt:.1f} s (includes the oracle's per-call projection)"}


def serving_replay(M, G, n_req=512, rate_hz=200.0, inflight=4, selective=True):
    """Poisson stream of render requests against the resident 3M-Gaussian,
    4-level scene: poses uniform on a sphere of radius 2-12 looking at the
    origin, 1920x1080 downscaled by a factor uniform over {1, 2, ..., 128}.
    Requests are submitted at their arrival times to the continuous-batching
    server; latency = completion - scheduled arrival (the server's completion
    minus submission time, plus how late the submission was)."""
    import numpy as np
    import torch
    ctx, dsc = c3_scene(M, G)
    stream = G.request_stream(seed=4, n=n_req, rate_hz=rate_hz)
    outs = [torch.empty((cam.height // d, cam.width // d, 3), device="cuda") for _, cam, d in stream]
    torch.cuda.synchronize()
    srv = M.Server(ctx, dsc, max_inflight=inflight)
    done = []
    late = np.zeros(n_req)
    t0 = time.perf_counter()
    for i, (arr, cam, d) in enumerate(stream):
        while time.perf_counter() - t0 < arr:
            done += srv.poll(64, 0)
            time.sleep(0.0002)
        late[i] = (time.perf_counter() - t0 - arr) * 1e3
        srv.submit(cam, outs[i], i, downscale=d, selective=selective)
    while len(done) < n_req:
        done += srv.poll(64, 1_000_000)
    srv.close()

    def latency(d):
        return (d["t_done_us"] - d["t_submit_us"]) / 1e3 + late[d["req_id"]]

    lat = np.array([latency(d) for d in done])
    ok = all(d["status"] == 0 for d in done)
    first = min(d["t_submit_us"] for d in done)
    last = max(d["t_done_us"] for d in done)
    per_ds = {}
    for d in done:
        per_ds.setdefault(stream[d["req_id"]][2], []).append(latency(d))
    return {"requests": n_req, "rate_hz": rate_hz, "inflight": inflight, "all_ok": ok,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "frames_per_s": n_req / ((last - first) / 1e6),
            "max_submit_lag_ms": float(late.max()),
            "blends": int(sum(d["n_blends"] for d in done)),
            "p50_ms_by_downscale": {str(k): float(np.percentile(v, 50)) for k, v in sorted(per_ds.items())}}


def c3_scene(M, G):
    """The resident 3M-Gaussian, 4-level scene (SH degree 3) with its
    selection ranges calibrated on the GPU at 1920x1080, shared by the
    serving replay and the differentiation configuration."""
    if not hasattr(c3_scene, "scene"):
        ctx = M.Context(0)
        sc = G.large_scene(3_000_000, 4, 3)
        dsc = M.DeviceScene(ctx, sc)
        M.calibrate(ctx, dsc, G.calibration_cameras(1003, 1920, 1080, 2250.0))
        c3_scene.scene = (ctx, dsc)
    return c3_scene.scene


def frame_timing(M, ctx, dsc, cam, ds, backward, reps=20):
    """One frame (forward, or forward + backward of a seeded upstream
    gradient): its counts, the sum of its stage spans in profiled eager runs
    (the library's HIP events around each stage, which add their own
    overhead), and the wall time per frame of a captured HIP graph of it
    (fixed tile-list capacity 1.25x the counted instances + 4096) replayed
    `reps` times back to back (the headline figures)."""
    import torch
    W, H = cam.width // ds, cam.height // ds
    g = torch.Generator().manual_seed(700 + ds)
    dl = torch.randn((H, W, 3), generator=g).cuda() * 1e-3 if backward else None

    def once(prof=False, capacity=0):
        _, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, profile=prof,
                         capacity=capacity)
        if backward:
            M.render_backward(ctx, fr, dl)
        return fr

    fr = once()
    st = fr.stats()
    fr.release()
    cap = int(st["n_instances"] * 1.25) + 4096
    dev_us = 0.0
    for _ in range(3):
        fr = once(prof=True)
        dev_us += sum(fr.stats()["stage_us"])
        fr.release()
    once(capacity=cap).release()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=side):
        _, gfr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, stream=side, capacity=cap)
        if backward:
            M.render_backward(ctx, gfr, dl, stream=side)
    for _ in range(3):
        gr.replay()
    torch.cuda.synchronize()
    assert gfr.stats()["n_blends"] == st["n_blends"]
    t0 = time.perf_counter()
    for _ in range(reps):
        gr.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    del gr
    torch.cuda.synchronize()
    gfr.release()
    return {"width": W, "height": H, "n_selected": st["n_selected"],
            "n_instances": st["n_instances"], "blends": st["n_blends"],
            "ms_per_frame": ms, "frames_per_s": 1e3 / ms,
            "blends_per_s": st["n_blends"] / (ms / 1e3),
            "stage_us_sum_profiled": dev_us / 3, "reps": reps}


def other_configs(M, G):
    """The two other workloads of the method's benchmark set, timed frame by
    frame: the single-level 10k-Gaussian scene at 128x128 (forward only) and
    the 3M-Gaussian, 4-level scene at 1920x1080, 1x and 8x (forward plus the
    adjoint backward)."""
    import numpy as np
    ctx = M.Context(0)
    sc1 = G.single_level_scene()
    d1 = M.DeviceScene(ctx, sc1)
    cam1 = G.Camera(R=np.eye(3, dtype=np.float32).reshape(9), t=np.array([0, 0, 3], np.float32),
                    fx=150.0, fy=150.0, cx=64.0, cy=64.0, width=128, height=128)
    out = {"single_level_10k_128px": dict(frame_timing(M, ctx, d1, cam1, 1, False, reps=200),
                                          n_gaussians=sc1.n, passes="forward")}
    d1.close()
    ctx3, d3 = c3_scene(M, G)
    cam3 = G.Camera(R=np.eye(3, dtype=np.float32).reshape(9), t=np.array([0, 0, 3], np.float32),
                    fx=2250.0, fy=2250.0, cx=960.0, cy=540.0, width=1920, height=1080)
    out["four_level_3m_1080p"] = {
        str(ds): dict(frame_timing(M, ctx3, d3, cam3, ds, True), passes="forward + backward")
        for ds in (1, 8)}
    return out


def aggregation_bench(M, G, reps=3):
    """Alg. 1 on the GPU: the level-0 Gaussians of the 3M-Gaussian scene
    (2,258,824 of them, SH degree 3) and 8 training cameras at radius 3,
    1920x1080; level 1 (downscale 4, 200^3 voxels) and then level 2 (16,
    133^3) built on top of it, as msgs_build_levels does.  Timed per level:
    one aggregate_level call on the resident scene (minimal coverage over the
    cameras, voxel keys, sort, segmented average pooling, enlargement), device
    synchronised on both sides."""
    import dataclasses
    import torch
    sc = G.large_scene(3_000_000, 4, 3)
    keep = sc.level == 0
    base = dataclasses.replace(sc, n=int(keep.sum()), n_levels=3, means=sc.means[:, keep].copy(),
                               scales=sc.scales[:, keep].copy(), quats=sc.quats[:, keep].copy(),
                               opacity=sc.opacity[keep].copy(), sh=sc.sh[:, keep].copy(),
                               level=sc.level[keep].copy(), s_max=sc.s_max[keep].copy(),
                               s_min=sc.s_min[keep].copy())
    cams = G.calibration_cameras(1003, 1920, 1080, 2250.0)
    ctx = M.Context(0)
    res = {}
    scene = base
    for level in (1, 2):
        dsc = M.DeviceScene(ctx, scene)
        part = M.aggregate_level(ctx, dsc, cams, level)  # warm-up (library defaults)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            part = M.aggregate_level(ctx, dsc, cams, level)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        below = int(scene.n)
        added = int(part["opacity"].numel())
        dt = sorted(ts)[len(ts) // 2]
        res[str(level)] = {"gaussians_below": below, "added": added, "ms": dt * 1e3,
                           "gaussians_per_s": below / dt, "cameras": len(cams)}
        host = {k: v.cpu().numpy() for k, v in part.items()}
        dsc.close()
        import numpy as np
        scene = dataclasses.replace(
            scene, n=scene.n + added,
            means=np.ascontiguousarray(np.concatenate([scene.means, host["means"]], 1)),
            scales=np.ascontiguousarray(np.concatenate([scene.scales, host["scales"]], 1)),
            quats=np.ascontiguousarray(np.concatenate([scene.quats, host["quats"]], 1)),
            opacity=np.ascontiguousarray(np.concatenate([scene.opacity, host["opacity"]])),
            sh=np.ascontiguousarray(np.concatenate([scene.sh, host["sh"]], 1)),
            level=np.concatenate([scene.level, np.full(added, level, np.uint8)]),
            s_max=np.concatenate([scene.s_max, np.zeros(added, np.float32)]),
            s_min=np.concatenate([scene.s_min, np.full(added, np.inf, np.float32)]))
    return {"workload": "level 0 of the 3M-Gaussian scene (2,258,824 Gaussians, SH degree 3), "
                        "8 cameras at 1920x1080; levels 1 and 2 aggregated in turn", "levels": res}


def prefilter_effect(M, ctx, dsc, cam, reps=5):
    """Projection-stage device time of the C2 frames with the pre-splat coverage
    bound on and off (the results are identical either way), and how many
    Gaussians the bound settled before the rotation load and the EWA."""
    import numpy as np
    out = {}
    for ds in DOWNSCALES:
        row = {}
        for on in (True, False):
            us, nf = [], 0
            for _ in range(reps):
                _, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, profile=True,
                                 prefilter=on)
                st = fr.stats()
                fr.release()
                us.append(st["stage_us"][0])
                nf = st["n_prefiltered"]
            row["on" if on else "off"] = {"project_us": float(np.median(us)), "prefiltered": nf}
        out[str(ds)] = row
    return out


def training_step(M, G, steps=5, warmup=2):
    """Multi-view training step on the 6M-Gaussian, 5-level scene: 8 views
    (seeded poses on a sphere of radius 2-12), one at each downscale 1, 2, ...,
    128 of 1920x1080, with the range update on, rendered by one multi-view call
    (one projection pass over the scene for the 8 views), then one multi-view
    backward into one set of gradient planes, all on one stream.  dL/dRGB is a
    fixed seeded tensor per view.  Timed eagerly (exact tile lists, one host
    synchronisation per step; also with one render call per view and one
    backward call per view, for comparison) and as one captured HIP graph
    (fixed tile-list capacities of 1.25x the eager counts, no host
    synchronisation).  Returns step times and blends per second."""
    import numpy as np
    import torch
    ctx = M.Context(0)
    sc = G.large_scene(6_000_000, 5, 5)
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(1005, 1920, 1080, 2250.0))
    poses = G.sphere_poses(8, 5, 2.0, 12.0)
    views = [(G.lookat_camera(poses[i], 1920, 1080, 2250.0), 2 ** i) for i in range(8)]
    dls = [torch.randn((1080 // d, 1920 // d, 3), generator=torch.Generator().manual_seed(900 + i))
           .cuda() * 1e-6 for i, (_, d) in enumerate(views)]
    outs = [torch.empty((1080 // d, 1920 // d, 3), device="cuda") for _, d in views]
    names = ("means", "scales", "quats", "opacity", "sh")
    grads = {k: torch.zeros_like(dsc.t[k]) for k in names}
    zeros = {k: torch.zeros_like(dsc.t[k]) for k in names}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    caps = [0] * len(views)

    def step(capacity=False, keep=False, mode="multi"):
        if mode == "multi":
            vl = [(cam, {"downscale": d, "update_range": True,
                         "capacity": caps[i] if capacity else 0})
                  for i, (cam, d) in enumerate(views)]
            _, frames = M.render_views(ctx, dsc, vl, keep_frames=True, outs=outs)
        else:
            frames = []
            if mode == "per_view_backward":
                for k in names:
                    grads[k].copy_(zeros[k])
            for i, ((cam, d), dl) in enumerate(zip(views, dls)):
                _, fr = M.render(ctx, dsc, cam, downscale=d, update_range=True, keep_frame=True,
                                 out=outs[i], capacity=caps[i] if capacity else 0)
                if mode == "per_view_backward":
                    M.render_backward(ctx, fr, dl, grads=grads, accumulate=True)
                frames.append(fr)
        if mode != "per_view_backward":
            M.render_backward_views(ctx, frames, dls, grads=grads)
        if keep:
            return frames
        for fr in frames:
            fr.release()
        return []

    with torch.cuda.stream(side):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        fr0 = step(keep=True)
        st0 = [f.stats() for f in fr0]
        blends = sum(s["n_blends"] for s in st0)
        for i, s in enumerate(st0):
            caps[i] = int(s["n_instances"] * 1.25) + 1024
        for f in fr0:
            f.release()
        torch.cuda.synchronize()
        t_eager = {}
        for mode in ("per_view_backward", "per_view", "multi"):
            step(mode=mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step(mode=mode)
            torch.cuda.synchronize()
            t_eager[mode] = (time.perf_counter() - t0) / steps
        # capture: warm the allocator on this stream with the same capacities
        for _ in range(2):
            step(capacity=True)
        torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        frames = step(capacity=True, keep=True)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    overflow = 0
    for f in frames:
        try:
            f.stats()
        except M.MsgsError:
            overflow += 1
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / steps
    del g
    torch.cuda.synchronize()
    for f in frames:
        f.release()
    dsc.close()
    return {"workload": "6M Gaussians over 5 levels (SH degree 3), 8 views at 1920x1080 / "
                        "{1,2,...,128}, range update on, gradients accumulated",
            "ms_per_step_eager": t_eager["multi"] * 1e3, "ms_per_step_graph": t_graph * 1e3,
            "ms_per_step_eager_render_per_view": t_eager["per_view"] * 1e3,
            "ms_per_step_eager_render_and_backward_per_view": t_eager["per_view_backward"] * 1e3,
            "blends_per_step": blends, "blends_per_s_eager": blends / t_eager["multi"],
            "blends_per_s_graph": blends / t_graph, "steps": steps,
            "execution": "one multi-view render call (one projection pass for the 8 views) and "
                         "one multi-view backward per step",
            "graph_capacity_overflows": overflow}


def serving_sweep(M, G, rates=(200, 400, 800, 1600, 3200, 6400), n_req=512):
    """The Poisson replay at increasing offered rates, selective and
    single-scale: frames/s, p50 and p99 per rate; capacity = the highest
    frames/s reached; sustainable rate = the highest offered rate served at
    95% or more of it with p99 at most 50 ms."""
    out = {}
    for selective in (True, False):
        curve = {}
        for r in rates:
            res = serving_replay(M, G, n_req=n_req, rate_hz=float(r), selective=selective)
            curve[str(r)] = {"frames_per_s": res["frames_per_s"], "p50_ms": res["p50_ms"],
                             "p99_ms": res["p99_ms"], "all_ok": res["all_ok"],
                             "max_submit_lag_ms": res["max_submit_lag_ms"]}
        ok = [r for r in rates if curve[str(r)]["frames_per_s"] >= 0.95 * r and
              curve[str(r)]["p99_ms"] <= 50.0]
        out["selective" if selective else "single_scale"] = {
            "by_offered_rate_hz": curve,
            "capacity_frames_per_s": max(v["frames_per_s"] for v in curve.values()),
            "sustainable_rate_hz": max(ok) if ok else None}
    return out


def traffic_for(kernel, launch):
    """HBM traffic of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken from the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    try:
        rec = json.loads(open(path).read().split("\n---\n")[0])
    except Exception:
        return None
    ent = rec.get(kernel, {}).get(launch)
    if not ent:
        return None
    src = os.path.join(ROOT, "paper_2311_17089_amd", "csrc", ent["source"])
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if h != ent["source_sha256_16"]:
        return None
    return ent["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-training", action="store_true")
    ap.add_argument("--no-aggregation", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=30)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run one serial step and a 1 GiB elementwise copy, for HBM counter runs")
    ap.add_argument("--serial", action="store_true",
                    help="render the frames of a step one after another on one stream")
    ap.add_argument("--eager", action="store_true",
                    help="time eager steps (exact tile lists, one host thread per frame) instead "
                         "of the replayed per-frame HIP graphs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X and the library "
              "has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_17089_amd import msgs as M
    from paper_2311_17089_amd import scenegen as G

    print("bench: building the 4-level scene", file=sys.stderr, flush=True)
    ctx = M.Context(0)
    sc = G.four_level_scene()
    dsc = M.DeviceScene(ctx, sc)
    M.calibrate(ctx, dsc, G.calibration_cameras(1002, W_FULL, H_FULL, FOCAL))
    cam = c2_camera(G)
    dls = {}
    for i, ds in enumerate(DOWNSCALES):
        g = torch.Generator().manual_seed(500 + i)
        dls[ds] = torch.randn((H_FULL // ds, W_FULL // ds, 3), generator=g).cuda() * 1e-3
    stream = torch.cuda.current_stream()
    # one stream and one host thread per frame: the four frames of a step are
    # independent, so the small ones run on the CUs the 1x frame leaves idle
    from concurrent.futures import ThreadPoolExecutor
    streams = {ds: torch.cuda.Stream() for ds in DOWNSCALES}
    pool = ThreadPoolExecutor(max_workers=len(DOWNSCALES))

    # per-launch device time of every stage, from the library's own HIP events
    # on the frame's stream, accumulated over the kernel-timing steps
    stage_acc = {ds: {s: 0.0 for s in STAGES} for ds in DOWNSCALES}

    # fixed tile-list capacities (set after the counting step) for the frames
    # that run without a host synchronisation: eager capacity-mode warm-up
    # and the captured graphs
    caps = {}

    def run_frame(ds, st=None, prof=False, capacity=False):
        _, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, profile=prof, stream=st,
                         capacity=caps[ds] if capacity else 0)
        M.render_backward(ctx, fr, dls[ds], stream=st)
        if prof:
            us = fr.stats()["stage_us"]  # waits for this frame's stream
            for s in STAGES:
                stage_acc[ds][s] += us[STAGE_IDX[s]]
        fr.release()

    def frame(ds, capacity=False):
        st = streams[ds]
        with torch.cuda.stream(st):
            run_frame(ds, st, capacity=capacity)

    def eager_step(prof=False, capacity=False):
        if args.serial or prof:
            for ds in DOWNSCALES:
                run_frame(ds, prof=prof)
            return
        for f in [pool.submit(frame, ds, capacity) for ds in DOWNSCALES]:
            f.result()

    graphs = {}

    def step(prof=False):
        if prof or not graphs:
            eager_step(prof=prof)
            return
        # one host thread replays the four frames' graphs, each on its stream
        cur = torch.cuda.current_stream()
        for ds in DOWNSCALES:
            streams[ds].wait_stream(cur)
            with torch.cuda.stream(streams[ds]):
                graphs[ds].replay()

    # counts of one step (deterministic)
    stats = {}
    dpasses = {}
    for ds in DOWNSCALES:
        _, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, profile=True)
        M.render_backward(ctx, fr, dls[ds])
        stats[ds] = fr.stats()
        dpasses[ds] = depth_sort_passes(fr)
        fr.release()
    blends_per_step = sum(stats[ds]["n_blends"] for ds in DOWNSCALES)
    for ds in DOWNSCALES:
        caps[ds] = int(stats[ds]["n_instances"] * 1.25) + 4096

    if args.traffic_probe:
        # the counters of this run give the HBM bytes of every kernel of one
        # step; the elementwise product below moves exactly 1 GiB in and 1 GiB
        # out and calibrates FETCH_SIZE / WRITE_SIZE
        args.serial = True
        step()
        torch.cuda.synchronize()
        x = torch.ones(1 << 28, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        print("bench: traffic probe done", file=sys.stderr, flush=True)
        return

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    def timed():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3

    print("bench: timed eager steps", file=sys.stderr, flush=True)
    ms_eager = timed()
    graph_frames = {}
    fwd_graphs = {}
    ms_fwd = None
    if not (args.eager or args.serial):
        # capture: one graph per frame (forward + backward) on the frame's
        # stream, each right after an eager capacity-mode frame on that stream,
        # whose freed blocks the captured frame then takes from the library's
        # block cache
        print("bench: capturing one graph per frame", file=sys.stderr, flush=True)
        for _ in range(2):
            eager_step(capacity=True)
        torch.cuda.synchronize()
        for ds in DOWNSCALES:
            with torch.cuda.stream(streams[ds]):
                run_frame(ds, streams[ds], capacity=True)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=streams[ds]):
                _, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, stream=streams[ds],
                                 capacity=caps[ds])
                gr = M.render_backward(ctx, fr, dls[ds], stream=streams[ds])
            graphs[ds] = g
            graph_frames[ds] = (fr, gr)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        for ds in DOWNSCALES:
            # a replayed frame did the counted work (and did not overflow)
            gs = graph_frames[ds][0].stats()
            for k in ("n_selected", "n_instances", "n_blends", "n_visits"):
                assert gs[k] == stats[ds][k], (ds, k, gs[k], stats[ds][k])
        print("bench: timed graph replays", file=sys.stderr, flush=True)
        ms_per_step = timed()
        # the same four frames forward only (the rendering workload as stated,
        # without the adjoint the headline step adds), one captured graph per
        # frame, replayed the same way
        print("bench: forward-only graph replays", file=sys.stderr, flush=True)
        for ds in DOWNSCALES:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=streams[ds]):
                _, fr = M.render(ctx, dsc, cam, downscale=ds, keep_frame=True, stream=streams[ds],
                                 capacity=caps[ds])
            fwd_graphs[ds] = (g, fr)

        def fwd_step():
            cur = torch.cuda.current_stream()
            for ds in DOWNSCALES:
                streams[ds].wait_stream(cur)
                with torch.cuda.stream(streams[ds]):
                    fwd_graphs[ds][0].replay()

        for _ in range(args.warmup):
            fwd_step()
        torch.cuda.synchronize()
        for ds in DOWNSCALES:
            gs = fwd_graphs[ds][1].stats()
            for k in ("n_selected", "n_instances", "n_blends", "n_visits"):
                assert gs[k] == stats[ds][k], (ds, k, gs[k], stats[ds][k])
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fwd_step()
        torch.cuda.synchronize()
        ms_fwd = (time.perf_counter() - t0) / args.steps * 1e3
    else:
        ms_per_step = ms_eager
    pool.shutdown()
    # kernel timing: the same steps with the frames one after another, so that
    # a kernel's launch time is its own and not shared with another frame's
    print("bench: kernel-timing steps", file=sys.stderr, flush=True)
    for _ in range(args.steps):
        step(prof=True)
    torch.cuda.synchronize()

    per_ds_stage = {ds: {s: v / args.steps for s, v in stage_acc[ds].items()} for ds in DOWNSCALES}
    stage_tot = {s: sum(per_ds_stage[ds][s] for ds in DOWNSCALES) for s in STAGES}
    dominant = max(STAGES, key=lambda s: stage_tot[s])
    print("bench: stage us per step " + json.dumps({k: round(v, 1) for k, v in stage_tot.items()}),
          file=sys.stderr, flush=True)

    # algorithmic work of every stage at every downscale
    def stage_work(ds):
        st = stats[ds]
        bits = max(1, int(np.ceil(np.log2(max(2, st["tiles_x"] * st["tiles_y"])))))
        b = stage_bytes(st, sc.n, sc.sh_degree, dpasses[ds], (bits + 7) // 8)
        b["blend"] = FLOPS_PER_VISIT * st["n_visits"] + FLOPS_PER_BLEND * st["n_blends"]
        b["blend_bwd"] = (FLOPS_PER_VISIT * st["n_visits"] +
                          FLOPS_PER_BLEND_BWD * st["n_blends"])
        return b

    work = {ds: stage_work(ds) for ds in DOWNSCALES}
    # roofline of the dominant kernel over all its launches of a step: total
    # algorithmic work / total launch time (= per-launch average over the four
    # frames, the figure a kernel-trace summary of the same run reports)
    tot_us = stage_tot[dominant]
    tot_work = sum(work[ds][dominant] for ds in DOWNSCALES)
    launches = len(DOWNSCALES)
    alu = dominant in ("blend", "blend_bwd")
    kname = {"blend": "k_blend", "blend_bwd": "k_blend_bwd"}.get(dominant, dominant)
    if alu:
        achieved = tot_work / (tot_us * 1e-6) / 1e12
        per = (f"fwd: {FLOPS_PER_VISIT} flops/visit + {FLOPS_PER_BLEND} flops/blend" if dominant == "blend"
               else f"bwd: {FLOPS_PER_VISIT} flops/visit + {FLOPS_PER_BLEND_BWD} flops/blend")
        roof = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / ALU_PEAK_TFLOPS}
    else:
        achieved = tot_work / (tot_us * 1e-6) / 1e9
        per = "bytes as listed in stage_bytes()"
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    roof.update({
        "kernel": kname, "launches_per_step": launches,
        "avg_launch_us": tot_us / launches,
        "algorithmic_per_launch": tot_work / launches,
        "algorithmic": per + "; visits/blends per launch averaged over the 1x, 4x, 16x, 64x frames",
        "frac_1x_launch": ((work[1][dominant] / (per_ds_stage[1][dominant] * 1e-6)) /
                           ((ALU_PEAK_TFLOPS * 1e12) if alu else (HBM_PEAK_GBS * 1e9))),
        "frac_by_downscale": {
            str(ds): round((work[ds][dominant] / (per_ds_stage[ds][dominant] * 1e-6)) /
                           ((ALU_PEAK_TFLOPS * 1e12) if alu else (HBM_PEAK_GBS * 1e9)), 4)
            for ds in DOWNSCALES if per_ds_stage[ds][dominant] > 0},
        "launch_us_by_downscale": {str(ds): round(per_ds_stage[ds][dominant], 2)
                                   for ds in DOWNSCALES},
        "measured": "HIP events on the frame's stream around each stage, averaged over "
                    f"{args.steps} steps run frame after frame after the timed region",
        "traffic": traffic_for(kname, "avg")})
    # HBM-bound stages: achieved algorithmic bandwidth per downscale
    hbm_stages = {}
    for s in ("project", "depth_sort", "count_scan", "emit", "tile_sort", "ranges", "zero_bwd",
              "chain_bwd"):
        hbm_stages[s] = {}
        for ds in DOWNSCALES:
            us = per_ds_stage[ds][s]
            gbs = work[ds][s] / (us * 1e-6) / 1e9 if us > 0 else 0.0
            hbm_stages[s][str(ds)] = {"us": round(us, 2), "bytes": int(work[ds][s]),
                                      "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}

    # per-downscale frame rate and latency, selective vs single-scale (forward)
    per_ds = {}
    for ds in DOWNSCALES:
        per_ds[str(ds)] = {}
        for sel in (True, False):
            for _ in range(2):
                M.render(ctx, dsc, cam, downscale=ds, selective=sel)
            torch.cuda.synchronize()
            lat = []
            for _ in range(args.latency_reps):
                t = time.perf_counter()
                M.render(ctx, dsc, cam, downscale=ds, selective=sel)
                torch.cuda.synchronize()
                lat.append((time.perf_counter() - t) * 1e3)
            _, fr = M.render(ctx, dsc, cam, downscale=ds, selective=sel, keep_frame=True,
                             profile=True)
            s = fr.stats()
            fr.release()
            lat = np.array(lat)
            per_ds[str(ds)]["selective" if sel else "single_scale"] = {
                "fps": float(1e3 / lat.mean()), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "device_ms": s["stage_us"][9] / 1e3,
                "blends": s["n_blends"], "instances": s["n_instances"],
                "selected": s["n_selected"], "blends_per_s": float(s["n_blends"] / lat.mean() * 1e3)}

    out = {
        "metric": "Gaussian-pixel blends/s",
        "value": blends_per_step / (ms_per_step / 1e3),
        "unit": "blends/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4-level scene, 531,250 Gaussians (400k/4^l per level, SH degree 3), "
                               "1600x1064 at 1x/4x/16x/64x, selective rendering, forward + backward "
                               "per downscale",
                   "n_gaussians": sc.n, "frames_per_step": len(DOWNSCALES),
                   "frames_in_flight": 1 if args.serial else len(DOWNSCALES),
                   "blends_per_step": blends_per_step,
                   "execution": ("eager, frames one after another on one stream" if args.serial
                                 else "eager, one host thread and stream per frame, exact tile "
                                      "lists" if (args.eager or not graphs)
                                 else "one captured HIP graph per frame (forward + backward, "
                                      "tile-list capacity 1.25x the counted instances + 4096), "
                                      "the four replayed on four streams")},
        "ms_per_step_eager": ms_eager,
        "roofline": roof,
        "stage_us_per_step": {s: round(v, 2) for s, v in stage_tot.items()},
        "stage_us_by_downscale": {str(ds): {s: round(v, 2) for s, v in per_ds_stage[ds].items()}
                                  for ds in DOWNSCALES},
        "depth_sort_passes": {str(ds): dpasses[ds] for ds in DOWNSCALES},
        "hbm_stages": hbm_stages,
        "per_downscale": per_ds,
        "prefilter": prefilter_effect(M, ctx, dsc, cam),
    }
    if ms_fwd is not None:
        out["forward_only"] = {
            "ms_per_step": ms_fwd, "blends_per_s": blends_per_step / (ms_fwd / 1e3),
            "execution": "the same four frames, forward only, one captured HIP graph per frame "
                         "replayed on four streams"}
    if not args.no_serving:
        print("bench: serving replay (3M-Gaussian scene, 512 requests at 200/s)", file=sys.stderr,
              flush=True)
        out["serving"] = {"selective": serving_replay(M, G, selective=True),
                          "single_scale": serving_replay(M, G, selective=False),
                          "saturation": serving_sweep(M, G)}
    if not args.no_other_configs:
        print("bench: 10k-Gaussian 128x128 and 3M-Gaussian 1080p frames", file=sys.stderr,
              flush=True)
        out["other_configs"] = other_configs(M, G)
    if not args.no_training:
        print("bench: training step (6M Gaussians, 8 views)", file=sys.stderr, flush=True)
        out["training_step"] = training_step(M, G)
    if not args.no_aggregation:
        print("bench: aggregation (Alg. 1, 2.26M level-0 Gaussians, 8 cameras)", file=sys.stderr,
              flush=True)
        out["aggregation"] = aggregation_bench(M, G)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline"]["cpu"] = cpu_info()
        out["cpu_baseline"].update(cpu_baseline_extra())
    print(json.dumps(out), flush=True)
    graphs.clear()
    fwd_frames = [fr for _, fr in fwd_graphs.values()]
    fwd_graphs.clear()
    torch.cuda.synchronize()
    for fr, _ in graph_frames.values():
        fr.release()
    for fr in fwd_frames:
        fr.release()
    dsc.close()
    del stream


if __name__ == "__main__":
    main()
