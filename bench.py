#!/usr/bin/env python
"""Benchmark of the batched randomized renderer on one MI355X.

Workload: 256 articulated hand-like scenes (25 capsule links of 512 triangles on a
24-hinge tree plus a 768-triangle cube, 13,568 triangles per scene) x 3 jittered
cameras = 768 frames at 200x200, each frame written as fp32 RGB, fp32 depth, fp32
view-space normal and int32 segmentation (32 B per pixel).  Synthetic, seeded inputs
stand in for the paper's Shadow-hand benchmark scene (which is not available).

A step is one orrb_render_batch over the whole batch (vertex stage, binning, raster,
shading, channel writes) with every input already resident in device memory.  The
line printed reports whole-job frames per second, the raster kernel's achieved write
bandwidth against the 8 TB/s HBM peak, the plain one-scene-per-launch form, and the
FP64 CPU oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_PIXEL = 32  # rgb 12 + depth 4 + normal 12 + seg 4
METRIC = "randomized 4-channel 200x200 frames/sec on 1 MI355X; shading-grad/sec; p99 ms"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_frame_traffic.json")
# the frame kernel's source: its file and the headers it includes
PROFILE_EVERY = 10  # timed region: the kernel of every 10th step bracketed by HIP events

KERNEL_SRCS = [os.path.join(ROOT, "paper_1906_11633_amd", "csrc", f)
               for f in ("orrb_kernels.hip", "orrb_primitives.h", "orrb_device.h", "orrb_post.h")]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per raster launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source (else None)."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_sha") != kernel_source_sha():
        return None
    return d.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch_fn, n_scenes_total: int, target_s: float, threads: int):
    """Time the FP64 oracle on the workload (its first scenes if the whole batch would
    take longer than target_s), repeating it until about target_s of work, and scale
    to frames per second."""
    import oracle
    oracle.build()
    probe = batch_fn(2)
    t0 = time.perf_counter()
    oracle.render(probe, threads=threads)
    per_scene = (time.perf_counter() - t0) / 2
    n = max(2, min(n_scenes_total, int(target_s / max(per_scene, 1e-6))))
    b = batch_fn(n)
    reps, frames = 0, 0
    t0 = time.perf_counter()
    while True:
        oracle.render(b, threads=threads)
        reps += 1
        frames += b.n_frames
        dt = time.perf_counter() - t0
        if dt >= target_s or reps >= 1000:
            break
    what = "the whole workload" if n == n_scenes_total else f"the first {n} of {n_scenes_total} scenes"
    return dict(value=frames / dt, unit="frames/s", cores=threads, kind="oracle",
                sample=f"{what} ({n} scenes, {b.n_frames} frames) rendered {reps}x by the FP64 oracle "
                       f"(OpenMP over frames, {threads} threads) in {dt:.1f} s")


def _timed(fn, reps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _event_times(fn, reps, torch, stream=None):
    """Per-call device durations (ms) from HIP events recorded on `stream` (default:
    torch's current stream, the one the library's calls are enqueued on)."""
    st = stream if stream is not None else torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(st)
        fn()
        e1.record(st)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def _pct(xs, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(xs), q)), 4)


def measure_aux(args, r, S, batch, job, torch, frame_ms_plain):
    """The same workload with every output on: the four channels, the transparency
    channel, the Tracker records and the post-processed 3 x 8-bit RGB (colour grading
    and grain randomized per frame), all written by the frame kernel: 36 B per pixel
    plus 3 B of 8-bit RGB (39 B), the Tracker records on top."""
    import ctypes as C
    from paper_1906_11633_amd import _lib
    post, grain = S.postprocess_params(2, batch.n_frames, batch.frame_scene)
    job.state["post"] = torch.from_numpy(post).cuda()
    job.state["grain"] = torch.from_numpy(grain).cuda()
    out = r.alloc_outputs(job, alpha=True, rgb8=True, track=True)
    lib, ctx = r.ctx.lib, r.ctx.handle
    for _ in range(3):
        r.render(job, out)
    torch.cuda.synchronize()
    n = max(10, args.steps // 4)
    _lib.check(lib.orrb_profile_enable(ctx, 1))
    dt = _timed(lambda: r.render(job, out), n, torch)
    kt = _lib.KernelTimes()
    _lib.check(lib.orrb_profile_read(ctx, C.byref(kt)))
    _lib.check(lib.orrb_profile_enable(ctx, 0))
    del job.state["post"], job.state["grain"]
    frame_ms = kt.frame_ms / max(kt.frame_launches, 1)
    fbytes = 39 * batch.total_pixels
    return dict(ms_per_step=round(dt * 1e3, 4), frames_per_s=round(batch.n_frames / dt, 1),
                k_frame_ms=round(frame_ms, 4), k_frame_ms_without=round(frame_ms_plain, 4),
                k_frame_overhead=round(frame_ms / frame_ms_plain - 1, 4) if frame_ms_plain else None,
                roofline=dict(bound="hbm", bytes_per_launch=fbytes, achieved=round(fbytes / (frame_ms * 1e-3) / 1e9, 1),
                              peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(fbytes / (frame_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))


def measure_rgb8_only(args, r, S, batch, job, torch):
    """The paper's benchmark format (Sec. 5: 200 x 200 images in 3 x 8-bit RGB): only the
    graded, grained, sRGB-encoded 8-bit planes are written, encoded by the frame kernel
    as it writes each tile (3 B per pixel)."""
    import ctypes as C
    from paper_1906_11633_amd import _lib
    post, grain = S.postprocess_params(2, batch.n_frames, batch.frame_scene)
    job.state["post"] = torch.from_numpy(post).cuda()
    job.state["grain"] = torch.from_numpy(grain).cuda()
    out = r.alloc_outputs(job, rgb8=True, base=())
    lib, ctx = r.ctx.lib, r.ctx.handle
    for _ in range(3):
        r.render(job, out)
    torch.cuda.synchronize()
    n = max(10, args.steps // 4)
    _lib.check(lib.orrb_profile_enable(ctx, 1))
    dt = _timed(lambda: r.render(job, out), n, torch)
    kt = _lib.KernelTimes()
    _lib.check(lib.orrb_profile_read(ctx, C.byref(kt)))
    _lib.check(lib.orrb_profile_enable(ctx, 0))
    del job.state["post"], job.state["grain"]
    frame_ms = kt.frame_ms / max(kt.frame_launches, 1)
    fbytes = 3 * batch.total_pixels
    return dict(ms_per_step=round(dt * 1e3, 4), frames_per_s=round(batch.n_frames / dt, 1),
                k_frame_ms=round(frame_ms, 4),
                roofline=dict(bound="hbm", bytes_per_launch=fbytes,
                              achieved=round(fbytes / (frame_ms * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=round(fbytes / (frame_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))


def measure_shadows(args, r, S, torch):
    """The workload lit like the paper's benchmark scene: three shadow-casting spot
    lights per scene (LightSetup placement, randomized angles), 128 x 128 shadow maps
    rendered by the same kernels (depth only) before the frames, 3 x 3 filtered."""
    b = S.with_spot_lights(S.config2(2, args.scenes, args.res), seed=2)
    job = r.prepare(b)
    out = r.alloc_outputs(job)
    for _ in range(3):
        r.render(job, out)
    n = max(10, args.steps // 4)
    dt = _timed(lambda: r.render(job, out), n, torch)
    ev = _event_times(lambda: r.render(job, out), n, torch)
    return dict(frames=b.n_frames, shadow_maps=int((b.light_type == 2).sum()), shadow_res=int(b.shadow_res),
                ms_per_step=round(dt * 1e3, 4), frames_per_s=round(b.n_frames / dt, 1),
                event_ms_median=_pct(ev, 50), event_ms_p90=_pct(ev, 90))


def measure_materials(args, r, S, torch):
    """The workload with randomized materials: pattern textures with random tiling and
    offset on about 70% of the objects, the block drawn by the fixed-hue sampler,
    sometimes emissive."""
    b = S.with_materials(S.config2(2, args.scenes, args.res), seed=2)
    job = r.prepare(b)
    out = r.alloc_outputs(job)
    for _ in range(3):
        r.render(job, out)
    n = max(10, args.steps // 4)
    dt = _timed(lambda: r.render(job, out), n, torch)
    return dict(frames=b.n_frames, textured_objects=int((b.object_texture >= 0).sum()),
                textures=len(b.textures), ms_per_step=round(dt * 1e3, 4), frames_per_s=round(b.n_frames / dt, 1))


def measure_grad(args, r, S):
    """Shading-gradient throughput: 64 scenes x 3 cameras at 200x200."""
    import torch
    from paper_1906_11633_amd.renderer import shade_backward
    ex = {}
    base, target = S.config4(4, 64, 200)
    job = r.prepare(base)
    out = r.render(job, vis=True)
    tgt = r.render(r.prepare(target))["rgb"]  # the target image, rendered by the same kernels
    grad_rgb = (2.0 * (out["rgb"] - tgt)).contiguous()
    ws = torch.empty(int(job.layout.info.grad_workspace_bytes), dtype=torch.uint8, device="cuda")
    step = lambda: shade_backward(r.ctx, job.layout, job.state, out["vis"], grad_rgb, ws)
    step()
    dt = _timed(step, 10, torch)
    ev = _event_times(step, 20, torch)
    # algorithmic bytes: the visibility key (8 B) and dL/drgb (12 B) of every pixel
    gbytes = 20 * base.total_pixels
    gms = sorted(ev)[len(ev) // 2]
    ex["shading_grad"] = dict(frames=base.n_frames, ms_per_backward=round(dt * 1e3, 3),
                              grad_frames_per_s=round(base.n_frames / dt, 1),
                              event_ms_median=_pct(ev, 50), event_ms_p90=_pct(ev, 90),
                              roofline=dict(bound="hbm", kernel="backward (vertex + k_grad_tile + k_grad_reduce)",
                                            bytes_per_call=gbytes, achieved=round(gbytes / (gms * 1e-3) / 1e9, 1),
                                            peak=HBM_PEAK_GBS, unit="GB/s",
                                            frac=round(gbytes / (gms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))
    print(f"[bench] backward {dt * 1e3:.3f} ms for {base.n_frames} frames", file=sys.stderr, flush=True)
    return ex


def measure_serving(args, r, S):
    """The serving loop: Poisson 2000 req/s of 1-32 scenes at 64/128/200 px."""
    from paper_1906_11633_amd.serving import ScenePool, Server, poisson_trace
    ex = {}
    pool = ScenePool(r.ctx, 256)
    warm = Server(r.ctx, pool)
    warm.run(poisson_trace(pool, 2000.0, 0.3, seed=99))
    srv = Server(r.ctx, pool)
    srv.layouts, srv.table_bytes = warm.layouts, warm.table_bytes
    # config 5: Poisson arrivals at 2000 req/s, statistics over the requests arriving
    # in the args.serving_seconds after a 1 s warm-up
    st = srv.run(poisson_trace(pool, 2000.0, args.serving_seconds, 1.0), warmup=1.0)
    assert st["wait_timeouts"] == 0, st
    ex["serving"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    ex["serving"].update(rate_req_per_s=2000.0, budget_gb=64, warmup_s=1.0, measured_s=args.serving_seconds)
    print(f"[bench] serving p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms", file=sys.stderr, flush=True)
    return ex


def _uneven_plain(r, b3, job3, out3):
    """Seconds per pass of the uneven batch rendered one scene (3 frames) per launch."""
    import torch
    from paper_1906_11633_amd.renderer import Layout, render_batch
    plain = []
    st3 = job3.state
    po = b3.pixel_offset
    for s in range(b3.n_scenes):
        ob, oe = int(b3.scene_object_begin[s]), int(b3.scene_object_begin[s + 1])
        lb, le = int(b3.scene_light_begin[s]), int(b3.scene_light_begin[s + 1])
        f0, f1 = 3 * s, 3 * s + 3
        sst = dict(object_pose=st3["object_pose"][ob:oe], object_seg=st3["object_seg"][ob:oe],
                   object_visible=st3["object_visible"][ob:oe], albedo=st3["albedo"][ob:oe],
                   roughness=st3["roughness"][ob:oe], specular=st3["specular"][ob:oe],
                   light_vec=st3["light_vec"][lb:le], light_intensity=st3["light_intensity"][lb:le],
                   view=st3["view"][f0:f1], intr=st3["intr"][f0:f1], near=st3["near"][f0:f1],
                   exposure=st3["exposure"][f0:f1])
        p0, p1 = int(po[f0]), int(po[f1])
        sout = dict(rgb=out3["rgb"][3 * p0:3 * p1], depth=out3["depth"][p0:p1], normal=out3["normal"][3 * p0:3 * p1],
                    seg=out3["seg"][p0:p1])
        plain.append((Layout(r.ctx, b3.select_scenes([s])), sst, sout))
    run_plain = lambda: [render_batch(r.ctx, lay, sst, sout, job3.workspace) for lay, sst, sout in plain]
    run_plain()
    return _timed(run_plain, 3, torch)


def measure_uneven(args, r, S):
    """The uneven batch (1024 scenes, 64-256 px, 2k-50k triangles) autotuned and
    replayed from a HIP graph, against its one-scene-per-launch form (unless
    --no-plain)."""
    import torch
    from paper_1906_11633_amd.renderer import Graph, Layout, autotune, render_batch
    ex = {}
    b3 = S.config3(3, 1024)
    job3 = r.prepare(b3)
    out3 = r.alloc_outputs(job3)
    tuning, _ = autotune(r.ctx, job3.layout, job3.state, out3, job3.workspace)
    inf3 = job3.layout.info
    g_nodes = int(inf3.render_kernels)  # kernel nodes of the captured graph
    stream = torch.cuda.Stream()
    g = Graph(r.ctx, job3.layout, job3.state, out3, job3.workspace, stream)
    with torch.cuda.stream(stream):
        for _ in range(3):
            g.replay(stream)
        dt3 = _timed(lambda: g.replay(stream), 20, torch)
        ev3 = _event_times(lambda: g.replay(stream), 20, torch, stream)
    g.close()
    bytes3 = BYTES_PER_PIXEL * b3.total_pixels
    ms3 = sorted(ev3)[len(ev3) // 2]
    dtp = None if args.no_plain else _uneven_plain(r, b3, job3, out3)
    ex["uneven_batch"] = dict(frames=b3.n_frames, pixels=b3.total_pixels, tuning=list(tuning),
                              ms_per_step=round(dt3 * 1e3, 3), frames_per_s=round(b3.n_frames / dt3, 1),
                              hbm_frac=round(bytes3 / dt3 / 1e9 / HBM_PEAK_GBS, 4),
                              plain_frames_per_s=round(b3.n_frames / dtp, 1) if dtp else None,
                              batched_over_plain=round(dtp / dt3, 2) if dtp else None,
                              graph_kernel_nodes=g_nodes, event_ms_median=_pct(ev3, 50), event_ms_p90=_pct(ev3, 90),
                              roofline=dict(bound="hbm", kernel="graph replay", bytes_per_call=bytes3,
                                            achieved=round(bytes3 / (ms3 * 1e-3) / 1e9, 1), peak=HBM_PEAK_GBS,
                                            unit="GB/s", frac=round(bytes3 / (ms3 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))
    print(f"[bench] uneven batch {dt3 * 1e3:.3f} ms/step (graph)" + (f", plain {dtp * 1e3:.3f} ms" if dtp else ""),
          file=sys.stderr, flush=True)
    return ex


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--scenes", type=int, default=256)
    ap.add_argument("--res", type=int, default=200)
    ap.add_argument("--tile", type=str, default="", help="tile_w,tile_h,bin_cap,persistent,path")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the gradient, serving and uneven-batch parts")
    ap.add_argument("--serving-seconds", type=float, default=10.0)
    ap.add_argument("--only", choices=["grad", "serving", "uneven", "aux", "materials", "shadows"],
                    help="run only this part and print its JSON (for profiling one kernel's workload)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this many MiB 5 times (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported in this build "
              "(frames shard by scene across GPUs with no exchange; see the design notes).", file=sys.stderr)
        return 2

    import torch
    from paper_1906_11633_amd import scenes as S
    from paper_1906_11633_amd import _lib
    from paper_1906_11633_amd.renderer import Renderer, Layout, render_batch
    import ctypes as C

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "launches": 5}), flush=True)
        return 0
    if args.only in ("grad", "serving", "uneven", "materials", "shadows"):
        part = dict(grad=measure_grad, serving=measure_serving, uneven=measure_uneven,
                    materials=lambda a, r, S: dict(materials=measure_materials(a, r, S, torch)),
                    shadows=lambda a, r, S: dict(spot_shadows=measure_shadows(a, r, S, torch)))[args.only]
        print(json.dumps(part(args, Renderer(0), S)), flush=True)
        return 0
    t_gen = time.perf_counter()
    batch = S.config2(2, args.scenes, args.res)
    print(f"[bench] generated {batch.n_frames} frames in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    r = Renderer(0)
    job = r.prepare(batch)
    if args.tile:
        job.layout.set_tuning(*(int(x) for x in args.tile.split(",")))
    out = r.alloc_outputs(job)
    lib, ctx = r.ctx.lib, r.ctx.handle
    F = batch.n_frames
    pixels = batch.total_pixels

    for _ in range(args.warmup):
        r.render(job, out)
    torch.cuda.synchronize()
    _lib.check(lib.orrb_profile_enable(ctx, PROFILE_EVERY))  # one timed launch in PROFILE_EVERY
    stats = torch.zeros(_lib.STATS_WORDS, dtype=torch.int32, device="cuda")
    out["stats"] = stats
    cur = torch.cuda.current_stream()
    # the timed region: K steps, with only the library's events around the kernel of one
    # step in PROFILE_EVERY (its mean duration for the roofline); events on every step
    # would add their own cost to each, so the step-time distribution is taken in a
    # separate pass below
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.render(job, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    del out["stats"]
    from paper_1906_11633_amd.renderer import read_stats
    counters = read_stats(stats)
    if counters["wait_timeouts"]:
        raise SystemExit(f"frame-kernel waits reached their bound: {counters}")
    kt = _lib.KernelTimes()
    _lib.check(lib.orrb_profile_read(ctx, C.byref(kt)))
    _lib.check(lib.orrb_profile_enable(ctx, 0))
    # step-time distribution (median / p90) from per-step HIP events, outside the timed region
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in step_ev:
        e0.record(cur)
        r.render(job, out)
        e1.record(cur)
    torch.cuda.synchronize()
    step_ms = [e0.elapsed_time(e1) for e0, e1 in step_ev]
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = F * args.steps / elapsed
    avg = lambda ms, n: ms / n if n else 0.0
    kernel_ms = dict(k_vertex=avg(kt.vertex_ms, kt.vertex_launches), k_raster_shade=avg(kt.raster_ms, kt.raster_launches),
                     k_frame=avg(kt.frame_ms, kt.frame_launches))
    # the dominant kernel writes every pixel of the frames it renders
    info = job.layout.info
    frame_pixels = sum(int(batch.width[f]) * int(batch.height[f]) for f in range(F)) if info.frame_path_frames == F else None
    if kernel_ms["k_frame"] >= kernel_ms["k_raster_shade"] and info.frame_path_frames == F:
        dom, dom_ms, dom_pixels = "k_frame", kernel_ms["k_frame"], frame_pixels
    else:
        dom, dom_ms, dom_pixels = "k_raster_shade", kernel_ms["k_raster_shade"], pixels if info.frame_path_frames == 0 else None
    if dom_pixels is None:
        raise SystemExit("bench.py expects every frame of the workload on one path")
    bytes_per_launch = BYTES_PER_PIXEL * dom_pixels
    achieved = bytes_per_launch / (dom_ms * 1e-3) / 1e9
    print(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, " +
          ", ".join(f"{k} {v:.3f} ms" for k, v in kernel_ms.items() if v), file=sys.stderr, flush=True)

    extra = dict(kernel_ms={k: round(v, 4) for k, v in kernel_ms.items() if v},
                 step_event_ms_median=_pct(step_ms, 50), step_event_ms_p90=_pct(step_ms, 90),
                 counters=counters,
                 tuning=list(job.layout.info.tuning.as_tuple()),
                 whole_step_hbm_frac=round(bytes_per_launch / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))

    # store-only ceiling: the same output buffers (same bytes, planar layout) filled by
    # the runtime's fill kernels, no rendering
    def fill_all():
        for k in ("rgb", "depth", "normal", "seg"):
            out[k].zero_()
    fill_all()
    fev = _event_times(fill_all, 20, torch)
    fms = sorted(fev)[len(fev) // 2]
    extra["store_ceiling_gbs"] = round(bytes_per_launch / (fms * 1e-3) / 1e9, 1)
    extra["store_ceiling_frac"] = round(bytes_per_launch / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    extra["aux_outputs"] = measure_aux(args, r, S, batch, job, torch, kernel_ms["k_frame"])
    extra["rgb8_only"] = measure_rgb8_only(args, r, S, batch, job, torch)
    print(f"[bench] rgb8 only (paper format): {extra['rgb8_only']['ms_per_step']:.3f} ms/step, "
          f"k_frame {extra['rgb8_only']['k_frame_ms']:.3f} ms", file=sys.stderr, flush=True)
    if args.only == "aux":
        print(json.dumps(dict(aux_outputs=extra["aux_outputs"], rgb8_only=extra["rgb8_only"])), flush=True)
        return 0
    print(f"[bench] with alpha, tracker and rgb8: {extra['aux_outputs']['ms_per_step']:.3f} ms/step, "
          f"k_frame {extra['aux_outputs']['k_frame_ms']:.3f} ms", file=sys.stderr, flush=True)
    extra["materials"] = measure_materials(args, r, S, torch)
    print(f"[bench] textured materials: {extra['materials']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    extra["spot_shadows"] = measure_shadows(args, r, S, torch)
    print(f"[bench] three shadow-casting spot lights: {extra['spot_shadows']['ms_per_step']:.3f} ms/step",
          file=sys.stderr, flush=True)
    for _ in range(2):
        r.render(job, out)  # the outputs hold the render again

    # with upload: the per-batch state (poses, materials, lights, cameras) copied from
    # pinned host memory before each render, on the same stream
    host = {k: v.cpu().pin_memory() for k, v in job.state.items()}
    state_bytes = sum(v.numel() * v.element_size() for v in host.values())

    def upload_and_render():
        for k, v in host.items():
            job.state[k].copy_(v, non_blocking=True)
        r.render(job, out)
    upload_and_render()
    dtu = _timed(upload_and_render, max(5, args.steps // 4), torch)
    extra["with_upload"] = dict(frames_per_s=round(F / dtu, 1), ms_per_step=round(dtu * 1e3, 4),
                                state_bytes=state_bytes)

    if not args.no_plain:
        # the plain form: the same kernels, one scene (3 frames) per launch, no graph
        ws = job.workspace
        lays = []
        st = job.state
        for s in range(batch.n_scenes):
            sub = batch.select_scenes([s])
            lay = Layout(r.ctx, sub)
            ob, oe = int(batch.scene_object_begin[s]), int(batch.scene_object_begin[s + 1])
            lb, le = int(batch.scene_light_begin[s]), int(batch.scene_light_begin[s + 1])
            fr = [int(f) for f in range(F) if batch.frame_scene[f] == s]
            f0, f1 = fr[0], fr[-1] + 1
            po = batch.pixel_offset
            sst = dict(object_pose=st["object_pose"][ob:oe], object_seg=st["object_seg"][ob:oe],
                       object_visible=st["object_visible"][ob:oe], albedo=st["albedo"][ob:oe],
                       roughness=st["roughness"][ob:oe], specular=st["specular"][ob:oe],
                       light_vec=st["light_vec"][lb:le], light_intensity=st["light_intensity"][lb:le],
                       view=st["view"][f0:f1], intr=st["intr"][f0:f1], near=st["near"][f0:f1],
                       exposure=st["exposure"][f0:f1])
            p0, p1 = int(po[f0]), int(po[f1])
            sout = dict(rgb=out["rgb"][3 * p0:3 * p1], depth=out["depth"][p0:p1], normal=out["normal"][3 * p0:3 * p1],
                        seg=out["seg"][p0:p1])
            lays.append((lay, sst, sout))
        plain_steps = max(3, args.steps // 20)
        for _ in range(2):
            for lay, sst, sout in lays:
                render_batch(r.ctx, lay, sst, sout, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            for lay, sst, sout in lays:
                render_batch(r.ctx, lay, sst, sout, ws)
        torch.cuda.synchronize()
        plain_fps = F * plain_steps / (time.perf_counter() - t0)
        extra["plain_form_frames_per_s"] = round(plain_fps, 1)
        extra["batched_over_plain"] = round(value / plain_fps, 2)

    if not args.no_extras:
        for part in (measure_grad, measure_serving, measure_uneven):
            extra.update(part(args, r, S))

    cpu = None
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = cpu_baseline(lambda n: S.config2(2, n, args.res), args.scenes, args.cpu_seconds, threads)
        cpu["value"] = round(cpu["value"], 3)
        one = cpu_baseline(lambda n: S.config2(2, n, args.res), args.scenes, args.cpu_seconds / 3, 1)
        extra["cpu_single_thread"] = dict(value=round(one["value"], 3), unit="frames/s", sample=one["sample"])
        c1 = cpu_baseline(lambda n: S.config1(1, n, 64), 4, 2.0, threads)  # the tiny correctness batch, whole
        extra["cpu_config1"] = dict(value=round(c1["value"], 3), unit="frames/s", cores=threads, sample=c1["sample"])
        extra["cpu_model"] = cpu_model()
        extra["cpu_threads_available"] = os.cpu_count()

    try:
        paper = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_throughput.json")))
        extra["paper_context"] = dict(images_per_s_1gpu=paper["table2_gpu_scaling"]["1"], hardware="1x V100 + 96 vCPU",
                                      output="200x200 RGB8 only, Unity/OpenGL", source=paper["source"])
    except (OSError, ValueError, KeyError):
        pass
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.scenes} hand-like scenes x 3 cameras at {args.res}x{args.res} "
                               f"({F} frames, 13568 triangles/scene, 1-4 point lights), 4 channels fp32 RGB/depth/"
                               "normal + int32 seg",
                   "frames_per_step": F, "pixels_per_step": pixels, "bytes_per_pixel": BYTES_PER_PIXEL},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic()},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
