"""Continuous-batching render server on one GPU.

ORRB serves batch-render requests from RL workers (Sec. 4.1, 4.5) through a pool of
render textures used round-robin with pre-allocated destinations and no GPU/CPU
stalls (Sec. 4.4).  This server is the in-process equivalent on one MI355X:

* scene state stays resident on the device: a pool of scene states (poses,
  materials, lights, cameras) lives in device memory, next to the shared meshes
  (Single Scene Multiple States, Sec. 3); a request names pool scenes and a
  resolution;
* admission by memory: a request is admitted when the device-memory budget (and a
  launch slot) has room for its outputs, its gathered state and the workspace of the
  launch it joins (frames on the tiled path need 16 B per vertex instance); the
  tables of the cached layouts count against the same budget for as long as they are
  cached; otherwise it waits, in arrival order;
* continuous batching: whenever a launch slot is free, every admitted request that
  is waiting is merged into one render launch (one layout, one kernel), while earlier
  launches are still running on other streams, so their work overlaps on the device;
* per request, latency = completion (stream event observed) - arrival, reported as
  p50 / p99 next to the frames/s served; each launch's counters (wait timeouts and
  the like) are read when it completes and summed into the statistics.

The per-pixel arithmetic does not depend on batch composition, so a request's
result is bit-identical alone and in any mix.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import scenes as S
from . import _lib
from .renderer import Context, Layout, render_batch

LIGHTS_PER_SCENE = 4   # lights padded with zero-intensity ones (they add exactly 0)
CAMS_PER_SCENE = 3
BYTES_PER_PIXEL = 32


@dataclass
class Request:
    rid: int
    scene_ids: np.ndarray
    res: int
    arrival: float                     # seconds since the start of the run
    t_admit: Optional[float] = None
    t_launch: Optional[float] = None
    t_done: Optional[float] = None
    result: Optional[Dict[str, torch.Tensor]] = None

    @property
    def n_frames(self) -> int:
        return CAMS_PER_SCENE * int(len(self.scene_ids))

    @property
    def pixels(self) -> int:
        return self.n_frames * self.res * self.res

    @property
    def out_bytes(self) -> int:
        return BYTES_PER_PIXEL * self.pixels


class ScenePool:
    """Device-resident states of `n_scenes` hand-like scenes (config-2 type)."""

    def __init__(self, ctx: Optional[Context], n_scenes: int = 256, seed: int = 5, device: str = "cuda"):
        """With ctx=None (and device="cpu") the pool holds host tensors only: enough to
        exercise the batching logic without a GPU."""
        b = S.config2(seed, n_scenes, 200)
        self.n_scenes = n_scenes
        self.meshes = b.meshes
        self.mesh_ids = [ctx.add_mesh(m) for m in b.meshes] if ctx is not None else list(range(len(b.meshes)))
        self.objs_per_scene = int(b.scene_object_begin[1])
        assert np.all(np.diff(b.scene_object_begin) == self.objs_per_scene)
        self.object_mesh = b.object_mesh[: self.objs_per_scene].copy()
        # lights padded to LIGHTS_PER_SCENE per scene
        lv = np.zeros((n_scenes, LIGHTS_PER_SCENE, 3), np.float32)
        li = np.zeros((n_scenes, LIGHTS_PER_SCENE), np.float32)
        lv[:, :, 2] = 10.0
        for s in range(n_scenes):
            l0, l1 = b.scene_light_begin[s], b.scene_light_begin[s + 1]
            lv[s, : l1 - l0] = b.light_vec[l0:l1]
            li[s, : l1 - l0] = b.light_intensity[l0:l1]
        assert np.all(b.light_type == 0)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(device)
        self.dev = dict(
            object_pose=t(b.object_pose, np.float32), object_seg=t(b.object_seg, np.int32),
            object_visible=t(b.object_visible, np.uint8), albedo=t(b.albedo, np.float32),
            roughness=t(b.roughness, np.float32), specular=t(b.specular, np.float32),
            light_vec=t(lv.reshape(-1, 3), np.float32), light_intensity=t(li.reshape(-1), np.float32),
            view=t(b.view, np.float32), near=t(b.near, np.float32), exposure=t(b.exposure, np.float32))
        self.device = device
        # gathered per-request state: objects (pose 48, seg 4, visible 1, albedo 12, roughness 4, specular 4),
        # lights (position 12, intensity 4), cameras (view 48, intrinsics 16, near 4, exposure 4)
        self.state_bytes_per_scene = (self.objs_per_scene * 73 + LIGHTS_PER_SCENE * 16 + CAMS_PER_SCENE * 72)

    def batch_desc(self, reqs: List[Request]):
        """Host structure (for a layout) and gather indices of a merged batch."""
        sids = np.concatenate([r.scene_ids for r in reqs]).astype(np.int64)
        n = sids.size
        ops = self.objs_per_scene
        desc = dict(
            n_scenes=n,
            scene_object_begin=(np.arange(n + 1) * ops).astype(np.int32),
            object_mesh=np.tile(np.asarray(self.mesh_ids, np.int32)[self.object_mesh], n),
            scene_light_begin=(np.arange(n + 1) * LIGHTS_PER_SCENE).astype(np.int32),
            light_type=np.zeros(n * LIGHTS_PER_SCENE, np.int32),
            frame_scene=np.repeat(np.arange(n), CAMS_PER_SCENE).astype(np.int32),
            width=np.concatenate([np.full(r.n_frames, r.res, np.int32) for r in reqs]),
            height=np.concatenate([np.full(r.n_frames, r.res, np.int32) for r in reqs]))
        obj_idx = (sids[:, None] * ops + np.arange(ops)[None]).reshape(-1)
        light_idx = (sids[:, None] * LIGHTS_PER_SCENE + np.arange(LIGHTS_PER_SCENE)[None]).reshape(-1)
        frame_idx = (sids[:, None] * CAMS_PER_SCENE + np.arange(CAMS_PER_SCENE)[None]).reshape(-1)
        intr = np.concatenate([np.tile(S.intrinsics(r.res, r.res), (r.n_frames, 1)) for r in reqs]).astype(np.float32)
        return desc, obj_idx, light_idx, frame_idx, intr

    def standalone_batch(self, req: Request) -> "S.Batch":
        """The request as a plain generator Batch (for checks that render it alone)."""
        desc, oi, li, fi, intr = self.batch_desc([req])
        cpu = {k: v.cpu().numpy() for k, v in self.dev.items()}
        return S.Batch(meshes=self.meshes, scene_object_begin=desc["scene_object_begin"],
                       object_mesh=np.tile(self.object_mesh, len(req.scene_ids)),
                       scene_light_begin=desc["scene_light_begin"], light_type=desc["light_type"],
                       frame_scene=desc["frame_scene"], width=desc["width"], height=desc["height"],
                       object_pose=cpu["object_pose"][oi], object_seg=cpu["object_seg"][oi],
                       object_visible=cpu["object_visible"][oi], albedo=cpu["albedo"][oi],
                       roughness=cpu["roughness"][oi], specular=cpu["specular"][oi],
                       light_vec=cpu["light_vec"][li], light_intensity=cpu["light_intensity"][li],
                       view=cpu["view"][fi], intr=intr, near=cpu["near"][fi], exposure=cpu["exposure"][fi],
                       name=f"request{req.rid}")


class _LayoutDesc:
    """Adapter: a layout description in the attribute form Layout() expects."""

    def __init__(self, desc, meshes, object_mesh_local):
        self.meshes = meshes
        self.scene_object_begin = desc["scene_object_begin"]
        self.object_mesh = object_mesh_local
        self.scene_light_begin = desc["scene_light_begin"]
        self.light_type = desc["light_type"]
        self.frame_scene = desc["frame_scene"]
        self.width = desc["width"]
        self.height = desc["height"]


@dataclass
class _Launch:
    reqs: List[Request]
    event: torch.cuda.Event
    stream: torch.cuda.Stream
    bytes: int
    stats: Optional[torch.Tensor] = None
    keep: list = field(default_factory=list)


class Server:
    """Continuous-batching renderer over a resident ScenePool."""

    def __init__(self, ctx: Context, pool: ScenePool, budget_bytes: int = 64 << 30, n_streams: int = 4,
                 max_batch_frames: int = 1536, max_inflight: int = 8, keep_results: bool = False,
                 layout_cache: int = 256, tuning=None):
        """`tuning` (tile_w, tile_h, bin_cap, persistent, path) is set on every layout
        the server builds (None: the default, frame path where scenes fit)."""
        self.ctx, self.pool = ctx, pool
        self.budget = int(budget_bytes)
        self.used = 0          # outputs, state and workspace of launches in flight
        self.table_bytes = 0   # device tables of the cached layouts
        self.tuning = tuning
        self.counters = {k: 0 for k in _lib.STAT_NAMES}
        self.streams = [torch.cuda.Stream(device=pool.device) for _ in range(n_streams)]
        self.next_stream = 0
        self.max_batch_frames = max_batch_frames
        self.max_inflight = max_inflight
        self.keep_results = keep_results
        self.queue: collections.deque = collections.deque()
        self.inflight: List[_Launch] = []
        self.done: List[Request] = []
        self.layouts: "collections.OrderedDict" = collections.OrderedDict()
        self.layout_cache = layout_cache
        self.launches = 0
        self.launch_frames = 0
        self.max_inflight_seen = 0
        # frame-path launches need only the workspace's work counters: one small buffer
        # per stream (launches on one stream run in order, on different streams they
        # overlap and must not share counters)
        self.small_ws = [torch.empty(256, dtype=torch.uint8, device=pool.device) for _ in range(n_streams)]

    # -- admission ------------------------------------------------------------------
    def data_bytes(self, r: Request) -> int:
        """Outputs and gathered state of a request."""
        return r.out_bytes + len(r.scene_ids) * self.pool.state_bytes_per_scene

    @staticmethod
    def _workspace_bytes(lay: Layout) -> int:
        n = int(lay.info.workspace_bytes)
        return n if n > 256 else 0  # frame-path launches use their stream's small buffer

    def need_bytes(self, r: Request) -> int:
        """Device bytes the request needs when launched alone: outputs, state and the
        workspace of its layout (the layout's tables are counted while it is cached)."""
        return self.data_bytes(r) + self._workspace_bytes(self._layout([r]))

    def submit(self, r: Request):
        need = self.need_bytes(r)
        if need + self.table_bytes > self.budget:
            raise ValueError(f"request {r.rid} needs {need} bytes (outputs, state, workspace) besides "
                             f"{self.table_bytes} bytes of layout tables: above the whole budget")
        self.queue.append(r)

    def _layout(self, reqs: List[Request]) -> Layout:
        key = tuple((len(r.scene_ids), r.res) for r in reqs)
        lay = self.layouts.get(key)
        if lay is None:
            desc, *_ = self.pool.batch_desc(reqs)
            local = np.tile(self.pool.object_mesh, int(desc["n_scenes"]))
            lay = Layout(self.ctx, _LayoutDesc(desc, self.pool.meshes, local),
                         mesh_ids=self.pool.mesh_ids)
            if self.tuning is not None:
                lay.set_tuning(*self.tuning)
            self.layouts[key] = lay
            self.table_bytes += int(lay.info.table_bytes)
            if len(self.layouts) > self.layout_cache:
                _, old = self.layouts.popitem(last=False)
                torch.cuda.synchronize()  # no launch may still use the evicted layout
                self.table_bytes -= int(old.info.table_bytes)
                old.close()
        else:
            self.layouts.move_to_end(key)
        return lay

    def _evict_except(self, keep: Layout):
        for key in [k for k, v in self.layouts.items() if v is not keep]:
            old = self.layouts.pop(key)
            self.table_bytes -= int(old.info.table_bytes)
            old.close()

    def _dispatch(self, now: float):
        """Merge every waiting request that fits into one launch on the next stream."""
        if not self.queue or len(self.inflight) >= self.max_inflight:
            return
        group, frames, data = [], 0, 0
        free = self.budget - self.used - self.table_bytes
        while self.queue:
            r = self.queue[0]
            nb = self.data_bytes(r)
            if data + nb > free or (group and frames + r.n_frames > self.max_batch_frames):
                break
            self.queue.popleft()
            group.append(r)
            frames += r.n_frames
            data += nb
        # the merged launch's workspace must fit as well: give back the latest requests
        # until it does (a request that fits alone waits for launches to complete)
        lay, need = None, 0
        while group:
            lay = self._layout(group)
            need = data + self._workspace_bytes(lay)
            if self.used + self.table_bytes + need <= self.budget:
                break
            if len(group) == 1 and not self.inflight:
                # alone with nothing running: drop the other cached layouts' tables
                self._evict_except(lay)
                if self.table_bytes + need <= self.budget:
                    break
                raise RuntimeError(f"request {group[0].rid} needs {need} bytes and its layout "
                                   f"{self.table_bytes}: it cannot run within the budget")
            r = group.pop()
            self.queue.appendleft(r)
            frames -= r.n_frames
            data -= self.data_bytes(r)
        if not group:
            return
        for r in group:
            r.t_admit = now
        desc, oi, li, fi, intr = self.pool.batch_desc(group)
        stream, small_ws = self.streams[self.next_stream], self.small_ws[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        dev = self.pool.device
        P = sum(r.pixels for r in group)
        with torch.cuda.stream(stream):
            idx = {k: torch.from_numpy(v).pin_memory().to(dev, non_blocking=True)
                   for k, v in (("o", oi), ("l", li), ("f", fi))}
            st = {}
            for k in ("object_pose", "object_seg", "object_visible", "albedo", "roughness", "specular"):
                st[k] = self.pool.dev[k].index_select(0, idx["o"])
            for k in ("light_vec", "light_intensity"):
                st[k] = self.pool.dev[k].index_select(0, idx["l"])
            for k in ("view", "near", "exposure"):
                st[k] = self.pool.dev[k].index_select(0, idx["f"])
            st["intr"] = torch.from_numpy(intr).pin_memory().to(dev, non_blocking=True)
            out = dict(rgb=torch.empty(3 * P, dtype=torch.float32, device=dev),
                       depth=torch.empty(P, dtype=torch.float32, device=dev),
                       normal=torch.empty(3 * P, dtype=torch.float32, device=dev),
                       seg=torch.empty(P, dtype=torch.int32, device=dev))
            # the kernels keep counters (and, on the tiled path or for scratch-held
            # scenes, vertex records and bins) in the workspace: launches in flight on
            # other streams must not share it
            ws_need = int(lay.info.workspace_bytes)
            ws = small_ws if ws_need <= 256 else torch.empty(ws_need, dtype=torch.uint8, device=dev)
            out["stats"] = torch.zeros(_lib.STATS_WORDS, dtype=torch.int32, device=dev)
            render_batch(self.ctx, lay, st, out, ws, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        t = time.perf_counter()
        p0 = 0
        for r in group:
            r.t_launch = t
            if self.keep_results:
                n = r.pixels
                r.result = dict(rgb=out["rgb"][3 * p0:3 * (p0 + n)], depth=out["depth"][p0:p0 + n],
                                normal=out["normal"][3 * p0:3 * (p0 + n)], seg=out["seg"][p0:p0 + n])
            p0 += r.pixels
        self.used += need
        self.inflight.append(_Launch(group, ev, stream, need, stats=out["stats"], keep=[st, out, idx, ws]))
        self.launches += 1
        self.launch_frames += frames
        self.max_inflight_seen = max(self.max_inflight_seen, len(self.inflight))

    def _poll(self, now_fn):
        still = []
        for L in self.inflight:
            if L.event.query():
                t = now_fn()
                for r in L.reqs:
                    r.t_done = t
                    self.done.append(r)
                self.used -= L.bytes
                if L.stats is not None:  # complete: a plain copy, no device-wide wait
                    v = L.stats.cpu().numpy().astype(np.int64) & 0xffffffff
                    for i, k in enumerate(_lib.STAT_NAMES):
                        self.counters[k] += int(v[i])
            else:
                still.append(L)
        self.inflight = still

    # -- driving ----------------------------------------------------------------------
    def run(self, requests: List[Request], drain: bool = True, warmup: float = 0.0) -> dict:
        """Replay `requests` (arrival offsets in seconds) in real time; statistics cover
        the requests arriving after `warmup` seconds."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        k = 0
        while k < len(reqs) or self.queue or (drain and self.inflight):
            t = now()
            while k < len(reqs) and reqs[k].arrival <= t:
                self.submit(reqs[k])
                k += 1
            self._poll(now)
            self._dispatch(now())
            if not self.queue and k < len(reqs) and not self.inflight:
                time.sleep(max(0.0, min(reqs[k].arrival - now(), 1e-3)))
        wall = now()
        return self.stats(wall, warmup)

    def stats(self, wall: float, warmup: float = 0.0) -> dict:
        done = [r for r in self.done if r.arrival >= warmup]
        lat = np.array([r.t_done - r.arrival for r in done]) * 1e3
        wait = np.array([r.t_admit - r.arrival for r in done]) * 1e3
        frames = sum(r.n_frames for r in done)
        span = max(wall - warmup, 1e-9)
        return dict(requests=len(done), frames=frames, wall_s=wall, frames_per_s=frames / span,
                    p50_ms=float(np.percentile(lat, 50)) if lat.size else None,
                    p99_ms=float(np.percentile(lat, 99)) if lat.size else None,
                    mean_queue_wait_ms=float(wait.mean()) if wait.size else None,
                    launches=self.launches, mean_requests_per_launch=len(self.done) / max(self.launches, 1),
                    mean_frames_per_launch=self.launch_frames / max(self.launches, 1),
                    max_inflight=self.max_inflight_seen, wait_timeouts=self.counters["wait_timeouts"])


def poisson_trace(pool: ScenePool, rate: float = 2000.0, duration: float = 10.0, warmup: float = 0.0, seed: int = 5,
                  max_scenes: int = 32, res_choices=S.C5_RES) -> List[Request]:
    """Poisson arrivals at `rate`; each request holds U{1..max_scenes} pool scenes at a
    resolution drawn from `res_choices` (config 5)."""
    rng = np.random.default_rng([seed, 0xA771])
    out, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > warmup + duration:
            break
        n = int(rng.integers(1, max_scenes + 1))
        out.append(Request(rid, rng.integers(0, pool.n_scenes, n), int(rng.choice(res_choices)), t))
        rid += 1
    return out


def main(argv=None):
    import argparse
    import json
    from .renderer import Renderer
    ap = argparse.ArgumentParser(description="serving loop benchmark (config 5)")
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--warmup", type=float, default=1.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--streams", type=int, default=4)
    args = ap.parse_args(argv)
    r = Renderer(0)
    pool = ScenePool(r.ctx, 256)
    warm = Server(r.ctx, pool, int(args.budget_gb * (1 << 30)), args.streams)
    warm.run(poisson_trace(pool, args.rate, 0.3, seed=99))
    srv = Server(r.ctx, pool, int(args.budget_gb * (1 << 30)), args.streams)
    srv.layouts = warm.layouts
    trace = poisson_trace(pool, args.rate, args.duration, args.warmup)
    st = srv.run(trace, warmup=args.warmup)
    st.update(rate=args.rate, duration=args.duration, budget_gb=args.budget_gb, streams=args.streams)
    print(json.dumps(st))


if __name__ == "__main__":
    main()
