"""Python binding of the batched renderer: argument marshalling over the C ABI.

Every step of rendering runs in the HIP kernels of liborrb.so; this module only
uploads host arrays into torch device tensors, passes their pointers and the current
HIP stream, and allocates destinations.

Typical use::

    r = Renderer(device=0)
    job = r.prepare(batch)              # upload meshes + layout + per-batch state
    out = r.render(job)                 # dict of device tensors (planar channels)
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np
import torch

from . import _lib as L

STATE_FIELDS = dict(
    object_pose=torch.float32, object_seg=torch.int32, object_visible=torch.uint8, albedo=torch.float32,
    roughness=torch.float32, specular=torch.float32, light_vec=torch.float32, light_intensity=torch.float32,
    view=torch.float32, intr=torch.float32, near=torch.float32, exposure=torch.float32)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, np.int32)


class Context:
    """A device context with its resident mesh pool."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        self.device = int(device)
        h = C.c_void_p()
        L.check(self.lib.orrb_create(self.device, C.byref(h)))
        self.handle = h
        self._mesh_ids: Dict[int, int] = {}
        self._tex_ids: Dict[int, int] = {}
        self._keep = []  # meshes whose ids are cached (keeps id() stable)

    def add_mesh(self, mesh) -> int:
        key = id(mesh)
        if key in self._mesh_ids:
            return self._mesh_ids[key]
        pos = np.ascontiguousarray(mesh.pos, np.float32)
        nrm = np.ascontiguousarray(mesh.nrm, np.float32)
        idx = np.ascontiguousarray(mesh.idx, np.int32)
        mid = C.c_int32()
        L.check(self.lib.orrb_add_mesh(self.handle, pos.ctypes.data_as(C.c_void_p), nrm.ctypes.data_as(C.c_void_p),
                                       int(pos.shape[0]), idx.ctypes.data_as(C.c_void_p), int(idx.shape[0]),
                                       C.byref(mid)))
        self._mesh_ids[key] = mid.value
        self._keep.append(mesh)
        uv = getattr(mesh, "uv", None)
        if uv is not None:
            uvc = np.ascontiguousarray(uv, np.float32)
            L.check(self.lib.orrb_set_mesh_uv(self.handle, mid.value, uvc.ctypes.data_as(C.c_void_p)))
        return mid.value

    def add_texture(self, rgb) -> int:
        """Upload a pattern texture (RGB [H, W, 3]) to the resident pool once; its id."""
        key = id(rgb)
        if key in self._tex_ids:
            return self._tex_ids[key]
        arr = np.ascontiguousarray(rgb, np.float32)
        tid = C.c_int32()
        L.check(self.lib.orrb_add_texture(self.handle, arr.ctypes.data_as(C.c_void_p), int(arr.shape[1]),
                                          int(arr.shape[0]), C.byref(tid)))
        self._tex_ids[key] = tid.value
        self._keep.append(rgb)
        return tid.value

    def wait_timeouts(self) -> int:
        """Frame-kernel waits that reached their bound on this device so far (0 unless
        a wave stalled; non-zero means some rendered pixels are unspecified)."""
        n = C.c_uint64()
        L.check(self.lib.orrb_wait_timeouts(self.handle, C.byref(n)))
        return int(n.value)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.orrb_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Layout:
    """Validated batch structure (host arrays copied into library-owned device tables)."""

    def __init__(self, ctx: Context, batch, mesh_ids=None):
        self.ctx = ctx
        if mesh_ids is None:
            mesh_ids = [ctx.add_mesh(m) for m in batch.meshes]
        mesh_ids = np.asarray(mesh_ids, np.int32)
        om = np.asarray(batch.object_mesh, np.int64)
        if om.size and (om.min() < 0 or om.max() >= mesh_ids.size):
            raise L.OrrbError(1, "object_mesh refers to a mesh outside batch.meshes")
        self._arrays = dict(
            sob=_i32(batch.scene_object_begin), om=_i32(mesh_ids[om] if om.size else om),
            slb=_i32(batch.scene_light_begin), lt=_i32(batch.light_type), fs=_i32(batch.frame_scene),
            w=_i32(batch.width), h=_i32(batch.height))
        a = self._arrays
        p = lambda x: x.ctypes.data_as(C.c_void_p)
        desc = L.LayoutDesc(int(a["sob"].shape[0] - 1), p(a["sob"]), p(a["om"]), p(a["slb"]), p(a["lt"]),
                            int(a["fs"].shape[0]), p(a["fs"]), p(a["w"]), p(a["h"]),
                            int(getattr(batch, "shadow_res", 0) or 0))
        h = C.c_void_p()
        L.check(ctx.lib.orrb_layout_create(ctx.handle, C.byref(desc), C.byref(h)))
        self.handle = h
        self.pixel_offset = np.concatenate([[0], np.cumsum(a["w"].astype(np.int64) * a["h"].astype(np.int64))])
        # tracker records: one per (frame, object of the frame's scene), frames in order
        per_frame = np.diff(a["sob"].astype(np.int64))[a["fs"]] if a["fs"].size else np.zeros(0, np.int64)
        self.track_base = np.concatenate([[0], np.cumsum(per_frame)]).astype(np.int64)
        self.n_track_records = int(self.track_base[-1])

    @property
    def info(self) -> L.LayoutInfo:
        inf = L.LayoutInfo()
        L.check(self.ctx.lib.orrb_layout_info_get(self.handle, C.byref(inf)))
        return inf

    def set_tuning(self, tile_w=32, tile_h=32, bin_cap=256, persistent=0, path=0):
        t = L.Tuning(tile_w, tile_h, bin_cap, persistent, path)
        L.check(self.ctx.lib.orrb_layout_set_tuning(self.handle, C.byref(t)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.ctx.lib.orrb_layout_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_state(batch, device="cuda") -> Dict[str, torch.Tensor]:
    """Per-batch state of a generator Batch as contiguous device tensors (plus the
    post-processing parameters and grain texture when the batch carries them)."""
    src = dict(object_pose=batch.object_pose, object_seg=batch.object_seg, object_visible=batch.object_visible,
               albedo=batch.albedo, roughness=batch.roughness, specular=batch.specular, light_vec=batch.light_vec,
               light_intensity=batch.light_intensity, view=batch.view, intr=batch.intr, near=batch.near,
               exposure=batch.exposure)
    out = {}
    for k, dt in STATE_FIELDS.items():
        arr = np.ascontiguousarray(src[k])
        t = torch.from_numpy(arr.astype({torch.float32: np.float32, torch.int32: np.int32,
                                         torch.uint8: np.uint8}[dt], copy=False))
        out[k] = t.to(device, non_blocking=False).contiguous()
    post = getattr(batch, "post", None)
    if post is not None:
        out["post"] = torch.from_numpy(np.ascontiguousarray(post, np.float32)).to(device)
    grain = getattr(batch, "grain", None)
    if grain is not None:
        out["grain"] = torch.from_numpy(np.ascontiguousarray(grain, np.float32)).to(device)
    for k in ("light_dir", "light_cone", "shadow_view", "shadow_intr", "tex_xform", "emission"):
        v = getattr(batch, k, None)
        if v is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device)
    return out


def texture_state(ctx: "Context", batch, device="cuda") -> Dict[str, torch.Tensor]:
    """Each object's resident pattern and normal texture ids (the batch's textures
    uploaded to the context once), as device tensors; empty if the batch has neither."""
    ot = getattr(batch, "object_texture", None)
    nt = getattr(batch, "object_normal_texture", None)
    if (ot is None and nt is None) or getattr(batch, "textures", None) is None:
        return {}
    ids = np.array([ctx.add_texture(t) for t in batch.textures], np.int32)

    def mapped(x):
        x = np.asarray(x, np.int64)
        m = np.where(x >= 0, ids[np.clip(x, 0, max(len(ids) - 1, 0))] if len(ids) else -1, -1).astype(np.int32)
        return torch.from_numpy(m).to(device)
    out = {}
    if ot is not None:
        out["texture"] = mapped(ot)
    if nt is not None:
        out["normal_texture"] = mapped(nt)
    return out


@dataclass
class Job:
    layout: Layout
    state: Dict[str, torch.Tensor]
    total_pixels: int
    workspace: Optional[torch.Tensor] = None
    extra: dict = field(default_factory=dict)


class Renderer:
    """Context + helpers to render generator batches."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP renderer needs a GPU (torch.cuda.is_available() is False)")
        self.device = device
        self.ctx = Context(device)

    def prepare(self, batch, state: Optional[Dict[str, torch.Tensor]] = None) -> Job:
        lay = Layout(self.ctx, batch)
        st = state if state is not None else device_state(batch, f"cuda:{self.device}")
        if state is None:
            st.update(texture_state(self.ctx, batch, f"cuda:{self.device}"))
        inf = lay.info
        ws = torch.empty(max(int(inf.workspace_bytes_any), 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return Job(lay, st, int(inf.total_pixels), ws)

    def alloc_outputs(self, job: Job, tri_id=False, vis=False, stats=False, alpha=False, rgb8=False,
                      track=False, base=("rgb", "depth", "normal", "seg")) -> Dict[str, torch.Tensor]:
        """Destinations for a render of `job`: the channels named in `base` (any of rgb,
        depth, normal, seg; rgb8 without rgb is encoded by the render kernels themselves,
        the paper's 3 x 8-bit format) plus the optional ones."""
        P = job.total_pixels
        dev = f"cuda:{self.device}"
        shapes = dict(rgb=(3 * P, torch.float32), depth=(P, torch.float32), normal=(3 * P, torch.float32),
                      seg=(P, torch.int32))
        out = {k: torch.empty(shapes[k][0], dtype=shapes[k][1], device=dev) for k in base}
        if tri_id:
            out["tri_id"] = torch.empty(P, dtype=torch.int32, device=dev)
        if vis:
            out["vis"] = torch.empty(P, dtype=torch.int64, device=dev)
        if stats:
            out["stats"] = torch.zeros(L.STATS_WORDS, dtype=torch.int32, device=dev)
        if alpha:
            out["alpha"] = torch.empty(P, dtype=torch.float32, device=dev)
        if rgb8:
            out["rgb8"] = torch.empty(3 * P, dtype=torch.uint8, device=dev)
        if track:
            n = int(job.layout.n_track_records)
            out["track"] = torch.empty(n * L.TRACK_BYTES, dtype=torch.uint8, device=dev)
        return out

    def render(self, job: Job, out: Optional[Dict[str, torch.Tensor]] = None, tri_id=False, vis=False,
               stream=None, stats=False, alpha=False, rgb8=False, track=False) -> Dict[str, torch.Tensor]:
        if out is None:
            out = self.alloc_outputs(job, tri_id, vis, stats, alpha, rgb8, track)
        render_batch(self.ctx, job.layout, job.state, out, job.workspace, stream)
        return out


def render_batch(ctx: Context, layout: Layout, state: Dict[str, torch.Tensor], out: Dict[str, torch.Tensor],
                 workspace: torch.Tensor, stream=None):
    """orrb_render_batch on `stream` (default: torch's current stream)."""
    sc, cam, par, o = _structs(state, out)
    st = stream if stream is not None else torch.cuda.current_stream(ctx.device)
    L.check(ctx.lib.orrb_render_batch(ctx.handle, layout.handle, C.byref(sc), C.byref(cam), C.byref(par), C.byref(o),
                                      _ptr(workspace), int(workspace.numel()), C.c_void_p(st.cuda_stream)))


def validate_batch(ctx: Context, layout: Layout, state: Dict[str, torch.Tensor], stats: torch.Tensor, stream=None):
    """orrb_validate_batch on `stream`: adds to stats["invalid_state"] the objects, lights
    and frames of `state` that break the render's preconditions."""
    sc, cam, par, _ = _structs(state, {})
    st = stream if stream is not None else torch.cuda.current_stream(ctx.device)
    L.check(ctx.lib.orrb_validate_batch(ctx.handle, layout.handle, C.byref(sc), C.byref(cam), C.byref(par),
                                        _ptr(stats), C.c_void_p(st.cuda_stream)))


def render_batch_noalloc(ctx: Context, layout: Layout, state: Dict[str, torch.Tensor], out: Dict[str, torch.Tensor],
                         stream=None):
    """orrb_render_batch_noalloc on `stream`: the workspace comes from the library's fixed
    per-device array, so the call allocates nothing.  Calls that overlap on one device
    race on that array."""
    sc, cam, par, o = _structs(state, out)
    st = stream if stream is not None else torch.cuda.current_stream(ctx.device)
    L.check(ctx.lib.orrb_render_batch_noalloc(ctx.handle, layout.handle, C.byref(sc), C.byref(cam), C.byref(par),
                                              C.byref(o), C.c_void_p(st.cuda_stream)))


def _params(state) -> L.Params:
    s = state
    grain = s.get("grain")
    gh, gw = (int(grain.shape[-2]), int(grain.shape[-1])) if grain is not None else (0, 0)
    return L.Params(_ptr(s["albedo"]), _ptr(s["roughness"]), _ptr(s["specular"]), _ptr(s["light_vec"]),
                    _ptr(s["light_intensity"]), _ptr(s["exposure"]), _ptr(s.get("post")), _ptr(grain), gw, gh,
                    _ptr(s.get("light_dir")), _ptr(s.get("light_cone")), _ptr(s.get("shadow_view")),
                    _ptr(s.get("shadow_intr")), _ptr(s.get("texture")), _ptr(s.get("tex_xform")),
                    _ptr(s.get("emission")), _ptr(s.get("normal_texture")))


def _structs(state, out):
    s = state
    sc = L.Scenes(_ptr(s["object_pose"]), _ptr(s["object_seg"]), _ptr(s["object_visible"]))
    cam = L.Cameras(_ptr(s["view"]), _ptr(s["intr"]), _ptr(s["near"]))
    o = L.Outputs(_ptr(out.get("rgb")), _ptr(out.get("depth")), _ptr(out.get("normal")), _ptr(out.get("seg")),
                  _ptr(out.get("tri_id")), _ptr(out.get("vis")), _ptr(out.get("stats")), _ptr(out.get("alpha")),
                  _ptr(out.get("rgb8")), _ptr(out.get("track")))
    return sc, cam, _params(state), o


def read_track(track: torch.Tensor) -> Dict[str, np.ndarray]:
    """Tracker records (orrb_track, 48 bytes each) as numpy arrays: count, bbox
    [n, 4] (i_min, j_min, i_max, j_max), sum_i, sum_j, origin [n, 3] (x, y, w)."""
    raw = track.detach().to("cpu").numpy().view(np.uint8)
    dt = np.dtype([("count", "<i4"), ("bbox", "<i4", 4), ("origin", "<f4", 3), ("sum_i", "<u8"), ("sum_j", "<u8")])
    assert dt.itemsize == L.TRACK_BYTES
    r = raw.view(dt)
    return dict(count=r["count"].astype(np.int64), bbox=r["bbox"].astype(np.int64), sum_i=r["sum_i"].astype(np.int64),
                sum_j=r["sum_j"].astype(np.int64), origin=r["origin"].astype(np.float64))


def autotune(ctx: Context, layout: Layout, state, out, workspace, stream=None, cache_path=None):
    """orrb_autotune: measure candidate tunings on this batch and keep the fastest.
    Returns (tuning tuple, ms per render)."""
    sc, cam, par, o = _structs(state, out)
    st = stream if stream is not None else torch.cuda.current_stream(ctx.device)
    t = L.Tuning()
    ms = C.c_double()
    L.check(ctx.lib.orrb_autotune(ctx.handle, layout.handle, C.byref(sc), C.byref(cam), C.byref(par), C.byref(o),
                                  _ptr(workspace), int(workspace.numel()), C.c_void_p(st.cuda_stream),
                                  None if cache_path is None else str(cache_path).encode(), C.byref(t), C.byref(ms)))
    return t.as_tuple(), ms.value


class Graph:
    """orrb_graph_*: one render call captured with fixed buffers; replay() re-renders
    whatever those buffers hold."""

    def __init__(self, ctx: Context, layout: Layout, state, out, workspace, stream):
        self.ctx = ctx
        self._keep = (layout, state, out, workspace)
        sc, cam, par, o = _structs(state, out)
        h = C.c_void_p()
        L.check(ctx.lib.orrb_graph_create(ctx.handle, layout.handle, C.byref(sc), C.byref(cam), C.byref(par),
                                          C.byref(o), _ptr(workspace), int(workspace.numel()),
                                          C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.handle = h

    def replay(self, stream=None):
        st = stream if stream is not None else torch.cuda.current_stream(self.ctx.device)
        L.check(self.ctx.lib.orrb_graph_launch(self.handle, C.c_void_p(st.cuda_stream)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.ctx.lib.orrb_graph_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shade_backward(ctx: Context, layout: Layout, state: Dict[str, torch.Tensor], vis: torch.Tensor,
                   grad_rgb: torch.Tensor, workspace: Optional[torch.Tensor] = None, stream=None) -> Dict[str, torch.Tensor]:
    """orrb_shade_backward: gradients of the loss with respect to albedo [O,3],
    roughness [O], specular [O], light_vec [L,3] (world), light_intensity [L] and
    exposure [F], given dL/d(rgb) and the forward visibility keys."""
    s = state
    dev = vis.device
    inf = layout.info
    if workspace is None or workspace.numel() < inf.grad_workspace_bytes:
        workspace = torch.empty(max(int(inf.grad_workspace_bytes), 256), dtype=torch.uint8, device=dev)
    O, Lc, F = int(inf.n_objects), int(inf.n_lights), int(inf.n_frames)
    g = dict(albedo=torch.empty((O, 3), dtype=torch.float32, device=dev),
             roughness=torch.empty(O, dtype=torch.float32, device=dev),
             specular=torch.empty(O, dtype=torch.float32, device=dev),
             light_vec=torch.empty((Lc, 3), dtype=torch.float32, device=dev),
             light_intensity=torch.empty(Lc, dtype=torch.float32, device=dev),
             exposure=torch.empty(F, dtype=torch.float32, device=dev))
    sc = L.Scenes(_ptr(s["object_pose"]), _ptr(s["object_seg"]), _ptr(s["object_visible"]))
    cam = L.Cameras(_ptr(s["view"]), _ptr(s["intr"]), _ptr(s["near"]))
    par = _params(s)
    gr = L.Grads(_ptr(g["albedo"]), _ptr(g["roughness"]), _ptr(g["specular"]), _ptr(g["light_vec"]),
                 _ptr(g["light_intensity"]), _ptr(g["exposure"]))
    grad_rgb = grad_rgb.contiguous()
    if grad_rgb.dtype != torch.float32 or grad_rgb.numel() != 3 * int(inf.total_pixels):
        raise ValueError("grad_rgb must be float32 with 3 * total_pixels elements")
    if vis.dtype != torch.int64 or vis.numel() != int(inf.total_pixels):
        raise ValueError("vis must be int64 with total_pixels elements")
    st = stream if stream is not None else torch.cuda.current_stream(ctx.device)
    L.check(ctx.lib.orrb_shade_backward(ctx.handle, layout.handle, C.byref(sc), C.byref(cam), C.byref(par), _ptr(vis),
                                        _ptr(grad_rgb), C.byref(gr), _ptr(workspace), int(workspace.numel()),
                                        C.c_void_p(st.cuda_stream)))
    return g


def frame_planes(arr: torch.Tensor, pixel_offset, f: int, width: int, height: int, planes: int = 1) -> torch.Tensor:
    po = int(pixel_offset[f])
    n = width * height
    return arr[planes * po: planes * po + planes * n].view(planes, height, width)


def read_stats(stats: torch.Tensor) -> Dict[str, int]:
    """The named counters of a stats destination (copied on its stream's order)."""
    v = stats.detach().to("cpu").numpy().astype(np.int64) & 0xffffffff
    return {k: int(v[i]) for i, k in enumerate(L.STAT_NAMES)}
