"""FP64 CPU oracle of the batched randomized renderer (ctypes wrapper of oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU
baseline of the benchmark, never by the product path.  It shares no code with the
HIP renderer and imports nothing from the product package: a batch is any object with
the structure-of-arrays attributes documented in ``_pack`` (the seeded generators'
``Batch`` has them).

Entry points
------------
``render(batch)``      -> dict of FP64/int32 planar channels plus the two-nearest
                          depths and per-pixel fragment counts (oracle.c, steps O1-O9).
``shade_grad(batch, target, pixel_weight)`` -> (loss, grads): the analytic adjoint of
                          the shading over the fixed visibility (step O10).
``loss(batch, target, pixel_weight)``       -> the FP64 loss alone (for finite
                          differences).
``near_tie(out, rel)``  -> bool mask of pixels whose two nearest fragments are within
                          ``rel`` relative depth (several visibility answers are right).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def open_library(path: str):
    """Open a compiled oracle library and declare its entry points."""
    lib = C.CDLL(path)
    P = C.c_void_p
    inputs = [P] * 17 + [C.c_int32] + [P] * 8 + [P] * 6 + [C.c_int32] + [P] * 7
    lib.oracle_render.argtypes = inputs + [P] * 9 + [C.c_int32]
    lib.oracle_render.restype = C.c_int
    lib.oracle_shade_grad.argtypes = inputs + [C.c_int32, P, P, P, P, P, P, P, P, P, P, C.c_int32]
    lib.oracle_shade_grad.restype = C.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = open_library(_LIB_PATH)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Packed:
    """Contiguous FP64 / int arrays of a batch, kept alive for the C call."""

    def __init__(self, b):
        meshes = b.meshes
        nv = np.array([m.pos.shape[0] for m in meshes], np.int64)
        nt = np.array([m.idx.shape[0] for m in meshes], np.int64)
        self.mesh_vbegin = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
        self.mesh_tbegin = np.concatenate([[0], np.cumsum(nt)]).astype(np.int64)
        self.mesh_pos = np.ascontiguousarray(np.concatenate([m.pos for m in meshes]), np.float64)
        self.mesh_nrm = np.ascontiguousarray(np.concatenate([m.nrm for m in meshes]), np.float64)
        self.mesh_idx = np.ascontiguousarray(np.concatenate([m.idx for m in meshes]), np.int32)
        i32 = lambda x: np.ascontiguousarray(x, np.int32)
        f64 = lambda x: np.ascontiguousarray(np.asarray(x, np.float32), np.float64)  # exact promotion
        self.scene_object_begin = i32(b.scene_object_begin)
        self.object_mesh = i32(b.object_mesh)
        self.object_pose = f64(b.object_pose)
        self.object_seg = i32(b.object_seg)
        self.object_visible = np.ascontiguousarray(b.object_visible, np.uint8)
        self.scene_light_begin = i32(b.scene_light_begin)
        self.light_type = i32(b.light_type)
        self.frame_scene = i32(b.frame_scene)
        self.view = f64(b.view)
        self.intr = f64(b.intr)
        self.near = f64(b.near)
        self.width = i32(b.width)
        self.height = i32(b.height)
        w = self.width.astype(np.int64) * self.height.astype(np.int64)
        self.pixel_offset = np.concatenate([[0], np.cumsum(w)]).astype(np.int64)
        # shading parameters may be given in FP64 (finite differences perturb them)
        p64 = lambda x: np.ascontiguousarray(x, np.float64)
        self.albedo = p64(b.albedo)
        self.roughness = p64(b.roughness)
        self.specular = p64(b.specular)
        self.light_vec = p64(b.light_vec)
        self.light_intensity = p64(b.light_intensity)
        self.exposure = p64(b.exposure)
        self.n_frames = int(self.frame_scene.shape[0])
        self.n_scenes = int(self.scene_object_begin.shape[0] - 1)
        self.total_pixels = int(self.pixel_offset[-1])
        lights = np.diff(self.scene_light_begin)
        if lights.size and lights.max() > 64:
            raise ValueError("oracle supports at most 64 lights per scene")
        # spot lights (type 2): axis, cone cosines, shadow camera; shadow maps are set
        # by render() once the shadow frames are rendered
        nl = int(self.light_type.shape[0])
        self.has_spot = bool((self.light_type == 2).any())
        opt = lambda name, shape: (p64(getattr(b, name)) if getattr(b, name, None) is not None
                                   else np.zeros(shape, np.float64))
        self.light_dir = opt("light_dir", (nl, 3))
        self.light_cone = opt("light_cone", (nl, 2))
        self.shadow_view = opt("shadow_view", (nl, 3, 4))
        self.shadow_intr = opt("shadow_intr", (nl, 4))
        self.shadow_res = int(getattr(b, "shadow_res", 0) or 0)
        self.shadow_slot = np.full(nl, -1, np.int32)
        self.shadow_slot[self.light_type == 2] = np.arange(int((self.light_type == 2).sum()), dtype=np.int32)
        self.shadow_maps = np.zeros(max(1, int((self.light_type == 2).sum())) * max(1, self.shadow_res) ** 2)
        # materials with pattern textures and emission (None when the batch has none)
        uvs = [getattr(m, "uv", None) for m in meshes]
        self.mesh_uv = (np.ascontiguousarray(np.concatenate(
            [np.asarray(u, np.float32) if u is not None else np.zeros((m.pos.shape[0], 2), np.float32)
             for u, m in zip(uvs, meshes)]), np.float64) if any(u is not None for u in uvs) else None)
        texs = getattr(b, "textures", None)
        ot = getattr(b, "object_texture", None)
        nt = getattr(b, "object_normal_texture", None)
        if texs is not None and ot is None and nt is not None:
            ot = np.full(len(nt), -1, np.int32)  # normal textures only
        if texs is not None and ot is not None:
            info, off = [], 0
            for t in texs:
                H, W = t.shape[0], t.shape[1]
                info.append((off, W, H))
                off += W * H
            self.tex_texels = np.ascontiguousarray(np.concatenate(
                [np.asarray(t, np.float32).reshape(-1, 3) for t in texs]), np.float64)
            self.tex_info = np.ascontiguousarray(info, np.int64)
            self.obj_tex = np.ascontiguousarray(ot, np.int32)
            self.obj_txf = p64(np.asarray(b.tex_xform, np.float32))
        else:
            self.tex_texels = self.tex_info = self.obj_tex = self.obj_txf = None
        self.obj_ntex = (np.ascontiguousarray(nt, np.int32) if texs is not None and nt is not None else None)
        em = getattr(b, "emission", None)
        self.emission = None if em is None else p64(np.asarray(em, np.float32))

    def args(self):
        return [_ptr(self.mesh_vbegin), _ptr(self.mesh_tbegin), _ptr(self.mesh_pos), _ptr(self.mesh_nrm),
                _ptr(self.mesh_idx), _ptr(self.scene_object_begin), _ptr(self.object_mesh),
                _ptr(self.object_pose), _ptr(self.object_seg), _ptr(self.object_visible),
                _ptr(self.albedo), _ptr(self.roughness), _ptr(self.specular),
                _ptr(self.scene_light_begin), _ptr(self.light_type), _ptr(self.light_vec),
                _ptr(self.light_intensity), self.n_frames, _ptr(self.frame_scene), _ptr(self.view),
                _ptr(self.intr), _ptr(self.near), _ptr(self.exposure), _ptr(self.width),
                _ptr(self.height), _ptr(self.pixel_offset), _ptr(self.light_dir), _ptr(self.light_cone),
                _ptr(self.shadow_view), _ptr(self.shadow_intr), _ptr(self.shadow_maps), _ptr(self.shadow_slot),
                self.shadow_res, _ptr(self.mesh_uv), _ptr(self.tex_texels), _ptr(self.tex_info), _ptr(self.obj_tex),
                _ptr(self.obj_txf), _ptr(self.emission), _ptr(self.obj_ntex)]


def _pack(batch):
    return _Packed(batch)


def shadow_batch(batch):
    """The shadow frames of a batch's spot lights (type 2): one N x N frame per spot
    light, of that light's scene, seen from its shadow camera (near 0.01 m).  Only their
    depth is used; their lights are made point lights so that rendering them needs no
    shadow map."""
    lt = np.asarray(batch.light_type)
    spots = np.nonzero(lt == 2)[0]
    slb = np.asarray(batch.scene_light_begin)
    scene_of = np.searchsorted(slb, spots, side="right") - 1
    N = int(batch.shadow_res)
    n = spots.size
    return batch.replace(
        light_type=np.where(lt == 2, 0, lt).astype(np.int32), frame_scene=scene_of.astype(np.int32),
        width=np.full(n, N, np.int32), height=np.full(n, N, np.int32),
        view=np.asarray(batch.shadow_view, np.float32)[spots], intr=np.asarray(batch.shadow_intr, np.float32)[spots],
        near=np.full(n, 0.01, np.float32), exposure=np.ones(n, np.float32), post=None)


def render(batch, threads: int = 0) -> dict:
    """FP64 render of every frame (planar layout, frames packed in order).

    Spot lights (type 2) cast shadows (Sec. 5: spot lights with soft shadows): their
    shadow maps are first rendered as depth frames from the lights' shadow cameras by
    this same oracle, then shading filters them (3 x 3 percentage-closer filtering).

    Keys: rgb f64[3*P], depth f64[P], normal f64[3*P], seg i32[P], tri_id i32[P],
    depth2 f64[P] (second-nearest fragment depth, +inf if none), frag_count i32[P],
    obj_id i32[P] (global object of the nearest fragment, -1 background),
    alpha f64[P] (1 covered, 0 background), pixel_offset i64[F+1]; P = total pixels."""
    pk = _pack(batch)
    P = pk.total_pixels
    shadow = None
    if pk.has_spot:
        if pk.shadow_res < 1:
            raise ValueError("spot lights need shadow_res >= 1")
        shadow = render(shadow_batch(batch), threads)
        pk.shadow_maps = np.ascontiguousarray(shadow["depth"], np.float64)
    out = dict(rgb=np.zeros(3 * P), depth=np.zeros(P), normal=np.zeros(3 * P),
               seg=np.zeros(P, np.int32), tri_id=np.zeros(P, np.int32), depth2=np.zeros(P),
               frag_count=np.zeros(P, np.int32), obj_id=np.zeros(P, np.int32), shadow_amb=np.zeros(P, np.uint8))
    rc = _load().oracle_render(*pk.args(), _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["normal"]),
                               _ptr(out["seg"]), _ptr(out["tri_id"]), _ptr(out["depth2"]),
                               _ptr(out["frag_count"]), _ptr(out["obj_id"]), _ptr(out["shadow_amb"]), int(threads))
    if shadow is not None:
        out["shadow_depth"] = shadow["depth"]
    if rc != 0:
        raise MemoryError("oracle_render failed")
    out["pixel_offset"] = pk.pixel_offset
    # Sec. 4.4: RGB "optionally with" a transparency channel.  No material is
    # transparent here, so alpha is the coverage of the pixel centre.
    out["alpha"] = (out["tri_id"] >= 0).astype(np.float64)
    return out


def shade_grad(batch, target_rgb=None, pixel_weight=None, threads: int = 0, dl_drgb=None):
    """FP64 loss sum w_px (rgb - target)^2 and its gradient over the fixed visibility.

    With ``dl_drgb`` (planar like rgb, [3 * total_pixels]) the loss is the linear
    sum w_px dl_drgb . rgb instead and ``target_rgb`` is ignored.

    Returns (loss, dict(albedo [O,3], roughness [O], specular [O], light_vec [L,3]
    (world-space gradient of each light's vector: position of a point light,
    direction of a directional light), light_intensity [L], exposure [F]))."""
    pk = _pack(batch)
    P = pk.total_pixels
    if dl_drgb is not None:
        upstream = np.ascontiguousarray(dl_drgb, np.float64).reshape(-1)
        if upstream.shape[0] != 3 * P:
            raise ValueError("dl_drgb must hold 3 * total_pixels values")
        target = None
    else:
        upstream = None
        if target_rgb is None:
            raise ValueError("target_rgb or dl_drgb is required")
        target = np.ascontiguousarray(target_rgb, np.float64).reshape(-1)
        if target.shape[0] != 3 * P:
            raise ValueError("target must hold 3 * total_pixels values")
    wmask = None if pixel_weight is None else np.ascontiguousarray(pixel_weight, np.uint8).reshape(-1)
    if wmask is not None and wmask.shape[0] != P:
        raise ValueError("pixel_weight must hold total_pixels values")
    O = int(pk.object_mesh.shape[0])
    L = int(pk.light_type.shape[0])
    g = dict(albedo=np.zeros((O, 3)), roughness=np.zeros(O), specular=np.zeros(O),
             light_vec=np.zeros((L, 3)), light_intensity=np.zeros(L), exposure=np.zeros(pk.n_frames))
    loss = np.zeros(1)
    if pk.has_spot:
        raise ValueError("the oracle's adjoint does not cover spot lights")
    if pk.obj_tex is not None or pk.emission is not None:
        raise ValueError("the oracle's adjoint does not cover textured or emissive materials")
    rc = _load().oracle_shade_grad(*pk.args(), pk.n_scenes, _ptr(target), _ptr(wmask), _ptr(upstream),
                                   _ptr(loss), _ptr(g["albedo"]), _ptr(g["roughness"]), _ptr(g["specular"]),
                                   _ptr(g["light_vec"]), _ptr(g["light_intensity"]), _ptr(g["exposure"]),
                                   int(threads))
    if rc != 0:
        raise MemoryError("oracle_shade_grad failed")
    return float(loss[0]), g


def loss(batch, target_rgb, pixel_weight=None, threads: int = 0) -> float:
    return shade_grad(batch, target_rgb, pixel_weight, threads)[0]


def near_tie(out: dict, rel: float = 1e-5) -> np.ndarray:
    """Pixels with a second fragment whose depth is within rel * d1 of the nearest."""
    d1, d2 = out["depth"], out["depth2"]
    return (out["tri_id"] >= 0) & np.isfinite(d2) & (d2 - d1 <= rel * d1)


def frame_view(arr: np.ndarray, pixel_offset, f: int, width: int, height: int, planes: int = 1) -> np.ndarray:
    """View of frame f's planes: [planes, H, W] (planes = 3 for rgb/normal)."""
    po = int(pixel_offset[f])
    n = width * height
    return arr[planes * po: planes * po + planes * n].reshape(planes, height, width)


# ----------------------------------------------------------------------------------
# Tracker (Sec. 4.3.2): auxiliary per-object outputs of a rendered frame
# ----------------------------------------------------------------------------------

TRACK_EMPTY_MIN = 2 ** 31 - 1  # i_min / j_min of an object with no visible pixel


def track(batch, out) -> dict:
    """Tracker outputs (Sec. 4.3.2: screen-space coordinates and bounding boxes of the
    tracked objects) for every (frame, object of the frame's scene), frames in order and
    a scene's objects in scene order.

    From the rendered visibility (``out`` of :func:`render`): ``count`` = pixels whose
    nearest fragment belongs to the object; ``bbox`` = (i_min, j_min, i_max, j_max), the
    inclusive pixel range of those pixels ((2^31-1, 2^31-1, -1, -1) when count is 0);
    ``sum_i`` / ``sum_j`` = sums of their column / row indices (the centroid is
    sum / count + 1/2 in pixel coordinates).  ``origin`` = (x, y, w): the object frame's
    origin projected with the frame's pinhole camera (origin at the image's top-left
    corner, y down) and its eye depth w along -z, in FP64; x = y = NaN when w <= 0."""
    b = batch
    po = out["pixel_offset"]
    obj_id = out["obj_id"]
    rows = []
    for f in range(b.n_frames):
        s = int(b.frame_scene[f])
        W, H = int(b.width[f]), int(b.height[f])
        ids = obj_id[po[f]: po[f] + W * H].reshape(H, W)
        V = np.asarray(b.view[f], np.float32).astype(np.float64)
        fx, fy, cx, cy = np.asarray(b.intr[f], np.float32).astype(np.float64)
        for o in range(int(b.scene_object_begin[s]), int(b.scene_object_begin[s + 1])):
            jj, ii = np.nonzero(ids == o)
            t = np.asarray(b.object_pose[o], np.float32).astype(np.float64)[:, 3]
            e = V[:, :3] @ t + V[:, 3]
            w = -e[2]
            x, y = (fx * e[0] / w + cx, -fy * e[1] / w + cy) if w > 0 else (np.nan, np.nan)
            n = ii.size
            rows.append((n, ii.min() if n else TRACK_EMPTY_MIN, jj.min() if n else TRACK_EMPTY_MIN,
                         ii.max() if n else -1, jj.max() if n else -1, int(ii.sum()), int(jj.sum()), x, y, w))
    a = np.array(rows, dtype=object).reshape(-1, 10)
    return dict(count=a[:, 0].astype(np.int64), bbox=a[:, 1:5].astype(np.int64), sum_i=a[:, 5].astype(np.int64),
                sum_j=a[:, 6].astype(np.int64), origin=a[:, 7:10].astype(np.float64))


# ----------------------------------------------------------------------------------
# Post-processing and 3 x 8-bit encoding (Sec. 4.3.1 PostprocessingRandomizer:
# colour grading hue, saturation, contrast, temperature, tint and grain; Sec. 5:
# 200 x 200 images in 3 x 8-bit RGB).  The paper names the parameters, not the
# formulas; the definitions below are this implementation's reading.
# ----------------------------------------------------------------------------------

POST_WORDS = 12  # per-frame parameter words (see postprocess)
LUMA = np.array([0.2126, 0.7152, 0.0722])  # Rec. 709 luma weights


def srgb_encode(x):
    """sRGB transfer function (IEC 61966-2-1) of linear values in [0, 1]."""
    x = np.asarray(x, np.float64)
    return np.where(x <= 0.0031308, 12.92 * x, 1.055 * np.power(x, 1.0 / 2.4) - 0.055)


def hue_rotation(h):
    """Rotation by angle h (radians) about the grey axis (1, 1, 1)/sqrt(3) (Rodrigues)."""
    u = np.ones(3) / np.sqrt(3.0)
    K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return np.cos(h) * np.eye(3) + np.sin(h) * K + (1 - np.cos(h)) * np.outer(u, u)


def postprocess(batch, rgb, post=None, grain=None):
    """Colour grading, grain and 8-bit encoding of linear rgb (planar like the render's
    rgb, exposure already applied), per frame and pixel, in FP64.

    ``post`` f[F, 12] per frame: 0 temperature T, 1 tint G, 2 hue h (radians),
    3 saturation s, 4 contrast k, 5 grain intensity I, 6 grain coloration kappa,
    7 grain size S (pixels, integer >= 1), 8-9 grain texture offset (ox, oy) (integer
    texels), 10-11 unused.  None = identity grading, no grain.  ``grain`` f[3, GH, GW]
    in [0, 1) or None (no grain).  Steps, each channel c of pixel (i, j):

    1. white balance: c *= (1 + T/5, 1 - G/5, 1 - T/5)[c]  (warm/cool, magenta/green);
    2. clamp to [0, 1] and encode with the sRGB transfer function;
    3. saturation about the Rec. 709 luma Y, then contrast about 1/2:
       c = 1/2 + k (Y + s (c - Y) - 1/2);
    4. hue: rotate (r, g, b) by h about the grey axis;
    5. grain: c += I ((1 - kappa) g0 + kappa gc - 1/2), g sampled at texel
       ((i div S + ox) mod GW, (j div S + oy) mod GH);
    6. v = 255 clamp(c, 0, 1); code = floor(v + 1/2).

    Returns (codes u8[3P], v f64[3P])."""
    b = batch
    rgb = np.asarray(rgb, np.float64).reshape(-1)
    po = b.pixel_offset
    codes = np.zeros(rgb.shape[0], np.uint8)
    vals = np.zeros(rgb.shape[0], np.float64)
    for f in range(b.n_frames):
        W, H = int(b.width[f]), int(b.height[f])
        P = W * H
        p = np.zeros(POST_WORDS) if post is None else np.asarray(post[f], np.float32).astype(np.float64)
        if post is None:
            p[3] = p[4] = p[7] = 1.0
        T, G, h, s, k, I, kap = p[:7]
        S = max(1, int(np.floor(p[7])))
        ox, oy = int(p[8]), int(p[9])
        c = rgb[3 * po[f]: 3 * po[f] + 3 * P].reshape(3, P).T.copy()  # [P, 3]
        c *= np.array([1 + T / 5, 1 - G / 5, 1 - T / 5])
        e = srgb_encode(np.clip(c, 0.0, 1.0))
        Y = e @ LUMA
        q = 0.5 + k * (Y[:, None] + s * (e - Y[:, None]) - 0.5)
        r = q @ hue_rotation(h).T
        if grain is not None and I != 0:
            g = np.asarray(grain, np.float32).astype(np.float64)
            GH, GW = g.shape[1], g.shape[2]
            jj, ii = np.divmod(np.arange(P), W)
            tx = (ii // S + ox) % GW
            ty = (jj // S + oy) % GH
            g0 = g[0, ty, tx]
            n = np.stack([(1 - kap) * g0 + kap * g[ch, ty, tx] - 0.5 for ch in range(3)], axis=1)
            r = r + I * n
        v = 255.0 * np.clip(r, 0.0, 1.0)
        vals[3 * po[f]: 3 * po[f] + 3 * P] = v.T.reshape(-1)
        codes[3 * po[f]: 3 * po[f] + 3 * P] = np.floor(v + 0.5).astype(np.uint8).T.reshape(-1)
    return codes, vals
