"""Seeded synthetic scene generators for the batched renderer.

This module only builds *inputs*: tessellated meshes, host forward kinematics of a
hinge tree, camera matrices, and sampled randomization parameters.  It holds none of
the rendering arithmetic (no projection, rasterization or shading), so the HIP path
and the FP64 CPU oracle can both consume its arrays unchanged.

Paper context (ORRB, arXiv:1906.11633):
  * Single Scene Multiple States (Sec. 3): geometry and the kinematic hierarchy are
    shared by every scene instance; only randomized parameters and the light-weight
    state differ.  Here: one shared mesh list plus per-scene structure-of-arrays.
  * Seeded determinism (Sec. 4.3): a seed re-initialises the random generator and the
    randomizers always run in the same order.  Here: every scene draws from
    ``np.random.default_rng([seed, scene_index])`` in a fixed order, so a scene's
    parameters never depend on which batch it is rendered in.
  * Randomizers (Sec. 4.3.1): material tint/metallic/glossiness (albedo, specular,
    roughness), camera jitter, joint positions, light intensity, post-processing
    (exposure).  Utility components (Sec. 4.3.2): LookAt for cameras, LightSetup for
    light placement by distance from and height above a target.

Conventions (shared by both renderers, stated here because the paper fixes none):
  * world frame is right-handed; poses are ``[s*R | t]`` (3x4, object -> world, rigid
    plus uniform scale);
  * view matrices are 3x4 world -> camera; the camera looks down its -z axis, +y up;
  * intrinsics are ``(fx, fy, cx, cy)`` in pixels, image origin at the top-left corner,
    x right, y down, pixel (i, j) centred at (i + 1/2, j + 1/2);
  * meshes are closed, counter-clockwise when seen from outside, with smooth
    (capsule) or per-face (box) vertex normals.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# ----------------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------------


@dataclass
class Mesh:
    pos: np.ndarray  # f32 [V,3]
    nrm: np.ndarray  # f32 [V,3]
    idx: np.ndarray  # i32 [T,3], counter-clockwise seen from outside
    uv: Optional[np.ndarray] = None  # f32 [V,2] texture coordinates

    @property
    def n_verts(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.idx.shape[0])


def capsule_mesh(radius: float, length: float, slices: int = 16, stacks: int = 8) -> Mesh:
    """Capsule along local z: a cylinder of ``length`` between two hemispheres.

    ``slices`` around the axis and ``stacks`` rings per hemisphere give
    ``4*slices*stacks`` triangles and ``2 + 2*slices*stacks`` vertices (16x8 -> 512
    triangles, 258 vertices).  Normals are the analytic smooth normals.
    """
    S, T = int(slices), int(stacks)
    r, h = float(radius), 0.5 * float(length)
    phis = 2.0 * np.pi * np.arange(S) / S
    pos = [(0.0, 0.0, h + r)]
    nrm = [(0.0, 0.0, 1.0)]
    uv = [(0.0, 0.0)]
    rings = []
    # top hemisphere rings, polar angle from +z
    for k in range(1, T + 1):
        th = k * (0.5 * np.pi) / T
        ring = []
        for ph in phis:
            d = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
            ring.append(len(pos))
            pos.append((r * d[0], r * d[1], h + r * d[2]))
            nrm.append(d)
            uv.append((ph / (2 * np.pi), (r - r * d[2]) / (2 * h + 2 * r)))
        rings.append(ring)
    # bottom hemisphere rings, from the equator down
    for k in range(T, 0, -1):
        th = k * (0.5 * np.pi) / T
        ring = []
        for ph in phis:
            d = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), -math.cos(th))
            ring.append(len(pos))
            pos.append((r * d[0], r * d[1], -h + r * d[2]))
            nrm.append(d)
            uv.append((ph / (2 * np.pi), (2 * h + r - r * d[2]) / (2 * h + 2 * r)))
        rings.append(ring)
    bottom = len(pos)
    pos.append((0.0, 0.0, -h - r))
    nrm.append((0.0, 0.0, -1.0))
    uv.append((0.0, 1.0))
    tris = []
    for s in range(S):
        s1 = (s + 1) % S
        tris.append((0, rings[0][s], rings[0][s1]))
    for i in range(len(rings) - 1):
        a, b = rings[i], rings[i + 1]
        for s in range(S):
            s1 = (s + 1) % S
            tris.append((a[s], b[s], b[s1]))
            tris.append((a[s], b[s1], a[s1]))
    last = rings[-1]
    for s in range(S):
        s1 = (s + 1) % S
        tris.append((last[s], bottom, last[s1]))
    return Mesh(np.asarray(pos, np.float32), np.asarray(nrm, np.float32), np.asarray(tris, np.int32),
                np.asarray(uv, np.float32))


_BOX_FACES = (  # (N, U, V) with U x V = N
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
)


def box_mesh(n: int = 1) -> Mesh:
    """Unit cube [-1/2, 1/2]^3, each face split into n x n quads (12 n^2 triangles,
    6 (n+1)^2 vertices), with flat per-face normals."""
    n = int(n)
    pos, nrm, tris, uv = [], [], [], []
    for N, U, V in _BOX_FACES:
        N, U, V = np.array(N, float), np.array(U, float), np.array(V, float)
        base = len(pos)
        for j in range(n + 1):
            for i in range(n + 1):
                p = (i / n - 0.5) * U + (j / n - 0.5) * V + 0.5 * N
                pos.append(p)
                nrm.append(N)
                uv.append((i / n, j / n))
        for j in range(n):
            for i in range(n):
                v00 = base + j * (n + 1) + i
                v10, v01, v11 = v00 + 1, v00 + (n + 1), v00 + (n + 1) + 1
                tris.append((v00, v10, v11))
                tris.append((v00, v11, v01))
    return Mesh(np.asarray(pos, np.float32), np.asarray(nrm, np.float32), np.asarray(tris, np.int32),
                np.asarray(uv, np.float32))


def plane_mesh(nx: int, ny: int, sx: float = 1.0, sy: float = 1.0) -> Mesh:
    """Tessellated rectangle in the local z = 0 plane, normal +z, spanning
    [-sx/2, sx/2] x [-sy/2, sy/2] with nx x ny quads (2 nx ny triangles).  Open
    surface, used by tests (watertightness, closed-form shading)."""
    pos, tris = [], []
    for j in range(ny + 1):
        for i in range(nx + 1):
            pos.append(((i / nx - 0.5) * sx, (j / ny - 0.5) * sy, 0.0))
    for j in range(ny):
        for i in range(nx):
            v00 = j * (nx + 1) + i
            v10, v01, v11 = v00 + 1, v00 + nx + 1, v00 + nx + 2
            tris.append((v00, v10, v11))
            tris.append((v00, v11, v01))
    pos = np.asarray(pos, np.float32)
    nrm = np.zeros_like(pos)
    nrm[:, 2] = 1.0
    uv = np.stack([pos[:, 0] / sx + 0.5, pos[:, 1] / sy + 0.5], 1).astype(np.float32)
    return Mesh(pos, nrm, np.asarray(tris, np.int32), uv)


def triangle_mesh(p0, p1, p2) -> Mesh:
    """A single triangle (counter-clockwise seen from the side its normal points to)."""
    pos = np.asarray([p0, p1, p2], np.float64)
    n = np.cross(pos[1] - pos[0], pos[2] - pos[0])
    n = n / np.linalg.norm(n)
    return Mesh(pos.astype(np.float32), np.tile(n, (3, 1)).astype(np.float32),
                np.asarray([[0, 1, 2]], np.int32))


# ----------------------------------------------------------------------------------
# rigid-transform helpers (FP64 on the host)
# ----------------------------------------------------------------------------------


def rot_axis(axis: str, angle: float) -> np.ndarray:
    c, s = math.cos(angle), math.sin(angle)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], float)
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], float)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], float)


def uniform_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation (Shoemake, Graphics Gems III, 1992)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ], float)


def make_pose(R: np.ndarray, t, scale: float = 1.0) -> np.ndarray:
    P = np.zeros((3, 4), float)
    P[:, :3] = scale * R
    P[:, 3] = t
    return P


def homog(P: np.ndarray) -> np.ndarray:
    H = np.eye(4)
    H[:3, :] = P
    return H


def look_at_c2w(eye, target, up) -> np.ndarray:
    """Camera-to-world 4x4 of a camera at ``eye`` looking at ``target`` (LookAt
    utility, Sec. 4.3.2): camera -z points at the target, +y is as close to ``up`` as
    possible."""
    eye, target, up = (np.asarray(v, float) for v in (eye, target, up))
    f = target - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    C = np.eye(4)
    C[:3, 0], C[:3, 1], C[:3, 2], C[:3, 3] = r, u, -f, eye
    return C


def jitter_c2w(C: np.ndarray, rng: np.random.Generator, trans: float, angle_deg: float) -> np.ndarray:
    """Camera Jitter mode (Sec. 4.3.1): per-axis translation U[-trans, trans] and
    per-axis camera-local XYZ Euler angles U[-angle, angle], applied after LookAt."""
    t = rng.uniform(-trans, trans, 3)
    a = np.deg2rad(rng.uniform(-angle_deg, angle_deg, 3))
    J = np.eye(4)
    J[:3, :3] = rot_axis("x", a[0]) @ rot_axis("y", a[1]) @ rot_axis("z", a[2])
    J[:3, 3] = t
    return C @ J


def view_from_c2w(C: np.ndarray) -> np.ndarray:
    R = C[:3, :3]
    V = np.zeros((3, 4))
    V[:, :3] = R.T
    V[:, 3] = -R.T @ C[:3, 3]
    return V


def intrinsics(width: int, height: int, fov_y_deg: float = 45.0) -> np.ndarray:
    """Pinhole intrinsics with square pixels and the principal point at the centre."""
    fy = 0.5 * height / math.tan(0.5 * math.radians(fov_y_deg))
    return np.array([fy, fy, 0.5 * width, 0.5 * height], float)


# ----------------------------------------------------------------------------------
# batch container
# ----------------------------------------------------------------------------------


@dataclass
class Batch:
    """A batch of scenes and frames as structure-of-arrays.

    Structure (which mesh each object uses, how many lights of which type a scene
    has, which scene and resolution each frame has) is the *layout*; everything else
    is per-batch *state* that randomizers change.
    """
    meshes: List[Mesh]
    # layout
    scene_object_begin: np.ndarray  # i32 [S+1]
    object_mesh: np.ndarray         # i32 [O]
    scene_light_begin: np.ndarray   # i32 [S+1]
    light_type: np.ndarray          # i32 [L] 0 = point, 1 = directional
    frame_scene: np.ndarray         # i32 [F]
    width: np.ndarray               # i32 [F]
    height: np.ndarray              # i32 [F]
    # state
    object_pose: np.ndarray         # f32 [O,3,4]
    object_seg: np.ndarray          # i32 [O]
    object_visible: np.ndarray      # u8  [O]
    albedo: np.ndarray              # f32 [O,3]
    roughness: np.ndarray           # f32 [O]
    specular: np.ndarray            # f32 [O]
    light_vec: np.ndarray           # f32 [L,3] world position (point) or direction (directional)
    light_intensity: np.ndarray     # f32 [L]
    view: np.ndarray                # f32 [F,3,4]
    intr: np.ndarray                # f32 [F,4]
    near: np.ndarray                # f32 [F]
    exposure: np.ndarray            # f32 [F]
    name: str = ""
    extra: dict = field(default_factory=dict)
    # post-processing of the 8-bit output (optional): per-frame parameters and the
    # grain noise texture (see with_postprocessing)
    post: Optional[np.ndarray] = None   # f32 [F, 12]
    grain: Optional[np.ndarray] = None  # f32 [3, GH, GW] in [0, 1)
    # spot lights (light_type 2), optional: axis, cone cosines (inner, outer), shadow
    # camera (world -> light camera, intrinsics of an N x N map) and N
    light_dir: Optional[np.ndarray] = None    # f32 [L, 3]
    light_cone: Optional[np.ndarray] = None   # f32 [L, 2]
    shadow_view: Optional[np.ndarray] = None  # f32 [L, 3, 4]
    shadow_intr: Optional[np.ndarray] = None  # f32 [L, 4]
    shadow_res: int = 0
    # materials with pattern textures and emission, optional: the resident texture pool
    # (RGB [H, W, 3] arrays), each object's texture (-1 none), its UV transform (su, sv,
    # ou, ov) and its emissive power
    textures: Optional[list] = None
    object_texture: Optional[np.ndarray] = None  # i32 [O]
    tex_xform: Optional[np.ndarray] = None       # f32 [O, 4]
    emission: Optional[np.ndarray] = None        # f32 [O]
    # each object's normal (bump) texture from the same pool (-1 none), sampled at the
    # same transformed UV
    object_normal_texture: Optional[np.ndarray] = None  # i32 [O]

    @property
    def n_scenes(self) -> int:
        return int(self.scene_object_begin.shape[0] - 1)

    @property
    def n_objects(self) -> int:
        return int(self.object_mesh.shape[0])

    @property
    def n_lights(self) -> int:
        return int(self.light_type.shape[0])

    @property
    def n_frames(self) -> int:
        return int(self.frame_scene.shape[0])

    @property
    def pixel_offset(self) -> np.ndarray:
        """i64 [F+1]: frames packed densely in order; frame f's planes start at
        pixel_offset[f] (depth, seg) and 3*pixel_offset[f] (rgb, normal)."""
        po = np.zeros(self.n_frames + 1, np.int64)
        np.cumsum(self.width.astype(np.int64) * self.height.astype(np.int64), out=po[1:])
        return po

    @property
    def total_pixels(self) -> int:
        return int(self.pixel_offset[-1])

    def scene_triangles(self, s: int) -> int:
        b, e = self.scene_object_begin[s], self.scene_object_begin[s + 1]
        return int(sum(self.meshes[m].n_tris for m in self.object_mesh[b:e]))

    def frame_triangles(self) -> np.ndarray:
        per_scene = np.array([self.scene_triangles(s) for s in range(self.n_scenes)], np.int64)
        return per_scene[self.frame_scene]

    def uniform_shape(self) -> Optional[tuple]:
        if self.n_frames and np.all(self.width == self.width[0]) and np.all(self.height == self.height[0]):
            return int(self.width[0]), int(self.height[0])
        return None

    def select_scenes(self, scenes) -> "Batch":
        """Sub-batch made of the given scenes (and all their frames), in that order."""
        scenes = [int(s) for s in scenes]
        ob, lb = self.scene_object_begin, self.scene_light_begin
        objs = np.concatenate([np.arange(ob[s], ob[s + 1]) for s in scenes]).astype(np.int64)
        lights = np.concatenate([np.arange(lb[s], lb[s + 1]) for s in scenes]).astype(np.int64)
        frames, fs = [], []
        for k, s in enumerate(scenes):
            fr = np.nonzero(self.frame_scene == s)[0]
            frames.extend(fr.tolist())
            fs.extend([k] * len(fr))
        frames = np.asarray(frames, np.int64)
        sob = np.zeros(len(scenes) + 1, np.int32)
        sob[1:] = np.cumsum([ob[s + 1] - ob[s] for s in scenes])
        slb = np.zeros(len(scenes) + 1, np.int32)
        slb[1:] = np.cumsum([lb[s + 1] - lb[s] for s in scenes])
        return Batch(
            meshes=self.meshes, scene_object_begin=sob, object_mesh=self.object_mesh[objs],
            scene_light_begin=slb, light_type=self.light_type[lights],
            frame_scene=np.asarray(fs, np.int32), width=self.width[frames], height=self.height[frames],
            object_pose=self.object_pose[objs], object_seg=self.object_seg[objs],
            object_visible=self.object_visible[objs], albedo=self.albedo[objs],
            roughness=self.roughness[objs], specular=self.specular[objs],
            light_vec=self.light_vec[lights], light_intensity=self.light_intensity[lights],
            view=self.view[frames], intr=self.intr[frames], near=self.near[frames],
            exposure=self.exposure[frames], name=self.name + "[sub]",
            post=None if self.post is None else self.post[frames], grain=self.grain,
            light_dir=None if self.light_dir is None else self.light_dir[lights],
            light_cone=None if self.light_cone is None else self.light_cone[lights],
            shadow_view=None if self.shadow_view is None else self.shadow_view[lights],
            shadow_intr=None if self.shadow_intr is None else self.shadow_intr[lights], shadow_res=self.shadow_res,
            textures=self.textures,
            object_texture=None if self.object_texture is None else self.object_texture[objs],
            object_normal_texture=None if self.object_normal_texture is None else self.object_normal_texture[objs],
            tex_xform=None if self.tex_xform is None else self.tex_xform[objs],
            emission=None if self.emission is None else self.emission[objs])

    def replace(self, **kw) -> "Batch":
        d = dict(self.__dict__)
        d.update(kw)
        return Batch(**d)


class _Builder:
    """Accumulates scenes into a Batch."""

    def __init__(self, meshes: List[Mesh]):
        self.meshes = meshes
        self.sob, self.slb = [0], [0]
        self.obj = {k: [] for k in ("mesh", "pose", "seg", "vis", "alb", "rough", "spec")}
        self.lig = {k: [] for k in ("type", "vec", "int")}
        self.frm = {k: [] for k in ("scene", "view", "intr", "near", "exp", "w", "h")}

    def add_object(self, mesh, pose, seg, albedo, rough=1.0, spec=0.0, visible=1):
        o = self.obj
        o["mesh"].append(mesh)
        o["pose"].append(pose)
        o["seg"].append(seg)
        o["vis"].append(visible)
        o["alb"].append(albedo)
        o["rough"].append(rough)
        o["spec"].append(spec)

    def add_light(self, ltype, vec, intensity):
        self.lig["type"].append(ltype)
        self.lig["vec"].append(vec)
        self.lig["int"].append(intensity)

    def end_scene(self):
        self.sob.append(len(self.obj["mesh"]))
        self.slb.append(len(self.lig["type"]))

    def add_frame(self, view, intr, width, height, exposure=1.0, near=0.01, scene=None):
        f = self.frm
        f["scene"].append(len(self.sob) - 2 if scene is None else scene)
        f["view"].append(view)
        f["intr"].append(intr)
        f["near"].append(near)
        f["exp"].append(exposure)
        f["w"].append(width)
        f["h"].append(height)

    def build(self, name="") -> Batch:
        o, l, f = self.obj, self.lig, self.frm
        f32 = lambda x, shape: np.asarray(x, np.float64).reshape(shape).astype(np.float32)
        return Batch(
            meshes=self.meshes,
            scene_object_begin=np.asarray(self.sob, np.int32),
            object_mesh=np.asarray(o["mesh"], np.int32),
            scene_light_begin=np.asarray(self.slb, np.int32),
            light_type=np.asarray(l["type"], np.int32),
            frame_scene=np.asarray(f["scene"], np.int32),
            width=np.asarray(f["w"], np.int32), height=np.asarray(f["h"], np.int32),
            object_pose=f32(o["pose"], (-1, 3, 4)), object_seg=np.asarray(o["seg"], np.int32),
            object_visible=np.asarray(o["vis"], np.uint8), albedo=f32(o["alb"], (-1, 3)),
            roughness=f32(o["rough"], (-1,)), specular=f32(o["spec"], (-1,)),
            light_vec=f32(l["vec"], (-1, 3)), light_intensity=f32(l["int"], (-1,)),
            view=f32(f["view"], (-1, 3, 4)), intr=f32(f["intr"], (-1, 4)),
            near=f32(f["near"], (-1,)), exposure=f32(f["exp"], (-1,)), name=name)


# ----------------------------------------------------------------------------------
# config 1: tiny plain scenes
# ----------------------------------------------------------------------------------

CONFIG1_MESHES = lambda: [box_mesh(1), capsule_mesh(0.02, 0.08, 16, 8)]


def config1(seed: int = 1, n_scenes: int = 4, res: int = 64, materials: bool = False) -> Batch:
    """4 scenes x 1 camera at 64x64: a cube (12 triangles, 0.1 m edge) and two capsules
    (512 triangles) posed uniformly in a 0.3 m box with uniform orientation; albedo
    U[0,1]^3; one directional light of intensity 1 from the camera-facing hemisphere;
    camera 0.6 m up +z looking at the origin, FOV 45 deg.  ``materials=True`` adds the
    config-2 roughness / specular / exposure draws."""
    b = _Builder(CONFIG1_MESHES())
    for s in range(n_scenes):
        rng = np.random.default_rng([seed, s])
        for k, (mesh, scale) in enumerate(((0, 0.1), (1, 1.0), (1, 1.0))):
            R = uniform_rotation(rng)
            t = rng.uniform(-0.15, 0.15, 3)
            alb = rng.uniform(0, 1, 3)
            rough, spec = 1.0, 0.0
            if materials:
                rough, spec = rng.uniform(0.05, 1.0), rng.uniform(0, 1)
            b.add_object(mesh, make_pose(R, t, scale), k, alb, rough, spec)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        u[2] = -abs(u[2])  # light travels toward -z: it comes from the camera side
        b.add_light(1, u, 1.0)
        b.end_scene()
        C = look_at_c2w((0, 0, 0.6), (0, 0, 0), (0, 1, 0))
        exposure = rng.uniform(0.7, 1.3) if materials else 1.0
        b.add_frame(view_from_c2w(C), intrinsics(res, res), res, res, exposure)
    return b.build("config1" + ("s" if materials else ""))


# ----------------------------------------------------------------------------------
# config 2: articulated hand-like scenes
# ----------------------------------------------------------------------------------

# (radius, cylinder length) of the five shared capsule link meshes, metres
HAND_CAPSULES = ((0.025, 0.050), (0.011, 0.040), (0.010, 0.030), (0.009, 0.022), (0.008, 0.015))
HAND_TARGET = np.array([0.0, 0.0, 0.11])


def hand_meshes(slices: int = 16, stacks: int = 8, box_n: int = 8) -> List[Mesh]:
    return [capsule_mesh(r, L, slices, stacks) for r, L in HAND_CAPSULES] + [box_mesh(box_n)]


def hand_tree():
    """24-hinge kinematic tree: a palm root, four 5-link fingers and a 4-link thumb.

    Returns a list of links (parent, mesh, offset, base_rotation, axis); link 0 is the
    palm.  A link's joint frame is parent_frame * T(offset) * R0 * Rot(axis, q)."""
    links = [(-1, 0, np.array([0.0, 0.0, 0.0]), np.eye(3), None)]
    palm_top = HAND_CAPSULES[0][1] + HAND_CAPSULES[0][0]
    finger_meshes = (1, 2, 3, 4, 4)
    for k, x in enumerate((-0.027, -0.009, 0.009, 0.027)):
        parent = 0
        for j, m in enumerate(finger_meshes):
            if j == 0:
                off, R0 = np.array([x, 0.0, palm_top]), np.eye(3)
                axis = "x" if k % 2 == 0 else "y"
            else:
                pr, pl = HAND_CAPSULES[finger_meshes[j - 1]]
                off, R0, axis = np.array([0.0, 0.0, pl + pr]), np.eye(3), "x"
            links.append((parent, m, off, R0, axis))
            parent = len(links) - 1
    thumb_meshes = (1, 2, 3, 4)
    parent = 0
    for j, m in enumerate(thumb_meshes):
        if j == 0:
            off, R0, axis = np.array([-0.03, -0.01, 0.02]), rot_axis("y", -0.9), "y"
        else:
            pr, pl = HAND_CAPSULES[thumb_meshes[j - 1]]
            off, R0, axis = np.array([0.0, 0.0, pl + pr]), np.eye(3), "x"
        links.append((parent, m, off, R0, axis))
        parent = len(links) - 1
    assert len(links) == 25
    return links


def hand_fk(q: np.ndarray) -> List[np.ndarray]:
    """FP64 forward kinematics: 24 joint angles -> 25 capsule poses (3x4, object ->
    world).  The capsule mesh is centred on its link, extending along local +z."""
    links = hand_tree()
    frames = []
    poses = []
    qi = 0
    for parent, m, off, R0, axis in links:
        F = np.eye(4)
        F[:3, :3] = R0
        F[:3, 3] = off
        if axis is not None:
            J = np.eye(4)
            J[:3, :3] = rot_axis(axis, q[qi])
            qi += 1
            F = F @ J
        if parent >= 0:
            F = frames[parent] @ F
        frames.append(F)
        r, L = HAND_CAPSULES[m]
        C = np.eye(4)
        C[2, 3] = 0.5 * L + r
        poses.append((F @ C)[:3, :])
    return poses


def _hand_scene(b: _Builder, rng: np.random.Generator, res_list, n_cams: int = 3,
                jitter: bool = True):
    """One config-2 scene drawn from ``rng`` in a fixed order, plus its frames."""
    q = rng.uniform(-0.5, 0.5, 24)
    poses = hand_fk(q)
    for k, P in enumerate(poses):
        m = hand_tree()[k][1]
        alb = rng.uniform(0, 1, 3)
        rough = rng.uniform(0.05, 1.0)
        spec = rng.uniform(0, 1)
        b.add_object(m, P, k, alb, rough, spec)
    R = uniform_rotation(rng)
    t = np.array([0.0, -0.06, 0.10]) + rng.uniform(-0.03, 0.03, 3)
    alb = rng.uniform(0, 1, 3)
    rough = rng.uniform(0.05, 1.0)
    spec = rng.uniform(0, 1)
    b.add_object(5, make_pose(R, t, 0.05), 25, alb, rough, spec)
    n_lights = int(rng.integers(1, 5))
    for _ in range(n_lights):
        az = rng.uniform(0, 2 * np.pi)
        rho = rng.uniform(0.4, 0.8)
        hgt = rng.uniform(0.3, 0.8)
        pos = HAND_TARGET + np.array([rho * math.cos(az), rho * math.sin(az), hgt])
        b.add_light(0, pos, rng.uniform(0.5, 2.0))
    b.end_scene()
    for c in range(n_cams):
        az = math.radians(120.0 * c)
        el = math.radians(25.0)
        eye = HAND_TARGET + 0.45 * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        C = look_at_c2w(eye, HAND_TARGET, (0, 0, 1))
        if jitter:
            C = jitter_c2w(C, rng, 0.02, 3.0)
        res = res_list[c] if isinstance(res_list, (list, tuple)) else res_list
        b.add_frame(view_from_c2w(C), intrinsics(res, res), res, res, rng.uniform(0.7, 1.3))


def config2(seed: int = 2, n_scenes: int = 256, res: int = 200, n_cams: int = 3,
            scene_ids=None) -> Batch:
    """Articulated hand-like scenes: 25 capsule links (512 triangles each) on a
    24-hinge tree with joint angles U[-0.5, 0.5] rad plus one 768-triangle cube;
    3 cameras at 200x200; albedo U[0,1]^3, roughness U[0.05,1], specular U[0,1],
    1-4 point lights of intensity U[0.5,2], exposure U[0.7,1.3], camera jitter
    +-2 cm / +-3 deg."""
    b = _Builder(hand_meshes())
    ids = range(n_scenes) if scene_ids is None else scene_ids
    for s in ids:
        _hand_scene(b, np.random.default_rng([seed, int(s)]), res, n_cams)
    return b.build(f"config2[{n_scenes}x{n_cams}@{res}]")


# ----------------------------------------------------------------------------------
# post-processing randomizer (colour grading and grain of the 8-bit output)
# ----------------------------------------------------------------------------------

POST_WORDS = 12
GRAIN_SIZE = (64, 64)  # grain noise texture, texels


def postprocess_params(seed: int, n_frames: int, frame_scene=None, grain_size=GRAIN_SIZE):
    """Per-frame colour-grading and grain parameters and one grain noise texture
    (the PostprocessingRandomizer's draws): temperature and tint U[-0.3, 0.3], hue
    U[-pi/12, pi/12], saturation U[0.7, 1.3], contrast U[0.8, 1.2], grain intensity
    U[0, 0.06], coloration U[0, 1], size U{1, 2, 3} px, texel offsets uniform.  A frame's
    draws come from default_rng([seed, 0x9057, scene, k]) with k its index among its
    scene's frames, so they do not depend on the batch composition."""
    fs = np.zeros(n_frames, np.int64) if frame_scene is None else np.asarray(frame_scene, np.int64)
    GH, GW = grain_size
    post = np.zeros((n_frames, POST_WORDS), np.float32)
    seen = {}
    for f in range(n_frames):
        s = int(fs[f])
        k = seen.get(s, 0)
        seen[s] = k + 1
        rng = np.random.default_rng([seed, 0x9057, s, k])
        post[f, 0:2] = rng.uniform(-0.3, 0.3, 2)
        post[f, 2] = rng.uniform(-math.pi / 12, math.pi / 12)
        post[f, 3] = rng.uniform(0.7, 1.3)
        post[f, 4] = rng.uniform(0.8, 1.2)
        post[f, 5] = rng.uniform(0.0, 0.06)
        post[f, 6] = rng.uniform(0.0, 1.0)
        post[f, 7] = rng.integers(1, 4)
        post[f, 8] = rng.integers(0, GW)
        post[f, 9] = rng.integers(0, GH)
    grain = np.random.default_rng([seed, 0x6A41]).uniform(0.0, 1.0, (3, GH, GW)).astype(np.float32)
    return post, grain


def with_postprocessing(batch: Batch, seed: int = 0) -> Batch:
    """The batch with randomized post-processing parameters and grain texture."""
    post, grain = postprocess_params(seed, batch.n_frames, batch.frame_scene)
    return batch.replace(post=post, grain=grain)


# ----------------------------------------------------------------------------------
# materials: pattern textures (MaterialRandomizer) and the fixed-hue HSV sampler
# (FixedHueMaterialRandomizer)
# ----------------------------------------------------------------------------------


def hsv_to_rgb(h, s, v) -> np.ndarray:
    """HSV (hue in turns, [0, 1)) to RGB, the hexcone model (Smith 1978)."""
    h = float(h) % 1.0
    i = int(math.floor(h * 6.0)) % 6
    f = h * 6.0 - math.floor(h * 6.0)
    p, q, t = v * (1 - s), v * (1 - f * s), v * (1 - (1 - f) * s)
    return np.array([(v, t, p), (q, v, p), (p, v, t), (p, q, v), (t, p, v), (v, p, q)][i], float)


def fixed_hue_material(rng: np.random.Generator, base_hsv, radius, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                       metallic=(0.0, 1.0), glossiness=(0.0, 0.95), emissive_prob=0.0, emissive_power=(0.0, 0.0)):
    """A material near calibrated values: hue, saturation and value each moved by
    U[-radius, radius] around base_hsv (hue wrapping around the colour circle) and
    clamped to [lo, hi]; metallic level and glossiness uniform in their ranges; emissive
    with probability emissive_prob, with power uniform in its range.  Returns (albedo
    RGB, roughness = 1 - glossiness, specular = metallic, emission)."""
    d = rng.uniform(-1.0, 1.0, 3) * np.asarray(radius, float)
    hsv = np.asarray(base_hsv, float) + d
    hsv[0] %= 1.0
    hsv = np.clip(hsv, lo, hi)
    spec = rng.uniform(*metallic)
    rough = 1.0 - rng.uniform(*glossiness)
    emit = rng.uniform(*emissive_power) if rng.uniform() < emissive_prob else 0.0
    return hsv_to_rgb(*hsv), rough, spec, emit


def pattern_texture(rng: np.random.Generator, size: int = 64, cells: int = 8) -> np.ndarray:
    """A random pattern texture: a cells x cells checker of random colours with a
    random stripe overlay (RGB in [0, 1], [size, size, 3])."""
    cols = rng.uniform(0.2, 1.0, (cells, cells, 3))
    idx = np.arange(size) * cells // size
    tex = cols[idx[:, None], idx[None, :]]
    period = int(rng.integers(4, 16))
    stripe = ((np.arange(size)[None, :] + np.arange(size)[:, None]) // period) % 2
    return (tex * (0.75 + 0.25 * stripe[..., None])).astype(np.float32)


def bump_texture(rng: np.random.Generator, size: int = 64, waves: int = 4, slope: float = 0.6) -> np.ndarray:
    """A random normal (bump) texture: the normals of a periodic height field, a sum of
    `waves` plane waves with integer frequencies 1..6 per axis and random phases, scaled
    so the steepest slope is about `slope`; stored as RGB = (n + 1) / 2 ([size, size, 3]),
    tangent-space z up, so it tiles without seams."""
    y, x = np.mgrid[0:size, 0:size] / size
    gx = np.zeros((size, size))
    gy = np.zeros((size, size))
    for _ in range(waves):
        fx, fy = rng.integers(1, 7, 2)
        ph = rng.uniform(0, 2 * np.pi)
        arg = 2 * np.pi * (fx * x + fy * y) + ph
        gx += 2 * np.pi * fx * np.cos(arg)
        gy += 2 * np.pi * fy * np.cos(arg)
    k = slope / max(np.abs(gx).max(), np.abs(gy).max(), 1e-9)
    n = np.stack([-k * gx, -k * gy, np.ones_like(gx)], -1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    return ((n + 1) / 2).astype(np.float32)


def with_materials(batch: Batch, seed: int = 0, n_textures: int = 8, textured_prob: float = 0.7,
                   block_hsv=(0.08, 0.8, 0.8), block_radius=(0.04, 0.1, 0.1), n_normal_textures: int = 4,
                   normal_prob: float = 0.5) -> Batch:
    """The batch with randomized materials: each object gets, with probability
    textured_prob, one of n_textures random pattern textures and, with probability
    normal_prob, one of n_normal_textures normal textures, with tiling U[0.5, 4] and
    offset U[0, 1) per axis shared by both (MaterialRandomizer); each scene's last object
    (the hand scenes' block) is redrawn near a calibrated hue by the fixed-hue sampler,
    emissive with probability 0.2.  Draws come from default_rng([seed, 0x7E47, scene])."""
    pool_rng = np.random.default_rng([seed, 0x7E47])
    textures = [pattern_texture(pool_rng) for _ in range(n_textures)]
    textures += [bump_texture(pool_rng) for _ in range(n_normal_textures)]
    O = batch.n_objects
    tex = np.full(O, -1, np.int32)
    ntex = np.full(O, -1, np.int32)
    xf = np.tile(np.array([1, 1, 0, 0], np.float32), (O, 1))
    em = np.zeros(O, np.float32)
    alb = batch.albedo.copy()
    rough = batch.roughness.copy()
    spec = batch.specular.copy()
    for sc in range(batch.n_scenes):
        rng = np.random.default_rng([seed, 0x7E47, sc])
        ob, oe = int(batch.scene_object_begin[sc]), int(batch.scene_object_begin[sc + 1])
        for o in range(ob, oe):
            if rng.uniform() < textured_prob:
                tex[o] = int(rng.integers(0, n_textures))
            if n_normal_textures and rng.uniform() < normal_prob:
                ntex[o] = n_textures + int(rng.integers(0, n_normal_textures))
            if tex[o] >= 0 or ntex[o] >= 0:
                xf[o, :2] = rng.uniform(0.5, 4.0, 2)
                xf[o, 2:] = rng.uniform(0.0, 1.0, 2)
        if oe > ob:
            a, r, k, e = fixed_hue_material(rng, block_hsv, block_radius, emissive_prob=0.2, emissive_power=(0.1, 0.5))
            alb[oe - 1], rough[oe - 1], spec[oe - 1], em[oe - 1] = a, max(r, 0.05), k, e
    return batch.replace(textures=textures, object_texture=tex, tex_xform=xf, emission=em, albedo=alb,
                         roughness=rough, specular=spec, object_normal_texture=ntex if n_normal_textures else None)


# ----------------------------------------------------------------------------------
# spot lights with shadow maps (the paper's benchmark scene: three spot lights with
# soft shadows; LightRandomizer: intensities and spotlight angles; LightSetup:
# distance from and height above a target)
# ----------------------------------------------------------------------------------

SPOT_SHADOW_RES = 128


def spot_light(rng: np.random.Generator, target, res: int = SPOT_SHADOW_RES):
    """One spot light placed like LightSetup (horizontal distance U[0.4, 0.8] m, height
    U[0.3, 0.8] m, azimuth U[0, 2 pi) around the target), aimed at the target within
    +-3 cm, outer half-angle U[20, 35] deg, inner = outer * U[0.5, 0.9], intensity
    U[0.5, 2]; its shadow camera looks along the axis with a field of view of twice the
    outer angle plus 2 deg over an N x N map.  Returns (pos, axis, (cos inner, cos
    outer), intensity, view 3x4, intrinsics)."""
    target = np.asarray(target, float)
    az = rng.uniform(0, 2 * np.pi)
    rho = rng.uniform(0.4, 0.8)
    hgt = rng.uniform(0.3, 0.8)
    pos = target + np.array([rho * math.cos(az), rho * math.sin(az), hgt])
    aim = target + rng.uniform(-0.03, 0.03, 3)
    axis = (aim - pos) / np.linalg.norm(aim - pos)
    outer = math.radians(rng.uniform(20.0, 35.0))
    inner = outer * rng.uniform(0.5, 0.9)
    inten = rng.uniform(0.5, 2.0)
    C = look_at_c2w(pos, pos + axis, (0, 0, 1))
    view = view_from_c2w(C)
    K = intrinsics(res, res, 2 * math.degrees(outer) + 2.0)
    return pos, axis, (math.cos(inner), math.cos(outer)), inten, view, K


def with_spot_lights(batch: Batch, seed: int = 0, n_lights: int = 3, res: int = SPOT_SHADOW_RES,
                     target=None) -> Batch:
    """The batch with every scene's lights replaced by n_lights shadow-casting spot
    lights (type 2) aimed at `target` (default: the hand scenes' target).  Draws come
    from default_rng([seed, 0x5907, scene])."""
    tgt = HAND_TARGET if target is None else np.asarray(target, float)
    S_ = batch.n_scenes
    L = S_ * n_lights
    vec = np.zeros((L, 3)); inten = np.zeros(L); dirs = np.zeros((L, 3)); cone = np.zeros((L, 2))
    views = np.zeros((L, 3, 4)); intr = np.zeros((L, 4))
    for sc in range(S_):
        rng = np.random.default_rng([seed, 0x5907, sc])
        for k in range(n_lights):
            pos, axis, cs, I, V, K = spot_light(rng, tgt, res)
            l = sc * n_lights + k
            vec[l], dirs[l], cone[l], inten[l], views[l], intr[l] = pos, axis, cs, I, V, K
    f32 = lambda x: np.asarray(x, np.float64).astype(np.float32)
    return batch.replace(scene_light_begin=(np.arange(S_ + 1) * n_lights).astype(np.int32),
                         light_type=np.full(L, 2, np.int32), light_vec=f32(vec), light_intensity=f32(inten),
                         light_dir=f32(dirs), light_cone=f32(cone), shadow_view=f32(views), shadow_intr=f32(intr),
                         shadow_res=int(res))


# ----------------------------------------------------------------------------------
# config 3: uneven batch
# ----------------------------------------------------------------------------------

C3_CAPSULES = [(S, T) for S in (8, 16, 32) for T in (4, 8, 16)]
C3_BOXES = (1, 2, 4, 8, 16)
C3_RES = (64, 128, 200, 256)


def config3_meshes() -> List[Mesh]:
    return [capsule_mesh(0.012, 0.04, S, T) for S, T in C3_CAPSULES] + [box_mesh(n) for n in C3_BOXES]


def config3(seed: int = 3, n_scenes: int = 1024, n_cams: int = 3, min_tris: float = 2000,
            max_tris: float = 50000, res_choices=C3_RES) -> Batch:
    """Uneven batch: per-scene resolution from {64,128,200,256}^2 and a target triangle
    count log-uniform in [2k, 50k], filled with procedurally tessellated capsules
    (S in {8,16,32}, T in {4,8,16}) and subdivided boxes (n in {1,2,4,8,16}) posed in a
    0.3 m box; randomization as config 2."""
    meshes = config3_meshes()
    b = _Builder(meshes)
    nc = len(C3_CAPSULES)
    for s in range(n_scenes):
        rng = np.random.default_rng([seed, s])
        res = int(rng.choice(res_choices))
        target = math.exp(rng.uniform(math.log(min_tris), math.log(max_tris)))
        tris, k = 0, 0
        while tris < target:
            if rng.random() < 0.7:
                m = int(rng.integers(0, nc))
                scale = rng.uniform(0.6, 1.4)
            else:
                m = nc + int(rng.integers(0, len(C3_BOXES)))
                scale = rng.uniform(0.02, 0.06)
            R = uniform_rotation(rng)
            t = HAND_TARGET + rng.uniform(-0.15, 0.15, 3)
            b.add_object(m, make_pose(R, t, scale), k, rng.uniform(0, 1, 3), rng.uniform(0.05, 1.0), rng.uniform(0, 1))
            tris += meshes[m].n_tris
            k += 1
        for _ in range(int(rng.integers(1, 5))):
            az, rho, hgt = rng.uniform(0, 2 * np.pi), rng.uniform(0.4, 0.8), rng.uniform(0.3, 0.8)
            b.add_light(0, HAND_TARGET + np.array([rho * math.cos(az), rho * math.sin(az), hgt]), rng.uniform(0.5, 2.0))
        b.end_scene()
        for c in range(n_cams):
            az, el = math.radians(120.0 * c), math.radians(25.0)
            eye = HAND_TARGET + 0.6 * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
            C = jitter_c2w(look_at_c2w(eye, HAND_TARGET, (0, 0, 1)), rng, 0.02, 3.0)
            b.add_frame(view_from_c2w(C), intrinsics(res, res), res, res, rng.uniform(0.7, 1.3))
    return b.build(f"config3[{n_scenes}]")


# ----------------------------------------------------------------------------------
# config 4: targets with perturbed materials and lights
# ----------------------------------------------------------------------------------


def config4(seed: int = 4, n_scenes: int = 64, res: int = 200):
    """Differentiable-shading workload: config-2 scenes and a copy whose materials,
    lights and exposures are perturbed (albedo + N(0, 0.05) clipped to [0,1];
    roughness x U[0.8,1.2] clipped to [0.05,1]; light position + N(0, 0.05 m);
    intensity x U[0.8,1.2]; exposure x U[0.9,1.1]).  Returns (batch, target_batch)."""
    base = config2(seed, n_scenes, res)
    rng = np.random.default_rng([seed, 0x7A6])
    alb = np.clip(base.albedo + rng.normal(0, 0.05, base.albedo.shape), 0, 1)
    rough = np.clip(base.roughness * rng.uniform(0.8, 1.2, base.roughness.shape), 0.05, 1.0)
    lpos = base.light_vec + rng.normal(0, 0.05, base.light_vec.shape)
    inten = base.light_intensity * rng.uniform(0.8, 1.2, base.light_intensity.shape)
    expo = base.exposure * rng.uniform(0.9, 1.1, base.exposure.shape)
    target = base.replace(albedo=alb.astype(np.float32), roughness=rough.astype(np.float32),
                          light_vec=lpos.astype(np.float32), light_intensity=inten.astype(np.float32),
                          exposure=expo.astype(np.float32), name=base.name + "[target]")
    return base, target


# ----------------------------------------------------------------------------------
# config 5: serving requests
# ----------------------------------------------------------------------------------

C5_RES = (64, 128, 200)


def config5_requests(seed: int = 5, rate: float = 2000.0, duration: float = 10.0,
                     warmup: float = 1.0, max_scenes: int = 32):
    """Poisson arrivals at ``rate`` req/s over warmup + duration seconds; each request
    holds U{1..32} config-2 scenes (3 cameras) at a resolution from {64,128,200}^2.
    Returns a list of (arrival_time_s, n_scenes, res, first_scene_id)."""
    rng = np.random.default_rng([seed, 0xA771])
    t, out, sid = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > warmup + duration:
            break
        n = int(rng.integers(1, max_scenes + 1))
        res = int(rng.choice(C5_RES))
        out.append((t, n, res, sid))
        sid += n
    return out


def config5_request_batch(n_scenes: int, res: int, first_scene: int, seed: int = 5) -> Batch:
    return config2(seed, n_scenes, res, scene_ids=range(first_scene, first_scene + n_scenes))


# ----------------------------------------------------------------------------------
# small fixtures for tests
# ----------------------------------------------------------------------------------


def single_object_batch(mesh: Mesh, pose, *, res=(64, 64), view=None, intr=None,
                        albedo=(0.5, 0.5, 0.5), rough=1.0, spec=0.0, lights=((1, (0, 0, -1), 1.0),),
                        exposure=1.0, near=0.01, seg=7, fov=45.0, extra_objects=()) -> Batch:
    """One scene holding ``mesh`` (and optional extra (mesh_index, pose) objects sharing
    the same mesh list), one frame.  Default camera: identity view (camera at the
    origin looking down -z)."""
    meshes = [mesh] + [m for m, _ in extra_objects]
    b = _Builder(meshes)
    b.add_object(0, np.asarray(pose, float), seg, albedo, rough, spec)
    for k, (_, p) in enumerate(extra_objects):
        b.add_object(k + 1, np.asarray(p, float), seg + 1 + k, albedo, rough, spec)
    for lt, v, inten in lights:
        b.add_light(lt, v, inten)
    b.end_scene()
    W, H = res
    V = np.hstack([np.eye(3), np.zeros((3, 1))]) if view is None else np.asarray(view, float)
    K = intrinsics(W, H, fov) if intr is None else np.asarray(intr, float)
    b.add_frame(V, K, W, H, exposure, near)
    return b.build("fixture")
