"""Pins of the oracle's spot lights with shadow maps (CPU only): the paper's benchmark
scene uses spot lights with soft shadows (Sec. 5), and the LightRandomizer draws
spotlight angles (Sec. 4.3.1).  A ground plane under a spot light, with and without a
square occluder between them, against geometry computed here: the occluder's shadow is
its central projection from the light, the cone's inside matches the point light, its
outside is dark, and the filtered edge is soft."""
import math

import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S

LIGHT_H = 2.0     # light height above the ground plane (z = 0)
OCC_H = 1.0       # occluder height
OCC_SIDE = 0.4    # occluder side: its shadow on the ground has side OCC_SIDE * LIGHT_H / (LIGHT_H - OCC_H)
N = 128           # shadow map size


def _scene(occluder=True, inner_deg=30.0, outer_deg=38.0, res=(96, 96), light_xy=(0.0, 0.0), ground_side=4.0):
    ground = S.plane_mesh(16, 16, ground_side, ground_side)
    occ = S.plane_mesh(2, 2, OCC_SIDE, OCC_SIDE)
    extra = [(occ, S.make_pose(np.eye(3), (0.0, 0.0, OCC_H)))] if occluder else []
    C = S.look_at_c2w((0.0, -0.8, 3.2), (0.0, 0.0, 0.0), (0, 0, 1))
    b = S.single_object_batch(ground, S.make_pose(np.eye(3), (0.0, 0.0, 0.0)), res=res, view=S.view_from_c2w(C),
                              albedo=(0.8, 0.6, 0.4), lights=((0, (0, 0, 0), 1.0),), extra_objects=extra)
    pos = np.array([light_xy[0], light_xy[1], LIGHT_H])
    axis = np.array([0.0, 0.0, -1.0])
    Cs = S.look_at_c2w(pos, pos + axis, (0, 1, 0))
    f32 = lambda x: np.asarray(x, np.float64).astype(np.float32)
    return b.replace(light_type=np.array([2], np.int32), light_vec=f32([pos]), light_intensity=f32([3.0]),
                     light_dir=f32([axis]),
                     light_cone=f32([[math.cos(math.radians(inner_deg)), math.cos(math.radians(outer_deg))]]),
                     shadow_view=f32([S.view_from_c2w(Cs)]), shadow_intr=f32([S.intrinsics(N, N, 2 * outer_deg + 2)]),
                     shadow_res=N)


def _ground_points(b, out):
    """World position of every covered ground pixel (ray from the camera to z = 0) and
    the pixel's rgb."""
    W, H = int(b.width[0]), int(b.height[0])
    V = b.view[0].astype(np.float64)
    fx, fy, cx, cy = b.intr[0].astype(np.float64)
    Rc, cam = V[:, :3].T, -V[:, :3].T @ V[:, 3]
    j, i = np.mgrid[0:H, 0:W]
    d = np.stack([(i + 0.5 - cx) / fx, -(j + 0.5 - cy) / fy, -np.ones_like(i, float)], -1) @ Rc.T
    t = -cam[2] / d[..., 2]
    P = cam + t[..., None] * d
    rgb = oracle.frame_view(out["rgb"], out["pixel_offset"], 0, W, H, 3).transpose(1, 2, 0)
    obj = out["obj_id"].reshape(H, W)
    return P, rgb, obj


def test_occluder_shadow_is_its_central_projection():
    """Ground points whose shadow-map neighbourhood lies well inside the occluder's
    projected square are black; those well outside it (and inside the inner cone) get
    the unoccluded light."""
    b = _scene(occluder=True)
    out = oracle.render(b)
    free = oracle.render(_scene(occluder=False))
    P, rgb, obj = _ground_points(b, out)
    _, rgb_free, _ = _ground_points(b, free)
    half = 0.5 * OCC_SIDE * LIGHT_H / (LIGHT_H - OCC_H)
    texel = 2 * LIGHT_H * math.tan(math.radians(39.0)) / N  # ground size of a shadow-map texel
    ground = obj == 0
    m = np.maximum(np.abs(P[..., 0]), np.abs(P[..., 1]))
    inside = ground & (m < half - 3 * texel)
    outside = ground & (m > half + 3 * texel) & (np.hypot(P[..., 0], P[..., 1]) < LIGHT_H * math.tan(math.radians(29)))
    assert inside.sum() > 100 and outside.sum() > 300
    assert np.all(rgb[inside] == 0)
    np.testing.assert_allclose(rgb[outside], rgb_free[outside], rtol=1e-12)
    assert np.all(rgb_free[inside] > 0)


def test_soft_shadow_edge_takes_intermediate_values():
    """3 x 3 filtering: along the shadow's edge the light arrives in fractions k/9."""
    b = _scene(occluder=True)
    out = oracle.render(b)
    free = oracle.render(_scene(occluder=False))
    P, rgb, obj = _ground_points(b, out)
    _, rgb_free, _ = _ground_points(b, free)
    ok = (obj == 0) & (rgb_free[..., 0] > 1e-6)
    ratio = rgb[..., 0][ok] / rgb_free[..., 0][ok]
    k = ratio * 9
    assert np.allclose(k, np.round(k), atol=1e-9)  # multiples of 1/9
    assert ((k > 0.5) & (k < 8.5)).sum() > 20        # a soft edge, not a hard step


def test_spot_cone_inside_equals_point_light_outside_dark():
    """Without occluder: inside the inner cone the spot light is the point light; beyond
    the outer cone it is dark; in between it lies between the two and falls off
    outward."""
    b = _scene(occluder=False, inner_deg=12.0, outer_deg=20.0, res=(128, 128))
    out = oracle.render(b)
    pt = oracle.render(b.replace(light_type=np.array([0], np.int32)))
    P, rgb, obj = _ground_points(b, out)
    _, rgb_pt, _ = _ground_points(b, pt)
    ang = np.degrees(np.arctan2(np.hypot(P[..., 0], P[..., 1]), LIGHT_H))
    g = obj == 0
    inner, outer = g & (ang < 11.5), g & (ang > 20.5)
    mid = g & (ang > 12.5) & (ang < 19.5)
    assert inner.sum() > 200 and outer.sum() > 200 and mid.sum() > 200
    np.testing.assert_allclose(rgb[inner], rgb_pt[inner], rtol=1e-12)
    assert np.all(rgb[outer] == 0)
    r = rgb[..., 0][mid] / rgb_pt[..., 0][mid]
    assert np.all((r > 0) & (r < 1))
    order = np.argsort(ang[mid])
    assert np.all(np.diff(r[order]) <= 1e-12)  # falls off with the angle


def test_lone_plane_is_fully_lit_and_cone_is_smoothstep():
    """A plane smaller than the light's footprint, alone: it only meets itself in the
    shadow map (within the bias) and empty texels beyond its edges, so every pixel gets
    the full light; inside the inner cone the spot light is the point light, and
    between the cones it is the point light times smoothstep of the cosine of the angle
    to the axis between the two cone cosines."""
    inner, outer = 10.0, 25.0
    b = _scene(occluder=False, inner_deg=inner, outer_deg=outer, res=(128, 128), ground_side=1.2)
    out = oracle.render(b)
    pt = oracle.render(b.replace(light_type=np.array([0], np.int32)))
    P, rgb, obj = _ground_points(b, out)
    _, rgb_pt, _ = _ground_points(b, pt)
    g = (obj == 0) & (rgb_pt[..., 0] > 0)
    c = LIGHT_H / np.sqrt(P[..., 0] ** 2 + P[..., 1] ** 2 + LIGHT_H ** 2)  # cos of the angle to the axis
    ci, co = np.cos(np.radians(inner)), np.cos(np.radians(outer))
    t = np.clip((c - np.float32(co)) / (np.float32(ci) - np.float32(co)), 0, 1)
    expect = rgb_pt[..., 0] * t * t * (3 - 2 * t)
    assert g.sum() > 2000 and (g & (t > 0.05) & (t < 0.95)).sum() > 300
    # the shaded point comes from snapped vertices: within ~1e-5 of the exact ray hit
    np.testing.assert_allclose(rgb[..., 0][g], expect[g], rtol=2e-4, atol=1e-12)


def test_shadow_map_is_the_depth_render_from_the_light():
    """The shadow frame of the occluder scene holds the occluder at its distance
    LIGHT_H - OCC_H and the ground at LIGHT_H, seen straight down."""
    b = _scene(occluder=True)
    out = oracle.render(b)
    z = out["shadow_depth"].reshape(N, N)
    assert np.allclose(z[N // 2 - 3:N // 2 + 3, N // 2 - 3:N // 2 + 3], LIGHT_H - OCC_H, rtol=1e-9)
    assert np.isclose(z[5, 5], LIGHT_H, rtol=1e-9)


def test_light_behind_a_ground_point_and_ambiguity_report():
    """Moving the light sideways (in x and y) moves the shadow by the projection ratio;
    the pixels the oracle reports as ambiguous lie along the shadow's edge only."""
    lx, ly = 0.3, 0.2
    b = _scene(occluder=True, light_xy=(lx, ly))
    out = oracle.render(b)
    P, rgb, obj = _ground_points(b, out)
    half = 0.5 * OCC_SIDE * LIGHT_H / (LIGHT_H - OCC_H)
    k = LIGHT_H / (LIGHT_H - OCC_H)
    cx, cy = lx - lx * k, ly - ly * k  # shadow centre: the occluder's centre projected from the light
    texel = 2 * LIGHT_H * math.tan(math.radians(39.0)) / N
    m = np.maximum(np.abs(P[..., 0] - cx), np.abs(P[..., 1] - cy))
    inside = (obj == 0) & (m < half - 3 * texel)
    assert inside.sum() > 100 and np.all(rgb[inside] == 0)
    amb = out["shadow_amb"].reshape(rgb.shape[:2]).astype(bool)
    far = (obj == 0) & ((m < half - 4 * texel) | (m > half + 4 * texel))
    assert amb.sum() < 0.1 * (obj == 0).sum() and not (amb & far & (rgb[..., 0] == 0)).any()


def test_adjoint_rejects_spot_lights():
    b = _scene(occluder=False)
    with pytest.raises(ValueError):
        oracle.shade_grad(b, np.zeros(3 * b.total_pixels))
