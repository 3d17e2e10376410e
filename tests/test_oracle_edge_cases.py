"""Pins of the oracle's edge cases (CPU only): the guard band, the clamp of the
point-light distance, a directional light seen through a rotated camera (and the
gradients of directional lights), and the second-nearest depth that decides which
pixels are near-ties.

Each case is checked against brute-force ray casting or a closed form written in
world space, and is built so that the plausible mistake named in its docstring
fails it.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import brute

ID34 = np.hstack([np.eye(3), np.zeros((3, 1))])
GUARD = 1 << 24  # sub-pixel units (65,536 px)


# ---------------------------------------------------------------------------------
# guard band
# ---------------------------------------------------------------------------------


def guard_batch(axis: str, far_sub: int):
    """One front-facing triangle, two corners on a 16x16 screen, the third at snapped
    coordinate ``far_sub`` (1/256 px) along ``axis`` ('x': screen x, 'y': screen y,
    down).  Intrinsics (32, 32, 8, 8), eye depth 2: for |far_sub| <= 2^24 + 1 every
    view-space coordinate is an fp32 number and every step of the projection is exact,
    so the snapped coordinate is exactly ``far_sub``."""
    fx = fy = 32.0
    cx = cy = 8.0
    w = 2.0
    X = lambda sub: (sub - 256 * cx) / (256 * fx) * w    # sx = sub / 256
    Y = lambda sub: -(sub - 256 * cy) / (256 * fy) * w
    sub = lambda px: int(round(px * 256))
    near = sub(2.5) if far_sub > 0 else sub(13.5)  # the edge the wedge grows from
    if axis == "x":
        a, b, c = (near, sub(2.5)), (near, sub(12.5)), (far_sub, sub(12.5))
    else:
        a, b, c = (sub(2.5), near), (sub(12.5), near), (sub(2.5), far_sub)
    # front-facing: negative signed area on the y-down screen
    if (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]) > 0:
        b, c = c, b
    pos = np.array([[X(p[0]), Y(p[1]), -w] for p in (a, b, c)])
    mesh = S.Mesh(pos.astype(np.float32), np.tile([0, 0, 1.0], (3, 1)).astype(np.float32),
                  np.array([[0, 1, 2]], np.int32))
    assert np.array_equal(mesh.pos.astype(np.float64), pos), "guard fixture is not exactly representable"
    return S.single_object_batch(mesh, ID34, res=(16, 16), intr=(fx, fy, cx, cy))


GUARD_CASES = [("x", GUARD, True), ("x", GUARD + 1, False), ("y", GUARD, True), ("y", GUARD + 1, False),
               ("x", -60000 * 256, True), ("x", -70000 * 256, False),
               ("y", -60000 * 256, True), ("y", -70000 * 256, False)]


@pytest.mark.parametrize("axis,far_sub,kept", GUARD_CASES)
def test_guard_band_discards_triangles_beyond_65536_px(axis, far_sub, kept):
    """A vertex whose snapped |X| or |Y| exceeds 2^24 (65,536 px) discards its
    triangle, although the triangle covers pixels on screen; at exactly 2^24 it is
    kept and its coverage is the ray-cast coverage.  Exact boundary cases on the
    positive side pin the constant and the inclusive compare; far cases on the
    negative side pin the absolute value.  Mistakes caught: no guard, a guard in
    pixels instead of sub-pixels, a strict compare, a one-sided compare, X tested
    without Y."""
    b = guard_batch(axis, far_sub)
    out = oracle.render(b)
    ref = brute.cast(b, 0)
    hit = ref["tri"] >= 0
    assert hit.sum() >= 20  # the triangle does cover part of the screen
    tri = out["tri_id"]
    if not kept:
        assert np.all(tri == -1)
        return
    band = brute.edge_dist(b, 0) <= 2.0 / 256
    assert np.array_equal(tri[~band] >= 0, hit[~band])
    assert (tri >= 0).sum() >= 20


# ---------------------------------------------------------------------------------
# point light within 1 cm of a surface: A = I / max(|d|^2, 1e-4)
# ---------------------------------------------------------------------------------


def clamp_batch(k_s=0.0):
    """A camera-facing plane 0.1 m from the eye (64 px across 8.3 cm) lit by a point
    light 4 mm in front of it: pixels within 9.2 mm of the light's foot have
    |d|^2 < 1e-4 m^2."""
    q = (0.003, -0.002, -0.1 + 0.004)
    return S.single_object_batch(S.plane_mesh(4, 4, 4.0, 4.0), S.make_pose(np.eye(3), (0.0, 0.0, -0.1)), res=(64, 64),
                                 albedo=(0.5, 0.7, 0.2), spec=k_s, rough=1.0, lights=((0, q, 0.01),), exposure=1.3)


def _clamp_geometry(b, out):
    p = brute.pixel_rays(b, 0) * out["depth"][:, None]
    q = b.light_vec[0].astype(np.float64)
    d = q - p
    D = (d * d).sum(1)
    return p, d, D


def test_point_light_distance_clamp_closed_form():
    """rgb = e * I * albedo * max(0, n.l) / max(|d|^2, 1e-4) on a Lambertian plane
    whose point light is 4 mm away: about 150 pixels sit in the clamped region, where
    the unclamped falloff would be larger by up to 6x.  Mistakes caught: no clamp, the
    clamp on |d| instead of |d|^2, a different epsilon."""
    b = clamp_batch()
    out = oracle.render(b)
    assert np.all(out["tri_id"] >= 0)
    _, d, D = _clamp_geometry(b, out)
    n = np.array([0.0, 0.0, 1.0])
    ndl = np.maximum(0.0, d @ n / np.sqrt(D))
    e, I = float(b.exposure[0]), float(b.light_intensity[0])
    alb = b.albedo[0].astype(np.float64)
    expect = e * I * ndl[:, None] * alb[None] / np.maximum(D, 1e-4)[:, None]
    rgb = oracle.frame_view(out["rgb"], out["pixel_offset"], 0, 64, 64, 3).reshape(3, -1).T
    np.testing.assert_allclose(rgb, expect, rtol=1e-10)
    clamped = D < 1e-4
    assert 100 <= clamped.sum() <= 250
    unclamped = e * I * ndl[:, None] * alb[None] / D[:, None]
    assert np.all(np.abs(unclamped[clamped] - rgb[clamped]) > 1e-3 * rgb[clamped])
    # the light sits 4 mm from the plane: the clamp changes the brightest pixel by 6x
    assert unclamped[clamped].max() / rgb[clamped].max() > 5.0


def _linear_fd(b, c, w3, name, idx, h):
    from tests import fd
    lp = (c * w3 * oracle.render(fd.perturbed(b, name, idx, h))["rgb"]).sum()
    lm = (c * w3 * oracle.render(fd.perturbed(b, name, idx, -h))["rgb"]).sum()
    return (lp - lm) / (2 * h)


def _planar3(b, mask):
    return np.concatenate([np.tile(mask[b.pixel_offset[f]:b.pixel_offset[f + 1]], 3)
                           for f in range(b.n_frames)]).astype(np.float64)


@pytest.mark.parametrize("k_s", [0.0, 0.5])
def test_point_light_clamp_gradient_matches_differences(k_s):
    """Inside the clamp A = I / 1e-4 does not depend on the light position, so the
    adjoint drops dA/dd there.  Central differences of the linear loss sum c . rgb
    (two forward renders, no adjoint code) agree with the adjoint on the light's
    position and intensity; pixels whose |d|^2 is within the step of 1e-4 are held
    out.  Mistakes caught: dA/dd kept in the clamped region, dA/dI = 1/|d|^2 there."""
    b = clamp_batch(k_s)
    out = oracle.render(b)
    _, _, D = _clamp_geometry(b, out)
    mask = (np.abs(D - 1e-4) > 1e-7).astype(np.uint8)
    assert mask.sum() > 4000 and (mask.astype(bool) & (D < 1e-4)).sum() > 100
    c = np.random.default_rng(5).uniform(-1, 1, 3 * b.total_pixels)
    _, g = oracle.shade_grad(b, dl_drgb=c, pixel_weight=mask)
    w3 = _planar3(b, mask)
    for name, idx in (("light_vec", 0), ("light_vec", 1), ("light_vec", 2), ("light_intensity", 0)):
        a = g[name].reshape(-1)[idx]
        dfd = _linear_fd(b, c, w3, name, idx, 1e-6)
        assert abs(a - dfd) <= 1e-6 * abs(dfd) + 1e-9, (name, idx, a, dfd)


# ---------------------------------------------------------------------------------
# directional light through a rotated camera
# ---------------------------------------------------------------------------------


def _rotated_camera():
    c = np.array([0.2, -0.1, 0.3])
    C = S.look_at_c2w(np.array([0.9, -2.4, 1.6]), c, (0, 0, 1))
    V = S.view_from_c2w(C)
    return c, V


# a direction that mirrors the eye about the plane near its centre (a highlight)
MIRROR_U = (0.542, -2.326, 0.237)


def directional_batch(k_s, rough, lights=None, u=(0.9, 1.8, -1.3)):
    Rw = S.rot_axis("z", 0.4) @ S.rot_axis("x", -0.3)
    c, V = _rotated_camera()
    if lights is None:
        lights = ((1, u, 1.7),)
    return S.single_object_batch(S.plane_mesh(4, 4, 4.0, 4.0), S.make_pose(Rw, c), res=(48, 40), view=V,
                                 albedo=(0.9, 0.4, 0.15), spec=k_s, rough=rough, lights=lights, exposure=1.2)


def _world_terms(b, out):
    """World-space n (plane normal), camera centre o, and per-pixel hit points."""
    P = b.object_pose[0].astype(np.float64)
    n = P[:, :3] @ [0, 0, 1.0]
    n /= np.linalg.norm(n)
    V = b.view[0].astype(np.float64)
    Rc = V[:, :3].T
    o = -Rc @ V[:, 3]
    pw = o + (brute.pixel_rays(b, 0) * out["depth"][:, None]) @ Rc.T
    return n, o, pw


def test_directional_light_rotated_camera_lambert():
    """A Lambertian plane under a directional light, seen through a LookAt camera
    whose rotation is far from symmetric: rgb = e * I * albedo * max(0, n . -u/|u|),
    all in world space, on every covered pixel.  Mistakes caught: R_V transposed in
    the light's view-space direction, a missing sign, a missing normalization."""
    b = directional_batch(0.0, 1.0)
    out = oracle.render(b)
    cov = out["tri_id"] >= 0
    assert cov.mean() > 0.3
    n, _, _ = _world_terms(b, out)
    u = b.light_vec[0].astype(np.float64)
    l = -u / np.linalg.norm(u)
    ndl = n @ l
    assert ndl > 0.3
    expect = float(b.exposure[0]) * float(b.light_intensity[0]) * b.albedo[0].astype(np.float64) * ndl
    rgb = oracle.frame_view(out["rgb"], out["pixel_offset"], 0, 48, 40, 3).reshape(3, -1).T
    # the fp32 view rotation is orthonormal only to ~1e-7
    np.testing.assert_allclose(rgb[cov], np.tile(expect, (cov.sum(), 1)), rtol=1e-6)
    # the same plane with the light direction rotated by R_V^T instead of R_V
    R = b.view[0].astype(np.float64)[:, :3]
    wrong = -(R.T @ R.T @ u)
    wrong /= np.linalg.norm(wrong)
    assert abs(n @ wrong - ndl) > 0.05


def test_directional_light_rotated_camera_specular():
    """With a highlight: rgb = e * I * (n.l) * (albedo + k_s * (n.h)^m), h the unit
    bisector of l and the direction to the eye, computed in world space from the
    pixel's hit point; the exponent m = 2/r^2 - 2 makes the highlight sensitive to any
    error in l."""
    b = directional_batch(0.6, 0.3, u=MIRROR_U)
    out = oracle.render(b)
    cov = out["tri_id"] >= 0
    n, o, pw = _world_terms(b, out)
    u = b.light_vec[0].astype(np.float64)
    l = -u / np.linalg.norm(u)
    v = o - pw[cov]
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    h = l + v
    h /= np.linalg.norm(h, axis=1, keepdims=True)
    ndh = np.maximum(0.0, h @ n)
    r = float(b.roughness[0])
    m = 2 / r ** 2 - 2
    s = ndh ** m
    e, I, ks = float(b.exposure[0]), float(b.light_intensity[0]), float(b.specular[0])
    expect = e * I * (n @ l) * (b.albedo[0].astype(np.float64)[None] + ks * s[:, None])
    rgb = oracle.frame_view(out["rgb"], out["pixel_offset"], 0, 48, 40, 3).reshape(3, -1).T
    np.testing.assert_allclose(rgb[cov], expect, rtol=2e-5)
    assert (s * ks).max() > 0.05  # the highlight is in the frame


def test_directional_and_point_gradients_rotated_camera():
    """Gradients of a directional light's direction and intensity and of a point
    light's position, through the rotated camera, against central differences of
    the linear loss sum c . rgb (two forward renders, no adjoint code).  |u| = 2.4,
    so the 1/|a| factor of the normalization matters.  Mistakes caught: a missing
    tangent projection (I - l l^T), a missing 1/|a|, R_V instead of R_V^T on the way
    back, a sign."""
    from tests import fd
    lights = ((1, MIRROR_U, 1.1), (0, (0.5, -0.9, 1.2), 1.6))
    b = directional_batch(0.6, 0.3, lights=lights)
    out = oracle.render(b)
    mask = fd.smooth_mask(b, out)
    assert mask.mean() > 0.98
    c = np.random.default_rng(9).uniform(-1, 1, 3 * b.total_pixels)
    _, g = oracle.shade_grad(b, dl_drgb=c, pixel_weight=mask)
    w3 = _planar3(b, mask)
    gl = g["light_vec"].reshape(-1)
    assert np.abs(gl[:3]).max() > 1e-2  # the direction gradient is not the silent zero
    for name, idx in [("light_vec", k) for k in range(6)] + [("light_intensity", 0), ("light_intensity", 1)]:
        a = g[name].reshape(-1)[idx]
        dfd = _linear_fd(b, c, w3, name, idx, 1e-5)
        assert abs(a - dfd) <= 1e-6 * abs(dfd) + 1e-8 * np.abs(gl).max(), (name, idx, a, dfd)


# ---------------------------------------------------------------------------------
# second-nearest depth (near-tie classification)
# ---------------------------------------------------------------------------------


def stacked_planes(order, rel_gap):
    """Three camera-facing planes: the nearest at 2 m, the second at 2 (1 + rel_gap),
    the third at 3 m, drawn in ``order`` (indices into near, second, third)."""
    depths = [2.0, 2.0 * (1.0 + rel_gap), 3.0]
    mesh = S.plane_mesh(2, 2, 4.0, 4.0)
    poses = [S.make_pose(np.eye(3), (0.0, 0.0, -depths[k])) for k in order]
    return S.single_object_batch(mesh, poses[0], res=(24, 20), extra_objects=[(mesh, p) for p in poses[1:]])


@pytest.mark.parametrize("order", [(1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 2, 1)])
@pytest.mark.parametrize("rel_gap", [3e-6, 3e-5])
def test_second_nearest_depth_and_near_ties(order, rel_gap):
    """The oracle's second-nearest depth equals the brute-force second hit (the second
    plane, not the third) whatever order the planes are drawn in, and a pixel is a
    near-tie iff that gap is within 1e-5 relative.  Mistakes caught: d2 not taking the
    old d1 when a nearer fragment arrives, d2 overwritten by a farther fragment, an
    absolute instead of a relative threshold."""
    b = stacked_planes(order, rel_gap)
    out = oracle.render(b)
    ref = brute.cast(b, 0)
    cov = out["tri_id"] >= 0
    assert cov.all()
    # off shared edges (where the ray cast counts a plane twice, the fill rule once)
    ok = brute.edge_dist(b, 0) > 2.0 / 256
    assert ok.sum() > 400
    np.testing.assert_allclose(out["depth"][ok], ref["depth"][ok], rtol=1e-12)
    np.testing.assert_allclose(out["depth2"][ok], ref["depth2"][ok], rtol=1e-12)
    d2 = -float(np.float32(b.object_pose[order.index(1)][2, 3]))  # the second plane's fp32 depth
    np.testing.assert_allclose(out["depth2"], d2, rtol=1e-12)
    assert np.all(out["frag_count"] == 3)
    d1 = out["depth"]
    expect_tie = (d2 - d1) <= 1e-5 * d1
    assert bool(expect_tie.all()) == (rel_gap < 1e-5)
    assert np.array_equal(oracle.near_tie(out), expect_tie)
    # the nearest plane wins: its object's segmentation id
    assert np.all(out["seg"] == 7 + order.index(0))
