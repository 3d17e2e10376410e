"""Pins of the oracle's RGB channel (CPU only): closed forms of flat surfaces under
directional and point lights, the Blinn-Phong special cases, and linearity."""
import math

import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import brute

ID34 = np.hstack([np.eye(3), np.zeros((3, 1))])


def _plane_batch(R, c, res=(48, 40), **kw):
    return S.single_object_batch(S.plane_mesh(4, 4, 4.0, 4.0), S.make_pose(R, c, 1.0), res=res, **kw)


def _rgb(out, W, H):
    return oracle.frame_view(out["rgb"], out["pixel_offset"], 0, W, H, 3).reshape(3, -1).T


def test_lambert_plane_directional_light_is_constant():
    """A Lambertian plane (k_s = 0) under a directional light has
    rgb = e * I * albedo * max(0, n.l) on every covered pixel."""
    R = S.rot_axis("x", 0.35) @ S.rot_axis("y", 0.2)
    d = np.array([0.3, -0.5, -0.8])
    d /= np.linalg.norm(d)
    alb = (0.9, 0.4, 0.15)
    b = _plane_batch(R, (0.1, -0.1, -3.0), albedo=alb, lights=((1, d, 1.7),), exposure=1.2)
    out = oracle.render(b)
    rgb = _rgb(out, 48, 40)
    cov = out["tri_id"] >= 0
    assert cov.mean() > 0.5
    n = b.object_pose[0].astype(np.float64)[:, :3] @ [0, 0, 1.0]
    n /= np.linalg.norm(n)
    l = -b.light_vec[0].astype(np.float64)
    l /= np.linalg.norm(l)
    expect = float(b.exposure[0]) * float(b.light_intensity[0]) * np.asarray(b.albedo[0], np.float64) * max(0.0, n @ l)
    np.testing.assert_allclose(rgb[cov], np.tile(expect, (cov.sum(), 1)), rtol=1e-12)
    assert np.all(rgb[~cov] == 0)


def test_lambert_plane_point_light_closed_form():
    """Under a point light: rgb(p) = e * I * albedo * n.(q - p) / |q - p|^3 with p the
    exact ray-plane hit, all in world space through a general camera, within the
    depth error that snapping allows."""
    Rw = S.rot_axis("z", 0.4) @ S.rot_axis("x", -0.3)
    c = np.array([0.2, -0.1, 0.3])
    eye = np.array([0.9, -2.4, 1.6])
    C = S.look_at_c2w(eye, c, (0, 0, 1))
    q = np.array([-0.6, -1.2, 1.9])
    b = _plane_batch(Rw, c, view=S.view_from_c2w(C), albedo=(0.5, 0.7, 0.2), lights=((0, q, 2.0),), exposure=0.9)
    out = oracle.render(b)
    rgb = _rgb(out, 48, 40)
    P = b.object_pose[0].astype(np.float64)
    n = P[:, :3] @ [0, 0, 1.0]
    n /= np.linalg.norm(n)
    V = b.view[0].astype(np.float64)
    Rc = V[:, :3].T                       # camera-to-world rotation
    o = -Rc @ V[:, 3]                     # camera centre in world space
    r = brute.pixel_rays(b, 0) @ Rc.T     # world-space ray directions
    e, I = float(b.exposure[0]), float(b.light_intensity[0])

    def shade(t):
        p = o + r * t[:, None]
        d = b.light_vec[0].astype(np.float64) - p
        dist = np.linalg.norm(d, axis=1)
        cosl = np.maximum(0, d @ n / dist)
        return e * I * cosl[:, None] * np.asarray(b.albedo[0], np.float64)[None] / dist[:, None] ** 2

    cov = out["tri_id"] >= 0
    assert cov.mean() > 0.3
    # 1) at the rasterized depth (pinned by the tilted-plane test): equal up to the
    # fp32 view matrix not being exactly orthonormal (~1e-7 relative)
    dep = out["depth"]
    np.testing.assert_allclose(rgb[cov], shade(dep)[cov], rtol=1e-6, atol=1e-14)
    # 2) at the exact ray-plane hit: within what the snapped depth error allows
    t = (n @ (P[:, 3] - o)) / (r @ n)
    band = brute.edge_dist(b, 0) <= 2.0 / 256
    ok = cov & ~band
    rel_dz = np.abs(dep[ok] - t[ok]) / t[ok]
    tt = t.reshape(40, 48)
    snap_bound = 4 * (np.abs(np.diff(tt, axis=1)).max() + np.abs(np.diff(tt, axis=0)).max()) / 512
    assert np.abs(dep[ok] - t[ok]).max() <= snap_bound
    ref = shade(t)[ok]
    np.testing.assert_allclose(rgb[ok], ref, rtol=0, atol=np.abs(ref).max() * 10 * rel_dz.max() + 1e-12)


def test_mirror_highlight_independent_of_roughness():
    """Plane facing the camera, directional light from the eye, pixel on the optical
    axis: n = l = v, so n.h = 1 and the highlight is 1 for any roughness:
    rgb = e * I * (albedo + k_s)."""
    res = 33
    intr = (40.0, 40.0, 16.5, 16.5)  # pixel 16's centre sits on the optical axis
    for rough in (0.05, 0.3, 1.0):
        b = _plane_batch(np.eye(3), (0, 0, -2.0), res=(res, res), intr=intr, albedo=(0.2, 0.3, 0.4),
                         rough=rough, spec=0.7, lights=((1, (0, 0, -1), 1.5),), exposure=1.1)
        out = oracle.render(b)
        rgb = _rgb(out, res, res).reshape(res, res, 3)
        expect = float(b.exposure[0]) * float(b.light_intensity[0]) * (b.albedo[0].astype(np.float64) + float(b.specular[0]))
        np.testing.assert_allclose(rgb[16, 16], expect, rtol=1e-12)


@pytest.mark.parametrize("theta", [0.2, 0.5, 0.9])
@pytest.mark.parametrize("rough", [0.08, 0.4])
def test_off_mirror_highlight_half_angle(theta, rough):
    """On the optical axis (v = n = +z) with a directional light at angle theta from n:
    h bisects l and v, so n.h = cos(theta/2) and
    rgb = e * I * cos(theta) * (albedo + k_s * cos(theta/2)^m), m = 2/r^2 - 2."""
    res = 33
    intr = (40.0, 40.0, 16.5, 16.5)
    dirn = -np.array([math.sin(theta), 0.0, math.cos(theta)])  # light travels along dirn
    b = _plane_batch(np.eye(3), (0, 0, -2.0), res=(res, res), intr=intr, albedo=(0.2, 0.6, 0.1),
                     rough=rough, spec=0.8, lights=((1, dirn, 1.3),))
    out = oracle.render(b)
    rgb = _rgb(out, res, res).reshape(res, res, 3)[16, 16]
    d = b.light_vec[0].astype(np.float64)
    l = -d / np.linalg.norm(d)
    th = math.acos(l[2])  # the fp32-stored direction's own angle
    r = float(b.roughness[0])
    m = 2 / r ** 2 - 2
    expect = float(b.light_intensity[0]) * math.cos(th) * (b.albedo[0].astype(np.float64) + float(b.specular[0]) * math.cos(th / 2) ** m)
    np.testing.assert_allclose(rgb, expect, rtol=1e-10)


def test_roughness_one_is_lambert_with_albedo_plus_specular():
    """r = 1 gives m = 0, so the highlight is 1 wherever n.h > 0: the image equals a
    Lambert render with albedo a + k_s."""
    b = S.config1(n_scenes=2, materials=True)
    ks = np.full(b.specular.shape, 0.6)  # FP64 shading parameters
    b1 = b.replace(roughness=np.ones_like(b.roughness), specular=ks)
    b2 = b.replace(roughness=np.ones_like(b.roughness), specular=np.zeros_like(ks),
                   albedo=(b.albedo.astype(np.float64) + 0.6))
    o1, o2 = oracle.render(b1), oracle.render(b2)
    # pixels whose every light has n.h > 0 (true for these camera-facing lights)
    np.testing.assert_allclose(o1["rgb"], o2["rgb"], rtol=1e-12, atol=1e-14)


def test_linearity_in_exposure_intensity_albedo():
    """rgb is linear in exposure and in each light's intensity; with k_s = 0 it is
    linear in albedo."""
    b = S.config2(2, 1, 64)
    o = oracle.render(b)
    o_e = oracle.render(b.replace(exposure=b.exposure.astype(np.float64) * 2.5))
    np.testing.assert_allclose(o_e["rgb"], 2.5 * o["rgb"], rtol=1e-13, atol=1e-15)
    # intensities: rgb = sum of per-light images
    parts = []
    for k in range(b.n_lights):
        I = np.zeros(b.n_lights)
        I[k] = b.light_intensity[k]
        parts.append(oracle.render(b.replace(light_intensity=I))["rgb"])
    np.testing.assert_allclose(sum(parts), o["rgb"], rtol=1e-12, atol=1e-14)
    b0 = b.replace(specular=np.zeros_like(b.specular))
    o0 = oracle.render(b0)
    o3 = oracle.render(b0.replace(albedo=b0.albedo.astype(np.float64) * 3.0))
    np.testing.assert_allclose(o3["rgb"], 3.0 * o0["rgb"], rtol=1e-13, atol=1e-15)


def test_light_behind_surface_gives_black():
    """A directional light hitting the back of a camera-facing plane contributes 0."""
    b = _plane_batch(np.eye(3), (0, 0, -2.0), lights=((1, (0.2, 0.1, 1.0), 1.0),), spec=1.0, rough=0.3)
    out = oracle.render(b)
    assert np.any(out["tri_id"] >= 0)
    assert np.all(out["rgb"] == 0)


def test_background_channels():
    b = S.single_object_batch(S.box_mesh(1), S.make_pose(np.eye(3), (5.0, 0, -3.0), 0.2), res=(16, 16))
    out = oracle.render(b)
    assert np.all(out["tri_id"] == -1) and np.all(out["seg"] == -1)
    assert np.all(out["rgb"] == 0) and np.all(out["depth"] == 0) and np.all(out["normal"] == 0)
