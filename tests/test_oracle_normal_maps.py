"""Pins of the oracle's normal (bump) textures (CPU only; Sec. 4.3.1 MaterialRandomizer:
random pattern and normal textures with tiling and offset).  A flat plane facing the
camera, its UVs running with +x and +y, lit by one directional light without specular:
the shading normal is the decoded texel expressed in the (x, y, z) frame, so the render
is albedo * I * max(0, n'.l) in closed form; mirrored UVs flip the bitangent, flat maps
and degenerate UVs change nothing, and the normal channel keeps the geometric normal."""
import math

import numpy as np

import oracle
from paper_1906_11633_amd import scenes as S

RES = 64
ALB = (0.9, 0.7, 0.5)


def _plane(ntex, light_dir=(0.0, 0.0, 1.0), mesh=None, xform=(1, 1, 0, 0)):
    """A 2 x 2 m plane 2 m in front of a 64 x 64 camera (f = 64): pixel centre (i, j) sees
    u = (i + 1/2)/64, v = 1 - (j + 1/2)/64; one directional light towards light_dir."""
    d = np.asarray(light_dir, float)
    d = d / np.linalg.norm(d)
    m = mesh if mesh is not None else S.plane_mesh(4, 4, 2.0, 2.0)
    b = S.single_object_batch(m, S.make_pose(np.eye(3), (0, 0, -2.0)), res=(RES, RES),
                              intr=(64.0, 64.0, 32.0, 32.0), albedo=ALB, lights=((1, tuple(-d), 1.0),))
    if ntex is None:
        return b
    return b.replace(textures=[np.asarray(ntex, np.float32)], object_texture=np.array([-1], np.int32),
                     object_normal_texture=np.array([0], np.int32), tex_xform=np.asarray([xform], np.float32))


def _towards(ld):
    """The direction to the light as the render sees it: the stored (fp32) propagation
    direction, negated and normalized."""
    d = np.asarray(ld, float)
    d = -np.float32(-d / np.linalg.norm(d)).astype(np.float64)
    return d / np.linalg.norm(d)


def _rgb(out):
    return oracle.frame_view(out["rgb"], out["pixel_offset"], 0, RES, RES, 3).transpose(1, 2, 0)


def _encode(n):
    n = np.asarray(n, float)
    return ((n / np.linalg.norm(n, axis=-1, keepdims=True) + 1) / 2).astype(np.float32)


def test_flat_map_changes_nothing():
    flat = np.broadcast_to(_encode([0, 0, 1]), (8, 8, 3))
    for ld in [(0, 0, 1), (0.3, -0.2, 1)]:
        a = _rgb(oracle.render(_plane(flat, ld)))
        b = _rgb(oracle.render(_plane(None, ld)))
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


def test_tilt_along_u_follows_the_tangent():
    """A constant map tilted by a towards +t (the +u direction, world +x): under a light
    tilted by b in the x-z plane the diffuse term is cos(a - b)."""
    for a, b in [(0.3, 0.0), (0.3, 0.5), (0.3, -0.4), (-0.5, 0.2)]:
        tex = np.broadcast_to(_encode([math.sin(a), 0, math.cos(a)]), (4, 4, 3))
        rgb = _rgb(oracle.render(_plane(tex, (math.sin(b), 0, math.cos(b)))))
        t = np.float32(_encode([math.sin(a), 0, math.cos(a)])).astype(np.float64) * 2 - 1
        t /= np.linalg.norm(t)
        l = _towards((math.sin(b), 0, math.cos(b)))
        expect = np.asarray(ALB, np.float32).astype(np.float64) * max(0.0, t @ l)
        np.testing.assert_allclose(rgb.reshape(-1, 3), np.broadcast_to(expect, (RES * RES, 3)), rtol=1e-12)


def test_tilt_along_v_follows_the_bitangent_and_mirrored_uvs_flip_it():
    """Tilting towards +v goes to world +y; with v mirrored (v' = 1 - v) it goes to -y."""
    a, b = 0.4, 0.3
    tex = np.broadcast_to(_encode([0, math.sin(a), math.cos(a)]), (4, 4, 3))
    t = np.float32(_encode([0, math.sin(a), math.cos(a)])).astype(np.float64) * 2 - 1
    t /= np.linalg.norm(t)
    alb = np.asarray(ALB, np.float32).astype(np.float64)
    l = _towards((0, math.sin(b), math.cos(b)))
    rgb = _rgb(oracle.render(_plane(tex, (0, math.sin(b), math.cos(b)))))
    np.testing.assert_allclose(rgb[10, 10], alb * (t[1] * l[1] + t[2] * l[2]), rtol=1e-12)
    m = S.plane_mesh(4, 4, 2.0, 2.0)
    mir = S.Mesh(m.pos, m.nrm, m.idx, np.stack([m.uv[:, 0], 1 - m.uv[:, 1]], 1).astype(np.float32))
    rgb = _rgb(oracle.render(_plane(tex, (0, math.sin(b), math.cos(b)), mesh=mir)))
    np.testing.assert_allclose(rgb[10, 10], alb * (-t[1] * l[1] + t[2] * l[2]), rtol=1e-12)


def test_tangent_turns_with_the_pose():
    """The plane turned 90 degrees about its normal: +u now runs along world +y, so a map
    tilted towards +u leans towards +y."""
    a, b = 0.35, 0.25
    tex = np.broadcast_to(_encode([math.sin(a), 0, math.cos(a)]), (4, 4, 3))
    t = np.float32(_encode([math.sin(a), 0, math.cos(a)])).astype(np.float64) * 2 - 1
    t /= np.linalg.norm(t)
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    b0 = _plane(tex, (0, math.sin(b), math.cos(b)))
    bt = b0.replace(object_pose=np.asarray([S.make_pose(Rz, (0, 0, -2.0))], np.float32))
    l = _towards((0, math.sin(b), math.cos(b)))
    rgb = _rgb(oracle.render(bt))
    np.testing.assert_allclose(rgb[20, 20], np.asarray(ALB, np.float32).astype(np.float64) * (t[0] * l[1] + t[2] * l[2]),
                               rtol=1e-12)


def test_bump_texture_pixel_by_pixel():
    """A random 64 x 64 bump texture: each pixel centre lands on a texel centre, so pixel
    (i, j) is lit with the texel of column i and row 63 - j, decoded and normalized."""
    tex = S.bump_texture(np.random.default_rng(3))
    ld = np.array([0.2, -0.3, 1.0])
    rgb = _rgb(oracle.render(_plane(tex, ld)))
    ld = _towards(ld)
    t = tex.astype(np.float64)[::-1] * 2 - 1
    t /= np.linalg.norm(t, axis=-1, keepdims=True)
    expect = np.asarray(ALB, np.float32).astype(np.float64) * np.maximum(0, t @ ld)[..., None]
    np.testing.assert_allclose(rgb, expect, rtol=1e-11, atol=1e-13)
    assert np.std(t @ ld) > 0.05  # the texture does perturb the shading


def test_degenerate_uvs_and_normal_channel():
    """Zero UV area leaves the normal unchanged; the normal channel is the geometric one."""
    tex = np.broadcast_to(_encode([0.5, 0.2, 0.8]), (4, 4, 3))
    m = S.plane_mesh(4, 4, 2.0, 2.0)
    flat_uv = S.Mesh(m.pos, m.nrm, m.idx, np.full_like(m.uv, 0.25))
    ld = (0.3, 0.1, 1.0)
    a = oracle.render(_plane(tex, ld, mesh=flat_uv))
    b = oracle.render(_plane(None, ld, mesh=flat_uv))
    np.testing.assert_allclose(_rgb(a), _rgb(b), rtol=1e-12)
    c = oracle.render(_plane(tex, ld))
    assert not np.allclose(_rgb(c), _rgb(b))
    np.testing.assert_array_equal(c["normal"], b["normal"])


def test_hand_scene_flat_maps_match_untextured():
    """On the curved capsules of a hand scene (tangents from their UVs) a flat normal map
    gives the untextured render."""
    base = S.config2(4, 1, 64)
    flat = np.broadcast_to(_encode([0, 0, 1]), (4, 4, 3)).copy()
    O = base.n_objects
    b = base.replace(textures=[flat], object_texture=np.full(O, -1, np.int32),
                     object_normal_texture=np.zeros(O, np.int32),
                     tex_xform=np.tile(np.array([1, 1, 0, 0], np.float32), (O, 1)))
    np.testing.assert_allclose(oracle.render(b)["rgb"], oracle.render(base)["rgb"], rtol=1e-11, atol=1e-14)


def test_adjoint_rejects_normal_textures():
    import pytest
    b = _plane(np.broadcast_to(_encode([0, 0, 1]), (4, 4, 3)))
    with pytest.raises(ValueError):
        oracle.shade_grad(b, np.zeros(3 * b.total_pixels))
