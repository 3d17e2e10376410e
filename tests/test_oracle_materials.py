"""Pins of the oracle's materials (CPU only): pattern textures with tiling and offset
(Sec. 4.3.1 MaterialRandomizer), emission, and the fixed-hue HSV sampler (Sec. 4.3.1
FixedHueMaterialRandomizer), against the hexcone HSV model, the exact texel a pixel
centre lands on, bilinear weights, periodicity and the untextured render."""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S

RES = 64


def _plane(tex, xform=(1, 1, 0, 0), emission=None, intensity=1.0):
    """A 2 x 2 m plane (4 x 4 quads) facing the camera 2 m away, seen by a 64 x 64 camera
    with f = 64: pixel centre (i, j) sees u = (i + 1/2)/64, v = 1 - (j + 1/2)/64 exactly."""
    b = S.single_object_batch(S.plane_mesh(4, 4, 2.0, 2.0), S.make_pose(np.eye(3), (0, 0, -2.0)), res=(RES, RES),
                              intr=(64.0, 64.0, 32.0, 32.0), albedo=(0.9, 0.7, 0.5),
                              lights=((1, (0, 0, -1), intensity),))
    return b.replace(textures=[np.asarray(tex, np.float32)], object_texture=np.array([0], np.int32),
                     tex_xform=np.asarray([xform], np.float32),
                     emission=None if emission is None else np.asarray([emission], np.float32))


def _rgb(b, out):
    return oracle.frame_view(out["rgb"], out["pixel_offset"], 0, RES, RES, 3).transpose(1, 2, 0)


def test_hsv_hexcone_values():
    for hsv, rgb in [((0, 1, 1), (1, 0, 0)), ((1 / 3, 1, 1), (0, 1, 0)), ((2 / 3, 1, 1), (0, 0, 1)),
                     ((1 / 6, 1, 1), (1, 1, 0)), ((0.5, 1, 0.5), (0, 0.5, 0.5)), ((0.3, 0, 0.7), (0.7, 0.7, 0.7)),
                     ((1.0, 1, 1), (1, 0, 0))]:
        np.testing.assert_allclose(S.hsv_to_rgb(*hsv), rgb, atol=1e-12)


def test_fixed_hue_sampler_stays_in_radius_and_clamps():
    rng = np.random.default_rng(0)
    base, rad, lo, hi = (0.1, 0.7, 0.6), (0.05, 0.2, 0.3), (0.0, 0.0, 0.5), (1.0, 0.8, 0.8)
    import colorsys
    for _ in range(200):
        a, r, k, e = S.fixed_hue_material(rng, base, rad, lo, hi, glossiness=(0.2, 0.6), emissive_prob=0.5,
                                          emissive_power=(1.0, 2.0))
        h, s, v = colorsys.rgb_to_hsv(*a)
        dh = min(abs(h - base[0]), 1 - abs(h - base[0]))
        assert dh <= rad[0] + 1e-9 and lo[1] - 1e-9 <= s <= hi[1] + 1e-9 and lo[2] - 1e-9 <= v <= hi[2] + 1e-9
        assert 0.4 <= r <= 0.8 and (e == 0 or 1.0 <= e <= 2.0)


def test_pixel_centres_on_texel_centres_show_the_texels():
    """With a 64 x 64 texture each pixel centre lands on a texel centre: the render is the
    Lambert plane times that texel (texture rows run with v, image rows against it)."""
    tex = np.random.default_rng(1).uniform(0, 1, (64, 64, 3))
    b = _plane(tex)
    rgb = _rgb(b, oracle.render(b))
    expect = np.asarray(b.albedo[0], np.float64) * tex.astype(np.float32).astype(np.float64)[::-1, :, :]
    np.testing.assert_allclose(rgb, expect, rtol=1e-12, atol=1e-13)


def test_bilinear_weights_quarter_texel():
    """A 32 x 32 texture puts each pixel centre a quarter texel from a texel centre: the
    sample is 3/4 of the nearer texel and 1/4 of the next one, in each axis."""
    tex = np.random.default_rng(2).uniform(0, 1, (32, 32, 3)).astype(np.float32).astype(np.float64)
    b = _plane(tex)
    rgb = _rgb(b, oracle.render(b)) / np.asarray(b.albedo[0], np.float64)
    i = np.arange(RES)
    x = (i + 0.5) / 64 * 32 - 0.5  # texel coordinate of pixel column i
    k0 = np.floor(x).astype(int)
    w = x - k0
    assert set(np.round(w, 6)) == {0.25, 0.75}
    j = 5
    y = (1 - (j + 0.5) / 64) * 32 - 0.5
    l0 = int(np.floor(y))
    wy = y - l0
    row = (1 - wy) * tex[l0 % 32] + wy * tex[(l0 + 1) % 32]
    expect = (1 - w)[:, None] * row[k0 % 32] + w[:, None] * row[(k0 + 1) % 32]
    np.testing.assert_allclose(rgb[j], expect, rtol=1e-12, atol=1e-13)


def test_tiling_and_offset_are_periodic_shifts():
    """u' = 2 u + 1/4 repeats every 32 pixels; an offset of 1/2 at tiling 1 shifts the
    image by 32 columns (wrapping)."""
    tex = np.random.default_rng(3).uniform(0, 1, (16, 16, 3))
    tiled = _rgb(None, oracle.render(_plane(tex, (2, 1, 0.25, 0))))
    np.testing.assert_allclose(tiled[:, :32], tiled[:, 32:], rtol=1e-12, atol=1e-13)
    base = _rgb(None, oracle.render(_plane(tex, (1, 1, 0, 0))))
    shifted = _rgb(None, oracle.render(_plane(tex, (1, 1, 0.5, 0))))
    np.testing.assert_allclose(shifted, np.roll(base, -32, axis=1), rtol=1e-12, atol=1e-13)
    # the offset applies after the tiling: at tiling 2 an offset of 1/4 is 8 columns
    t2 = _rgb(None, oracle.render(_plane(tex, (2, 1, 0, 0))))
    t2o = _rgb(None, oracle.render(_plane(tex, (2, 1, 0.25, 0))))
    np.testing.assert_allclose(t2o, np.roll(t2, -8, axis=1), rtol=1e-12, atol=1e-13)


def test_white_texture_is_the_untextured_render():
    b = _plane(np.ones((8, 8, 3)))
    plain = b.replace(textures=None, object_texture=None, tex_xform=None)
    np.testing.assert_allclose(oracle.render(b)["rgb"], oracle.render(plain)["rgb"], rtol=1e-15)


def test_emission_adds_power_times_albedo():
    """Without light, an emissive textured plane shows exposure x power x albedo x texel."""
    tex = np.random.default_rng(4).uniform(0, 1, (64, 64, 3))
    b = _plane(tex, emission=0.6, intensity=0.0)
    rgb = _rgb(b, oracle.render(b))
    expect = np.float32(0.6) * np.asarray(b.albedo[0], np.float64) * tex.astype(np.float32).astype(np.float64)[::-1]
    np.testing.assert_allclose(rgb, expect, rtol=1e-12, atol=1e-13)
    lit = _rgb(b, oracle.render(b.replace(light_intensity=np.array([1.0], np.float32))))
    no_em = _rgb(b, oracle.render(b.replace(light_intensity=np.array([1.0], np.float32), emission=None)))
    np.testing.assert_allclose(lit - no_em, expect, rtol=1e-10, atol=1e-12)


def test_generators_give_uvs_in_range():
    for m in (S.capsule_mesh(0.02, 0.08), S.box_mesh(3), S.plane_mesh(3, 2)):
        assert m.uv is not None and m.uv.shape == (m.n_verts, 2)
        assert m.uv.min() >= 0 and m.uv.max() <= 1


def test_adjoint_rejects_textured_materials():
    b = _plane(np.ones((4, 4, 3)))
    with pytest.raises(ValueError):
        oracle.shade_grad(b, np.zeros(3 * b.total_pixels))
