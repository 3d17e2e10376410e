"""Pins of the oracle's auxiliary outputs (CPU only): the transparency channel and the
Tracker (Sec. 4.4, Sec. 4.3.2), and the post-processing / 8-bit encoding stage
(Sec. 4.3.1 PostprocessingRandomizer, Sec. 5's 3 x 8-bit RGB) against closed forms,
textbook values and invariants."""
import math

import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S


def _head_on_cube(off=(0.0, 0.0), D=3.1, res=64, fx=40.0):
    pose = S.make_pose(np.eye(3), (off[0], off[1], -D))
    intr = (fx, fx, res / 2, res / 2)
    return S.single_object_batch(S.box_mesh(1), pose, res=(res, res), intr=intr), intr


# ---------------------------------------------------------------- alpha, tracker

@pytest.mark.parametrize("off", [(0.0, 0.0), (0.3, 0.2), (-0.25, 0.35)])
def test_tracker_head_on_cube_closed_form(off):
    """A head-on cube covers the pixel centres strictly inside its projected front
    square: count, bounding box and index sums follow in closed form, and the origin
    (the cube's centre, D in front of the camera) projects to (cx + f x/D, cy - f y/D)."""
    D, res, fx = 3.1, 64, 40.0
    b, (fx, fy, cx, cy) = _head_on_cube(off, D, res, fx)
    out = oracle.render(b)
    t = oracle.track(b, out)
    zf = -float(b.object_pose[0, 2, 3]) - 0.5
    x0, x1 = cx + fx * (off[0] - 0.5) / zf, cx + fx * (off[0] + 0.5) / zf
    y0, y1 = cy - fy * (off[1] + 0.5) / zf, cy - fy * (off[1] - 0.5) / zf
    i = np.arange(res)
    cols = i[(i + 0.5 > x0) & (i + 0.5 < x1)]
    rows = i[(i + 0.5 > y0) & (i + 0.5 < y1)]
    assert t["count"][0] == cols.size * rows.size
    assert list(t["bbox"][0]) == [cols.min(), rows.min(), cols.max(), rows.max()]
    assert t["sum_i"][0] == cols.sum() * rows.size and t["sum_j"][0] == rows.sum() * cols.size
    Dz = -float(b.object_pose[0, 2, 3])
    ox = float(b.object_pose[0, 0, 3])
    oy = float(b.object_pose[0, 1, 3])
    np.testing.assert_allclose(t["origin"][0], [cx + fx * ox / Dz, cy - fy * oy / Dz, Dz], rtol=1e-12)
    alpha = out["alpha"].reshape(res, res)
    assert alpha.sum() == t["count"][0] and set(np.unique(alpha)) == {0.0, 1.0}


def test_tracker_origin_at_look_at_target_is_principal_point():
    """A LookAt camera aimed at an object's origin sees that origin at the principal
    point, at eye depth |eye - target|, whatever the camera's rotation."""
    target = np.array([0.12, -0.07, 0.05])
    eye = np.array([0.7, -0.9, 0.6])
    V = S.view_from_c2w(S.look_at_c2w(eye, target, (0, 0, 1)))
    b = S.single_object_batch(S.box_mesh(2), S.make_pose(S.rot_axis("z", 0.3), target, 0.2), res=(48, 40), view=V)
    t = oracle.track(b, oracle.render(b))
    K = b.intr[0].astype(np.float64)
    tgt = b.object_pose[0, :, 3].astype(np.float64)
    Vd = b.view[0].astype(np.float64)
    cam = -Vd[:, :3].T @ Vd[:, 3]  # camera centre in world space
    np.testing.assert_allclose(t["origin"][0, :2], K[2:], atol=1e-5)
    np.testing.assert_allclose(t["origin"][0, 2], np.linalg.norm(tgt - cam), rtol=1e-6)
    assert t["count"][0] > 0


def test_tracker_behind_camera_and_hidden_object():
    """An object behind the camera has w < 0 and NaN screen coordinates; a hidden
    object has no pixels (empty box markers) but its origin is still reported."""
    mesh = S.box_mesh(1)
    b = S.single_object_batch(mesh, S.make_pose(np.eye(3), (0, 0, 2.0)), res=(32, 32),
                              extra_objects=((mesh, S.make_pose(np.eye(3), (0.1, 0, -3.0))),))
    b = b.replace(object_visible=np.array([1, 0], np.uint8))
    t = oracle.track(b, oracle.render(b))
    assert t["origin"][0, 2] == -2.0 and np.isnan(t["origin"][0, :2]).all()
    assert t["count"][1] == 0 and list(t["bbox"][1]) == [oracle.TRACK_EMPTY_MIN] * 2 + [-1, -1]
    assert t["origin"][1, 2] == 3.0 and np.isfinite(t["origin"][1, :2]).all()


def test_tracker_invariants_config1():
    """Per frame: the objects' counts add up to the covered pixels; each object's pixels
    (its triangle-ID range, derived here from the mesh sizes, not from obj_id) lie in its
    box, touch all four sides of it, and give its index sums."""
    b = S.config1()
    out = oracle.render(b)
    t = oracle.track(b, out)
    po = out["pixel_offset"]
    row = 0
    for f in range(b.n_frames):
        s = b.frame_scene[f]
        W, H = int(b.width[f]), int(b.height[f])
        tri = out["tri_id"][po[f]: po[f] + W * H].reshape(H, W)
        objs = range(b.scene_object_begin[s], b.scene_object_begin[s + 1])
        base = 0
        total = 0
        for o in objs:
            nt = b.meshes[b.object_mesh[o]].n_tris
            jj, ii = np.nonzero((tri >= base) & (tri < base + nt))
            base += nt
            assert t["count"][row] == ii.size
            total += ii.size
            if ii.size:
                assert list(t["bbox"][row]) == [ii.min(), jj.min(), ii.max(), jj.max()]
                assert t["sum_i"][row] == ii.sum() and t["sum_j"][row] == jj.sum()
            row += 1
        assert total == (tri >= 0).sum()
    assert row == t["count"].shape[0]


# ---------------------------------------------------------------- post-processing

def _identity_post(n_frames):
    p = np.zeros((n_frames, oracle.POST_WORDS), np.float32)
    p[:, 3] = p[:, 4] = p[:, 7] = 1.0
    return p


def _flat_batch(W=8, H=4):
    b = S.single_object_batch(S.box_mesh(1), S.make_pose(np.eye(3), (0, 0, -3.0)), res=(W, H))
    return b


def test_srgb_transfer_textbook_values():
    """IEC 61966-2-1: linear 0.18 -> 0.46136, 0.5 -> 0.73536, 0.2140 -> 0.5,
    continuity at the 0.0031308 knee (0.04045), and the end points."""
    e = oracle.srgb_encode([0.0, 0.0031308, 0.18, 0.5, 0.21404114, 1.0])
    np.testing.assert_allclose(e, [0.0, 0.040449936, 0.46135613, 0.73535698, 0.5, 1.0], atol=2e-8)


def test_identity_grading_is_plain_srgb8():
    """With identity parameters and no grain the codes are round(255 sRGB(clamp(x)))."""
    b = _flat_batch()
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.2, 1.4, 3 * b.total_pixels)
    codes, v = oracle.postprocess(b, x, _identity_post(1))
    codes2, _ = oracle.postprocess(b, x, None)
    expect = np.floor(255 * oracle.srgb_encode(np.clip(x, 0, 1)) + 0.5)
    assert np.array_equal(codes, expect.astype(np.uint8)) and np.array_equal(codes, codes2)
    assert codes[x >= 1].min() == 255 and codes[x <= 0].max() == 0


@pytest.mark.parametrize("turns, perm", [(1, (2, 0, 1)), (-1, (1, 2, 0)), (3, (0, 1, 2))])
def test_hue_rotation_by_thirds_permutes_channels(turns, perm):
    """Rotating colours by 120 degrees about the grey axis cycles the channels exactly
    (r -> g -> b for +120 degrees); a full turn is the identity."""
    b = _flat_batch()
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 1.0, 3 * b.total_pixels)
    p = _identity_post(1)
    p[0, 2] = turns * 2 * math.pi / 3
    _, v = oracle.postprocess(b, x, p)
    _, v0 = oracle.postprocess(b, x, None)
    P = b.total_pixels
    # the angle is stored in fp32 (within 2e-7 of a multiple of 2 pi/3)
    np.testing.assert_allclose(v.reshape(3, P), v0.reshape(3, P)[list(perm)], atol=1e-4)


def test_zero_saturation_gives_rec709_luma_and_zero_contrast_gives_mid_grey():
    b = _flat_batch()
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, 3 * b.total_pixels)
    P = b.total_pixels
    p = _identity_post(1)
    p[0, 3] = 0.0
    _, v = oracle.postprocess(b, x, p)
    e = oracle.srgb_encode(x.reshape(3, P))
    Y = 0.2126 * e[0] + 0.7152 * e[1] + 0.0722 * e[2]
    for c in range(3):
        np.testing.assert_allclose(v.reshape(3, P)[c], 255 * Y, atol=1e-9)
    p = _identity_post(1)
    p[0, 4] = 0.0
    codes, v = oracle.postprocess(b, x, p)
    assert np.all(v == 127.5) and np.all(codes == 128)  # floor(127.5 + 0.5)


def test_white_balance_orders_grey_channels():
    """A warm temperature (T > 0) makes a grey pixel red > green > blue; a positive tint
    removes green (magenta cast, red = blue > green)."""
    b = _flat_batch()
    x = np.full(3 * b.total_pixels, 0.3)
    P = b.total_pixels
    p = _identity_post(1)
    p[0, 0] = 0.8
    _, v = oracle.postprocess(b, x, p)
    v = v.reshape(3, P)
    assert np.all(v[0] > v[1]) and np.all(v[1] > v[2])
    p = _identity_post(1)
    p[0, 1] = 0.8
    _, v = oracle.postprocess(b, x, p)
    v = v.reshape(3, P)
    assert np.all(v[0] == v[2]) and np.all(v[1] < v[0])


def test_grain_shift_coloration_size_and_wrap():
    """Grain adds I((1 - kappa) g0 + kappa gc - 1/2): a texture of 1/2 adds nothing; with
    kappa = 0 every channel gets the plane-0 value; with kappa = 1 each its own plane; the
    noise is constant over S x S pixel blocks and repeats every GW S pixels."""
    W, H = 40, 12
    b = _flat_batch(W, H)
    P = W * H
    x = np.full(3 * P, 0.2)
    _, v0 = oracle.postprocess(b, x, None)
    g = np.full((3, 4, 5), 0.5, np.float32)
    p = _identity_post(1)
    p[0, 5] = 0.1
    _, v = oracle.postprocess(b, x, p, g)
    assert np.array_equal(v, v0)
    rng = np.random.default_rng(6)
    g = rng.uniform(0, 1, (3, 4, 5)).astype(np.float32)
    for kap in (0.0, 1.0):
        p[0, 6] = kap
        p[0, 7] = 2.0
        p[0, 8], p[0, 9] = 3.0, 1.0
        _, v = oracle.postprocess(b, x, p, g)
        d = (v - v0).reshape(3, H, W)
        if kap == 0.0:
            assert np.allclose(d[0], d[1]) and np.allclose(d[1], d[2])
        else:
            assert not np.allclose(d[0], d[1])
        # blocks of 2 x 2 pixels share one texel; period 5 texels x 2 px = 10 px in x, 8 px in y
        assert np.allclose(d[:, ::2, ::2], d[:, 1::2, 1::2])
        assert np.allclose(d[:, :, :30], d[:, :, 10:40]) and np.allclose(d[:, :4], d[:, 8:12])
        # texel (0, 0) is used by the 2 x 2 block with i div 2 = 2 (2 + 3 = 0 mod 5) and j div 2 = 3
        gc = g[0, 0, 0] if kap == 0.0 else g[:, 0, 0]
        np.testing.assert_allclose(d[:, 6, 4], 255 * 0.1 * (np.asarray(gc) - 0.5) * np.ones(3), atol=1e-9)
