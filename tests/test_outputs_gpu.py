"""GPU parity of the auxiliary outputs: the transparency channel, the Tracker records
(Sec. 4.4, Sec. 4.3.2) and the post-processed 3 x 8-bit RGB (Sec. 4.3.1
PostprocessingRandomizer, Sec. 5), through the C ABI, against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import parity

pytestmark = pytest.mark.gpu

TUNINGS = [None, (32, 32, 256, 0, 1), (16, 16, 512, 1, 1)]
TUNING_IDS = ["frame-path", "tiled", "tiled-persistent"]


@pytest.fixture(scope="module")
def renderer():
    import torch
    from paper_1906_11633_amd.renderer import Renderer
    assert torch.cuda.is_available()
    return Renderer(0)


def _render(renderer, batch, tuning=None):
    import torch
    from paper_1906_11633_amd.renderer import read_track
    job = renderer.prepare(batch)
    if tuning is not None:
        job.layout.set_tuning(*tuning)
    print(f"[outputs] {batch.name} frames={batch.n_frames} tuning={job.layout.info.tuning.as_tuple()}", flush=True)
    out = renderer.render(job, tri_id=True, alpha=True, rgb8=batch.post is not None, track=True, stats=True)
    torch.cuda.synchronize()
    res = parity.to_numpy({k: v for k, v in out.items() if k != "track"})
    res["track"] = read_track(out["track"])
    res["stats"] = out["stats"].cpu().numpy()
    return res


def _object_of_triangles(batch, tri_id):
    """Global object of each pixel's triangle (scene-local IDs run over the scene's
    objects in order), -1 for background."""
    po = batch.pixel_offset
    obj = np.full(tri_id.shape, -1, np.int32)
    for f in range(batch.n_frames):
        s = batch.frame_scene[f]
        t = tri_id[po[f]: po[f + 1]]
        base = 0
        for o in range(batch.scene_object_begin[s], batch.scene_object_begin[s + 1]):
            nt = batch.meshes[batch.object_mesh[o]].n_tris
            obj[po[f]: po[f + 1]][(t >= base) & (t < base + nt)] = o
            base += nt
    return obj


def _check_tracker(batch, gpu, ref):
    # Where the two nearest fragments are a near tie, the GPU's triangle is as valid as
    # the oracle's: take the records of the visibility the GPU chose (its tri_id is
    # bit-exact against the oracle's elsewhere), and the oracle's FP64 projections.
    mine = dict(ref)
    mine["obj_id"] = _object_of_triangles(batch, gpu["tri_id"])
    expect = oracle.track(batch, mine)
    t = gpu["track"]
    for k in ("count", "bbox", "sum_i", "sum_j"):
        assert np.array_equal(t[k], expect[k]), k
    o, e = t["origin"], expect["origin"]
    assert np.array_equal(np.isnan(o), np.isnan(e))
    fin = np.isfinite(e)
    np.testing.assert_allclose(o[fin], e[fin], rtol=1e-5, atol=1e-4)
    assert int(t["count"].sum()) == int((gpu["tri_id"] >= 0).sum())


@pytest.mark.parametrize("tuning", TUNINGS, ids=TUNING_IDS)
def test_alpha_and_tracker_config1(renderer, tuning):
    b = S.config1()
    gpu = _render(renderer, b, tuning)
    ref = oracle.render(b)
    parity.compare(b, gpu, ref)
    assert np.array_equal(gpu["alpha"], (gpu["tri_id"] >= 0).astype(np.float32))
    _check_tracker(b, gpu, ref)
    assert int(gpu["stats"][0]) == 0


@pytest.mark.parametrize("tuning", TUNINGS, ids=TUNING_IDS)
def test_tracker_config2_ragged_and_hidden(renderer, tuning):
    """Hand scenes at a ragged size (77 px: partial 64 x 4 tiles), with some objects
    hidden and one camera looking away from every object (empty frame)."""
    b = S.config2(2, 3, 77)
    vis = b.object_visible.copy()
    vis[::5] = 0
    view = b.view.copy()
    view[4, :, 3] += np.array([0.0, 0.0, 50.0], np.float32)  # everything behind the camera
    b = b.replace(object_visible=vis, view=view)
    gpu = _render(renderer, b, tuning)
    ref = oracle.render(b)
    parity.compare(b, gpu, ref)
    _check_tracker(b, gpu, ref)
    po = b.pixel_offset
    assert (gpu["tri_id"][po[4]: po[5]] < 0).all()


def _check_rgb8(batch, gpu, ref, band=1e-3):
    """8-bit codes: the oracle's FP64 post-processing of the GPU's own fp32 rgb must give
    the GPU's codes, except where the FP64 value lies within `band` of a rounding
    boundary (the fp32 chain's error is far below it); end to end against the oracle's
    FP64 rgb the codes differ by at most 1."""
    codes, v = oracle.postprocess(batch, gpu["rgb"].astype(np.float64), batch.post, batch.grain)
    near = np.abs((v - np.floor(v)) - 0.5) < band
    bad = (codes != gpu["rgb8"]) & ~near
    assert not bad.any(), (int(bad.sum()), np.nonzero(bad)[0][:8])
    codes2, _ = oracle.postprocess(batch, ref["rgb"], batch.post, batch.grain)
    assert np.abs(codes2.astype(int) - gpu["rgb8"].astype(int)).max() <= 1
    print("rgb8 near-boundary fraction", near.mean(), "end-to-end off-by-one", (codes2 != gpu["rgb8"]).mean(),
          flush=True)


@pytest.mark.parametrize("tuning", TUNINGS, ids=TUNING_IDS)
def test_rgb8_postprocessing_config2(renderer, tuning):
    b = S.with_postprocessing(S.config2(2, 2, 200), seed=5)
    gpu = _render(renderer, b, tuning)
    ref = oracle.render(b)
    parity.compare(b, gpu, ref)
    _check_rgb8(b, gpu, ref)


def test_rgb8_unaligned_sizes_identity_and_no_grain(renderer):
    """Widths that are not multiples of 4 (scalar byte stores), identity grading (the
    plain sRGB8 encoding) and a batch without a grain texture."""
    b = S.config2(3, 2, 77)
    b = b.replace(post=np.tile(np.array([0, 0, 0, 1, 1, 0, 0, 1, 0, 0, 0, 0], np.float32), (b.n_frames, 1)))
    gpu = _render(renderer, b)
    ref = oracle.render(b)
    _check_rgb8(b, gpu, ref)
    plain = np.floor(255 * oracle.srgb_encode(np.clip(gpu["rgb"].astype(np.float64), 0, 1)) + 0.5)
    v = 255 * oracle.srgb_encode(np.clip(gpu["rgb"].astype(np.float64), 0, 1))
    ok = np.abs(v - np.floor(v) - 0.5) >= 1e-3
    assert np.array_equal(plain[ok].astype(np.uint8), gpu["rgb8"][ok])


def test_rgb8_grain_on_unaligned_widths(renderer):
    """Grain on 77-pixel-wide frames: four-pixel groups that span two rows, so the
    grain texel is recomputed inside a group."""
    b = S.with_postprocessing(S.config2(3, 2, 77), seed=7)
    assert (b.post[:, 5] > 0).all() and (b.post[:, 7] > 1).any()
    gpu = _render(renderer, b)
    ref = oracle.render(b)
    _check_rgb8(b, gpu, ref)


FUSED = [
    ("config2-frame-path", lambda: S.with_postprocessing(S.config2(2, 2, 200), seed=5), None),
    ("config2-tiled", lambda: S.with_postprocessing(S.config2(2, 2, 200), seed=5), (32, 32, 256, 0, 1)),
    ("width77-frame-path", lambda: S.with_postprocessing(S.config2(3, 2, 77), seed=7), None),
    ("width77-tiled-persistent", lambda: S.with_postprocessing(S.config2(3, 2, 77), seed=7), (16, 16, 512, 1, 1)),
    ("uneven-one-launch", lambda: S.with_postprocessing(S.config3(3, 4), seed=3), (32, 32, 512, 0, 2)),
]


@pytest.mark.parametrize("name,make,tuning", FUSED, ids=[c[0] for c in FUSED])
def test_rgb8_alone_is_encoded_by_the_render_kernels(renderer, name, make, tuning):
    """rgb8 requested without the fp32 rgb (the paper's 3 x 8-bit format): the render
    kernels encode while writing, and give the same bytes as the separate pass that
    encodes a rendered fp32 rgb; the other channels are unchanged."""
    import torch
    b = make()
    job = renderer.prepare(b)
    if tuning is not None:
        job.layout.set_tuning(*tuning)
    print(f"[outputs] fused rgb8 {name} frames={b.n_frames} tuning={job.layout.info.tuning.as_tuple()}", flush=True)
    both = renderer.render(job, rgb8=True)
    alone = renderer.alloc_outputs(job, rgb8=True, base=("depth", "seg"))
    alone["rgb8"].fill_(0x5A)
    renderer.render(job, alone)
    torch.cuda.synchronize()
    for k in ("rgb8", "depth", "seg"):
        assert torch.equal(both[k], alone[k]), k
    if name == "config2-frame-path":  # and against the oracle
        gpu = parity.to_numpy(both)
        _check_rgb8(b, gpu, oracle.render(b))


def test_outputs_bit_identical_across_tunings(renderer):
    b = S.with_postprocessing(S.config2(4, 2, 96), seed=2)
    base = _render(renderer, b)
    for tuning in TUNINGS[1:]:
        other = _render(renderer, b, tuning)
        for k in ("alpha", "rgb8", "tri_id", "rgb"):
            assert np.array_equal(base[k], other[k]), (tuning, k)
        for k in ("count", "bbox", "sum_i", "sum_j"):
            assert np.array_equal(base["track"][k], other["track"][k]), (tuning, k)
        np.testing.assert_array_equal(base["track"]["origin"], other["track"]["origin"])
